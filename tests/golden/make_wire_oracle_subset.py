"""Writes wire_oracle_subset.txt: the FP64 oracle's replay of every 2nd
avalanche (ids 0, 2, ..., 2046) of the wire-chamber workload (argon-like
gas, 25 um wire in a 5 mm tube at 1500 V as a 512 x 64 polar map, 0.5 T
along the wire, primaries at rest at rho = 1 mm; seed 5), run to
termination with the banded majorant (100-bin bands, helical bound,
lookahead 1).  One line per avalanche: id, electrons (gain), electrons
that reached the wire, and over those the summed arrival times t1, the
summed drift times t1 - t0 and the summed radial displacements
rho0 - rho1 (mean arrival time; radial drift velocity).  Calls only the oracle and the seeded input description.

    python tests/golden/make_wire_oracle_subset.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2509_15377_amd import workloads as W  # noqa: E402

MODULUS = 2
OUT = os.path.join(HERE, "wire_oracle_subset.txt")


def main():
    wl = W.wire(band_bins=100)
    idx = W.subset_primaries(wl.primaries, MODULUS)
    t = time.time()
    ep = O.run(O.Gas(wl.gas, band_bins=100), wl.field, wl.primaries[idx], wl.seed, banded=True,
               ids=idx, band_lookahead=1.0)
    dt = time.time() - t
    avals = wl.primaries["aval"][idx]
    n = np.bincount(ep["aval"], minlength=wl.n_aval)
    w = ep["status"] == 4
    nw = np.bincount(ep["aval"][w], minlength=wl.n_aval)
    t1 = np.bincount(ep["aval"][w], weights=ep["t1"][w], minlength=wl.n_aval)
    st = np.bincount(ep["aval"][w], weights=(ep["t1"] - ep["t0"])[w], minlength=wl.n_aval)
    r0 = np.hypot(ep["x0"], ep["y0"])
    r1 = np.hypot(ep["x1"], ep["y1"])
    sr = np.bincount(ep["aval"][w], weights=(r0 - r1)[w], minlength=wl.n_aval)
    with open(OUT, "w") as fh:
        fh.write(f"# FP64 oracle, wire chamber, avalanches with id % {MODULUS} == 0, banded (100 bins), "
                 "lookahead 1, seed 5; written by make_wire_oracle_subset.py\n")
        fh.write("# aval electrons at_wire sum_t1_ns sum_t1_minus_t0_ns sum_rho0_minus_rho1_cm\n")
        for a in avals:
            fh.write(f"{a} {n[a]} {nw[a]} {t1[a]:.17g} {st[a]:.17g} {sr[a]:.17g}\n")
    print(f"{avals.size} avalanches, {ep.size} electrons, {dt:.0f} s")


if __name__ == "__main__":
    main()
