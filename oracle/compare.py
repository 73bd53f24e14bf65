"""Per-trajectory comparison of an endpoint set against the oracle's.

TEST INFRASTRUCTURE ONLY.  Both inputs are numpy structured arrays with the
136-byte endpoint layout (fields x0..e1, eid, parent, aval, status, the
per-electron counters and the decision trace); nothing here imports the HIP
package.

Electrons are joined on their id (primaries 2^63 | index, secondaries a
63-bit id drawn from the parent's random stream), which is unique within a
run with overwhelming probability.  A matched electron is

* a *decision flip* when its own decisions differ from the oracle's: its
  decision trace (a hash over its real collisions, masked nulls and band
  cuts, with their flight indices and channels), a counter, its status or
  its parent differ.  Rounding can flip a decision whose margin is within
  a few ulps; the descendants of a flipped electron carry different ids and
  show up as unmatched, not as flips.
* a *coordinate mismatch* (drift) when its decisions are the same but a
  start or end coordinate differs by more than the tolerance (|d| <= rtol *
  max(|ref|, floor), floors 1e-4 cm, 1e-3 ns, 1e-3 eV).  With the same
  decisions the arithmetic between them is the same up to rounding, but
  ulp-level differences are not always damped along a trajectory: the
  oracle against its own build with fused multiply-adds
  (tests/test_oracle_rounding.py) shows, with the global majorant (tens of
  thousands of flights per electron), about one electron in 1e5 drifting
  past 1e-9 with every decision the same.  Some endpoints are also
  ill-conditioned: a secondary born 1.5e-9 cm below the anode (argon-like
  gas, 40 kV/cm) gains E (z_hi - z0) = 6e-5 eV on its way out, so a
  difference of 3e-17 cm in its birth height (some twenty ulps, carried
  from its parent's flights) is 1.2e-12 eV in its final energy, past
  1e-9 of the 1e-3 eV floor.  Both are rounding-induced deviations with
  identical decisions; they share the 0.1 % budget of the flips and are
  bounded on their own by max_drift_fraction.
"""
from __future__ import annotations

import numpy as np

FLOORS = {"x0": 1e-4, "y0": 1e-4, "z0": 1e-4, "t0": 1e-3, "e0": 1e-3,
          "x1": 1e-4, "y1": 1e-4, "z1": 1e-4, "t1": 1e-3, "e1": 1e-3}
DECISIONS = ("aval", "status", "n_real", "n_ion", "n_null", "n_masked", "n_band", "n_overflow",
             "parent", "trace")


def compare(got, ref, rtol=1e-9):
    g_eid = got["eid"]
    r_eid = ref["eid"]
    if np.unique(g_eid).size != g_eid.size or np.unique(r_eid).size != r_eid.size:
        raise AssertionError("duplicate electron ids inside one run")
    common, gi, ri = np.intersect1d(g_eid, r_eid, assume_unique=True, return_indices=True)
    G = got[gi]
    R = ref[ri]
    flip = np.zeros(common.size, dtype=bool)
    for f in DECISIONS:
        flip |= G[f] != R[f]
    coord_bad = np.zeros(common.size, dtype=bool)
    max_rel = {}
    for f, floor in FLOORS.items():
        d = np.abs(G[f] - R[f])
        scale = np.maximum(np.abs(R[f]), floor)
        rel = d / scale
        same = rel[~flip]
        max_rel[f] = float(same.max()) if same.size else 0.0
        coord_bad |= ~(rel <= rtol)
    mismatch = coord_bad & ~flip
    n_match = int(common.size)
    return {
        "n_got": int(got.size), "n_ref": int(ref.size), "matched": n_match,
        "unmatched_got": int(got.size - n_match), "unmatched_ref": int(ref.size - n_match),
        "flips": int(flip.sum()), "flip_fraction": float(flip.sum() / max(n_match, 1)),
        "coord_mismatches": int(mismatch.sum()),
        "max_rel": max_rel,
        "flipped_eids": common[flip][:20].tolist(),
        "mismatched_eids": common[mismatch][:20].tolist(),
    }


def assert_parity(got, ref, rtol=1e-9, max_flip_fraction=1e-3, max_unmatched_fraction=0.01,
                  max_flips=None, max_drift_fraction=1e-4):
    """Decision flips and coordinate drifts (same decisions, a coordinate
    beyond rtol) together: below max_flip_fraction of the matched
    electrons; drifts alone at most max_drift_fraction; flips at most
    max_flips when given (0 where a path reproduces every decision)."""
    rep = compare(got, ref, rtol)
    assert rep["n_ref"] > 0
    drift = rep["coord_mismatches"] / max(rep["matched"], 1)
    assert drift <= max_drift_fraction, rep
    assert rep["flip_fraction"] + drift < max_flip_fraction, rep
    if max_flips is not None:
        assert rep["flips"] <= max_flips, rep
    unm = max(rep["unmatched_got"], rep["unmatched_ref"]) / rep["n_ref"]
    assert unm <= max_unmatched_fraction, rep
    if rep["flips"] == 0:
        # with no flip there is nothing to explain unmatched electrons by
        assert rep["unmatched_got"] == 0 and rep["unmatched_ref"] == 0, rep
    return rep
