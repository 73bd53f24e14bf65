"""FP32-mixed against FP64 on the wire chamber: the benchmark's batched
FP32-mixed workload with a polar field map (argon-like gas, 25 um wire in
a 5 mm tube at 1500 V, 512 x 64 map), 0.5 T along the wire and the
helical band bound, 2048 avalanches from primaries at rest at rho = 1 mm.

In this geometry rounding differences grow exponentially along a
trajectory, so the FP32 and FP64 runs of one seed decorrelate long before
the electrons reach the wire (paired correlation of the per-avalanche
gains ~0): the two precisions are independent samples, and with a
per-avalanche gain spread of ~0.89 of its mean, the 1 % gate on the mean
gain needs of order 1e5 avalanches per precision (NSEEDS seeds of the
2048-avalanche workload).  Gates (as for the slab workloads): mean gain
within 1 %, radial drift velocity within 0.5 %, KS p > 0.01 on the
per-avalanche gain and mean arrival time and on the arrival time, energy
and axial position of one electron per avalanche (the one with the
smallest id: independent samples).  Both precisions are also compared in
distribution with the FP64 oracle's replay of every 2nd avalanche of
seed 5, run to termination (tests/golden/wire_oracle_subset.txt)."""
import math
import os

import numpy as np
import pytest
from scipy import stats

from paper_2509_15377_amd import workloads as W

pytestmark = pytest.mark.gpu

NSEEDS = 48
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "wire_oracle_subset.txt")


@pytest.fixture(scope="module")
def A():
    from paper_2509_15377_amd import avm
    if avm.device_count() < 1:
        pytest.fail("no HIP device visible: the GPU tests need an MI355X")
    return avm


def _per_avalanche(A, r, n_aval):
    """Per-avalanche gain; over the electrons that reached the wire, their
    number and summed arrival times t1, drift times t1 - t0 and radial
    displacements; and the arrival time, energy and z of the avalanche's
    secondary with the smallest id (ids are random draws: a random
    electron).  Reduced on the device."""
    import torch
    gain = r.avalanche_counts()["n_endpoints"].astype(np.float64)
    t = r.endpoint_tensors(("t0", "t1", "x0", "y0", "x1", "y1", "z1", "e1", "eid", "avalanche", "status"))
    a = t["avalanche"].long()
    w = t["status"] == 4
    zeros = torch.zeros(n_aval, dtype=torch.int64, device="cuda")

    def fixed_sum(v, unit):
        # per-avalanche sums over the wire arrivals in int64 fixed point
        # (exact; the device's float64 scatter-add is slow under contention)
        q = torch.where(w, torch.round(v / unit), torch.zeros_like(v)).long()
        return zeros.index_add(0, a, q).double().cpu().numpy() * unit

    n_w = zeros.index_add(0, a, w.long()).cpu().numpy().astype(np.float64)
    s_t1 = fixed_sum(t["t1"], 1e-9)
    s_t = fixed_sum(t["t1"] - t["t0"], 1e-9)
    s_r = fixed_sum(torch.hypot(t["x0"], t["y0"]) - torch.hypot(t["x1"], t["y1"]), 1e-12)
    big = torch.iinfo(torch.int64).max
    key = torch.where(t["eid"] < 0, torch.full_like(t["eid"], big), t["eid"])  # primaries: 2^63 | i
    emin = torch.full((n_aval,), big, dtype=torch.int64, device="cuda").scatter_reduce(0, a, key, reduce="amin")
    pick = torch.nonzero(key == emin[a]).squeeze(1)
    one = torch.stack([t["t1"][pick], t["e1"][pick], t["z1"][pick], a[pick].double()]).cpu().numpy()
    order = np.argsort(one[3])
    return {"gain": gain, "n_w": n_w, "s_t1": s_t1, "s_t": s_t, "s_r": s_r, "one": one[:3, order]}


@pytest.fixture(scope="module")
def wire_runs(A):
    wl = W.wire(band_bins=100)
    g = A.Gas(wl.gas)
    f = A.Field(wl.field)
    out = {}
    for name, prec in (("fp64", A.FP64), ("fp32", A.FP32_MIXED)):
        parts = []
        r = A.Run(g, f, wl.primaries, wl.n_aval, seed=wl.seed, majorant=A.BANDED, precision=prec,
                  band_lookahead=1.0, capacity=90_000_000, timeout_s=100.0)
        for s in range(NSEEDS):
            r.set_seed(wl.seed + 1000 * s)
            r.execute()
            r.sync()
            parts.append(_per_avalanche(A, r, wl.n_aval))
            if s % 8 == 7:
                print(f"wire {name}: {s + 1} of {NSEEDS} seeds", flush=True)
        r.close()
        out[name] = {k: np.concatenate([p[k] for p in parts], axis=-1) for k in parts[0]}
        out[name]["seed5"] = parts[0]
    return wl, out


def _summary(d):
    gain = d["gain"]
    return {"mean_gain": gain.mean(), "se": gain.std() / math.sqrt(gain.size) / gain.mean(),
            "drift": d["s_r"].sum() / d["s_t"].sum(), "mean_t": d["s_t1"] / np.maximum(d["n_w"], 1)}


def test_wire_fp32_against_fp64(wire_runs):
    wl, out = wire_runs
    a, b = out["fp64"], out["fp32"]
    sa, sb = _summary(a), _summary(b)
    rel = sb["mean_gain"] / sa["mean_gain"] - 1.0
    se = math.hypot(sa["se"], sb["se"])
    d = b["gain"] - a["gain"]
    paired_se = d.std() / math.sqrt(d.size) / sa["mean_gain"]
    corr = np.corrcoef(a["gain"], b["gain"])[0, 1]
    dv = sb["drift"] / sa["drift"] - 1.0
    ks = {"gain": stats.ks_2samp(a["gain"], b["gain"]).pvalue,
          "mean_t": stats.ks_2samp(sa["mean_t"], sb["mean_t"]).pvalue}
    for i, k in enumerate(("t1", "e1", "z1")):
        ks[k] = stats.ks_2samp(a["one"][i], b["one"][i]).pvalue
    print(f"wire, {a['gain'].size} avalanches per precision: mean gain fp64 {sa['mean_gain']:.1f} "
          f"fp32 {sb['mean_gain']:.1f}, rel {rel:+.4f} (unpaired se {se:.4f}; paired se {paired_se:.4f}, "
          f"corr {corr:.3f}); radial drift fp64 {sa['drift']:.6e} fp32 {sb['drift']:.6e} cm/ns, "
          f"rel {dv:+.2e}; KS {ks}")
    assert abs(rel) < 0.01
    assert abs(dv) < 0.005
    for k, p in ks.items():
        assert p > 0.01, k


def _golden():
    rows = np.loadtxt(GOLDEN, comments="#")
    return {"aval": rows[:, 0].astype(np.int64), "gain": rows[:, 1], "n_w": rows[:, 2],
            "s_t1": rows[:, 3], "s_t": rows[:, 4], "s_r": rows[:, 5]}


def test_wire_against_oracle_subset(wire_runs):
    """Seed 5's avalanches 0, 2, ..., 2046 in each precision against the
    oracle's replay of the same avalanches (independent samples here):
    mean gain and radial drift within three standard errors, KS p > 0.01
    on the per-avalanche gain and mean arrival time."""
    wl, out = wire_runs
    ref = _golden()
    assert ref["aval"].size == 1024
    rg = ref["gain"]
    rt = ref["s_t1"] / np.maximum(ref["n_w"], 1)
    rng = np.random.default_rng(0)
    boot = rng.integers(0, rg.size, (400, rg.size))
    v_ref = ref["s_r"].sum() / ref["s_t"].sum()
    v_se = np.std(ref["s_r"][boot].sum(1) / ref["s_t"][boot].sum(1))
    for name in ("fp64", "fp32"):
        d = out[name]["seed5"]
        sel = ref["aval"]
        g = d["gain"][sel]
        t = d["s_t1"][sel] / np.maximum(d["n_w"][sel], 1)
        v = d["s_r"][sel].sum() / d["s_t"][sel].sum()
        se = math.sqrt(rg.var() / rg.size + g.var() / g.size)
        p_g = stats.ks_2samp(rg, g).pvalue
        p_t = stats.ks_2samp(rt, t).pvalue
        print(f"{name} vs oracle (1024 avalanches): mean gain {g.mean():.1f} vs {rg.mean():.1f} "
              f"(se {se:.1f}); drift {v:.6e} vs {v_ref:.6e} (se {v_se:.1e}); KS gain {p_g:.3f} "
              f"mean arrival {p_t:.3f}")
        assert abs(g.mean() - rg.mean()) < 3 * se
        assert abs(v - v_ref) < 3 * math.hypot(v_se, v_se)
        assert p_g > 0.01 and p_t > 0.01
