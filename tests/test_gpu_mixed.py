"""FP32-mixed precision against FP64 (through the C-ABI).

The FP32-mixed path draws the same Philox blocks as the FP64 path (24-bit
uniforms from the same high words), so the two runs of one workload are
paired by avalanche.  Gates: mean gain within 1 %, drift velocity within
0.5 %, KS p > 0.01 on the endpoint and arrival-time distributions (pooled
endpoints, and per avalanche, where samples are independent).  The FP64 GPU
path itself matches the FP64 oracle per trajectory (test_gpu_parity.py), so
these are also the errors against the oracle; a direct comparison with the
oracle on a subset is included."""
import numpy as np
import pytest
from scipy import stats

from gates import statistical_gates
from oracle import compare as CMP
from paper_2509_15377_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    from paper_2509_15377_amd import avm
    if avm.device_count() < 1:
        pytest.fail("no HIP device visible: the GPU tests need an MI355X")
    return avm


def _run(A, wl, precision, **kw):
    kw.setdefault("timeout_s", 120.0)
    kw.setdefault("capacity", 16_000_000)
    return A.run(wl, precision=precision, majorant=A.BANDED, **kw)


def _drift(ep):
    m = ep["status"] == 2
    return (ep["z1"][m] - ep["z0"][m]).sum() / (ep["t1"][m] - ep["t0"][m]).sum()


@pytest.fixture(scope="module")
def argon_pair(A):
    wl = W.argon(band_bins=100)
    e64, t64, p64 = _run(A, wl, A.FP64)
    e32, t32, p32 = _run(A, wl, A.FP32_MIXED)
    return wl, (e64, t64, p64), (e32, t32, p32)


def test_mixed_gain_and_drift(argon_pair):
    wl, (e64, t64, p64), (e32, t32, p32) = argon_pair
    g64 = p64["n_endpoints"].astype(float)
    g32 = p32["n_endpoints"].astype(float)
    rel = abs(g32.mean() - g64.mean()) / g64.mean()
    d = g32 - g64
    se_paired = d.std() / np.sqrt(d.size) / g64.mean()
    corr = np.corrcoef(g64, g32)[0, 1]
    v64, v32 = _drift(e64), _drift(e32)
    print(f"mean gain fp64 {g64.mean():.2f} fp32 {g32.mean():.2f} rel {rel:.2e} "
          f"(paired se {se_paired:.2e}, corr {corr:.3f}); drift {v64:.6e} {v32:.6e} "
          f"rel {abs(v32 - v64) / v64:.2e}")
    assert rel < 0.01
    assert abs(v32 - v64) / v64 < 0.005
    # bookkeeping holds in FP32 too
    assert t32["n_endpoints"] == wl.n_aval + t32["n_ion"]
    assert np.array_equal(p32["n_endpoints"], 1 + p32["n_ion"])


def test_mixed_distributions(argon_pair):
    wl, (e64, _, p64), (e32, _, p32) = argon_pair
    m64, m32 = e64["status"] == 2, e32["status"] == 2
    pooled = {k: stats.ks_2samp(e64[k][m64], e32[k][m32]).pvalue for k in ("t1", "e1", "x1")}
    per_aval = stats.ks_2samp(p64["n_endpoints"], p32["n_endpoints"]).pvalue

    def mean_t(ep):
        s = np.bincount(ep["aval"], weights=ep["t1"], minlength=wl.n_aval)
        return s / np.bincount(ep["aval"], minlength=wl.n_aval)

    t_aval = stats.ks_2samp(mean_t(e64), mean_t(e32)).pvalue
    print("KS pooled", pooled, "per-avalanche gain", per_aval, "mean arrival", t_aval)
    for p in list(pooled.values()) + [per_aval, t_aval]:
        assert p > 0.01


def test_mixed_against_oracle_subset(A, oracle_mod):
    """Every 10th avalanche of the benchmark workload in FP32-mixed, against
    the FP64 oracle on the same 100 avalanches (which it replays exactly on
    its own), with the accuracy gates; the primaries match it per
    trajectory to 1e-4 up to their first rounding-induced decision flip."""
    wl = W.argon(band_bins=100)
    idx = W.subset_primaries(wl.primaries, 10)
    ref = oracle_mod.run(oracle_mod.Gas(wl.gas, band_bins=100), wl.field, wl.primaries[idx], wl.seed,
                         banded=True, ids=idx)
    ep32, _, _ = _run(A, wl, A.FP32_MIXED)
    sub = ep32[(ep32["aval"] % 10) == 0]
    rep = CMP.compare(sub, ref, rtol=1e-4)
    print("fp32 vs oracle", {k: rep[k] for k in ("n_got", "n_ref", "matched", "flips")})
    prim = ref[ref["parent"] == 0]
    assert rep["matched"] >= prim.size
    statistical_gates(ref, sub, "argon fp32 vs oracle (every 10th avalanche)", wl.n_aval)


def test_mixed_batched_equals_plain(A):
    wl = W.toy(64)
    a, ta, _ = A.run(wl, precision=A.FP32_MIXED, mode=A.PLAIN, capacity=100000, timeout_s=60.0)
    b, tb, _ = A.run(wl, precision=A.FP32_MIXED, mode=A.BATCHED, capacity=100000, timeout_s=60.0)
    assert a.tobytes() == b.tobytes()
    assert ta == tb


def test_mixed_tables_beyond_the_lds_copies(A):
    """FP32-mixed with 1000 bands (more than the 512 staged in LDS: the
    kernel instance with index tests) against FP64 at the same band width
    (itself matched to the oracle per trajectory in test_gpu_parity.py),
    paired by avalanche, with the accuracy gates."""
    wl = W.argon(400, band_bins=20)
    e64, t64, p64 = _run(A, wl, A.FP64)
    e32, t32, p32 = _run(A, wl, A.FP32_MIXED)
    assert t32["n_endpoints"] == e32.size == wl.n_aval + t32["n_ion"]
    assert t32["n_band"] > 0 and t32["truncated"] == 0
    statistical_gates(e64, e32, "1000 bands fp32 vs fp64", wl.n_aval)
