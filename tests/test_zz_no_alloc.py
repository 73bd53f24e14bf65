"""avm_run_noalloc (the batched transport into caller-owned outputs, with
its working memory in the library's static scratch array) against the
allocating entry points (avm_run_create / execute / sync) on the same
inputs and options: endpoints bit for bit after sorting by (avalanche,
id), per-avalanche counters and totals equal.  Two calls in a row on one
GPU share the scratch array; the second has a smaller input (and the
FP32-mixed precision), so stale contents of the first would show."""
import numpy as np
import pytest

from paper_2509_15377_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    from paper_2509_15377_amd import avm
    if avm.device_count() < 1:
        pytest.fail("no HIP device visible: the GPU tests need an MI355X")
    return avm


def _reference(A, g, f, prim_np, n_aval, seed, cap, **kw):
    ep, tot, per = A.run(gas=g, field=f, primaries=prim_np, n_aval=n_aval, seed=seed, capacity=cap,
                         mode=A.BATCHED, timeout_s=60.0, **kw)
    return ep, tot, per


def _noalloc(A, g, f, prim_np, n_aval, seed, cap, **kw):
    import torch
    dev = torch.from_numpy(prim_np.view(np.uint8).copy()).to("cuda:0")
    out = A.noalloc_outputs(cap, n_aval)
    s = torch.cuda.current_stream()
    A.run_noalloc(g, f, dev, n_aval, out, seed=seed, stream=s, timeout_s=60.0, **kw)
    s.synchronize()
    return A.noalloc_results(out, n_aval)


def _same(a, b):
    ea, ta, pa = a
    eb, tb, pb, flags = b
    assert flags == 0
    assert ea.size == eb.size == ta["n_endpoints"]
    assert ea.tobytes() == eb.tobytes()
    assert ta == tb
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), k


def test_noalloc_matches_run_twice(A):
    wl = W.argon(band_bins=100)
    g = A.Gas(wl.gas)
    f = A.Field(wl.field)
    # call 1: 48 avalanches, FP64, banded with lookahead
    prim = wl.primaries[wl.primaries["aval"] < 48]
    kw = dict(majorant=A.BANDED, band_lookahead=1.0)
    print("noalloc call 1: argon, 48 avalanches, FP64 banded", flush=True)
    ref1 = _reference(A, g, f, prim, 48, wl.seed, 1_000_000, **kw)
    got1 = _noalloc(A, g, f, prim, 48, wl.seed, 1_000_000, **kw)
    _same(ref1, got1)
    assert ref1[1]["n_endpoints"] > 48 * 100
    # call 2: a smaller input, FP32-mixed
    prim2 = wl.primaries[wl.primaries["aval"] < 12]
    kw2 = dict(majorant=A.BANDED, precision=A.FP32_MIXED)
    print("noalloc call 2: argon, 12 avalanches, FP32-mixed banded", flush=True)
    ref2 = _reference(A, g, f, prim2, 12, wl.seed, 300_000, **kw2)
    got2 = _noalloc(A, g, f, prim2, 12, wl.seed, 300_000, **kw2)
    _same(ref2, got2)


def test_noalloc_polar_map_crossings(A):
    """The polar-map kernel through avm_run_noalloc: wire-chamber electrons
    that end on the wire and beyond the tube within 4000 flights (the
    boundary crossings found after the pass), against the allocating entry
    points, with the helical band bound."""
    import math
    wl = W.wire()
    g = A.Gas(wl.gas, band_bins=100)
    f = A.Field(wl.field)
    p = W.primaries_at_rest(16)
    phi = np.linspace(0.0, 2.0 * math.pi, 8, endpoint=False) + 0.1
    rho = np.r_[np.full(8, 40e-4), np.full(8, 0.4999)]
    p["x"] = rho * np.cos(np.r_[phi, phi])
    p["y"] = rho * np.sin(np.r_[phi, phi])
    p["e"][8:] = 2.0
    p["dx"][8:] = np.cos(phi)
    p["dy"][8:] = np.sin(phi)
    p["dz"][8:] = 0.0
    kw = dict(majorant=A.BANDED, k_max=4000)
    print("noalloc: wire chamber near the boundaries, FP64 banded", flush=True)
    ref = _reference(A, g, f, p, 16, wl.seed, 200_000, **kw)
    got = _noalloc(A, g, f, p, 16, wl.seed, 200_000, **kw)
    _same(ref, got)
    st = ref[1]["n_status"]
    assert st[4] > 0 and st[5] > 0


def test_noalloc_truncation_and_errors(A):
    import torch
    wl = W.toy(40)
    g = A.Gas(wl.gas)
    f = A.Field(wl.field)
    dev = torch.from_numpy(wl.primaries.view(np.uint8).copy()).to("cuda:0")
    out = A.noalloc_outputs(100, 40)
    s = torch.cuda.current_stream()
    A.run_noalloc(g, f, dev, 40, out, seed=1, stream=s, timeout_s=60.0)
    s.synchronize()
    ep, tot, per, flags = A.noalloc_results(out, 40)
    assert flags == A.NOALLOC_TRUNCATED and tot["truncated"] == 1 and tot["n_requested"] > 100
    assert ep.size == 100
    # beyond the scratch limit, the plain mode, graph capture: refused
    with pytest.raises(A.AvmError) as e:
        A.run_noalloc(g, f, dev, 40, A.noalloc_outputs(A.NOALLOC_MAX_ELECTRONS + 1, 40), seed=1)
    assert e.value.status == A.AVM_E_ARG and "scratch" in str(e.value)
