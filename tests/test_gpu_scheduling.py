"""Scheduling of the batched persistent kernel through the C-ABI: results do
not depend on the pass length, and a run that drops secondaries at its
capacity still ends (terminations and drops are counted on `ended`, created
electrons on `tail`; the kernel leaves when the two agree)."""
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


def _sorted(ep):
    return ep[np.lexsort((ep["eid"], ep["aval"]))]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_pass_length_does_not_change_results(A, precision):
    """One flight per pass (an exchange after every flight), an odd length,
    the other precision's default and a long one give the same bits as the
    default (40 flights in FP64, 48 in FP32-mixed) on 40 argon avalanches,
    banded with lookahead."""
    wl = W.argon(40)
    g = A.Gas(wl.gas, band_bins=100)
    f = A.Field(wl.field)
    kw = dict(seed=wl.seed, majorant=A.BANDED, band_lookahead=1.0, capacity=4_000_000, timeout_s=60.0,
              precision=A.FP64 if precision == "fp64" else A.FP32_MIXED)
    ref = None
    for fpp in (0, 1, 7, 40, 48, 100):
        r = A.Run(g, f, wl.primaries, wl.n_aval, flights_per_pass=fpp, **kw)
        r.execute()
        r.sync()
        ep = _sorted(r.endpoints())
        c = r.counts()
        r.close()
        assert c["n_endpoints"] == ep.size == wl.n_aval + c["n_ion"]
        if ref is None:
            ref = ep
        else:
            assert ep.tobytes() == ref.tobytes(), fpp
    print(precision, "pass lengths 1, 7, 40, 48, 100 and the default agree on", ref.size, "electrons")


@pytest.mark.parametrize("graph", [False, True])
def test_truncated_banded_run_ends(A, graph):
    """40 argon avalanches need ~1.1e5 slots; with 3e4 most secondaries are
    dropped.  The run must still end (well inside its time budget), report
    the truncation and keep exactly `capacity` records, on every execute."""
    wl = W.argon(40)
    g = A.Gas(wl.gas, band_bins=100)
    f = A.Field(wl.field)
    r = A.Run(g, f, wl.primaries, wl.n_aval, seed=wl.seed, majorant=A.BANDED, band_lookahead=1.0,
              capacity=30_000, timeout_s=30.0, graph=graph)
    for _ in range(3):
        r.execute()
        assert r.sync(allow_truncation=True) is False
        c = r.counts()
        assert c["truncated"] == 1 and c["n_requested"] > 30_000
        assert r.num_endpoints() == 30_000
        ep = r.endpoints()
        # every stored record is a finished electron of a valid avalanche
        assert np.all(ep["status"] > 0) and np.all(ep["aval"] < wl.n_aval)
        assert np.unique(ep["eid"]).size == ep.size
    r.close()


def test_repeated_executes_agree(A):
    """The run counters (tail, queue, ended, epoch) are reset by every
    execute: three executes of one run give the same electrons."""
    wl = W.argon(16)
    g = A.Gas(wl.gas, band_bins=100)
    f = A.Field(wl.field)
    r = A.Run(g, f, wl.primaries, wl.n_aval, seed=wl.seed, majorant=A.BANDED, capacity=2_000_000,
              timeout_s=60.0)
    out = []
    for _ in range(3):
        r.execute()
        r.sync()
        out.append(_sorted(r.endpoints()))
    r.close()
    assert out[0].tobytes() == out[1].tobytes() == out[2].tobytes()


@pytest.mark.parametrize("graph", [False, True])
def test_set_seed_equals_a_new_run(A, graph):
    """A seed changed between executes (avm_run_set_seed; a captured graph
    is captured again) gives the bits of a new run created with that seed,
    and changing it back gives the first run's bits again."""
    wl = W.argon(24)
    g = A.Gas(wl.gas, band_bins=100)
    f = A.Field(wl.field)
    kw = dict(majorant=A.BANDED, capacity=2_000_000, timeout_s=60.0, band_lookahead=1.0)
    r = A.Run(g, f, wl.primaries, wl.n_aval, seed=wl.seed, graph=graph, **kw)
    r.execute(); r.sync()
    first = _sorted(r.endpoints())
    r.set_seed(77)
    r.execute(); r.sync()
    second = _sorted(r.endpoints())
    fresh = A.Run(g, f, wl.primaries, wl.n_aval, seed=77, graph=graph, **kw)
    fresh.execute(); fresh.sync()
    assert second.tobytes() == _sorted(fresh.endpoints()).tobytes()
    assert r.counts() == fresh.counts()
    assert second.tobytes() != first.tobytes()
    fresh.close()
    r.set_seed(wl.seed)
    r.execute(); r.sync()
    assert _sorted(r.endpoints()).tobytes() == first.tobytes()
    r.close()
