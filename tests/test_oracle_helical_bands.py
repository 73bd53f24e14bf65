"""Banded majorant with a magnetic field (helical flights): the pins.

Along a helical flight in frozen E and B the energy is not convex in time,
so the band rule uses a bound that grows with time: 2 k_a e(s) <=
(|v_par| + |a_par| s)^2 + (|w| + |u0|)^2 (w the E x B drift, u0 the
gyration velocity).  The band is raised until the bound at the flight start
is below its edge, and the flight is cut where the bound reaches the edge.
Pins: the bound holds along sampled flights and its root lies on the edge;
no decision ever sees a rate above the majorant in use; banded and global
majorants agree in distribution (wire geometry with 0.5 T, slab with axial
B); the banded majorant cuts the null fraction."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2509_15377_amd import workloads as W


def _vec(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dp(a):
    import ctypes
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _bound(L, v, E, B):
    out = np.zeros(5)
    L.orc_helical_bound(_dp(_vec(v)), _dp(_vec(E)), _dp(_vec(B)), _dp(out))
    return out


def _bval(b, s):
    vp, ap, p, q, m = b
    return (vp + ap * s) ** 2 + min(p + q * s, m) ** 2


def test_bound_holds_along_flights(oracle_mod):
    L = oracle_mod.lib()
    ka = L.orc_k_a()
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(300):
        v = rng.normal(size=3) * rng.uniform(0.01, 0.3)
        E = rng.normal(size=3) * rng.uniform(1e2, 1e5)
        B = rng.normal(size=3) * rng.uniform(0.05, 2.0)
        b = _bound(L, v, E, B)
        assert _bval(b, 0.0) == pytest.approx(v @ v, rel=1e-12)  # exact at the start
        for si in np.linspace(0.0, rng.uniform(1e-3, 0.2), 64):
            _, vv = oracle_mod.propagate([0, 0, 0], v, E, B, si)
            worst = max(worst, (vv @ vv - _bval(b, si)) / _bval(b, si))
        # the root lies on the requested edge, on either branch of the bound
        e0 = (v @ v) / (2 * ka)
        for edge in (e0 * 1.0001, e0 * rng.uniform(1.01, 3.0), e0 * 50.0):
            sc = L.orc_helical_bound_root(_dp(b), edge)
            if math.isfinite(sc):
                assert _bval(b, sc) / (2 * ka) == pytest.approx(edge, rel=1e-10)
            else:
                assert b[1] == 0.0 and _bval(b, 1e9) / (2 * ka) < edge
        assert L.orc_helical_bound_root(_dp(b), e0 * 0.5) == 0.0
    assert worst <= 1e-12


def _run(O, wl, prim, banded, **kw):
    g = O.Gas(wl.gas, band_bins=100)
    return O.run(g, wl.field, prim, wl.seed, banded=banded, **kw)


def _per_aval(ep, n):
    """Independent per-avalanche samples: gain, mean arrival time, and the
    primary electron's arrival time and energy (electrons inside one
    avalanche are correlated, so pooled endpoints are not iid)."""
    a = ep["aval"].astype(np.int64)
    gain = np.bincount(a, minlength=n)
    mean_t = np.bincount(a, weights=ep["t1"], minlength=n) / gain
    prim = ep[ep["parent"] == 0]
    order = np.argsort(prim["aval"])
    return {"gain": gain, "mean_t1": mean_t, "prim_t1": prim["t1"][order], "prim_e1": prim["e1"][order]}


def test_wire_banded_equals_global_in_distribution(oracle_mod):
    O = oracle_mod
    L = O.lib()
    n = 400
    wl = W.wire(n)
    prim = wl.primaries.copy()
    phi = np.random.default_rng(7).uniform(0.0, 2.0 * math.pi, n)
    prim["x"], prim["y"] = 0.01 * np.cos(phi), 0.01 * np.sin(phi)  # rho = 100 um: avalanches
    L.orc_reset_majorant_violations()
    eg = _run(O, wl, prim, False, t_max=3.0)
    eb = _run(O, wl, prim, True, t_max=3.0)
    assert L.orc_majorant_violations() == 0
    fl = lambda ep: float((ep["n_real"].astype(float) + ep["n_null"] + ep["n_masked"] + ep["n_band"]).sum())
    null = lambda ep: (ep["n_null"].astype(float) + ep["n_masked"]).sum() / fl(ep)
    print("wire: electrons", eg.size, eb.size, "null fraction", null(eg), null(eb),
          "flights", fl(eg), fl(eb))
    pg, pb = _per_aval(eg, n), _per_aval(eb, n)
    for key in pg:
        assert stats.ks_2samp(pg[key], pb[key]).pvalue > 1e-3, key
    g, b = pg["gain"].astype(float), pb["gain"].astype(float)
    assert abs(g.mean() - b.mean()) < 4.0 * math.sqrt(g.var() / n + b.var() / n)
    assert fl(eb) < 0.5 * fl(eg)


def test_slab_axial_b_banded_equals_global(oracle_mod):
    O = oracle_mod
    L = O.lib()
    gas = W.toy_gas()
    field = W.slab(20e-4, 4e4, (0.0, 0.0, 2.0))
    wl = W.Workload("t", gas, field, W.primaries_at_rest(3000), 3000, 13, "")
    L.orc_reset_majorant_violations()
    eg = _run(O, wl, wl.primaries, False)
    eb = _run(O, wl, wl.primaries, True)
    assert L.orc_majorant_violations() == 0
    ng = np.bincount(eg["aval"], minlength=3000)
    nb = np.bincount(eb["aval"], minlength=3000)
    print("slab B: mean gain", ng.mean(), nb.mean(), "band cuts", eb["n_band"].sum())
    assert eb["n_band"].sum() > 0
    assert stats.ks_2samp(ng, nb).pvalue > 1e-3
    for key in ("t1", "e1", "x1"):
        a, b = eg[eg["status"] == 2][key], eb[eb["status"] == 2][key]
        assert stats.ks_2samp(a, b).pvalue > 1e-3, key
    se = math.sqrt(ng.var() / ng.size + nb.var() / nb.size)
    assert abs(ng.mean() - nb.mean()) < 4 * se


def test_no_majorant_violation_without_b(oracle_mod):
    O = oracle_mod
    L = O.lib()
    wl = W.argon(20, band_bins=100)
    L.orc_reset_majorant_violations()
    _run(O, wl, wl.primaries, True)
    _run(O, wl, wl.primaries, False)
    assert L.orc_majorant_violations() == 0
