"""Pins of the oracle's induced signal (Shockley-Ramo on the readout
electrode, binned in time; paper Sec. 3.2 names the induced signal as the
step users take after the avalanche).

* sum rule: over bins covering every electron's life, the signal of an
  avalanche is the sum over its electrons of phi_w(end) - phi_w(start),
  taken from the endpoints alone (slab and wire geometries);
* ballistic closed form: with a gas that has no real collision below its
  last node, an electron released at rest moves as z = k_a E t^2 / 2 until
  it leaves, so each bin holds (z(T_j+1) - z(T_j)) / d (also with B along z,
  which leaves z(t) unchanged: the helical code path);
* additivity over finer bins, invariance under a shift of the bin origin by
  whole bins, independence of the processing order and thread count;
* argument errors."""
import math

import numpy as np
import pytest

from paper_2509_15377_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore")


def _phi_slab(z, field):
    return (z - field.z_lo_cm) / (field.z_hi_cm - field.z_lo_cm)


def test_weighting_potentials(oracle_mod):
    f = oracle_mod.Field(W.slab(0.01, 3e4))
    assert f.weighting([0.3, -2.0, 0.0]) == 0.0
    assert f.weighting([0.0, 0.0, 0.0025]) == pytest.approx(0.25, rel=1e-15)
    wf = W.wire_polar_map()
    fw = oracle_mod.Field(wf)
    assert fw.weighting([wf.a_cm, 0.0, 0.0]) == pytest.approx(1.0, rel=1e-15)
    assert fw.weighting([0.0, wf.b_cm, 1.0]) == pytest.approx(0.0, abs=1e-15)
    r = 0.1
    assert fw.weighting([r / math.sqrt(2), r / math.sqrt(2), 0.0]) == pytest.approx(
        math.log(wf.b_cm / r) / math.log(wf.b_cm / wf.a_cm), rel=1e-14)


def test_sum_rule_slab(oracle_mod):
    wl = W.toy(40)
    ep, sig = oracle_mod.run(wl.gas, wl.field, wl.primaries, wl.seed, signal=(0.0, 0.01, 200, 40))
    assert ep["t1"].max() < 2.0  # the bins cover every life
    d = wl.field.z_hi_cm - wl.field.z_lo_cm
    expect = np.bincount(ep["aval"], weights=(ep["z1"] - ep["z0"]) / d, minlength=40)
    assert np.allclose(sig.sum(axis=1), expect, rtol=1e-12, atol=1e-12)
    # electrons drift to the readout plane: the induced charge grows there
    assert (sig.sum(axis=1) > 0).all()


def test_sum_rule_wire(oracle_mod):
    wl = W.wire(2)
    of = oracle_mod.Field(wl.field)
    ep, sig = oracle_mod.run(wl.gas, wl.field, wl.primaries, wl.seed, k_max=20000,
                             signal=(0.0, 0.05, 400, 2))
    assert ep["t1"].max() < 20.0
    phi = lambda x, y: np.array([of.weighting([a, b, 0.0]) for a, b in zip(x, y)])
    dphi = phi(ep["x1"], ep["y1"]) - phi(ep["x0"], ep["y0"])
    expect = np.bincount(ep["aval"], weights=dphi, minlength=2)
    assert np.allclose(sig.sum(axis=1), expect, rtol=1e-11, atol=1e-13)


def _null_gas():
    """One elastic channel whose rate is zero at every node but the last: below
    the last bin every collision is null, so electrons move ballistically."""
    n = 400
    vals = np.zeros(n + 1)
    vals[-1] = 1e3
    ch = W.Channel(W.ELASTIC, vals, values_kind=W.VALUES_RATE)
    return W.Gas(400.0, n, W.GAS_DENSITY, [ch], 0)


@pytest.mark.parametrize("B", [(0.0, 0.0, 0.0), (0.0, 0.0, 0.7)])
def test_ballistic_closed_form(oracle_mod, B):
    E0, gap = 2e4, 0.01
    field = W.slab(gap, E0, B)
    prim = W.primaries_at_rest(1)
    dt, nb = 0.002, 40
    ep, sig = oracle_mod.run(_null_gas(), field, prim, 7, signal=(0.0, dt, nb, 1))
    assert ep.size == 1 and ep["status"][0] == 2 and ep["n_real"][0] == 0
    a = oracle_mod.lib().orc_k_a() * E0
    t_exit = math.sqrt(2.0 * gap / a)
    assert ep["t1"][0] == pytest.approx(t_exit, rel=1e-9)
    T = np.arange(nb + 1) * dt
    z = np.minimum(0.5 * a * np.minimum(T, t_exit) ** 2, gap)
    expect = np.diff(z) / gap
    assert np.allclose(sig[0], expect, rtol=1e-9, atol=1e-13)
    assert sig[0].sum() == pytest.approx(1.0, rel=1e-12)


def test_additivity_shift_and_order(oracle_mod):
    wl = W.toy(12)
    g = oracle_mod.Gas(wl.gas)
    f = oracle_mod.Field(wl.field)
    _, s1 = oracle_mod.run(g, f, wl.primaries, wl.seed, signal=(0.0, 0.01, 100, 12))
    _, s2 = oracle_mod.run(g, f, wl.primaries, wl.seed, signal=(0.0, 0.005, 200, 12))
    assert np.allclose(s2.reshape(12, 100, 2).sum(axis=2), s1, rtol=1e-10, atol=1e-12)
    _, s3 = oracle_mod.run(g, f, wl.primaries, wl.seed, signal=(-0.05, 0.01, 105, 12))
    assert np.allclose(s3[:, 5:], s1, rtol=1e-10, atol=1e-12)
    assert np.abs(s3[:, :5]).max() == 0.0  # nothing before the first electron is born
    _, s4 = oracle_mod.run(g, f, wl.primaries, wl.seed, fifo=True, threads=1,
                           signal=(0.0, 0.01, 100, 12))
    assert np.allclose(s4, s1, rtol=1e-12, atol=1e-13)


def test_signal_argument_errors(oracle_mod):
    wl = W.toy(2)
    for bad in ((0.0, 0.01, 0, 2), (0.0, 0.0, 10, 2), (0.0, -1.0, 10, 2), (math.nan, 0.01, 10, 2),
                (0.0, 0.01, 10, 1)):
        with pytest.raises(ValueError):
            oracle_mod.run(wl.gas, wl.field, wl.primaries, wl.seed, signal=bad)
