"""Pins of the oracle's rate table: the majorant bounds the interpolated
rate everywhere, the interpolation is exactly linear between nodes, bands
are prefix maxima, and bad inputs are rejected."""
import math

import numpy as np
import pytest

from paper_2509_15377_amd import workloads as W


def _nu_nodes(gas, ka):
    """Rates at the nodes from the gas description: N sigma sqrt(2 k_a e)."""
    e = W.energy_nodes(gas.e_max_eV, gas.n_bins)
    sp = np.sqrt(2 * ka * e)
    out = []
    for ch in gas.channels:
        v = np.asarray(ch.values, dtype=np.float64)
        out.append(v if ch.values_kind == W.VALUES_RATE else gas.density_cm3 * v * sp)
    return e, np.array(out)


@pytest.mark.parametrize("make", [W.toy_gas, lambda: W.argon_like_gas(attachment=True)])
def test_majorant_bounds_rate_on_dense_scan(oracle_mod, make):
    O = oracle_mod
    gas = make()
    g = O.Gas(gas, band_bins=gas.n_bins // 40)
    gamma = g.gamma
    rng = np.random.default_rng(21)
    es = np.concatenate([rng.uniform(0, gas.e_max_eV * 1.2, 30000),
                         W.energy_nodes(gas.e_max_eV, gas.n_bins)[::7]])
    for e in es:
        nu, tot, over = g.rates(e)
        assert tot <= gamma * (1 + 1e-15)
        b = g.band_of(e)
        gb, edge = g.band(b)
        assert e < edge
        assert tot <= gb * (1 + 1e-15)
        assert (nu >= -1e-9 * tot).all()
        assert over == (e >= gas.e_max_eV)
    # the bound is tight: Gamma is attained at a node
    _, nus = _nu_nodes(gas, O.k_a())
    assert gamma == pytest.approx(nus.sum(axis=0).max(), rel=1e-14)


def test_band_majorants_are_prefix_maxima(oracle_mod):
    O = oracle_mod
    gas = W.argon_like_gas()
    g = O.Gas(gas, band_bins=200)
    assert g.n_bands == 100
    prev = 0.0
    for b in range(g.n_bands):
        gb, edge = g.band(b)
        assert gb >= prev
        prev = gb
        if b < g.n_bands - 1:
            assert edge == pytest.approx((b + 1) * 200 * gas.e_max_eV / gas.n_bins, rel=1e-15)
            assert g.band_of(edge) == b + 1
            assert g.band_of(math.nextafter(edge, 0)) == b
        else:
            assert edge == math.inf and gb == g.gamma
    assert g.band_of(0.0) == 0
    assert g.band_of(1e9) == g.n_bands - 1


def test_interpolation_is_linear_between_nodes(oracle_mod):
    O = oracle_mod
    gas = W.toy_gas()
    g = O.Gas(gas)
    e_nodes, nus = _nu_nodes(gas, O.k_a())
    rng = np.random.default_rng(22)
    for k in rng.integers(0, gas.n_bins, 200):
        for f in (0.0, 0.25, 0.5, 0.9):
            e = e_nodes[k] + f * (e_nodes[k + 1] - e_nodes[k])
            nu, tot, _ = g.rates(e)
            want = (1 - f) * nus[:, k] + f * nus[:, k + 1]
            assert np.allclose(nu, want, rtol=1e-9, atol=1e-9 * want.sum())
    # above the table the rates stay at the last node's values
    nu, tot, over = g.rates(gas.e_max_eV * 3)
    assert over and np.allclose(nu, nus[:, -1], rtol=1e-12)


def test_cumulative_table_is_ordered(oracle_mod):
    O = oracle_mod
    gas = W.argon_like_gas(attachment=True)
    g = O.Gas(gas)
    cum = g.cumulative()
    assert cum.shape == (gas.n_bins + 1, 33)
    assert (np.diff(cum, axis=1) >= 0).all()
    # the interpolated cumulative rates stay ordered across channels
    rng = np.random.default_rng(23)
    for e in rng.uniform(0, 400, 2000):
        nu, tot, _ = g.rates(e)
        assert (nu >= 0).all()


def test_constant_rate_table(oracle_mod):
    O = oracle_mod
    g = O.Gas(W.constant_rate_gas(1234.5))
    assert g.gamma == 1234.5
    for e in (0.0, 1e-9, 3.3, 999.0, 5e4):
        assert g.rates(e)[1] == 1234.5


def test_bad_tables_are_rejected(oracle_mod):
    O = oracle_mod
    gas = W.toy_gas()
    bad = W.toy_gas()
    bad.channels[0].values = bad.channels[0].values.copy()
    bad.channels[0].values[5] = -1e-20
    with pytest.raises(ValueError):
        O.Gas(bad)
    bad.channels[0].values[5] = math.nan
    with pytest.raises(ValueError):
        O.Gas(bad)
    zero = W.Gas(gas.e_max_eV, gas.n_bins, gas.density_cm3,
                 [W.Channel(W.ELASTIC, np.zeros(gas.n_bins + 1))])
    with pytest.raises(ValueError):
        O.Gas(zero)  # no collisions at all
    thr = W.toy_gas()
    thr.channels[1].e_lo_eV = 5.0  # excitation window opening below its loss
    with pytest.raises(ValueError):
        O.Gas(thr)
