"""Pin of the whole null-collision transport against an independent
brute-force integrator (small time steps, no null collisions, numpy random
numbers, its own table interpolation and scattering frames) on a tiny
avalanche case: toy gas, 10 um gap, 50 kV/cm (gain ~1.8)."""
import numpy as np
import pytest
from scipy import stats

from oracle import bruteforce as BF
from paper_2509_15377_amd import workloads as W


@pytest.mark.slow
def test_oracle_matches_small_step_integration(oracle_mod):
    O = oracle_mod
    gas = W.toy_gas()
    gap, E0, n = 10e-4, 50e3, 3000
    ep = O.run(gas, W.slab(gap, E0), W.primaries_at_rest(n), seed=51)
    bf = BF.simulate(gas, gap, E0, n, 1e-6, np.random.default_rng(52), block=64)
    go = np.bincount(ep["aval"], minlength=n)
    gb = np.bincount(bf["aval"], minlength=n)
    assert stats.ks_2samp(go, gb).pvalue > 1e-3
    se = np.sqrt(go.var() / n + gb.var() / n)
    assert abs(go.mean() - gb.mean()) < 4 * se
    assert go.mean() > 1.5  # the case really multiplies
    mo, mb = ep["status"] == 2, bf["status"] == 2
    assert mo.mean() > 0.99 and mb.mean() > 0.99
    for a, b in ((ep["t1"][mo], bf["t"][mb]), (ep["e1"][mo], bf["e"][mb])):
        assert stats.ks_2samp(a, b).pvalue > 1e-3
        # first-order time-step bias of the integrator: ~0.5 % at dt = 1e-6 ns
        assert abs(a.mean() - b.mean()) < 4 * np.sqrt(a.var() / a.size + b.var() / b.size) + 0.01 * abs(a.mean())


# ---- the argon-like gas: screened Rutherford elastic, 30 excitations,
# Opal-Beaty ionisation, as the transport loop calls them
_ARGON = {}


def _argon_bf():
    """Brute force on the tiny argon case (10 um, 60 kV/cm, gain ~2),
    computed once per session."""
    if "bf" not in _ARGON:
        _ARGON["bf"] = BF.simulate(W.argon_like_gas(), 10e-4, 60e3, 3000, 1e-6,
                                   np.random.default_rng(62), block=64)
    return _ARGON["bf"]


def _argon_checks(O):
    """p-values and standardised mean differences (oracle vs brute force) of
    the per-avalanche gain, the arrival time and energy at the anode and the
    secondaries' birth energies."""
    n = 3000
    ep = O.run(W.argon_like_gas(), W.slab(10e-4, 60e3), W.primaries_at_rest(n), seed=61)
    bf = _argon_bf()
    go = np.bincount(ep["aval"], minlength=n)
    gb = np.bincount(bf["aval"], minlength=n)
    mo, mb = ep["status"] == 2, bf["status"] == 2
    pairs = {"gain": (go, gb), "t": (ep["t1"][mo], bf["t"][mb]), "e": (ep["e1"][mo], bf["e"][mb]),
             "sec_e": (ep["e0"][ep["parent"] != 0], bf["sec_e"])}
    out = {}
    for k, (a, b) in pairs.items():
        z = abs(a.mean() - b.mean()) / np.sqrt(a.var() / a.size + b.var() / b.size)
        out[k] = (stats.ks_2samp(a, b).pvalue, z, a.mean(), b.mean())
    return out


@pytest.mark.slow
def test_argon_gas_matches_small_step_integration(oracle_mod):
    """Screened-Rutherford elastic scattering and the Opal-Beaty split, as
    wired into the transport loop, against the brute-force integrator (its
    own rejection samplers of the two laws)."""
    res = _argon_checks(oracle_mod)
    print(res)
    assert res["gain"][2] > 1.5  # the case really multiplies
    for k, (p, z, _, _) in res.items():
        assert p > 1e-3, k
        # time-step bias of the integrator at dt = 1e-6 ns: below 1 %
        assert z < 4.0 or abs(res[k][2] - res[k][3]) < 0.01 * abs(res[k][3]), k


@pytest.mark.slow
@pytest.mark.parametrize("macro", ["ORC_PLANT_SR_ISOTROPIC", "ORC_PLANT_OB_AVAIL"])
def test_argon_planted_mistakes_are_caught(oracle_mod, macro):
    with oracle_mod.planted(macro):
        res = _argon_checks(oracle_mod)
    assert min(p for p, _, _, _ in res.values()) < 1e-6, res
