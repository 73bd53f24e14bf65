"""Penning transfer in the oracle (an excitation followed, with probability
p, by an extra electron of a given energy born where it happened; random
blocks j = 2, 3 of the flight as for an ionisation).  Pins: the parent's
own trajectory does not depend on p; with the same seed the children at
p = 0.3 are exactly the subset of the p = 1 children whose decision
uniform is below 0.3 (about 30 % of them, binomial); children carry the
transfer energy; p = 0 is the gas without transfer bit for bit; bookkeeping
holds; bad settings are rejected."""
import math

import numpy as np
import pytest

from paper_2509_15377_amd import workloads as W


def _run(O, p, n=24, t_max=0.06):
    wl = W.penning(n, prob=p) if p is not None else W.argon(n)
    ep = O.run(wl.gas, wl.field, wl.primaries, wl.seed if p is not None else 6, t_max=t_max)
    return wl, ep


def test_parent_trajectory_independent_of_transfer(oracle_mod):
    _, e0 = _run(oracle_mod, 0.0)
    _, e1 = _run(oracle_mod, 1.0)
    p0, p1 = e0[e0["parent"] == 0], e1[e1["parent"] == 0]
    assert p0.size == p1.size == 24
    for k in ("x1", "y1", "z1", "t1", "e1", "status", "n_real", "n_null", "n_masked"):
        assert np.array_equal(p0[k], p1[k]), k
    assert (p1["n_ion"] > p0["n_ion"]).any()
    assert e1.size > e0.size


def test_children_subset_and_yield(oracle_mod):
    _, e1 = _run(oracle_mod, 1.0, n=160, t_max=0.1)
    _, e3 = _run(oracle_mod, 0.3, n=160, t_max=0.1)
    prim_ids = set(e1["eid"][e1["parent"] == 0].tolist())
    kids1 = set(e1["eid"][np.isin(e1["parent"], list(prim_ids))].tolist())
    kids3 = set(e3["eid"][np.isin(e3["parent"], list(prim_ids))].tolist())
    # ionisation children are common to both runs; transfer children of
    # the 0.3 run must all appear in the p = 1 run
    assert kids3 <= kids1
    wl = W.penning(2, prob=1.0)
    thr = {round(c.penning_energy_eV, 12) for c in wl.gas.channels if c.penning_prob > 0}
    e_child = lambda ep, ids: ep["e0"][np.isin(ep["eid"], list(ids))]
    pen1 = {i for i, e in zip(e1["eid"], e1["e0"]) if i in kids1 and round(e, 12) in thr}
    pen3 = {i for i in kids3 if i in pen1}
    n = len(pen1)
    assert n > 200
    frac = len(pen3) / n
    assert abs(frac - 0.3) < 4.0 * math.sqrt(0.3 * 0.7 / n), (frac, n)


def test_transfer_energy_and_bookkeeping(oracle_mod):
    wl, e = _run(oracle_mod, 0.5)
    energies = {round(c.penning_energy_eV, 12) for c in wl.gas.channels if c.penning_prob > 0}
    kids = e[e["parent"] != 0]
    at_transfer = np.array([round(x, 12) in energies for x in kids["e0"]])
    assert at_transfer.sum() > 0
    assert (kids["e0"][at_transfer] >= 1.0).all() and (kids["e0"][at_transfer] <= 4.5).all()
    pa = oracle_mod.per_avalanche(e, wl.n_aval)
    assert np.array_equal(pa["n_endpoints"], 1 + pa["n_ion"])


def test_zero_probability_is_the_plain_gas(oracle_mod):
    wl0 = W.penning(16, prob=0.0)
    wa = W.argon(16)
    a = oracle_mod.run(wl0.gas, wl0.field, wl0.primaries, 6)
    b = oracle_mod.run(wa.gas, wa.field, wa.primaries, 6)
    assert a.tobytes() == b.tobytes()


def test_bad_penning_settings(oracle_mod):
    L = oracle_mod.lib()
    g = oracle_mod.Gas(W.argon_like_gas())
    assert L.orc_gas_set_penning(g.h, 0, 0.5, 1.0) != 0     # elastic channel
    assert L.orc_gas_set_penning(g.h, 1, 1.5, 1.0) != 0     # probability > 1
    assert L.orc_gas_set_penning(g.h, 1, 0.5, -1.0) != 0    # negative energy
    assert L.orc_gas_set_penning(g.h, 99, 0.5, 1.0) != 0    # no such channel
    assert L.orc_gas_set_penning(g.h, 1, 0.5, 1.0) == 0
