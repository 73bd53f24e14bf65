"""Pins of the oracle's counter-based generator (Philox4x32-10) and of the
uniform maps built on it.

The generator is pinned against rocRAND's header-only Philox engine (an
implementation that shares nothing with the oracle), compiled on the fly
from tests/golden/philox_rocrand_kat.cpp.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rocrand_kat(lines, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND known-answer program")
    exe = str(tmp_path / "philox_kat")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(GOLDEN, "philox_rocrand_kat.cpp")],
                   check=True, capture_output=True, cwd=str(tmp_path))
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    return [tuple(int(w, 16) for w in o.split()) for o in out if o.strip()]


def test_philox_matches_rocrand(oracle_mod, tmp_path):
    rng = np.random.default_rng(1234)
    cases = [((0, 0, 0, 0), (0, 0)), ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0))]
    for _ in range(200):
        c = tuple(int(x) for x in rng.integers(0, 2 ** 32, 4, dtype=np.uint64))
        k = tuple(int(x) for x in rng.integers(0, 2 ** 32, 2, dtype=np.uint64))
        cases.append((c, k))
    # counters of the method's own layout: (4k+j, aval, eid_lo, eid_hi)
    for kk in (0, 1, 7, (1 << 30) - 1):
        for j in range(4):
            eid = (1 << 63) | 12345
            cases.append(((4 * kk + j, 999, eid & 0xFFFFFFFF, eid >> 32), (2, 0)))
    lines = ["%x %x %x %x %x %x" % (c + k) for c, k in cases]
    ref = _rocrand_kat(lines, tmp_path)
    assert len(ref) == len(cases)
    for (c, k), r in zip(cases, ref):
        assert oracle_mod.philox(c, k) == r


def test_u53_extremes_and_exactness(oracle_mod):
    O = oracle_mod
    assert O.u53(0, 0) == 2.0 ** -53
    assert O.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0
    assert O.u53(0, 63) == 2.0 ** -53          # low 6 bits of w_lo dropped
    assert O.u53(0, 64) == 2.0 * 2.0 ** -53
    assert O.u53(31, 0) == 2.0 ** -53          # low 5 bits of w_hi dropped
    assert O.u53(32, 0) == (2.0 ** 26 + 1) * 2.0 ** -53
    rng = np.random.default_rng(7)
    for hi, lo in rng.integers(0, 2 ** 32, (500, 2), dtype=np.uint64):
        m = (int(hi) >> 5) * 2 ** 26 + (int(lo) >> 6)
        assert O.u53(int(hi), int(lo)) == (m + 1) / 2.0 ** 53   # exact in binary64
        assert 0.0 < O.u53(int(hi), int(lo)) <= 1.0


def test_u24_extremes_and_shared_high_word(oracle_mod):
    O = oracle_mod
    assert O.u24(0) == np.float32(2.0 ** -24)
    assert O.u24(0xFFFFFFFF) == np.float32(1.0)
    rng = np.random.default_rng(8)
    for hi, lo in rng.integers(0, 2 ** 32, (500, 2), dtype=np.uint64):
        f = O.u24(int(hi))
        d = O.u53(int(hi), int(lo))
        assert f == np.float32(((int(hi) >> 8) + 1) / 2.0 ** 24)
        # the FP32 and FP64 uniforms of one word pair are common random numbers
        assert abs(float(f) - d) <= 2.0 ** -24


def test_philox_uniformity(oracle_mod):
    """Chi-square of the U53 uniforms of 20000 consecutive flight blocks."""
    from scipy import stats
    O = oracle_mod
    u = []
    for k in range(20000):
        w = O.philox((4 * k, 3, 77, 1 << 31), (5, 0))
        u.append(O.u53(w[0], w[1]))
        u.append(O.u53(w[2], w[3]))
    h, _ = np.histogram(u, bins=50, range=(0, 1))
    assert stats.chisquare(h).pvalue > 1e-3
