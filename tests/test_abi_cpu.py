"""The C-ABI library on a machine without a GPU: it loads, exports every
symbol include/avm.h declares, and rejects bad arguments before touching a
device."""
import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2509_15377_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def A():
    from paper_2509_15377_amd import avm
    if not os.path.exists(avm.LIB_PATH):
        from paper_2509_15377_amd import build
        build.build()
    avm.lib()
    return avm


def _declared():
    txt = open(os.path.join(ROOT, "include", "avm.h")).read()
    return sorted(set(re.findall(r"^(?:avm_status|void|const char\*|int32_t)\s+(avm_\w+)\(", txt, re.M)))


def test_library_exports_every_declared_symbol(A):
    names = _declared()
    assert len(names) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", A.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (avm_\w+)", out))
    assert set(names) <= exported
    assert set(names) == set(A.EXPORTED)
    L = A.lib()
    for n in names:
        assert getattr(L, n) is not None


def test_abi_version_and_sizes(A):
    assert A.lib().avm_abi_version() == 3
    assert A.ENDPOINT_DTYPE.itemsize == 136
    assert A.END_RECORD_DTYPE.itemsize == 72
    assert W.PRIMARY_DTYPE.itemsize == 72
    assert C.sizeof(A._Counts) == 8 * 18 + 8
    assert C.sizeof(A._Opts) == 72
    assert C.sizeof(A._TuneResult) == 48
    assert C.sizeof(A._EndpointArrays) == 9 * 8
    assert C.sizeof(A._NoallocOut) == 12 * 8


def test_record_layouts_match_the_header(A, tmp_path):
    """The binding's record layouts against what a C compiler makes of
    include/avm.h: sizes and field offsets."""
    fields = {"avm_counts": [n for n in A.COUNTS_DTYPE.names if n != "_pad"],
              "avm_end_record": A.END_RECORD_DTYPE.names,
              "avm_endpoint": [n if n != "aval" else "avalanche" for n in A.ENDPOINT_DTYPE.names
                               if n != "_pad"]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "avm.h"', "int main(void) {"]
    for t, names in fields.items():
        lines.append(f'  printf("{t} size %zu\\n", sizeof({t}));')
        for n in names:
            lines.append(f'  printf("{t} {n} %zu\\n", offsetof({t}, {n}));')
    for t in ("avm_endpoint_arrays", "avm_noalloc_out"):
        lines.append(f'  printf("{t} size %zu\\n", sizeof({t}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n"):
        if line:
            t, n, v = line.split()
            got[(t, n)] = int(v)
    assert got[("avm_counts", "size")] == A.COUNTS_DTYPE.itemsize
    for n in A.COUNTS_DTYPE.names:
        if n != "_pad":
            assert got[("avm_counts", n)] == A.COUNTS_DTYPE.fields[n][1], n
    assert got[("avm_end_record", "size")] == A.END_RECORD_DTYPE.itemsize
    for n in A.END_RECORD_DTYPE.names:
        assert got[("avm_end_record", n)] == A.END_RECORD_DTYPE.fields[n][1], n
    assert got[("avm_endpoint", "size")] == A.ENDPOINT_DTYPE.itemsize
    for n in A.ENDPOINT_DTYPE.names:
        if n != "_pad":
            assert got[("avm_endpoint", "avalanche" if n == "aval" else n)] == A.ENDPOINT_DTYPE.fields[n][1], n
    assert got[("avm_endpoint_arrays", "size")] == C.sizeof(A._EndpointArrays)
    assert got[("avm_noalloc_out", "size")] == C.sizeof(A._NoallocOut)


def test_argument_errors_without_a_device(A):
    L = A.lib()
    h = C.c_void_p()
    # gas: no channels, bad sizes, negative cross-section
    assert L.avm_gas_create(0, 100.0, 10, 1e19, 0, None, 0, C.byref(h)) == A.AVM_E_ARG
    assert b"channel" in L.avm_last_error()
    gas = W.toy_gas()
    chans = (A._Channel * 3)()
    keep = []
    for i, ch in enumerate(gas.channels):
        v = np.ascontiguousarray(ch.values, dtype=np.float64).copy()
        if i == 0:
            v[3] = -1.0
        keep.append(v)
        chans[i] = A._Channel(ch.kind, ch.angular, ch.split, ch.values_kind, ch.loss_eV, ch.e_lo_eV,
                              ch.e_hi_eV, ch.mass_ratio, ch.split_w_eV, ch.screening_eV,
                              v.ctypes.data_as(C.POINTER(C.c_double)))
    assert L.avm_gas_create(0, gas.e_max_eV, gas.n_bins, gas.density_cm3, 3, chans, 0, C.byref(h)) == A.AVM_E_ARG
    assert b"bad value" in L.avm_last_error()
    assert L.avm_gas_create(0, -1.0, gas.n_bins, 1e19, 3, chans, 0, C.byref(h)) == A.AVM_E_ARG
    assert L.avm_gas_create(0, 100.0, 0, 1e19, 3, chans, 0, C.byref(h)) == A.AVM_E_ARG
    assert not h.value
    # fields
    E = np.array([0.0, 0.0, -1e4])
    dp = C.POINTER(C.c_double)
    assert L.avm_field_slab(0, 1.0, 0.0, 1, E.ctypes.data_as(dp), None, C.byref(h)) == A.AVM_E_ARG
    Bx = np.array([0.1, 0.0, 0.0])
    assert L.avm_field_slab(0, 0.0, 1.0, 1, E.ctypes.data_as(dp), Bx.ctypes.data_as(dp),
                            C.byref(h)) == A.AVM_E_UNSUPPORTED
    bad = np.array([0.0, math.nan, 0.0])
    assert L.avm_field_slab(0, 0.0, 1.0, 1, bad.ctypes.data_as(dp), None, C.byref(h)) == A.AVM_E_ARG
    fp = C.POINTER(C.c_float)
    m = np.zeros((4, 4), dtype=np.float32)
    assert L.avm_field_polar_map(0, 1.0, 0.5, 4, 4, m.ctypes.data_as(fp), m.ctypes.data_as(fp), None,
                                 C.byref(h)) == A.AVM_E_ARG
    # runs: NULL handles
    o = A._Opts()
    assert L.avm_run_create(None, None, None, 0, 0, 0, C.byref(o), C.byref(h)) == A.AVM_E_ARG
    assert L.avm_run_execute(None) == A.AVM_E_ARG
    assert L.avm_run_sync(None) == A.AVM_E_ARG
    assert L.avm_gas_get_info(None, None) == A.AVM_E_ARG
    assert L.avm_gas_set_band_bins(None, 10) == A.AVM_E_ARG
    assert L.avm_gas_set_penning(None, 1, 0.5, 1.0) == A.AVM_E_ARG
    assert L.avm_run_set_signal(None, 0.0, 0.01, 10) == A.AVM_E_ARG
    assert L.avm_run_signal(None, 0, 0, None) == A.AVM_E_ARG
    assert L.avm_run_set_seed(None, 1) == A.AVM_E_ARG
    res = A._TuneResult()
    assert L.avm_autotune(None, None, None, 0, 0, 0, C.byref(o), 0, None, C.byref(res)) == A.AVM_E_ARG
    L.avm_gas_destroy(None)
    L.avm_field_destroy(None)
    L.avm_run_destroy(None)


def test_product_path_fails_loudly_without_library(A, monkeypatch, tmp_path):
    monkeypatch.setattr(A, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(A, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        A.lib()
