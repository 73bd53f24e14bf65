"""Python binding of libavm (include/avm.h): argument marshalling only.

Every step of the transport runs in the HIP library; this module converts
workload descriptions into the C structures, passes torch device pointers
and streams through, and copies results into numpy arrays.  It raises
immediately if the library is missing -- there is no fallback path.

The C entry points are available under their own names (``avm_gas_create``
and so on, see ``lib()``); ``Gas``, ``Field`` and ``Run`` wrap them with
ownership, and ``run()`` does a whole avalanche simulation in one call.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "_lib", "libavm.so")

AVM_OK, AVM_E_ARG, AVM_E_NOMEM, AVM_E_HIP, AVM_E_CAPACITY, AVM_E_UNSUPPORTED, AVM_E_TIMEOUT, AVM_E_STATE = range(8)
FP64, FP32_MIXED = 0, 1
GLOBAL, BANDED = 0, 1
PLAIN, BATCHED = 0, 1

ENDPOINT_DTYPE = np.dtype([
    ("x0", "<f8"), ("y0", "<f8"), ("z0", "<f8"), ("t0", "<f8"), ("e0", "<f8"),
    ("x1", "<f8"), ("y1", "<f8"), ("z1", "<f8"), ("t1", "<f8"), ("e1", "<f8"),
    ("eid", "<u8"), ("parent", "<u8"),
    ("aval", "<u4"), ("status", "<u4"), ("n_real", "<u4"), ("n_ion", "<u4"),
    ("n_null", "<u4"), ("n_masked", "<u4"), ("n_band", "<u4"), ("n_overflow", "<u4"),
    ("trace", "<u4"), ("_pad", "<u4"),
])
assert ENDPOINT_DTYPE.itemsize == 136


class AvmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"avm status {status}: {msg}")
        self.status = status


class _Channel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("angular", C.c_int32), ("split", C.c_int32),
                ("values_kind", C.c_int32), ("loss_eV", C.c_double), ("e_lo_eV", C.c_double),
                ("e_hi_eV", C.c_double), ("mass_ratio", C.c_double), ("split_w_eV", C.c_double),
                ("screening_eV", C.c_double), ("values", C.POINTER(C.c_double))]


class _GasInfo(C.Structure):
    _fields_ = [("gamma", C.c_double), ("e_max_eV", C.c_double), ("n_bins", C.c_int32),
                ("n_channels", C.c_int32), ("n_bands", C.c_int32), ("band_bins", C.c_int32)]


class _Opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("precision", C.c_int32), ("majorant", C.c_int32),
                ("mode", C.c_int32), ("flights_per_pass", C.c_int32), ("t_max_ns", C.c_double),
                ("capacity", C.c_uint64), ("k_max", C.c_uint32), ("waves_per_cu", C.c_int32),
                ("timeout_s", C.c_double), ("hip_stream", C.c_void_p), ("graph", C.c_int32),
                ("band_lookahead", C.c_float)]


class _Counts(C.Structure):
    _fields_ = [("n_endpoints", C.c_uint64), ("n_ion", C.c_uint64), ("n_att", C.c_uint64),
                ("n_real", C.c_uint64), ("n_null", C.c_uint64), ("n_masked", C.c_uint64),
                ("n_band", C.c_uint64), ("n_overflow", C.c_uint64), ("n_status", C.c_uint64 * 9),
                ("n_requested", C.c_uint64), ("truncated", C.c_uint32), ("_pad", C.c_uint32)]


# numpy view of an array of avm_counts records
COUNTS_DTYPE = np.dtype([(n, "<u8") for n in ("n_endpoints", "n_ion", "n_att", "n_real", "n_null",
                                               "n_masked", "n_band", "n_overflow")]
                        + [("n_status", "<u8", (9,)), ("n_requested", "<u8"), ("truncated", "<u4"),
                           ("_pad", "<u4")])
assert COUNTS_DTYPE.itemsize == C.sizeof(_Counts)


class _TuneResult(C.Structure):
    _fields_ = [("flights_per_pass", C.c_int32), ("waves_per_cu", C.c_int32),
                ("band_bins", C.c_int32), ("trials", C.c_int32), ("from_cache", C.c_int32),
                ("band_lookahead", C.c_float), ("best_ms", C.c_double), ("start_ms", C.c_double),
                ("key", C.c_uint64)]


TUNE_BANDS = 1


# The start of each electron is stored as arrays (name, numpy kind); its end
# as one avm_end_record of 72 bytes (name, numpy kind, byte offset).
_START_ARRAYS = (("x0", "f8"), ("y0", "f8"), ("z0", "f8"), ("t0", "f8"), ("e0", "f8"),
                 ("eid", "u8"), ("parent", "u8"), ("avalanche", "u4"))
END_RECORD_DTYPE = np.dtype([
    ("x1", "<f8"), ("y1", "<f8"), ("z1", "<f8"), ("t1", "<f8"), ("e1", "<f8"),
    ("status", "<u4"), ("n_real", "<u4"), ("n_ion", "<u4"), ("n_null", "<u4"),
    ("n_masked", "<u4"), ("n_band", "<u4"), ("n_overflow", "<u4"), ("trace", "<u4"),
])
assert END_RECORD_DTYPE.itemsize == 72
_END_FIELDS = tuple((n, END_RECORD_DTYPE[n].str[1:], END_RECORD_DTYPE.fields[n][1])
                    for n in END_RECORD_DTYPE.names)


class _EndpointArrays(C.Structure):
    _fields_ = [(n, C.c_void_p) for n, _ in _START_ARRAYS] + [("end", C.c_void_p)]


NOALLOC_MAX_ELECTRONS = 4194304
NOALLOC_TIMEOUT, NOALLOC_BAD_AVALANCHE, NOALLOC_TRUNCATED = 1, 2, 4


class _NoallocOut(C.Structure):
    _fields_ = [(n, C.c_void_p) for n, _ in _START_ARRAYS] + [
        ("end", C.c_void_p), ("aval_counts", C.c_void_p), ("counts", C.c_void_p),
        ("flags", C.c_void_p)]


# C entry points: name -> (argtypes, restype)
_VP = C.c_void_p
_DP = C.POINTER(C.c_double)
_FP = C.POINTER(C.c_float)
_SIGS = {
    "avm_last_error": ([], C.c_char_p),
    "avm_abi_version": ([], C.c_int32),
    "avm_device_count": ([], C.c_int32),
    "avm_gas_create": ([C.c_int32, C.c_double, C.c_int32, C.c_double, C.c_int32,
                        C.POINTER(_Channel), C.c_int32, C.POINTER(_VP)], C.c_int),
    "avm_gas_get_info": ([_VP, C.POINTER(_GasInfo)], C.c_int),
    "avm_gas_get_tables": ([_VP, _DP, _DP, _DP], C.c_int),
    "avm_gas_set_band_bins": ([_VP, C.c_int32], C.c_int),
    "avm_gas_set_penning": ([_VP, C.c_int32, C.c_double, C.c_double], C.c_int),
    "avm_gas_destroy": ([_VP], None),
    "avm_field_slab": ([C.c_int32, C.c_double, C.c_double, C.c_uint32, _DP, _DP, C.POINTER(_VP)], C.c_int),
    "avm_field_polar_map": ([C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_int32, _FP, _FP,
                             _DP, C.POINTER(_VP)], C.c_int),
    "avm_field_destroy": ([_VP], None),
    "avm_run_create": ([_VP, _VP, _VP, C.c_int32, C.c_uint64, C.c_uint32, C.POINTER(_Opts),
                        C.POINTER(_VP)], C.c_int),
    "avm_run_execute": ([_VP], C.c_int),
    "avm_run_sync": ([_VP], C.c_int),
    "avm_run_counts": ([_VP, C.POINTER(_Counts)], C.c_int),
    "avm_run_avalanche_counts": ([_VP, C.c_uint32, C.c_uint32, _VP], C.c_int),
    "avm_run_num_endpoints": ([_VP, C.POINTER(C.c_uint64)], C.c_int),
    "avm_run_endpoints": ([_VP, C.c_uint64, C.c_uint64, _VP], C.c_int),
    "avm_run_endpoint_arrays": ([_VP, C.POINTER(_EndpointArrays)], C.c_int),
    "avm_run_timing": ([_VP, _DP, C.POINTER(C.c_uint32)], C.c_int),
    "avm_run_set_seed": ([_VP, C.c_uint64], C.c_int),
    "avm_run_destroy": ([_VP], None),
    "avm_run_set_signal": ([_VP, C.c_double, C.c_double, C.c_int32], C.c_int),
    "avm_run_signal": ([_VP, C.c_uint32, C.c_uint32, _DP], C.c_int),
    "avm_autotune": ([_VP, _VP, _VP, C.c_int32, C.c_uint64, C.c_uint32, C.POINTER(_Opts), C.c_uint32,
                      C.c_char_p, C.POINTER(_TuneResult)], C.c_int),
    "avm_run_noalloc": ([_VP, _VP, _VP, C.c_uint64, C.c_uint32, C.POINTER(_Opts),
                         C.POINTER(_NoallocOut)], C.c_int),
}
EXPORTED = tuple(_SIGS)

_lib = None


def lib():
    """The loaded libavm.so with typed entry points (raises if missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libavm.so not found at {LIB_PATH}: build it with "
                               "__graft_entry__.build() (hipcc, gfx950); there is no CPU fallback")
        # torch ships its own HIP runtime; loading it first makes libavm bind
        # to the same runtime, so device pointers and streams are shared
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc, what=""):
    if rc != AVM_OK:
        msg = lib().avm_last_error().decode(errors="replace")
        raise AvmError(rc, f"{what}: {msg}" if what else msg)


def __getattr__(name):
    # the C entry points under their own names: avm.avm_gas_create(...)
    if name in _SIGS:
        return getattr(lib(), name)
    raise AttributeError(name)


def device_count() -> int:
    return lib().avm_device_count()


class Gas:
    def __init__(self, gas, device: int = 0, band_bins: Optional[int] = None):
        chans = (_Channel * len(gas.channels))()
        keep = []
        for i, ch in enumerate(gas.channels):
            v = np.ascontiguousarray(ch.values, dtype=np.float64)
            if v.size != gas.n_bins + 1:
                raise ValueError("channel values must have n_bins+1 entries")
            keep.append(v)
            chans[i] = _Channel(ch.kind, ch.angular, ch.split, ch.values_kind, ch.loss_eV, ch.e_lo_eV,
                                ch.e_hi_eV, ch.mass_ratio, ch.split_w_eV, ch.screening_eV,
                                v.ctypes.data_as(_DP))
        h = _VP()
        bb = gas.band_bins if band_bins is None else band_bins
        _check(lib().avm_gas_create(device, gas.e_max_eV, gas.n_bins, gas.density_cm3,
                                    len(gas.channels), chans, bb, C.byref(h)), "avm_gas_create")
        self.h = h
        for i, ch in enumerate(gas.channels):
            if float(getattr(ch, "penning_prob", 0.0)) > 0.0:
                self.set_penning(i, ch.penning_prob, ch.penning_energy_eV)
        info = _GasInfo()
        _check(lib().avm_gas_get_info(h, C.byref(info)))
        self.gamma = info.gamma
        self.n_bins = info.n_bins
        self.n_channels = info.n_channels
        self.n_bands = info.n_bands
        self.band_bins = info.band_bins

    def _refresh(self):
        info = _GasInfo()
        _check(lib().avm_gas_get_info(self.h, C.byref(info)))
        self.n_bands = info.n_bands
        self.band_bins = info.band_bins

    def set_penning(self, channel: int, probability: float, energy_eV: float):
        """Penning transfer of an excitation channel (avm_gas_set_penning)."""
        _check(lib().avm_gas_set_penning(self.h, int(channel), float(probability), float(energy_eV)),
               "avm_gas_set_penning")

    def set_band_bins(self, band_bins: int):
        """Rebuild the band majorants with a new band width (avm_gas_set_band_bins)."""
        _check(lib().avm_gas_set_band_bins(self.h, int(band_bins)), "avm_gas_set_band_bins")
        self._refresh()

    def tables(self):
        cum = np.zeros((self.n_bins + 1, self.n_channels))
        bg = np.zeros(self.n_bands)
        be = np.zeros(self.n_bands)
        _check(lib().avm_gas_get_tables(self.h, cum.ctypes.data_as(_DP), bg.ctypes.data_as(_DP),
                                        be.ctypes.data_as(_DP)))
        return cum, bg, be

    def close(self):
        if getattr(self, "h", None):
            lib().avm_gas_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may be gone
            pass


class Field:
    def __init__(self, field, device: int = 0):
        h = _VP()
        B = np.ascontiguousarray(getattr(field, "B_T", np.zeros(3)), dtype=np.float64)
        if hasattr(field, "z_lo_cm"):
            E = np.ascontiguousarray(field.E_vcm, dtype=np.float64).reshape(-1, 3)
            _check(lib().avm_field_slab(device, field.z_lo_cm, field.z_hi_cm, E.shape[0],
                                        E.ctypes.data_as(_DP), B.ctypes.data_as(_DP), C.byref(h)),
                   "avm_field_slab")
        else:
            er = np.ascontiguousarray(field.E_r, dtype=np.float32)
            ep = np.ascontiguousarray(field.E_phi, dtype=np.float32)
            _check(lib().avm_field_polar_map(device, field.a_cm, field.b_cm, er.shape[0], er.shape[1],
                                             er.ctypes.data_as(_FP), ep.ctypes.data_as(_FP),
                                             B.ctypes.data_as(_DP), C.byref(h)), "avm_field_polar_map")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().avm_field_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may be gone
            pass


def _counts_dict(c: _Counts):
    d = {k: int(getattr(c, k)) for k in ("n_endpoints", "n_ion", "n_att", "n_real", "n_null",
                                         "n_masked", "n_band", "n_overflow", "n_requested",
                                         "truncated")}
    d["n_status"] = [int(x) for x in c.n_status]
    return d


def _primaries_arg(primaries):
    """(pointer, on_device, count, object to keep alive) for primary records:
    a numpy structured array of 72-byte records, or a GPU torch tensor
    holding them."""
    if hasattr(primaries, "data_ptr"):  # torch tensor
        if not primaries.is_cuda:
            raise ValueError("torch primaries must live on the GPU")
        if primaries.numel() * primaries.element_size() % 72:
            raise ValueError("primary tensor size is not a multiple of 72 bytes")
        return (C.c_void_p(primaries.data_ptr()), 1,
                primaries.numel() * primaries.element_size() // 72, primaries)
    p = np.ascontiguousarray(primaries)
    if p.dtype.itemsize != 72:
        raise ValueError("primary records must be 72 bytes")
    return C.c_void_p(p.ctypes.data), 0, p.size, p


def _make_opts(seed, precision, majorant, mode, flights_per_pass, t_max, capacity, k_max,
               waves_per_cu, timeout_s, stream, graph, band_lookahead=0.0):
    st = None
    if stream is not None:
        st = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    return _Opts(int(seed), precision, majorant, mode, int(flights_per_pass), float(t_max),
                 int(capacity), int(k_max), int(waves_per_cu), float(timeout_s), st,
                 int(bool(graph)), float(band_lookahead))


def autotune(gas: Gas, field: Field, primaries, n_aval: int, *, seed: int, precision=FP64,
             majorant=GLOBAL, capacity=0, t_max=math.inf, k_max=0, timeout_s=0.0, stream=None,
             tune_bands=True, cache=None):
    """Choose flights_per_pass, waves_per_cu and (banded) the gas's band
    width for a batched run of these primaries (avm_autotune).  Returns a
    dict; pass its flights_per_pass, waves_per_cu and band_lookahead to Run."""
    ptr, on_dev, n_prim, keep = _primaries_arg(primaries)
    o = _make_opts(seed, precision, majorant, BATCHED, 0, t_max, capacity, k_max, 0, timeout_s,
                   stream, False)
    res = _TuneResult()
    path = None if cache is None else os.fsencode(cache)
    _check(lib().avm_autotune(gas.h, field.h, ptr, on_dev, n_prim, int(n_aval), C.byref(o),
                              TUNE_BANDS if tune_bands else 0, path, C.byref(res)), "avm_autotune")
    del keep
    gas._refresh()
    return {k: getattr(res, k) for k, _ in res._fields_ if not k.startswith("_")}


class Run:
    """One run (avm_run_*).  ``primaries``: a numpy structured array of
    72-byte primary records (host) or a torch uint8/any tensor on the GPU
    holding the same records (device, prim_on_device=1)."""

    def __init__(self, gas: Gas, field: Field, primaries, n_aval: int, *, seed: int,
                 precision=FP64, majorant=GLOBAL, mode=BATCHED, capacity=0, t_max=math.inf,
                 k_max=0, flights_per_pass=0, waves_per_cu=0, timeout_s=0.0, stream=None,
                 graph=False, band_lookahead=0.0):
        self._keep = [gas, field, primaries]
        ptr, on_dev, n_prim, keep = _primaries_arg(primaries)
        self._keep.append(keep)
        o = _make_opts(seed, precision, majorant, mode, flights_per_pass, t_max, capacity, k_max,
                       waves_per_cu, timeout_s, stream, graph, band_lookahead)
        h = _VP()
        _check(lib().avm_run_create(gas.h, field.h, ptr, on_dev, n_prim, int(n_aval), C.byref(o),
                                    C.byref(h)), "avm_run_create")
        self.h = h
        self.n_aval = int(n_aval)
        self.n_prim = n_prim

    def execute(self):
        _check(lib().avm_run_execute(self.h), "avm_run_execute")

    def sync(self, allow_truncation=False):
        rc = lib().avm_run_sync(self.h)
        if rc == AVM_E_CAPACITY and allow_truncation:
            return False
        _check(rc, "avm_run_sync")
        return True

    def counts(self):
        c = _Counts()
        _check(lib().avm_run_counts(self.h, C.byref(c)))
        return _counts_dict(c)

    def avalanche_counts(self):
        a = np.zeros(self.n_aval, dtype=COUNTS_DTYPE)
        if self.n_aval:
            _check(lib().avm_run_avalanche_counts(self.h, 0, self.n_aval, C.c_void_p(a.ctypes.data)))
        keys = ("n_endpoints", "n_ion", "n_att", "n_real", "n_null", "n_masked", "n_band", "n_overflow")
        return {k: a[k].astype(np.int64) for k in keys}

    def num_endpoints(self):
        n = C.c_uint64()
        _check(lib().avm_run_num_endpoints(self.h, C.byref(n)))
        return n.value

    def endpoints(self, first=0, n=None):
        total = self.num_endpoints()
        if n is None:
            n = total - first
        out = np.zeros(n, dtype=ENDPOINT_DTYPE)
        if n:
            _check(lib().avm_run_endpoints(self.h, first, n, C.c_void_p(out.ctypes.data)))
        return out

    def endpoint_arrays(self):
        a = _EndpointArrays()
        _check(lib().avm_run_endpoint_arrays(self.h, C.byref(a)))
        return {name: getattr(a, name) for name, _ in a._fields_}

    def endpoint_tensors(self, fields=None):
        """The stored endpoints as torch tensors on the device, without a
        copy (avm_run_endpoint_arrays; valid until the run is closed or
        executed again): a dict of 1-D tensors of num_endpoints() entries."""
        import torch
        n = self.num_endpoints()
        ptrs = self.endpoint_arrays()
        # unsigned fields come back as signed tensors of the same bits; the
        # end fields are strided views into the 72-byte end records
        typestrs = {"f8": "<f8", "u8": "<i8", "u4": "<i4"}
        views = [(name, k, ptrs[name] or 0, None) for name, k in _START_ARRAYS]
        views += [(name, k, (ptrs["end"] or 0) + off, (END_RECORD_DTYPE.itemsize,))
                  for name, k, off in _END_FIELDS]
        out = {}
        for name, k, ptr, strides in views:
            if fields is not None and name not in fields:
                continue
            cai = {"shape": (n,), "typestr": typestrs[k], "data": (ptr, False), "version": 2}
            if strides is not None:
                cai["strides"] = strides

            class _View:
                __cuda_array_interface__ = cai
            out[name] = torch.as_tensor(_View(), device="cuda")
        return out

    def set_signal(self, t0_ns: float, dt_ns: float, n_bins: int):
        """Request the induced signal on the readout electrode (avm_run_set_signal)."""
        _check(lib().avm_run_set_signal(self.h, float(t0_ns), float(dt_ns), int(n_bins)),
               "avm_run_set_signal")
        self.n_signal_bins = int(n_bins)

    def signal(self):
        """The induced signal [n_aval, n_bins] of the last execute (avm_run_signal)."""
        out = np.zeros((self.n_aval, self.n_signal_bins))
        _check(lib().avm_run_signal(self.h, 0, self.n_aval, out.ctypes.data_as(_DP)), "avm_run_signal")
        return out

    def set_seed(self, seed: int):
        """The seed of the following executes (avm_run_set_seed)."""
        _check(lib().avm_run_set_seed(self.h, int(seed)), "avm_run_set_seed")

    def timing(self):
        ms = C.c_double()
        it = C.c_uint32()
        _check(lib().avm_run_timing(self.h, C.byref(ms), C.byref(it)))
        return ms.value, it.value

    def close(self):
        if getattr(self, "h", None):
            lib().avm_run_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: the library may be gone
            pass


def noalloc_outputs(capacity: int, n_aval: int, device="cuda:0"):
    """Output tensors for avm_run_noalloc (the caller's memory: allocated
    here, by torch, before the call)."""
    import torch
    dt = {"f8": torch.float64, "u8": torch.int64, "u4": torch.int32}
    out = {n: torch.zeros(capacity, dtype=dt[k], device=device) for n, k in _START_ARRAYS}
    out["end"] = torch.zeros((capacity, END_RECORD_DTYPE.itemsize), dtype=torch.uint8, device=device)
    out["aval_counts"] = torch.zeros((max(n_aval, 1), 8), dtype=torch.int64, device=device)
    out["counts"] = torch.zeros(C.sizeof(_Counts), dtype=torch.uint8, device=device)
    out["flags"] = torch.zeros(1, dtype=torch.int32, device=device)
    return out


def run_noalloc(gas: Gas, field: Field, primaries, n_aval: int, out: dict, *, seed: int,
                precision=FP64, majorant=GLOBAL, t_max=math.inf, k_max=0, flights_per_pass=0,
                waves_per_cu=0, timeout_s=0.0, stream=None, band_lookahead=0.0):
    """avm_run_noalloc: the batched transport into the caller's output
    tensors ``out`` (see noalloc_outputs; capacity = their length), with the
    primaries a GPU tensor of 72-byte records.  Enqueued on ``stream``;
    returns at once."""
    ptr, on_dev, n_prim, keep = _primaries_arg(primaries)
    if not on_dev:
        raise ValueError("avm_run_noalloc takes device primaries")
    cap = out["x0"].numel()
    o = _make_opts(seed, precision, majorant, BATCHED, flights_per_pass, t_max, cap, k_max,
                   waves_per_cu, timeout_s, stream, False, band_lookahead)
    if out["end"].numel() != cap * END_RECORD_DTYPE.itemsize:
        raise ValueError("run_noalloc: out['end'] must hold one 72-byte record per slot")
    st = _NoallocOut(*[C.c_void_p(out[n].data_ptr()) for n, _ in _START_ARRAYS],
                     C.c_void_p(out["end"].data_ptr()), C.c_void_p(out["aval_counts"].data_ptr()),
                     C.c_void_p(out["counts"].data_ptr()), C.c_void_p(out["flags"].data_ptr()))
    _check(lib().avm_run_noalloc(gas.h, field.h, ptr, n_prim, int(n_aval), C.byref(o), C.byref(st)),
           "avm_run_noalloc")
    del keep


def noalloc_results(out: dict, n_aval: int):
    """(endpoints sorted by (avalanche, eid), totals dict, per-avalanche
    counts dict, flags) from the output tensors of a finished run_noalloc."""
    c = _Counts.from_buffer_copy(out["counts"].cpu().numpy().tobytes())
    tot = _counts_dict(c)
    n = min(tot["n_requested"], out["x0"].numel())
    ep = np.zeros(n, dtype=ENDPOINT_DTYPE)
    names = {"avalanche": "aval"}
    for name, _ in _START_ARRAYS:
        ep[names.get(name, name)] = out[name][:n].cpu().numpy().view(ENDPOINT_DTYPE[names.get(name, name)])
    end = out["end"][:n].cpu().numpy().reshape(-1).view(END_RECORD_DTYPE)
    for name in END_RECORD_DTYPE.names:
        ep[name] = end[name]
    ep = ep[np.lexsort((ep["eid"], ep["aval"]))]
    ac = out["aval_counts"][:n_aval].cpu().numpy().view(np.uint64).astype(np.int64)
    keys = ("n_endpoints", "n_ion", "n_att", "n_real", "n_null", "n_masked", "n_band", "n_overflow")
    per = {k: ac[:, j] for j, k in enumerate(keys)}
    return ep, tot, per, int(out["flags"].cpu().item())


def run(workload=None, *, gas=None, field=None, primaries=None, n_aval=None, seed=None,
        device=0, band_bins=None, sort=True, signal=None, **kw):
    """Whole simulation in one call.  Returns (endpoints sorted by
    (avalanche, eid), totals dict, per-avalanche counts dict), plus the
    induced signal [n_aval, n_bins] when ``signal=(t0_ns, dt_ns, n_bins)``."""
    if workload is not None:
        gas = gas or workload.gas
        field = field or workload.field
        primaries = workload.primaries if primaries is None else primaries
        n_aval = workload.n_aval if n_aval is None else n_aval
        seed = workload.seed if seed is None else seed
    g = gas if isinstance(gas, Gas) else Gas(gas, device, band_bins)
    f = field if isinstance(field, Field) else Field(field, device)
    r = Run(g, f, primaries, n_aval, seed=seed, **kw)
    if signal is not None:
        r.set_signal(*signal)
    r.execute()
    r.sync()
    ep = r.endpoints()
    tot = r.counts()
    per = r.avalanche_counts()
    sig = r.signal() if signal is not None else None
    r.close()
    if sort:
        ep = ep[np.lexsort((ep["eid"], ep["aval"]))]
    if signal is not None:
        return ep, tot, per, sig
    return ep, tot, per
