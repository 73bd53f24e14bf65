"""ctypes wrapper of the FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product path never does.  It imports nothing
from the HIP package: gases, fields and primaries are plain objects with the
attributes of the seeded workload descriptions (duck typing), and the
endpoints come back as a numpy structured array.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "avm_oracle.c")

ENDPOINT_DTYPE = np.dtype([
    ("x0", "<f8"), ("y0", "<f8"), ("z0", "<f8"), ("t0", "<f8"), ("e0", "<f8"),
    ("x1", "<f8"), ("y1", "<f8"), ("z1", "<f8"), ("t1", "<f8"), ("e1", "<f8"),
    ("eid", "<u8"), ("parent", "<u8"),
    ("aval", "<u4"), ("status", "<u4"), ("n_real", "<u4"), ("n_ion", "<u4"),
    ("n_null", "<u4"), ("n_masked", "<u4"), ("n_band", "<u4"), ("n_overflow", "<u4"),
    ("trace", "<u4"), ("_pad", "<u4"),
])
assert ENDPOINT_DTYPE.itemsize == 136

K_MAX_DEFAULT = (1 << 30) - 1


def build(force: bool = True, path: str = LIB_PATH, defines=()) -> str:
    """Compile liboracle.so with gcc (plain C, FP64, no contraction).
    ``defines``: extra macros (the ORC_PLANT_* switches of the pin tests)."""
    if force or not os.path.exists(path):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall",
               "-fPIC", "-shared", "-pthread"] + ["-D" + d for d in defines] + [
               "-o", path + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(path + ".tmp", path)
    return path


class _Channel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("angular", C.c_int32), ("split", C.c_int32),
                ("values_kind", C.c_int32), ("loss_eV", C.c_double), ("e_lo_eV", C.c_double),
                ("e_hi_eV", C.c_double), ("mass_ratio", C.c_double), ("split_w_eV", C.c_double),
                ("screening_eV", C.c_double), ("values", C.POINTER(C.c_double))]


class _Opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("banded", C.c_int32), ("fifo", C.c_int32),
                ("t_max_ns", C.c_double), ("k_max", C.c_uint32), ("n_threads", C.c_int32),
                ("band_lookahead", C.c_double)]


class _Signal(C.Structure):
    _fields_ = [("t0_ns", C.c_double), ("dt_ns", C.c_double), ("n_bins", C.c_int32),
                ("n_rows", C.c_uint32), ("out", C.POINTER(C.c_double))]


_lib = None
_variants = {}


def _load(path):
    L = C.CDLL(path)
    _declare(L)
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(SRC) > os.path.getmtime(LIB_PATH):
            build()
        _lib = _load(LIB_PATH)
    return _lib


class planted:
    """Context in which the oracle is a build with one planted mistake
    (``with planted("ORC_PLANT_PHI_SWAP"): ...``): the pin tests use it to
    show that their pin fails on that mistake.  Objects made inside the
    context belong to that build."""

    def __init__(self, macro):
        self.macro = macro

    def __enter__(self):
        global _lib
        if self.macro not in _variants:
            d = os.path.join(HERE, "_variants")
            os.makedirs(d, exist_ok=True)
            path = os.path.join(d, f"liboracle_{self.macro.lower()}.so")
            build(True, path, (self.macro,))
            _variants[self.macro] = _load(path)
        lib()
        self._saved = _lib
        _lib = _variants[self.macro]
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


def _declare(L):
    """Argument and result types of the C entry points."""
    dp, vp, u32p = C.POINTER(C.c_double), C.c_void_p, C.POINTER(C.c_uint32)
    L.orc_gas_create.argtypes = [C.c_double, C.c_int32, C.c_double, C.c_int32,
                                 C.POINTER(_Channel), C.c_int32, C.POINTER(vp)]
    L.orc_gas_destroy.argtypes = [vp]
    L.orc_gas_set_penning.argtypes = [vp, C.c_int32, C.c_double, C.c_double]
    L.orc_gas_gamma.argtypes = [vp]
    L.orc_gas_gamma.restype = C.c_double
    L.orc_gas_n_bands.argtypes = [vp]
    L.orc_gas_band.argtypes = [vp, C.c_int32, dp, dp]
    L.orc_gas_set_gamma.argtypes = [vp, C.c_double]
    L.orc_gas_rates.argtypes = [vp, C.c_double, dp, dp]
    L.orc_gas_cumulative.argtypes = [vp, dp]
    L.orc_gas_band_of.argtypes = [vp, C.c_double]
    L.orc_field_slab.argtypes = [C.c_double, C.c_double, C.c_uint32, dp, dp, C.POINTER(vp)]
    fp = C.POINTER(C.c_float)
    L.orc_field_polar.argtypes = [C.c_double, C.c_double, C.c_int32, C.c_int32, fp, fp, dp,
                                  C.POINTER(vp)]
    L.orc_field_destroy.argtypes = [vp]
    L.orc_field_eval.argtypes = [vp, dp, C.c_uint32, dp]
    L.orc_run.argtypes = [vp, vp, vp, C.POINTER(C.c_uint64), C.c_uint64, C.POINTER(_Opts),
                          C.POINTER(vp), C.POINTER(C.c_int32)]
    L.orc_run_signal.argtypes = [vp, vp, vp, C.POINTER(C.c_uint64), C.c_uint64,
                                 C.POINTER(_Opts), C.POINTER(_Signal), C.POINTER(vp),
                                 C.POINTER(C.c_int32)]
    L.orc_weighting.argtypes = [vp, dp]
    L.orc_weighting.restype = C.c_double
    L.orc_result_count.argtypes = [vp]
    L.orc_result_count.restype = C.c_uint64
    L.orc_result_copy.argtypes = [vp, vp]
    L.orc_result_destroy.argtypes = [vp]
    L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
    L.orc_u53.argtypes = [C.c_uint32, C.c_uint32]
    L.orc_u53.restype = C.c_double
    L.orc_u24.argtypes = [C.c_uint32]
    L.orc_u24.restype = C.c_float
    L.orc_cos_screened_rutherford.argtypes = [C.c_double, C.c_double, C.c_double]
    L.orc_cos_screened_rutherford.restype = C.c_double
    L.orc_split_energy.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double]
    L.orc_split_energy.restype = C.c_double
    L.orc_rotate.argtypes = [dp, C.c_double, C.c_double, dp]
    L.orc_elastic.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp]
    L.orc_slab_exit.argtypes = [C.c_double] * 6 + [dp]
    L.orc_band_root.argtypes = [dp, dp, C.c_double]
    L.orc_band_root.restype = C.c_double
    L.orc_propagate.argtypes = [dp, dp, dp, dp, C.c_double, dp, dp]
    L.orc_helical_bound.argtypes = [dp, dp, dp, dp]
    L.orc_helical_bound_root.argtypes = [dp, C.c_double]
    L.orc_helical_bound_root.restype = C.c_double
    L.orc_majorant_violations.restype = C.c_uint64
    L.orc_k_a.restype = C.c_double
    L.orc_k_b.restype = C.c_double


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Gas:
    """Rate table built by the oracle from a gas description."""

    def __init__(self, gas, band_bins=None):
        L = lib()
        self._L = L
        self._keep = []
        chans = (_Channel * len(gas.channels))()
        for i, ch in enumerate(gas.channels):
            v = np.ascontiguousarray(ch.values, dtype=np.float64)
            if v.size != gas.n_bins + 1:
                raise ValueError("channel values must have n_bins+1 entries")
            self._keep.append(v)
            chans[i] = _Channel(ch.kind, ch.angular, ch.split, ch.values_kind, ch.loss_eV,
                                ch.e_lo_eV, ch.e_hi_eV, ch.mass_ratio, ch.split_w_eV,
                                ch.screening_eV, _dptr(v))
        h = C.c_void_p()
        bb = gas.band_bins if band_bins is None else band_bins
        rc = L.orc_gas_create(gas.e_max_eV, gas.n_bins, gas.density_cm3, len(gas.channels),
                              chans, bb, C.byref(h))
        if rc:
            raise ValueError(f"orc_gas_create failed ({rc})")
        self.h = h
        for i, ch in enumerate(gas.channels):
            p = float(getattr(ch, "penning_prob", 0.0))
            if p > 0.0:
                rc = L.orc_gas_set_penning(h, i, p, float(getattr(ch, "penning_energy_eV", 0.0)))
                if rc:
                    raise ValueError(f"orc_gas_set_penning failed ({rc})")
        self.n_ch = len(gas.channels)
        self.n_bins = gas.n_bins

    def __del__(self):
        if getattr(self, "h", None):
            self._L.orc_gas_destroy(self.h)
            self.h = None

    @property
    def gamma(self):
        return self._L.orc_gas_gamma(self.h)

    @property
    def n_bands(self):
        return self._L.orc_gas_n_bands(self.h)

    def band(self, b):
        g, e = C.c_double(), C.c_double()
        if self._L.orc_gas_band(self.h, b, C.byref(g), C.byref(e)):
            raise IndexError(b)
        return g.value, e.value

    def band_of(self, e):
        return self._L.orc_gas_band_of(self.h, e)

    def set_gamma(self, gamma):
        if self._L.orc_gas_set_gamma(self.h, gamma):
            raise ValueError("gamma below the table maximum")

    def rates(self, e):
        nu = np.zeros(self.n_ch)
        tot = C.c_double()
        over = self._L.orc_gas_rates(self.h, float(e), _dptr(nu), C.byref(tot))
        return nu, tot.value, bool(over)

    def cumulative(self):
        out = np.zeros((self.n_bins + 1, self.n_ch))
        self._L.orc_gas_cumulative(self.h, _dptr(out))
        return out


class Field:
    def __init__(self, field):
        L = lib()
        self._L = L
        h = C.c_void_p()
        B = np.ascontiguousarray(getattr(field, "B_T", np.zeros(3)), dtype=np.float64)
        self._keep = [B]
        if hasattr(field, "z_lo_cm"):
            E = np.ascontiguousarray(field.E_vcm, dtype=np.float64).reshape(-1, 3)
            self._keep.append(E)
            rc = L.orc_field_slab(field.z_lo_cm, field.z_hi_cm, E.shape[0], _dptr(E), _dptr(B),
                                  C.byref(h))
        else:
            er = np.ascontiguousarray(field.E_r, dtype=np.float32)
            ep = np.ascontiguousarray(field.E_phi, dtype=np.float32)
            self._keep += [er, ep]
            fp = C.POINTER(C.c_float)
            rc = L.orc_field_polar(field.a_cm, field.b_cm, er.shape[0], er.shape[1],
                                   er.ctypes.data_as(fp), ep.ctypes.data_as(fp), _dptr(B),
                                   C.byref(h))
        if rc:
            raise ValueError(f"oracle field creation failed ({rc})")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            self._L.orc_field_destroy(self.h)
            self.h = None

    def weighting(self, r):
        """Weighting potential of the readout electrode at r (orc_weighting)."""
        rr = np.ascontiguousarray(r, dtype=np.float64)
        return self._L.orc_weighting(self.h, _dptr(rr))

    def eval(self, r, aval=0):
        r = np.ascontiguousarray(r, dtype=np.float64)
        E = np.zeros(3)
        self._L.orc_field_eval(self.h, _dptr(r), aval, _dptr(E))
        return E


def run(gas, field, primaries, seed, *, banded=False, fifo=False, t_max=math.inf,
        k_max=K_MAX_DEFAULT, threads=0, ids=None, return_threads=False, signal=None,
        band_lookahead=0.0):
    """Transport the primaries; returns endpoints sorted by (aval, eid).

    ``gas``/``field`` are oracle ``Gas``/``Field`` objects or workload
    descriptions (built on the fly).  ``ids`` gives the primary ids used for
    the electron ids (default: array positions).  ``signal=(t0_ns, dt_ns,
    n_bins, n_rows)`` also returns the induced-signal array [n_rows, n_bins]
    (see orc_run_signal): the result is then (endpoints, signal)."""
    L = lib()
    g = gas if isinstance(gas, Gas) else Gas(gas)
    f = field if isinstance(field, Field) else Field(field)
    if g._L is not L or f._L is not L:
        raise ValueError("gas or field built by another oracle build (planted context)")
    prim = np.ascontiguousarray(primaries)
    if prim.dtype.itemsize != 72:
        raise ValueError("primary records must be 72 bytes")
    idp = None
    if ids is not None:
        ida = np.ascontiguousarray(ids, dtype=np.uint64)
        idp = ida.ctypes.data_as(C.POINTER(C.c_uint64))
    o = _Opts(int(seed), int(bool(banded)), int(bool(fifo)), float(t_max), int(k_max), int(threads),
              float(band_lookahead))
    h = C.c_void_p()
    used = C.c_int32()
    sig = None
    sp = None
    if signal is not None:
        t0, dt, nb, nr = signal
        sig = np.zeros((int(nr), int(nb)))
        sp = C.byref(_Signal(float(t0), float(dt), int(nb), int(nr), _dptr(sig)))
    rc = L.orc_run_signal(g.h, f.h, prim.ctypes.data_as(C.c_void_p), idp, prim.size, C.byref(o),
                          sp, C.byref(h), C.byref(used))
    if rc:
        raise ValueError(f"orc_run failed ({rc})")
    n = L.orc_result_count(h)
    out = np.zeros(n, dtype=ENDPOINT_DTYPE)
    if n:
        L.orc_result_copy(h, out.ctypes.data_as(C.c_void_p))
    L.orc_result_destroy(h)
    out = out[np.lexsort((out["eid"], out["aval"]))]
    res = out if sig is None else (out, sig)
    if return_threads:
        return res, used.value
    return res


def per_avalanche(ep, n_aval):
    """Per-avalanche sums of the endpoint counters."""
    a = ep["aval"].astype(np.int64)
    res = {"n_endpoints": np.bincount(a, minlength=n_aval)}
    for key in ("n_real", "n_ion", "n_null", "n_masked", "n_band", "n_overflow"):
        res[key] = np.bincount(a, weights=ep[key].astype(np.float64), minlength=n_aval).astype(np.int64)
    res["n_att"] = np.bincount(a, weights=(ep["status"] == 3).astype(np.float64),
                               minlength=n_aval).astype(np.int64)
    return res


# scalar helpers for the pins
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(o)


def u53(hi, lo):
    return lib().orc_u53(hi, lo)


def u24(w):
    return lib().orc_u24(w)


def k_a():
    return lib().orc_k_a()


def k_b():
    return lib().orc_k_b()


def cos_screened_rutherford(u, e, screening):
    return lib().orc_cos_screened_rutherford(u, e, screening)


def split_energy(split, u, e_avail, w):
    return lib().orc_split_energy(split, u, e_avail, w)


def rotate(d, cos_t, phi):
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_rotate(_dptr(d), cos_t, phi, _dptr(out))
    return out


def elastic(e, mu, cos_chi):
    eo, cl = C.c_double(), C.c_double()
    lib().orc_elastic(e, mu, cos_chi, C.byref(eo), C.byref(cl))
    return eo.value, cl.value


def slab_exit(z0, vz, az, z_lo, z_hi, T):
    s = C.c_double()
    side = lib().orc_slab_exit(z0, vz, az, z_lo, z_hi, T, C.byref(s))
    return side, (s.value if side else None)


def band_root(v, a, e_edge):
    v = np.ascontiguousarray(v, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    return lib().orc_band_root(_dptr(v), _dptr(a), e_edge)


def propagate(r0, v0, E, B, s):
    r0, v0, E, B = (np.ascontiguousarray(x, dtype=np.float64) for x in (r0, v0, E, B))
    r, v = np.zeros(3), np.zeros(3)
    lib().orc_propagate(_dptr(r0), _dptr(v0), _dptr(E), _dptr(B), s, _dptr(r), _dptr(v))
    return r, v
