"""Thin ctypes binding of libpa.so (argument marshalling only).

Every function keeps the C name and signature of ``include/pa.h``; the
``Population`` class is a convenience wrapper that calls them.  All compute
runs in the library's HIP kernels: if libpa.so is missing this module raises
instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libpa.so")

PA_OK, PA_EINVAL, PA_ENOMEM, PA_ECAPACITY, PA_EDEVICE, PA_ESTATE, PA_EEMPTY = (
    0, -1, -2, -3, -4, -5, -6)
PA_FERRO, PA_PMJ = 0, 1
PA_INT8, PA_BITS = 0, 1
KERNEL_CLASSES = ("init", "sweep", "hist", "counts", "scatter", "gather")


class pa_config(C.Structure):
    _fields_ = [("L", C.c_int32), ("model", C.c_int32),
                ("J", C.c_void_p), ("R_target", C.c_int64),
                ("capacity", C.c_int64), ("layout", C.c_int32),
                ("rows_per_lane", C.c_int32), ("seed", C.c_uint64),
                ("population_id", C.c_uint32), ("stream", C.c_void_p)]


class pa_obs(C.Structure):
    _fields_ = [("R", C.c_int64), ("beta", C.c_double), ("e", C.c_double),
                ("abs_m", C.c_double), ("m2", C.c_double), ("C", C.c_double),
                ("sumE", C.c_int64), ("sumE2", C.c_int64),
                ("sumAbsM", C.c_int64), ("sumM2", C.c_int64),
                ("Emin", C.c_int32), ("Emax", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pa_timing(C.Structure):
    _fields_ = [("ms", C.c_double * 6), ("launches", C.c_int64 * 6),
                ("bytes", C.c_int64 * 6), ("attempts", C.c_int64)]


class PAError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed: %s (%d)" % (what, strerror(code), code))
        self.code = code


_lib = None


def lib():
    """Load libpa.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(
                "libpa.so is not built (run paper_2006_00561_amd/build.py); "
                "there is no fallback path")
        L = C.CDLL(SO_PATH)
        P, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        sig = {
            "pa_init": ([C.POINTER(pa_config), C.POINTER(P)], C.c_int),
            "pa_sweep": ([P, d, i32], C.c_int),
            "pa_resample": ([P, d, C.POINTER(i64)], C.c_int),
            "pa_observables": ([P, C.POINTER(pa_obs)], C.c_int),
            "pa_free_energy": ([P, C.POINTER(d), C.POINTER(d)], C.c_int),
            "pa_state": ([P, C.POINTER(i64), C.POINTER(d), C.POINTER(i32)],
                         C.c_int),
            "pa_get_population": ([P, P, P, P, i64], C.c_int),
            "pa_get_replicas": ([P, P, i64, P, P, P], C.c_int),
            "pa_get_counts": ([P, P, i64, C.POINTER(i64)], C.c_int),
            "pa_set_population": ([P, P, i64], C.c_int),
            "pa_histogram": ([P, P, i64, C.POINTER(i32), C.POINTER(i32)],
                             C.c_int),
            "pa_overlap": ([P, d, C.POINTER(d)], C.c_int),
            "pa_bisect_dbeta": ([P, d, d, C.POINTER(d)], C.c_int),
            "pa_set_timing": ([P, i32], C.c_int),
            "pa_get_timing": ([P, C.POINTER(pa_timing)], C.c_int),
            "pa_destroy": ([P], None),
            "pa_strerror": ([C.c_int], C.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def strerror(code):
    return lib().pa_strerror(code).decode()


def _ck(rc, what):
    if rc != PA_OK:
        raise PAError(rc, what)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Population:
    """One population on the device, driven through the C ABI."""

    def __init__(self, L, R_target, seed=1, population_id=0, J=None,
                 layout=PA_INT8, capacity=0, rows_per_lane=0, stream=None):
        self.L, self.N = L, L * L
        self._J = None if J is None else np.ascontiguousarray(J, np.int8)
        cfg = pa_config()
        cfg.L = L
        cfg.model = PA_FERRO if J is None else PA_PMJ
        cfg.J = _ptr(self._J)
        cfg.R_target = R_target
        cfg.capacity = capacity
        cfg.layout = layout
        cfg.rows_per_lane = rows_per_lane
        cfg.seed = seed
        cfg.population_id = population_id
        cfg.stream = stream
        h = C.c_void_p()
        _ck(lib().pa_init(C.byref(cfg), C.byref(h)), "pa_init")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().pa_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- the hot path
    def sweep(self, beta, theta):
        _ck(lib().pa_sweep(self._h, beta, theta), "pa_sweep")

    def resample(self, beta_next):
        Rn = C.c_int64()
        _ck(lib().pa_resample(self._h, beta_next, C.byref(Rn)), "pa_resample")
        return Rn.value

    def resample_rc(self, beta_next):
        Rn = C.c_int64()
        rc = lib().pa_resample(self._h, beta_next, C.byref(Rn))
        return rc, Rn.value

    def observables(self):
        o = pa_obs()
        _ck(lib().pa_observables(self._h, C.byref(o)), "pa_observables")
        return o.as_dict()

    def free_energy(self):
        z, q = C.c_double(), C.c_double()
        _ck(lib().pa_free_energy(self._h, C.byref(z), C.byref(q)),
            "pa_free_energy")
        return z.value, q.value

    # --- state and export
    def state(self):
        R, b, s = C.c_int64(), C.c_double(), C.c_int32()
        _ck(lib().pa_state(self._h, C.byref(R), C.byref(b), C.byref(s)),
            "pa_state")
        return R.value, b.value, s.value

    @property
    def R(self):
        return self.state()[0]

    @property
    def beta(self):
        return self.state()[1]

    @property
    def step(self):
        return self.state()[2]

    def population(self):
        R = self.R
        s = np.empty((R, self.L, self.L), np.int8)
        E = np.empty(R, np.int32)
        M = np.empty(R, np.int32)
        _ck(lib().pa_get_population(self._h, _ptr(s), _ptr(E), _ptr(M), R),
            "pa_get_population")
        return s, E, M

    def energies(self):
        R = self.R
        E = np.empty(R, np.int32)
        M = np.empty(R, np.int32)
        _ck(lib().pa_get_population(self._h, None, _ptr(E), _ptr(M), R),
            "pa_get_population")
        return E, M

    def replicas(self, slots):
        sl = np.ascontiguousarray(slots, np.int64)
        k = len(sl)
        s = np.empty((k, self.L, self.L), np.int8)
        E = np.empty(k, np.int32)
        M = np.empty(k, np.int32)
        _ck(lib().pa_get_replicas(self._h, _ptr(sl), k, _ptr(s), _ptr(E),
                                  _ptr(M)), "pa_get_replicas")
        return s, E, M

    def counts(self, cap=None):
        cap = self.R * 4 + 1024 if cap is None else cap
        n = np.empty(max(cap, 1), np.uint32)
        ln = C.c_int64()
        _ck(lib().pa_get_counts(self._h, _ptr(n), cap, C.byref(ln)),
            "pa_get_counts")
        return n[:ln.value].copy()

    def set_population(self, spins):
        s = np.ascontiguousarray(spins, np.int8)
        _ck(lib().pa_set_population(self._h, _ptr(s), s.shape[0]),
            "pa_set_population")

    def histogram(self):
        nb, st = C.c_int32(), C.c_int32()
        _ck(lib().pa_histogram(self._h, None, 0, C.byref(nb), C.byref(st)),
            "pa_histogram")
        h = np.empty(nb.value, np.uint32)
        _ck(lib().pa_histogram(self._h, _ptr(h), nb.value, C.byref(nb),
                               C.byref(st)), "pa_histogram")
        return h, st.value

    def overlap(self, dbeta):
        a = C.c_double()
        _ck(lib().pa_overlap(self._h, dbeta, C.byref(a)), "pa_overlap")
        return a.value

    def bisect_dbeta(self, target, beta_f):
        d = C.c_double()
        _ck(lib().pa_bisect_dbeta(self._h, target, beta_f, C.byref(d)),
            "pa_bisect_dbeta")
        return d.value

    def set_timing(self, enable=True):
        _ck(lib().pa_set_timing(self._h, 1 if enable else 0), "pa_set_timing")

    def timing(self):
        t = pa_timing()
        _ck(lib().pa_get_timing(self._h, C.byref(t)), "pa_get_timing")
        out = {}
        for i, k in enumerate(KERNEL_CLASSES):
            out[k] = {"ms": t.ms[i], "launches": t.launches[i],
                      "bytes": t.bytes[i]}
        out["attempts"] = t.attempts
        return out
