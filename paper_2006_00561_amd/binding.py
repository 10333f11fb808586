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

(PA_OK, PA_EINVAL, PA_ENOMEM, PA_ECAPACITY, PA_EDEVICE, PA_ESTATE, PA_EEMPTY,
 PA_EIO) = (0, -1, -2, -3, -4, -5, -6, -7)
PA_FERRO, PA_PMJ, PA_POTTS = 0, 1, 2
PA_INT8, PA_BITS = 0, 1
PA_NEAREST, PA_POISSON, PA_SYSTEMATIC, PA_RESIDUAL, PA_MULTINOMIAL = range(5)
PA_RNG_WORD, PA_RNG_PLANES = 0, 1
KERNEL_CLASSES = ("init", "sweep", "hist", "counts", "scatter", "gather")
PA_TIMING_ALL = -1


class pa_config(C.Structure):
    _fields_ = [("L", C.c_int32), ("model", C.c_int32),
                ("J", C.c_void_p), ("R_target", C.c_int64),
                ("capacity", C.c_int64), ("layout", C.c_int32),
                ("rows_per_lane", C.c_int32), ("seed", C.c_uint64),
                ("population_id", C.c_uint32), ("stream", C.c_void_p),
                ("resampling", C.c_int32), ("q", C.c_int32),
                ("rng_mode", C.c_int32)]


class pa_obs(C.Structure):
    _fields_ = [("R", C.c_int64), ("beta", C.c_double), ("e", C.c_double),
                ("abs_m", C.c_double), ("m2", C.c_double), ("C", C.c_double),
                ("sumE", C.c_int64), ("sumE2", C.c_int64),
                ("sumAbsM", C.c_int64), ("sumM2", C.c_int64),
                ("Emin", C.c_int32), ("Emax", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pa_family(C.Structure):
    _fields_ = [("R", C.c_int64), ("n0", C.c_int64), ("families", C.c_int64),
                ("largest", C.c_int64), ("rho_t", C.c_double),
                ("rho_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pa_combined(C.Structure):
    _fields_ = [("M", C.c_int32), ("R", C.c_int64), ("beta", C.c_double),
                ("e", C.c_double), ("abs_m", C.c_double), ("m2", C.c_double),
                ("C", C.c_double), ("varE", C.c_double), ("lnZ", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pa_timing(C.Structure):
    _fields_ = [("ms", C.c_double * 6), ("launches", C.c_int64 * 6),
                ("bytes", C.c_int64 * 6), ("attempts", C.c_int64)]


class PAError(RuntimeError):
    def __init__(self, code, what):
        msg = "%s failed: %s (%d)" % (what, strerror(code), code)
        if code == PA_EDEVICE:
            msg += ": " + lib().pa_last_error().decode()
        super().__init__(msg)
        self.code = code


_lib = None


def _torch_runtime_first():
    """Let torch bring up the HIP runtime before the library is loaded, so
    that the library shares it and torch's device memory and streams can be
    handed to the library (loaded the other way round, torch finds no
    device).  Nothing happens where torch or a GPU is absent."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def lib():
    """Load libpa.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(
                "libpa.so is not built (run paper_2006_00561_amd/build.py); "
                "there is no fallback path")
        _torch_runtime_first()
        L = C.CDLL(SO_PATH)
        P, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        sig = {
            "pa_init": ([C.POINTER(pa_config), C.POINTER(P)], C.c_int),
            "pa_sweep": ([P, d, i32], C.c_int),
            "pa_resample": ([P, d, C.POINTER(i64)], C.c_int),
            "pa_anneal": ([P, P, i32, i32, P, P, C.POINTER(i32)], C.c_int),
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
            "pa_set_timing_sample": ([P, i32], C.c_int),
            "pa_save": ([P, C.c_char_p], C.c_int),
            "pa_load": ([C.c_char_p, P, C.POINTER(P)], C.c_int),
            "pa_get_config": ([P, C.POINTER(pa_config)], C.c_int),
            "pa_start_heating": ([P, d], C.c_int),
            "pa_weighted_average": ([i32, P, P, i32, P, C.POINTER(d)],
                                    C.c_int),
            "pa_weighted_observables": ([i32, P, P, i32,
                                         C.POINTER(pa_combined)], C.c_int),
            "pa_get_families": ([P, P, i64, C.POINTER(i64), C.POINTER(i64)],
                                C.c_int),
            "pa_family_summary": ([P, i64, i64, C.POINTER(pa_family)],
                                  C.c_int),
            "pa_family_stats": ([P, C.POINTER(pa_family)], C.c_int),
            "pa_get_timing": ([P, C.POINTER(pa_timing)], C.c_int),
            "pa_destroy": ([P], None),
            "pa_strerror": ([C.c_int], C.c_char_p),
            "pa_last_error": ([], C.c_char_p),
            "pa_tune_rows_per_lane": ([i32, i32, i32, i64, i32, P,
                                       C.POINTER(i32), P], C.c_int),
            "pa_batch_init": ([P, i32, P, i32, C.POINTER(P)], C.c_int),
            "pa_batch_run": ([P, i32, P, i32, i32], C.c_int),
            "pa_batch_run_adaptive": ([P, d, d, i32, i32, i32,
                                       C.POINTER(i32)], C.c_int),
            "pa_batch_run_adaptive_tol": ([P, d, d, d, i32, i32, i32,
                                           C.POINTER(i32)], C.c_int),
            "pa_batch_state": ([P, i32, C.POINTER(i64), C.POINTER(d),
                                C.POINTER(i32), C.POINTER(d)], C.c_int),
            "pa_batch_trajectory": ([P, i32, P, P, i32, C.POINTER(i32)],
                                    C.c_int),
            "pa_batch_get_population": ([P, i32, P, P, P, i64], C.c_int),
            "pa_batch_get_families": ([P, i32, P, i64, C.POINTER(i64),
                                       C.POINTER(i64)], C.c_int),
            "pa_batch_set_sweep_blocks": ([P, i32, i32], C.c_int),
            "pa_batch_get_sweep_blocks": ([P, C.POINTER(i32), C.POINTER(i32)],
                                          C.c_int),
            "pa_batch_destroy": ([P], None),
            "pa_batch_run_learned": ([P, P, d, d, d, i32, i32, i32,
                                      C.POINTER(i32), P], C.c_int),
            "pa_batch_decisions": ([P, i32, P, P, P, P, i32,
                                    C.POINTER(i32)], C.c_int),
            "pa_batch_host_stats": ([P, C.POINTER(d), C.POINTER(i64), P],
                                    C.c_int),
            "pa_mlp_create": ([i32, i32, i32, C.c_uint64, P, C.POINTER(P)],
                              C.c_int),
            "pa_mlp_n_params": ([P, C.POINTER(i64)], C.c_int),
            "pa_mlp_set_params": ([P, P, i64], C.c_int),
            "pa_mlp_get_params": ([P, P, i64], C.c_int),
            "pa_mlp_set_norm": ([P, P, P, C.c_float, C.c_float], C.c_int),
            "pa_mlp_forward": ([P, P, i32, P], C.c_int),
            "pa_mlp_forward_noalloc": ([P, P, i32, P], C.c_int),
            "pa_mlp_loss_grad": ([P, P, P, i32, C.POINTER(C.c_float), P],
                                 C.c_int),
            "pa_mlp_train": ([P, P, P, i64, i32, i32, C.c_float, C.c_uint64,
                              C.POINTER(C.c_float)], C.c_int),
            "pa_mlp_destroy": ([P], None),
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
                 layout=PA_INT8, capacity=0, rows_per_lane=0, stream=None,
                 resampling=PA_NEAREST, q=0, rng_mode=PA_RNG_WORD):
        """J: +-J couplings (None = ferromagnet); q >= 2: the q-state Potts
        ferromagnet (spins are states 0..q-1); rng_mode: the sweep's
        random numbers (PA_RNG_WORD or PA_RNG_PLANES)."""
        self.L, self.N = L, L * L
        self._J = None if J is None else np.ascontiguousarray(J, np.int8)
        cfg = pa_config()
        cfg.L = L
        cfg.model = PA_POTTS if q else (PA_FERRO if J is None else PA_PMJ)
        cfg.q = q
        cfg.J = _ptr(self._J)
        cfg.R_target = R_target
        cfg.capacity = capacity
        cfg.layout = layout
        cfg.rows_per_lane = rows_per_lane
        cfg.seed = seed
        cfg.population_id = population_id
        cfg.stream = stream
        cfg.resampling = resampling
        cfg.rng_mode = rng_mode
        h = C.c_void_p()
        _ck(lib().pa_init(C.byref(cfg), C.byref(h)), "pa_init")
        self._h = h

    def start_heating(self, beta0):
        """Ground states at beta0 > 0 (heating protocol; ferromagnet)."""
        _ck(lib().pa_start_heating(self._h, beta0), "pa_start_heating")

    # --- checkpoint and resume
    def save(self, path):
        _ck(lib().pa_save(self._h, os.fsencode(path)), "pa_save")

    @classmethod
    def load(cls, path, stream=None):
        """A population restored from a pa_save file; it continues the run
        bit for bit."""
        h = C.c_void_p()
        _ck(lib().pa_load(os.fsencode(path), stream, C.byref(h)), "pa_load")
        self = cls.__new__(cls)
        self._h = h
        self._J = None
        cfg = pa_config()
        _ck(lib().pa_get_config(h, C.byref(cfg)), "pa_get_config")
        self.L, self.N = cfg.L, cfg.L * cfg.L
        return self

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

    def resample(self, beta_next, wait=True):
        """Resample to beta_next and return the new size; with wait=False
        the call may return before the size is known (returns None) and the
        next synchronising call brings it to the host."""
        if not wait:
            _ck(lib().pa_resample(self._h, beta_next, None), "pa_resample")
            return None
        Rn = C.c_int64()
        _ck(lib().pa_resample(self._h, beta_next, C.byref(Rn)), "pa_resample")
        return Rn.value

    def anneal_rc(self, betas, theta, as_dicts=True):
        """The whole loop over the schedule `betas` (pa_anneal): returns the
        status code, the number of completed steps, their observables (one
        dict per completed step, or with as_dicts=False a numpy structured
        array with pa_obs's fields) and their ln Q."""
        b = np.ascontiguousarray(betas, dtype=np.float64)
        K = len(b)
        obs = (pa_obs * max(1, K))()
        q = np.zeros(max(1, K), dtype=np.float64)
        done = C.c_int32()
        rc = lib().pa_anneal(self._h, _ptr(b), K, theta,
                             C.cast(obs, C.c_void_p), _ptr(q), C.byref(done))
        n = done.value
        if not as_dicts:
            return rc, n, np.ctypeslib.as_array(obs)[:n], q[:n]
        return rc, n, [obs[i].as_dict() for i in range(n)], list(q[:n])

    def anneal(self, betas, theta, as_dicts=True):
        """As anneal_rc, raising on failure; returns (observables, ln Q)."""
        rc, _, obs, q = self.anneal_rc(betas, theta, as_dicts)
        _ck(rc, "pa_anneal")
        return obs, q

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

    def families(self):
        """(family number of every replica, size of the founding
        population)."""
        ln, n0 = C.c_int64(), C.c_int64()
        _ck(lib().pa_get_families(self._h, None, 0, C.byref(ln), C.byref(n0)),
            "pa_get_families")
        f = np.empty(max(ln.value, 1), np.uint32)
        _ck(lib().pa_get_families(self._h, _ptr(f), ln.value, C.byref(ln),
                                  C.byref(n0)), "pa_get_families")
        return f[:ln.value].copy(), n0.value

    def family_stats(self):
        out = pa_family()
        _ck(lib().pa_family_stats(self._h, C.byref(out)), "pa_family_stats")
        return out.as_dict()

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

    def set_timing(self, enable=True, classes=None, every=1):
        """Start (zeroed) or stop the per-class kernel timing; classes is an
        iterable of KERNEL_CLASSES names to time (default: all); every: time
        the first launch of a class and then one in `every`."""
        if not enable:
            mask = 0
        elif classes is None:
            mask = PA_TIMING_ALL
        else:
            mask = 0
            for k in classes:
                mask |= 1 << KERNEL_CLASSES.index(k)
        _ck(lib().pa_set_timing(self._h, mask), "pa_set_timing")
        _ck(lib().pa_set_timing_sample(self._h, every),
            "pa_set_timing_sample")

    def timing(self):
        t = pa_timing()
        _ck(lib().pa_get_timing(self._h, C.byref(t)), "pa_get_timing")
        out = {}
        for i, k in enumerate(KERNEL_CLASSES):
            out[k] = {"ms": t.ms[i], "launches": t.launches[i],
                      "bytes": t.bytes[i]}
        out["attempts"] = t.attempts
        return out


def tune_rows_per_lane(L, layout=PA_INT8, model=PA_FERRO, R=4096, theta=4,
                       stream=None):
    """Fastest rows-per-lane sweep shape for side L (and the three times)."""
    best = C.c_int32()
    ms = (C.c_float * 4)()
    _ck(lib().pa_tune_rows_per_lane(L, layout, model, R, theta, stream,
                                    C.byref(best), ms),
        "pa_tune_rows_per_lane")
    return best.value, list(ms)


def family_summary(fam, n0):
    """Family statistics of a family array (pa_family_summary)."""
    f = np.ascontiguousarray(fam, np.uint32)
    out = pa_family()
    _ck(lib().pa_family_summary(_ptr(f), len(f), n0, C.byref(out)),
        "pa_family_summary")
    return out.as_dict()


def weighted_average(lnZ, values):
    """Weighted average over independent populations (pa_weighted_average):
    lnZ [M], values [M][k] of linear population averages; returns
    (averages [k], combined ln Z)."""
    z = np.ascontiguousarray(lnZ, np.float64)
    v = np.ascontiguousarray(values, np.float64).reshape(len(z), -1)
    out = np.zeros(v.shape[1], np.float64)
    lz = C.c_double()
    _ck(lib().pa_weighted_average(len(z), _ptr(z), _ptr(v), v.shape[1],
                                  _ptr(out), C.byref(lz)),
        "pa_weighted_average")
    return out, lz.value


def combine_observables(lnZ, obs, N):
    """Energy per spin, |m|, m^2, the energy variance and the specific heat
    of M independent populations together (pa_weighted_observables), from
    each population's pa_obs (a dict as returned by observables())."""
    z = np.ascontiguousarray(lnZ, np.float64)
    arr = (pa_obs * len(obs))()
    for i, o in enumerate(obs):
        for k, _ in pa_obs._fields_:
            setattr(arr[i], k, o[k])
    out = pa_combined()
    _ck(lib().pa_weighted_observables(len(z), _ptr(z), arr, int(N),
                                      C.byref(out)),
        "pa_weighted_observables")
    return out.as_dict()


class Batch:
    """Many independent populations advanced together (pa_batch_*)."""

    def __init__(self, pops, stream=None, autotune=False, tune_sweep=False):
        """pops: list of dicts with keys L, R (target), and optionally J,
        q (q-state Potts), seed, population_id, layout, capacity,
        rows_per_lane, rng_mode."""
        self.n = len(pops)
        self._keep = []
        cfgs = (pa_config * self.n)()
        self.L = []
        for i, p in enumerate(pops):
            c = cfgs[i]
            J = p.get("J")
            if J is not None:
                J = np.ascontiguousarray(J, np.int8)
                self._keep.append(J)
            c.L = p["L"]
            q = p.get("q", 0)
            c.model = PA_POTTS if q else (PA_FERRO if J is None else PA_PMJ)
            c.q = q
            c.J = _ptr(J)
            c.R_target = p["R"]
            c.capacity = p.get("capacity", 0)
            c.layout = p.get("layout", PA_INT8)
            c.rows_per_lane = p.get("rows_per_lane", 0)
            c.seed = p.get("seed", 1)
            c.population_id = p.get("population_id", i)
            c.rng_mode = p.get("rng_mode", PA_RNG_WORD)
            self.L.append(p["L"])
        h = C.c_void_p()
        flags = (1 if autotune else 0) | (2 if tune_sweep else 0)
        _ck(lib().pa_batch_init(cfgs, self.n, stream, flags, C.byref(h)),
            "pa_batch_init")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().pa_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, betas, theta, use_graph=True):
        """betas: array [steps][n] of next temperatures."""
        b = np.ascontiguousarray(betas, np.float64)
        if b.ndim == 1:
            b = np.repeat(b[:, None], self.n, axis=1).copy()
        assert b.shape[1] == self.n
        _ck(lib().pa_batch_run(self._h, b.shape[0], _ptr(b), theta,
                               1 if use_graph else 0), "pa_batch_run")

    def run_adaptive(self, target, beta_f, max_steps, theta, use_graph=True,
                     tol=0.0):
        """Overlap-targeted schedule by bisection; tol > 0 stops each
        bisection at the first step whose overlap is within tol of the
        target (pa_batch_run_adaptive_tol)."""
        st = C.c_int32()
        if tol > 0.0:
            _ck(lib().pa_batch_run_adaptive_tol(
                self._h, target, tol, beta_f, max_steps, theta,
                1 if use_graph else 0, C.byref(st)),
                "pa_batch_run_adaptive_tol")
        else:
            _ck(lib().pa_batch_run_adaptive(self._h, target, beta_f,
                                            max_steps, theta,
                                            1 if use_graph else 0,
                                            C.byref(st)),
                "pa_batch_run_adaptive")
        return st.value

    def state(self, p):
        R, b, s, z = C.c_int64(), C.c_double(), C.c_int32(), C.c_double()
        _ck(lib().pa_batch_state(self._h, p, C.byref(R), C.byref(b),
                                 C.byref(s), C.byref(z)), "pa_batch_state")
        return R.value, b.value, s.value, z.value

    def trajectory(self, p, cap=100000):
        obs = (pa_obs * cap)()
        z = np.zeros(cap, np.float64)
        ln = C.c_int32()
        _ck(lib().pa_batch_trajectory(self._h, p, obs, _ptr(z), cap,
                                      C.byref(ln)), "pa_batch_trajectory")
        return [obs[i].as_dict() for i in range(ln.value)], z[:ln.value]

    def population(self, p):
        R = self.state(p)[0]
        L = self.L[p]
        s = np.empty((R, L, L), np.int8)
        E = np.empty(R, np.int32)
        M = np.empty(R, np.int32)
        _ck(lib().pa_batch_get_population(self._h, p, _ptr(s), _ptr(E),
                                          _ptr(M), R),
            "pa_batch_get_population")
        return s, E, M

    def families(self, p):
        """(family number of every replica of population p, founding
        size)."""
        ln, n0 = C.c_int64(), C.c_int64()
        _ck(lib().pa_batch_get_families(self._h, p, None, 0, C.byref(ln),
                                        C.byref(n0)), "pa_batch_get_families")
        f = np.empty(max(ln.value, 1), np.uint32)
        _ck(lib().pa_batch_get_families(self._h, p, _ptr(f), ln.value,
                                        C.byref(ln), C.byref(n0)),
            "pa_batch_get_families")
        return f[:ln.value].copy(), n0.value

    def sweep_blocks(self):
        """(workgroups, items per queue atomic) of the persistent sweep."""
        bl, ch = C.c_int32(), C.c_int32()
        _ck(lib().pa_batch_get_sweep_blocks(self._h, C.byref(bl),
                                            C.byref(ch)),
            "pa_batch_get_sweep_blocks")
        return bl.value, ch.value

    def set_sweep_blocks(self, blocks, chunk=1):
        _ck(lib().pa_batch_set_sweep_blocks(self._h, blocks, chunk),
            "pa_batch_set_sweep_blocks")

    def run_learned(self, mlp, target, tol, beta_f, max_steps, theta,
                    use_graph=True):
        st = C.c_int32()
        src = np.zeros(5, np.int64)
        _ck(lib().pa_batch_run_learned(self._h, mlp._h, target, tol, beta_f,
                                       max_steps, theta, 1 if use_graph else 0,
                                       C.byref(st), _ptr(src)),
            "pa_batch_run_learned")
        return st.value, src

    def decisions(self, p, cap=100000, with_proposals=False):
        """(features [k][8] float32, dbeta [k], source [k]) of population p
        over the last run, and the network's log dbeta proposals if asked."""
        f = np.zeros((cap, 8), np.float32)
        db = np.zeros(cap, np.float64)
        src = np.zeros(cap, np.int32)
        prop = np.zeros(cap, np.float32)
        ln = C.c_int32()
        _ck(lib().pa_batch_decisions(self._h, p, _ptr(f), _ptr(db), _ptr(src),
                                     _ptr(prop), cap, C.byref(ln)),
            "pa_batch_decisions")
        k = ln.value
        if with_proposals:
            return f[:k], db[:k], src[:k], prop[:k]
        return f[:k], db[:k], src[:k]

    def host_stats(self):
        ms = C.c_double()
        ev = C.c_int64()
        src = np.zeros(5, np.int64)
        _ck(lib().pa_batch_host_stats(self._h, C.byref(ms), C.byref(ev),
                                      _ptr(src)), "pa_batch_host_stats")
        return {"host_ms": ms.value, "overlap_evals": ev.value,
                "sources": src.tolist()}


class MLP:
    """The temperature-step network (pa_mlp_*): FP32, trained and evaluated
    by the library's HIP kernels."""

    def __init__(self, n_in=8, width=64, depth=3, seed=1, stream=None):
        h = C.c_void_p()
        _ck(lib().pa_mlp_create(n_in, width, depth, seed, stream, C.byref(h)),
            "pa_mlp_create")
        self._h = h
        self.n_in, self.width, self.depth = n_in, width, depth
        n = C.c_int64()
        _ck(lib().pa_mlp_n_params(h, C.byref(n)), "pa_mlp_n_params")
        self.n_params = n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().pa_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        p = np.zeros(self.n_params, np.float32)
        _ck(lib().pa_mlp_get_params(self._h, _ptr(p), self.n_params),
            "pa_mlp_get_params")
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        _ck(lib().pa_mlp_set_params(self._h, _ptr(p), len(p)),
            "pa_mlp_set_params")

    def set_norm(self, mu, sigma, mu_y, sigma_y):
        mu = np.ascontiguousarray(mu, np.float32)
        sigma = np.ascontiguousarray(sigma, np.float32)
        _ck(lib().pa_mlp_set_norm(self._h, _ptr(mu), _ptr(sigma),
                                  float(mu_y), float(sigma_y)),
            "pa_mlp_set_norm")

    def forward(self, X):
        X = np.ascontiguousarray(X, np.float32)
        y = np.zeros(len(X), np.float32)
        _ck(lib().pa_mlp_forward(self._h, _ptr(X), len(X), _ptr(y)),
            "pa_mlp_forward")
        return y

    def forward_noalloc(self, X_dev, B, y_dev):
        """pa_mlp_forward_noalloc: X_dev and y_dev are device addresses
        (ints) of B x n_in and B floats; asynchronous on the network's
        stream."""
        _ck(lib().pa_mlp_forward_noalloc(self._h, C.c_void_p(X_dev), int(B),
                                         C.c_void_p(y_dev)),
            "pa_mlp_forward_noalloc")

    def loss_grad(self, X, T):
        X = np.ascontiguousarray(X, np.float32)
        T = np.ascontiguousarray(T, np.float32)
        g = np.zeros(self.n_params, np.float32)
        loss = C.c_float()
        _ck(lib().pa_mlp_loss_grad(self._h, _ptr(X), _ptr(T), len(X),
                                   C.byref(loss), _ptr(g)), "pa_mlp_loss_grad")
        return loss.value, g

    def train(self, X, T, batch=256, iters=2000, lr=1e-3, seed=7):
        X = np.ascontiguousarray(X, np.float32)
        T = np.ascontiguousarray(T, np.float32)
        loss = C.c_float()
        _ck(lib().pa_mlp_train(self._h, _ptr(X), _ptr(T), len(X), batch,
                               iters, lr, seed, C.byref(loss)),
            "pa_mlp_train")
        return loss.value
