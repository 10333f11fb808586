"""ctypes wrapper and build step of the C oracle (test infrastructure only).

The oracle is compiled with ``gcc -O2 -ffp-contract=off`` and no
architecture-specific flags, so that every double-precision operation is the
plain IEEE operation written in the source (no fused multiply-add, no
vectorised libm).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pa_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
# a planted-mistake build of the oracle can be loaded in place of the real
# one (only the tests of the oracle's mutants set this)
_SO_OVERRIDE = os.environ.get("PA_ORACLE_SO")

OK, EINVAL, ENOMEM, ECAPACITY, EEMPTY = 0, -1, -2, -3, -6


def build(force: bool = True, mutant: int = 0, out: str = "") -> str:
    """Compile liboracle.so in place and return its path.  mutant > 0
    builds a planted-mistake variant into `out` instead."""
    if mutant:
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC",
               "-shared", "-pthread", "-DORC_MUTANT=%d" % mutant, "-o", out, _SRC,
               "-lm"]
        subprocess.run(cmd, check=True)
        return out
    if force or not os.path.exists(_SO) or (
            os.path.getmtime(_SO) < os.path.getmtime(_SRC)):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-Wall",
               "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


class Obs(C.Structure):
    _fields_ = [("R", C.c_int64), ("beta", C.c_double), ("e", C.c_double),
                ("abs_m", C.c_double), ("m2", C.c_double), ("C", C.c_double),
                ("sumE", C.c_int64), ("sumE2", C.c_int64),
                ("sumAbsM", C.c_int64), ("sumM2", C.c_int64),
                ("Emin", C.c_int32), ("Emax", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _SO_OVERRIDE:
            L = C.CDLL(_SO_OVERRIDE)
        else:
            if not os.path.exists(_SO):
                build(force=False)
            L = C.CDLL(_SO)
        P = C.c_void_p
        i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_energy.argtypes = [C.c_int, P, i8p, C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32)]
        L.orc_energy.restype = None
        L.orc_create.argtypes = [C.c_int, P, C.c_int64, C.c_int64, C.c_uint64,
                                 C.c_uint32, C.POINTER(P)]
        L.orc_destroy.argtypes = [P]
        L.orc_destroy.restype = None
        L.orc_resample.argtypes = [P, C.c_double, C.POINTER(C.c_int64)]
        L.orc_sweep.argtypes = [P, C.c_int]
        L.orc_sweep_threads.argtypes = [P, C.c_int, C.c_int]
        L.orc_observables.argtypes = [P, C.POINTER(Obs)]
        L.orc_free_energy.argtypes = [P, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]
        L.orc_R.argtypes = [P]
        L.orc_R.restype = C.c_int64
        L.orc_beta.argtypes = [P]
        L.orc_beta.restype = C.c_double
        L.orc_step.argtypes = [P]
        L.orc_get_population.argtypes = [P, P, P, P, C.c_int64]
        L.orc_get_counts.argtypes = [P, u32p, C.c_int64]
        L.orc_get_families.argtypes = [P, u32p, C.c_int64,
                                       C.POINTER(C.c_int64)]
        L.orc_family_stats.argtypes = [u32p, C.c_int64, C.c_int64,
                                       C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int64),
                                       C.POINTER(C.c_double),
                                       C.POINTER(C.c_double)]
        L.orc_set_population.argtypes = [P, i8p, C.c_int64]
        L.orc_histogram.argtypes = [P, u32p]
        L.orc_set_visit_shuffle.argtypes = [P, C.c_uint64]
        L.orc_set_visit_shuffle.restype = None
        L.orc_multinomial_pick.argtypes = [
            C.c_uint64, np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS"),
            C.c_int64]
        L.orc_multinomial_pick.restype = C.c_int64
        L.orc_counts.argtypes = [C.c_int, i32p, C.c_int64, C.c_int64,
                                 C.c_double, C.c_uint64, C.c_uint32, C.c_int,
                                 C.c_int, u32p, C.POINTER(C.c_int64),
                                 C.POINTER(C.c_double)]
        L.orc_set_resampling.argtypes = [P, C.c_int]
        L.orc_start_heating.argtypes = [P, C.c_double]
        L.orc_create_potts.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_int64,
                                       C.c_uint64, C.c_uint32,
                                       C.POINTER(P)]
        L.orc_potts_energy.argtypes = [C.c_int, C.c_int, P, i32p, i32p]
        L.orc_potts_energy.restype = None
        L.orc_poisson_draw.argtypes = [C.c_double, C.c_uint32]
        L.orc_poisson_draw.restype = C.c_uint32
        L.orc_sweep_replica.argtypes = [C.c_int, P, i8p, C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int32), C.c_double,
                                        C.c_uint64, C.c_uint32, C.c_int,
                                        C.c_int, C.c_int, C.c_uint32]
        L.orc_sweep_potts_replica.argtypes = [
            C.c_int, C.c_int, i8p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
            C.c_double, C.c_uint64, C.c_uint32, C.c_int, C.c_int, C.c_int,
            C.c_uint32]
        L.orc_set_rng_mode.argtypes = [P, C.c_int]
        L.orc_site_draw.argtypes = [C.c_int, C.c_int, C.c_uint64, C.c_uint32,
                                    C.c_int, C.c_int, C.c_uint32, C.c_int,
                                    C.c_int]
        L.orc_site_draw.restype = C.c_uint32
        L.orc_sweep_replica_rng.argtypes = [
            C.c_int, P, i8p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
            C.c_double, C.c_uint64, C.c_uint32, C.c_int, C.c_int, C.c_int,
            C.c_uint32, C.c_int]
        L.orc_overlap.argtypes = [P, C.c_double, C.POINTER(C.c_double)]
        L.orc_bisect_dbeta.argtypes = [P, C.c_double, C.c_double,
                                       C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _check(rc, what):
    if rc != OK:
        raise RuntimeError("oracle %s failed with code %d" % (what, rc))


def _jptr(J):
    if J is None:
        return None, None
    Jc = np.ascontiguousarray(J, dtype=np.int8)
    return Jc, Jc.ctypes.data_as(C.c_void_p)


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: 4 uint32 words for a 4-word counter and a
    2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(c, k, out)
    return out


def energy(spins, J=None):
    """(E, M) of one L x L configuration of +-1 spins (Eq. Ham)."""
    s = np.ascontiguousarray(spins, dtype=np.int8)
    L = s.shape[-1]
    Jc, jp = _jptr(J)
    E, M = C.c_int32(), C.c_int32()
    lib().orc_energy(L, jp, s, C.byref(E), C.byref(M))
    return E.value, M.value


NEAREST, POISSON, SYSTEMATIC, RESIDUAL, MULTINOMIAL = 0, 1, 2, 3, 4
RNG_WORD, RNG_PLANES = 0, 1


def site_draw(mode, L, seed, pop, step, half_sweep, slot, y, x):
    """The 32-bit Metropolis random number of site (x, y)."""
    return int(lib().orc_site_draw(mode, L, seed, pop, step, half_sweep, slot,
                                   y, x))


def poisson_draw(rho, r):
    return int(lib().orc_poisson_draw(float(rho), int(r)))


def multinomial_pick(u, cum):
    """The replica a 64-bit multinomial draw u lands in (cum: the interval
    ends C_0 <= ... <= C_{R-1})."""
    cum = np.ascontiguousarray(cum, np.uint64)
    return int(lib().orc_multinomial_pick(int(u), cum, len(cum)))


def counts(N, E, R_t, dbeta, seed, pop, step_next, law=NEAREST):
    """Copy counts and ln Q for a population given by its energies."""
    E = np.ascontiguousarray(E, dtype=np.int32)
    n = np.zeros(len(E), np.uint32)
    Rn, lnQ = C.c_int64(), C.c_double()
    _check(lib().orc_counts(N, E, len(E), R_t, dbeta, seed, pop, step_next,
                            law, n, C.byref(Rn), C.byref(lnQ)), "counts")
    return n, Rn.value, lnQ.value


def family_stats(fam, n0):
    """Families alive, largest family, rho_t and rho_s of a family array."""
    f = np.ascontiguousarray(fam, np.uint32)
    nf, big = C.c_int64(), C.c_int64()
    rt, rs = C.c_double(), C.c_double()
    _check(lib().orc_family_stats(f, len(f), n0, C.byref(nf), C.byref(big),
                                  C.byref(rt), C.byref(rs)), "family_stats")
    return {"families": nf.value, "largest": big.value, "rho_t": rt.value,
            "rho_s": rs.value}


def sweep_replica(spins, E, M, beta, seed, pop, step, t0, theta, slot, J=None,
                  rng_mode=RNG_WORD):
    """theta sweeps of one replica; returns (spins, E, M)."""
    s = np.array(spins, dtype=np.int8, copy=True, order="C")
    L = s.shape[-1]
    Jc, jp = _jptr(J)
    e, m = C.c_int32(int(E)), C.c_int32(int(M))
    _check(lib().orc_sweep_replica_rng(L, jp, s, C.byref(e), C.byref(m), beta,
                                       seed, pop, step, t0, theta, slot,
                                       rng_mode), "sweep_replica")
    return s, e.value, m.value


def sweep_potts_replica(spins, E, M, beta, q, seed, pop, step, t0, theta,
                        slot):
    """theta sweeps of one q-state Potts replica; returns (states, E, M)."""
    s = np.array(spins, dtype=np.int8, copy=True, order="C")
    L = s.shape[-1]
    e, m = C.c_int32(int(E)), C.c_int32(int(M))
    _check(lib().orc_sweep_potts_replica(L, q, s, C.byref(e), C.byref(m),
                                         beta, seed, pop, step, t0, theta,
                                         slot), "sweep_potts_replica")
    return s, e.value, m.value


class OraclePA:
    """One population on the CPU oracle."""

    def __init__(self, L, R_target, seed=1, pop=0, J=None, capacity=0,
                 law=NEAREST, q=0, rng_mode=RNG_WORD):
        """q = 0: Ising spins (ferromagnet or the couplings J); q >= 2: the
        q-state Potts ferromagnet."""
        self.L, self.N, self.q = L, L * L, q
        self._Jc, jp = _jptr(J)
        h = C.c_void_p()
        if q:
            _check(lib().orc_create_potts(L, q, R_target, capacity, seed, pop,
                                          C.byref(h)), "create_potts")
        else:
            _check(lib().orc_create(L, jp, R_target, capacity, seed, pop,
                                    C.byref(h)), "create")
        self._h = h
        if law != NEAREST:
            _check(lib().orc_set_resampling(h, law), "set_resampling")
        if rng_mode != RNG_WORD:
            _check(lib().orc_set_rng_mode(h, rng_mode), "set_rng_mode")

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def R(self):
        return lib().orc_R(self._h)

    @property
    def beta(self):
        return lib().orc_beta(self._h)

    @property
    def step(self):
        return lib().orc_step(self._h)

    def start_heating(self, beta0):
        _check(lib().orc_start_heating(self._h, beta0), "start_heating")

    def resample(self, beta_next):
        Rn = C.c_int64()
        rc = lib().orc_resample(self._h, beta_next, C.byref(Rn))
        if rc != OK:
            raise RuntimeError("oracle resample failed with code %d (R_new=%d)"
                               % (rc, Rn.value))
        return Rn.value

    def resample_rc(self, beta_next):
        Rn = C.c_int64()
        rc = lib().orc_resample(self._h, beta_next, C.byref(Rn))
        return rc, Rn.value

    def sweep(self, theta, threads=1):
        if threads > 1:
            _check(lib().orc_sweep_threads(self._h, theta, threads), "sweep")
        else:
            _check(lib().orc_sweep(self._h, theta), "sweep")

    def observables(self):
        o = Obs()
        _check(lib().orc_observables(self._h, C.byref(o)), "observables")
        return o.as_dict()

    def free_energy(self):
        z, q = C.c_double(), C.c_double()
        _check(lib().orc_free_energy(self._h, C.byref(z), C.byref(q)), "lnZ")
        return z.value, q.value

    def population(self):
        R = self.R
        s = np.empty((R, self.L, self.L), np.int8)
        E = np.empty(R, np.int32)
        M = np.empty(R, np.int32)
        _check(lib().orc_get_population(self._h, s.ctypes.data, E.ctypes.data,
                                        M.ctypes.data, R), "get_population")
        return s, E, M

    def energies(self):
        R = self.R
        E = np.empty(R, np.int32)
        M = np.empty(R, np.int32)
        _check(lib().orc_get_population(self._h, None, E.ctypes.data,
                                        M.ctypes.data, R), "get_population")
        return E, M

    def counts(self, n_len):
        n = np.zeros(max(n_len, 1), np.uint32)
        _check(lib().orc_get_counts(self._h, n, n_len), "get_counts")
        return n[:n_len]

    def families(self):
        """(family of every replica, size of the founding population)."""
        f = np.zeros(max(self.R, 1), np.uint32)
        n0 = C.c_int64()
        _check(lib().orc_get_families(self._h, f, self.R, C.byref(n0)),
               "get_families")
        return f[:self.R], n0.value

    def set_population(self, spins):
        s = np.ascontiguousarray(spins, dtype=np.int8)
        _check(lib().orc_set_population(self._h, s, s.shape[0]),
               "set_population")

    def histogram(self):
        out = np.zeros(4 * self.N + 1, np.uint32)
        _check(lib().orc_histogram(self._h, out), "histogram")
        return out

    def set_visit_shuffle(self, seed):
        lib().orc_set_visit_shuffle(self._h, seed)

    def overlap(self, dbeta):
        a = C.c_double()
        _check(lib().orc_overlap(self._h, dbeta, C.byref(a)), "overlap")
        return a.value

    def bisect_dbeta(self, target, beta_f):
        d = C.c_double()
        _check(lib().orc_bisect_dbeta(self._h, target, beta_f, C.byref(d)),
               "bisect")
        return d.value
