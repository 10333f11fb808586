"""Exact results for the 2D Ising model on an L x L torus, independent of the
oracle and of the HIP path: they pin the oracle.

* ``enumerate_states`` lists every one of the 2^(L*L) configurations (L <= 5)
  and their energies and magnetisations with numpy, from the Hamiltonian of
  Sec. 3, Eq. Ham (H = -sum over the 2N bonds of J sigma sigma').
* ``kaufman_lnZ`` is the exact finite-torus partition function of Kaufman
  (Phys. Rev. 76, 1232 (1949)), as written by Ferdinand and Fisher
  (Phys. Rev. 185, 832 (1969)), evaluated with mpmath.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

BETA_C = float(mp.log(1 + mp.sqrt(2)) / 2)


def _all_configs(L):
    N = L * L
    idx = np.arange(1 << N, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(N)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8).reshape(-1, L, L)


@functools.lru_cache(maxsize=8)
def enumerate_states(L, J_bytes=None):
    """(E, M) arrays over all 2^(L*L) configurations.  J_bytes, if given, is
    the bytes of an int8 [2][L][L] coupling array (right, down)."""
    s = _all_configs(L).astype(np.int32)
    if J_bytes is None:
        Jr = np.ones((L, L), np.int32)
        Jd = np.ones((L, L), np.int32)
    else:
        J = np.frombuffer(J_bytes, np.int8).reshape(2, L, L).astype(np.int32)
        Jr, Jd = J[0], J[1]
    right = np.roll(s, -1, axis=2)
    down = np.roll(s, -1, axis=1)
    E = -(Jr[None] * s * right).sum(axis=(1, 2)) - (Jd[None] * s * down).sum(
        axis=(1, 2))
    M = s.sum(axis=(1, 2))
    return E.astype(np.int64), M.astype(np.int64)


def density_of_states(L, J=None):
    """{E: g(E)} by enumeration."""
    E, _ = enumerate_states(L, None if J is None else
                            np.ascontiguousarray(J, np.int8).tobytes())
    vals, cnt = np.unique(E, return_counts=True)
    return dict(zip(vals.tolist(), cnt.tolist()))


def brute_thermo(L, beta, J=None):
    """Exact ln Z, <E>/N, <|M|>/N, <M^2>/N^2 and the specific heat
    C = beta^2 (<E^2> - <E>^2) / N by enumeration (mpmath sums)."""
    E, M = enumerate_states(L, None if J is None else
                            np.ascontiguousarray(J, np.int8).tobytes())
    N = L * L
    mp.mp.dps = 40
    b = mp.mpf(beta)
    # group by (E, |M|) to keep the mpmath sums short
    keys, cnt = np.unique(np.stack([E, np.abs(M), M * M]), axis=1,
                          return_counts=True)
    Z = mp.mpf(0)
    sE = mp.mpf(0)
    sE2 = mp.mpf(0)
    sAM = mp.mpf(0)
    sM2 = mp.mpf(0)
    for (e, am, m2), c in zip(keys.T.tolist(), cnt.tolist()):
        w = c * mp.exp(-b * e)
        Z += w
        sE += w * e
        sE2 += w * e * e
        sAM += w * am
        sM2 += w * m2
    return {
        "lnZ": float(mp.log(Z)),
        "e": float(sE / Z / N),
        "abs_m": float(sAM / Z / N),
        "m2": float(sM2 / Z / N / N),
        "C": float(b * b * (sE2 / Z - (sE / Z) ** 2) / N),
    }


def kaufman_lnZ(L, beta, dps=50):
    """Exact ln Z of the L x L periodic ferromagnet (J = 1), K = beta:
    Z = 1/2 (2 sinh 2K)^(N/2) (Z1 + Z2 + Z3 + Z4), products over r < L of
    2cosh / 2sinh (L gamma_l / 2) with l = 2r+1 (Z1, Z2) and l = 2r (Z3, Z4),
    cosh gamma_l = cosh 2K coth 2K - cos(pi l / L) for l >= 1 and
    gamma_0 = 2K + ln tanh K (negative above the critical temperature)."""
    with mp.workdps(dps):
        K = mp.mpf(beta)
        n = L

        def gamma(l):
            if l == 0:
                return 2 * K + mp.log(mp.tanh(K))
            return mp.acosh(mp.cosh(2 * K) * mp.coth(2 * K) -
                            mp.cos(mp.pi * l / n))

        Z1 = Z2 = Z3 = Z4 = mp.mpf(1)
        for r in range(n):
            g1 = gamma(2 * r + 1)
            g0 = gamma(2 * r)
            Z1 *= 2 * mp.cosh(n * g1 / 2)
            Z2 *= 2 * mp.sinh(n * g1 / 2)
            Z3 *= 2 * mp.cosh(n * g0 / 2)
            Z4 *= 2 * mp.sinh(n * g0 / 2)
        Z = mp.mpf(1) / 2 * (2 * mp.sinh(2 * K)) ** (n * n / mp.mpf(2)) * (
            Z1 + Z2 + Z3 + Z4)
        return mp.log(Z)


def kaufman_energy(L, beta):
    """<E>/N = -(1/N) d ln Z / d beta, derivative taken in mpmath."""
    with mp.workdps(80):
        b = mp.mpf(beta)
        h = mp.mpf(10) ** -25
        d = (kaufman_lnZ(L, b + h, dps=80) - kaufman_lnZ(L, b - h, dps=80)) / (
            2 * h)
        return float(-d / (L * L))
