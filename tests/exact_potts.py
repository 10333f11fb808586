"""Exact results for the q-state Potts ferromagnet on an L x L torus
(H = -sum over the 2N bonds of delta(s, s')), independent of the oracle and
of the HIP path.

The density of states comes from a row transfer matrix whose entries are
polynomials in the number of satisfied bonds: T[a, b] counts the bonds
inside row a and between rows a and b, and the trace of T^L, as a
polynomial, has coefficient g(E = -m) at power m.  Row states are
enumerated (q^L of them), so L is small (q^L <= a few hundred).
"""
from __future__ import annotations

import functools
import itertools

import numpy as np


@functools.lru_cache(maxsize=8)
def density_of_states(L, q):
    """g[m] = number of configurations with m satisfied bonds (E = -m),
    m = 0..2N, as float64 (exact below 2^53)."""
    rows = np.array(list(itertools.product(range(q), repeat=L)), np.int64)
    nr = len(rows)
    intra = (rows == np.roll(rows, -1, axis=1)).sum(axis=1)
    inter = (rows[:, None, :] == rows[None, :, :]).sum(axis=2)
    deg = 2 * L * L
    T = np.zeros((nr, nr, deg + 1))
    for a in range(nr):
        for b in range(nr):
            T[a, b, intra[a] + inter[a, b]] = 1.0

    def mul(A, B):
        C = np.zeros((nr, nr, deg + 1))
        for i in range(deg + 1):
            Ai = A[:, :, i]
            if not Ai.any():
                continue
            # C[a, c, i + k] += sum_b A[a, b, i] B[b, c, k]
            C[:, :, i:] += np.tensordot(Ai, B[:, :, :deg + 1 - i], axes=(1, 0))
        return C

    P = T
    for _ in range(L - 1):
        P = mul(P, T)
    return np.array([np.trace(P[:, :, m]) for m in range(deg + 1)])


def thermo(L, q, beta):
    """ln Z, <E>/N and the energy distribution p(E = -m) at beta."""
    g = density_of_states(L, q)
    m = np.arange(len(g), dtype=np.float64)
    ok = g > 0
    x = np.log(g[ok]) + beta * m[ok]
    mx = x.max()
    Z = np.exp(x - mx).sum()
    lnZ = mx + np.log(Z)
    p = np.zeros(len(g))
    p[ok] = np.exp(x - lnZ)
    e = -(p * m).sum() / (L * L)
    return {"lnZ": float(lnZ), "e": float(e), "p": p}
