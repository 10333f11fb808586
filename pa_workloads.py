"""Seeded synthetic workloads of population annealing for the 2D Ising model.

This module only describes inputs: lattice sizes, population targets,
schedules, seeds and the +-J coupling instances.  It holds none of the
method's arithmetic, so both the HIP path and the oracle take their inputs
from it.

The paper's workload (Sec. 3, "Simulation task", and the footnotes on the
replica count): the L = 64 periodic ferromagnet, 20480 replicas per GPU,
beta from 0 to 1 in K = 200 equal steps (dbeta = 0.005), theta in {1, 10}
Metropolis sweeps per step, spins drawn uniformly at beta_0 = 0.  The
configurations below use the same model and schedule shape at the sizes the
benchmark and the tests run.
"""
from __future__ import annotations

import math

import numpy as np

# name -> (L, R_target, layout, beta_f, K, theta, seed[, q for Potts])
CONFIGS = {
    # small case the oracle finishes in seconds
    "C1": dict(L=16, R=1000, layout="int8", beta_f=1.0, K=100, theta=5,
               seed=1),
    # the benchmark workload: L = 64, R = 65536, beta 0 -> 1 in 200 steps
    "C2": dict(L=64, R=65536, layout="int8", beta_f=1.0, K=200, theta=10,
               seed=1),
    # the paper's total replica count on one device, bit-packed spins
    "C3a": dict(L=64, R=1 << 21, layout="bits", beta_f=0.5, K=100, theta=10,
                seed=1),
    "C3b": dict(L=128, R=1 << 18, layout="bits", beta_f=0.5, K=100,
                theta=10, seed=1),
    # the paper's own per-GPU shape (Sec. 3): 20480 replicas, dbeta = 0.005
    "CP1": dict(L=64, R=20480, layout="int8", beta_f=1.0, K=200, theta=1,
                seed=1),
    "CP10": dict(L=64, R=20480, layout="int8", beta_f=1.0, K=200, theta=10,
                 seed=1),
    # the q = 10 Potts ferromagnet (named with the heating protocol in
    # Sec. 2) at the same per-GPU shape, cooled across its first-order
    # transition at beta_c = ln(1 + sqrt(10))
    "CQ10": dict(L=64, R=20480, layout="int8", beta_f=1.6, K=200, theta=10,
                 seed=1, q=10),
}


def deferral_capacity(R: int) -> int:
    """Capacity at which a resampling never waits for its new size: the size
    is bounded by R_target + R_old, with R_old within R_target + 16 sqrt(R)
    + 1024 (the default capacity)."""
    return 2 * R + 16 * math.isqrt(R - 1) + 16 + 1024


def linear_schedule(beta_f: float, K: int, beta0: float = 0.0):
    """beta_i = beta0 + ((beta_f - beta0) * i) / K for i = 1..K, computed from
    i (never accumulated)."""
    return [beta0 + ((beta_f - beta0) * float(i)) / float(K)
            for i in range(1, K + 1)]


def pmj_couplings(L: int, instance_seed: int, p_neg: float = 0.5):
    """Bimodal +-J couplings of one Edwards-Anderson instance: int8 [2][L][L]
    (plane 0: bond to the right neighbour, plane 1: bond below), each -1 with
    probability p_neg, from numpy's PCG64 seeded by the instance."""
    rng = np.random.Generator(np.random.PCG64(instance_seed))
    neg = rng.random((2, L, L)) < p_neg
    return np.where(neg, -1, 1).astype(np.int8)


def gauge_couplings(L: int, seed: int):
    """A +-J instance that is a ferromagnet in disguise: J_xy = eps_x eps_y
    for random signs eps; returns (J, eps)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = np.where(rng.random((L, L)) < 0.5, -1, 1).astype(np.int8)
    J = np.empty((2, L, L), np.int8)
    J[0] = eps * np.roll(eps, -1, axis=1)
    J[1] = eps * np.roll(eps, -1, axis=0)
    return J, eps


def batched_glass_instances(n: int = 64, seed: int = 2006,
                            coupling_seed0: int = 1):
    """The batched workload: n independent +-J populations with L drawn
    uniformly from {8, 12, 16, 24, 32} and R log-uniform in [2^10, 2^16];
    instance k uses coupling seed coupling_seed0 + k and population id k."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ls = rng.choice([8, 12, 16, 24, 32], size=n)
    Rs = np.round(2.0 ** (10.0 + 6.0 * rng.random(n))).astype(np.int64)
    out = []
    for k in range(n):
        L = int(Ls[k])
        out.append(dict(L=L, R=int(Rs[k]),
                        J=pmj_couplings(L, coupling_seed0 + k),
                        population_id=k, seed=1))
    return out
