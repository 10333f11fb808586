"""Pins of the oracle's reweighting / resampling step (Eqs. part-Q, tau) and of
the free-energy recursion (Eq. Free-En), against direct evaluations of the
definitions and against invariants."""
import numpy as np
import pytest

import oracle


def _direct_rho_lnQ(E, R_t, dbeta):
    """rho_j = R_t exp(-dbeta E_j) / sum_k exp(-dbeta E_k) and
    ln Q = ln mean_j exp(-dbeta E_j), evaluated in extended precision
    from the definitions (no energy-level grouping, no shift by E_min
    inside the sum order)."""
    x = -dbeta * E.astype(np.longdouble)
    m = x.max()
    ex = np.exp(x - m)
    s = ex.sum()
    rho = R_t * ex / s
    lnQ = m + np.log(s / len(E))
    return rho.astype(np.float64), float(lnQ)


def _annealed(L=16, R=2000, steps=8, seed=7):
    p = oracle.OraclePA(L, R, seed=seed)
    for i in range(1, steps + 1):
        p.resample(0.05 * i)
        p.sweep(2)
    return p


@pytest.mark.parametrize("dbeta", [0.0, 0.01, 0.05, 0.3, -0.05, -0.3])
def test_counts_are_floor_or_ceil_of_mean(dbeta):
    p = _annealed()
    E, _ = p.energies()
    R_old = len(E)
    rho, lnQ = _direct_rho_lnQ(E, 2000, dbeta)
    Rn = p.resample(p.beta + dbeta)
    n = p.counts(R_old).astype(np.int64)
    fl = np.floor(rho)
    near_int = np.abs(rho - np.round(rho)) < 1e-9
    ok = (n == fl) | (n == fl + 1)
    assert np.all(ok | near_int)
    assert Rn == n.sum()
    # the +1 draws follow the fractional parts
    frac = rho - fl
    extra = (n - fl)[~near_int]
    mu = frac[~near_int].sum()
    sd = np.sqrt((frac * (1 - frac))[~near_int].sum()) + 1e-9
    assert abs(extra.sum() - mu) < 5 * sd + 1e-6
    # ln Q against the direct log-mean-exp
    z, q = p.free_energy()
    assert abs(q - lnQ) <= 1e-12 * max(1.0, abs(lnQ))


def test_population_size_is_controlled():
    """E[R_new] = R_target and Var(R_new) <= R/4 over independent draws."""
    R_t = 1000
    vals = []
    for seed in range(60):
        p = oracle.OraclePA(12, R_t, seed=100 + seed)
        vals.append(p.resample(0.3))
    vals = np.array(vals, dtype=np.float64)
    assert abs(vals.mean() - R_t) < 5 * np.sqrt(R_t / 4 / len(vals))
    assert vals.var() <= R_t / 4 * 1.6


def test_zero_step_is_identity():
    p = oracle.OraclePA(10, 500, seed=9)
    s0, E0, M0 = p.population()
    z0, _ = p.free_energy()
    Rn = p.resample(0.0)
    assert Rn == 500
    assert np.all(p.counts(500) == 1)
    s1, E1, M1 = p.population()
    assert np.array_equal(s0, s1) and np.array_equal(E0, E1)
    z1, q1 = p.free_energy()
    assert q1 == 0.0 and z1 == z0


def test_new_population_repeats_parents_in_order():
    p = _annealed(steps=4)
    s0, E0, M0 = p.population()
    p.resample(p.beta + 0.08)
    n = p.counts(len(E0))
    s1, E1, M1 = p.population()
    parent = np.repeat(np.arange(len(E0)), n)
    assert np.array_equal(s1, s0[parent])
    assert np.array_equal(E1, E0[parent]) and np.array_equal(M1, M0[parent])


def test_lnZ_starts_at_N_ln2_and_accumulates_lnQ():
    L = 8
    p = oracle.OraclePA(L, 400, seed=2)
    z, q = p.free_energy()
    assert z == L * L * np.log(2.0)
    total = z
    for i in range(1, 6):
        p.resample(0.1 * i)
        p.sweep(1)
        z, q = p.free_energy()
        total = total + q
        assert z == total


def test_capacity_overflow_leaves_population_untouched():
    """With capacity equal to the target, about half of the seeds overflow;
    the first one that does must leave the population as it was."""
    L = 6
    for seed in range(1, 40):
        p = oracle.OraclePA(L, 1000, seed=seed, capacity=1000)
        s0, E0, M0 = p.population()
        z0, _ = p.free_energy()
        rc, Rn = p.resample_rc(0.3)
        if rc == oracle.OK:
            assert Rn <= 1000
            continue
        assert rc == oracle.ECAPACITY and Rn > 1000
        assert p.R == 1000 and p.beta == 0.0 and p.free_energy()[0] == z0
        s, E, M = p.population()
        assert np.array_equal(s, s0) and np.array_equal(E, E0)
        return
    raise AssertionError("no seed overflowed")


def test_invalid_steps_are_rejected():
    p = oracle.OraclePA(6, 10, seed=4)
    p.resample(0.2)
    assert p.resample_rc(-0.1)[0] == oracle.EINVAL    # beta stays >= 0
    assert p.resample_rc(float("nan"))[0] == oracle.EINVAL


def test_counts_on_energies_match_full_resample():
    p = _annealed(steps=3)
    E, _ = p.energies()
    beta, step = p.beta, p.step
    n, Rn, lnQ = oracle.counts(p.N, E, 2000, 0.07, 7, 0, step + 1)
    Rp = p.resample(beta + 0.07)
    assert Rp == Rn and np.array_equal(p.counts(len(E)), n)
    assert p.free_energy()[1] == lnQ
