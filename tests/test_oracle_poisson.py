"""Pins of the oracle's Poisson resampling law: the inverse-CDF draw against
scipy's Poisson distribution, and the copy counts and population sizes it
gives against their Poisson means and variances."""
import numpy as np
import pytest
from scipy import stats

import oracle

TWO32 = 1 << 32


def _thresholds(rho, kmax):
    """U_k = the smallest r whose draw exceeds k, by bisection over r (the
    draw is non-decreasing in r)."""
    U = []
    for k in range(kmax):
        lo, hi = 0, TWO32
        while lo < hi:
            mid = (lo + hi) // 2
            if oracle.poisson_draw(rho, mid) > k:
                hi = mid
            else:
                lo = mid + 1
        U.append(lo)
    return np.array(U, dtype=np.float64)


@pytest.mark.parametrize("rho", [0.05, 0.7, 1.0, 1.9, 6.5, 40.0])
def test_draw_inverts_the_poisson_cdf(rho):
    kmax = int(rho + 8 * np.sqrt(rho) + 8)
    U = _thresholds(rho, kmax)
    cdf = stats.poisson.cdf(np.arange(kmax), rho)
    # each threshold is floor(C(k) 2^32): within one 32-bit step of the CDF
    assert np.all(np.abs(U / TWO32 - cdf) <= 1.0 / TWO32 + 1e-12)


def test_draw_edges():
    assert oracle.poisson_draw(0.0, 0) == 0
    assert oracle.poisson_draw(0.0, TWO32 - 1) == 0
    for rho in (0.3, 3.0, 300.0):
        top = oracle.poisson_draw(rho, TWO32 - 1)
        assert top <= np.ceil(rho + 64 * np.sqrt(rho) + 64)
        assert stats.poisson.sf(top, rho) < 2.0 ** -31
        # r = 0: the smallest k whose CDF reaches one 32-bit step
        k0 = oracle.poisson_draw(rho, 0)
        assert abs(k0 - stats.poisson.ppf(2.0 ** -32, rho)) <= 1


def test_counts_follow_poisson_on_one_level():
    """All replicas at one energy: every mean is R_t / R, the counts are
    Poisson with that mean (chi-square against the pmf)."""
    R, R_t = 20000, 30000
    E = np.full(R, -32, np.int32)
    n, Rn, lnQ = oracle.counts(16, E, R_t, 0.3, 11, 2, 5, law=oracle.POISSON)
    rho = R_t / R
    assert Rn == n.sum()
    k = np.arange(12)
    obs = np.array([(n == v).sum() for v in k[:-1]] + [(n >= 11).sum()])
    exp = R * np.append(stats.poisson.pmf(k[:-1], rho),
                        stats.poisson.sf(10, rho))
    chi2 = ((obs - exp) ** 2 / exp)[exp > 5].sum()
    assert chi2 < stats.chi2.ppf(0.999, (exp > 5).sum() - 1)
    assert abs(n.mean() - rho) < 5 * np.sqrt(rho / R)


def test_poisson_counts_have_the_right_means_and_ln_Q():
    rng = np.random.default_rng(3)
    E = (rng.integers(-64, 64, 6000) * 4).astype(np.int32)   # N = 256
    dbeta = 0.02
    n_p, R_p, q_p = oracle.counts(256, E, 6000, dbeta, 5, 1, 3,
                                  law=oracle.POISSON)
    n_n, R_n, q_n = oracle.counts(256, E, 6000, dbeta, 5, 1, 3)
    assert q_p == q_n                      # the law does not enter ln Q
    w = np.exp(-dbeta * (E - E.min()).astype(np.float64))
    rho = 6000 * w / w.sum()
    assert abs(n_p.sum() - rho.sum()) < 5 * np.sqrt(rho.sum())
    # per energy level: counts around rho with Poisson spread
    z = (n_p - rho) / np.sqrt(rho)
    assert abs(z.mean()) < 5 / np.sqrt(len(z)) and 0.9 < z.std() < 1.1
    # energies outside [-2N, 2N] are rejected, not indexed
    bad = np.array([-2 * 256 - 4, 0], np.int32)
    with pytest.raises(Exception):
        oracle.counts(256, bad, 10, 0.1, 5, 1, 3)


def test_population_size_fluctuates_as_poisson():
    """E[R_new] = R_t and Var(R_new) = R_t over independent draws."""
    R_t, vals = 1500, []
    for seed in range(50):
        p = oracle.OraclePA(8, R_t, seed=seed, law=oracle.POISSON)
        vals.append(p.resample(0.1))
        p.close()
    v = np.array(vals, np.float64)
    assert abs(v.mean() - R_t) < 5 * np.sqrt(R_t / len(v))
    assert 0.4 * R_t < v.var(ddof=1) < 1.8 * R_t
