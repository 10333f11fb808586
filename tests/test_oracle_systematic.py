"""Pins of the oracle's systematic, residual and multinomial resampling
(variants of the resampling step in the review the paper cites).
Systematic: one comb of unit-spaced points over the mean copy numbers laid
end to end; every count is the floor or the ceiling of its mean, the size is
the target up to one, and the counts are unbiased over the comb offset.
Residual: the floors for certain and multinomial draws over the fractions.
Multinomial: R_target independent draws weighted by the means."""
import numpy as np
import pytest

import oracle


def _energies(seed, R, L=16):
    rng = np.random.default_rng(seed)
    N = L * L
    return N, (rng.integers(-N // 2, N // 2, R) * 4).astype(np.int32)


def _rho(E, R_t, dbeta):
    x = -dbeta * E.astype(np.longdouble)
    ex = np.exp(x - x.max())
    return (R_t * ex / ex.sum()).astype(np.float64)


@pytest.mark.parametrize("dbeta,R_t", [(0.0, 3000), (0.01, 3000),
                                       (0.05, 2000), (0.2, 5000),
                                       (-0.03, 3000)])
def test_counts_are_floor_or_ceiling_and_size_is_exact(dbeta, R_t):
    N, E = _energies(1, 3000)
    n, Rn, lnQ = oracle.counts(N, E, R_t, dbeta, 9, 3, 4,
                               law=oracle.SYSTEMATIC)
    rho = _rho(E, R_t, dbeta)
    fl = np.floor(rho)
    near = np.abs(rho - np.round(rho)) < 1e-9
    ok = (n == fl) | (n == fl + 1)
    assert np.all(ok | near)
    assert Rn == n.sum() and R_t - 1 <= Rn <= R_t
    # the law does not enter ln Q
    assert lnQ == oracle.counts(N, E, R_t, dbeta, 9, 3, 4)[2]


def test_counts_are_unbiased_over_the_comb_offset():
    N, E = _energies(2, 400)
    R_t, dbeta = 400, 0.04
    rho = _rho(E, R_t, dbeta)
    acc = np.zeros(len(E))
    K = 400
    for step in range(1, K + 1):          # a fresh offset U at every step
        acc += oracle.counts(N, E, R_t, dbeta, 5, 1, step,
                             law=oracle.SYSTEMATIC)[0]
    mean = acc / K
    frac = rho - np.floor(rho)
    sd = np.sqrt(frac * (1 - frac) / K) + 1e-12
    z = (mean - rho) / sd
    assert np.all(np.abs(z[frac > 0.02]) < 6)
    assert abs(z[frac > 0.02].mean()) < 6 / np.sqrt((frac > 0.02).sum())


def test_systematic_population_runs():
    """A full anneal under the systematic law keeps R at the target (or one
    below) at every step."""
    p = oracle.OraclePA(8, 700, seed=3, law=oracle.SYSTEMATIC)
    for i in range(1, 21):
        Rn = p.resample(0.05 * i)
        assert 699 <= Rn <= 700
        p.sweep(2)


@pytest.mark.parametrize("dbeta", [0.0, 0.02, 0.2, -0.05])
def test_residual_keeps_the_floors_and_draws_over_the_fractions(dbeta):
    """Residual resampling: floor(rho) copies for certain, then
    R_target - sum floor(rho) multinomial draws weighted by the fractional
    parts: no count is below its floor, the size is exactly the target, and
    the extra copies follow the fractions."""
    N, E = _energies(4, 2500)
    R_t = 2500
    n, Rn, _ = oracle.counts(N, E, R_t, dbeta, 3, 2, 7, law=oracle.RESIDUAL)
    rho = _rho(E, R_t, dbeta)
    fl = np.floor(rho)
    near = np.abs(rho - np.round(rho)) < 1e-9
    assert np.all((n >= fl) | near)
    assert np.all(n[near] >= np.round(rho[near]) - 1)
    assert Rn == n.sum() == R_t
    # a replica whose mean is an integer gets exactly that many copies
    whole = np.abs(rho - np.round(rho)) < 1e-12
    if whole.any():
        assert np.all(n[whole] == np.round(rho[whole]))


@pytest.mark.parametrize("R,R_t", [(500, 500), (500, 1000), (300, 301),
                                   (400, 1201)])
def test_residual_at_zero_step_is_exact_or_one_draw(R, R_t):
    """At dbeta = 0 every replica has mean R_t / R: an integer mean gives
    exactly that many copies of each replica (no draws), and a target one
    above a multiple of the population is one draw over equal fractions."""
    N, E = _energies(7, R)
    n, Rn, _ = oracle.counts(N, E, R_t, 0.0, 3, 2, 5, law=oracle.RESIDUAL)
    assert Rn == R_t == n.sum()
    base = R_t // R
    assert np.all((n == base) | (n == base + 1))
    assert (n == base + 1).sum() == R_t - base * R


def test_residual_counts_are_unbiased():
    N, E = _energies(5, 300)
    R_t, dbeta = 300, 0.05
    rho = _rho(E, R_t, dbeta)
    fl = np.floor(rho)
    frac = rho - fl
    D = R_t - fl.sum()
    p = frac / frac.sum()
    acc = np.zeros(len(E))
    K = 300
    for step in range(1, K + 1):
        acc += oracle.counts(N, E, R_t, dbeta, 8, 1, step,
                             law=oracle.RESIDUAL)[0]
    sd = np.sqrt(D * p * (1 - p) / K) + 1e-12
    z = (acc / K - rho) / sd
    assert np.all(np.abs(z[frac > 0.02]) < 6)
    assert abs(z[frac > 0.02].mean()) < 6 / np.sqrt((frac > 0.02).sum())


def test_multinomial_draws_follow_the_weights():
    """Multinomial resampling: exactly R_target copies in total, each
    replica's count binomial with the probability of its weight."""
    N, E = _energies(6, 500)
    R_t, dbeta = 20000, 0.004
    n, Rn, lnQ = oracle.counts(N, E, R_t, dbeta, 4, 2, 9,
                               law=oracle.MULTINOMIAL)
    assert Rn == R_t == n.sum()
    assert lnQ == oracle.counts(N, E, R_t, dbeta, 4, 2, 9)[2]
    rho = _rho(E, R_t, dbeta)            # expected counts
    p = rho / R_t
    big = rho > 5
    assert big.sum() > 300
    z = ((n - rho) / np.sqrt(R_t * p * (1 - p)))[big]
    assert abs(z.mean()) < 5 / np.sqrt(len(z)) and 0.85 < z.std() < 1.15
    # a replica of zero weight is never drawn
    E2 = E.copy()
    E2[0] = 4 * N // 2                   # far above the rest
    n2 = oracle.counts(N, E2, R_t, 3.0, 4, 2, 9, law=oracle.MULTINOMIAL)[0]
    assert n2[0] == 0


def test_multinomial_draw_maps_exactly_at_interval_ends():
    """A 64-bit draw u lands at x = floor(u C / 2^64): for each interval
    [C_{j-1}, C_j) the smallest u that reaches it is ceil(C_{j-1} 2^64 / C)
    (exact integers), so u one below lands in the previous nonempty
    interval and u itself in j.  Intervals far below 2^-32 of the axis
    (a replica with a tiny mean) are still reached by their exact share of
    the 2^64 draws."""
    import numpy as np
    rng = np.random.default_rng(5)
    for R, big in ((5, False), (40, True), (300, True)):
        P = rng.integers(1, 1 << 40, size=R, dtype=np.uint64)
        if big:
            # one replica with mean 1e-6 copies among weights of order 2^32
            P[R // 2] = 4295
            P[:R // 2] = (rng.integers(1, 8, size=R // 2, dtype=np.uint64)
                          << np.uint64(32))
        cum = np.cumsum(P).astype(np.uint64)
        C = int(cum[-1])
        for j in range(R):
            lo_end = 0 if j == 0 else int(cum[j - 1])
            first_u = -(-(lo_end << 64) // C)          # ceil
            if first_u >= 1 << 64:
                continue
            assert oracle.multinomial_pick(first_u, cum) == j
            if first_u > 0:
                assert oracle.multinomial_pick(first_u - 1, cum) < j
            # the share of the 2^64 draws of interval j is its length
            # over C to within one draw in 2^64 (exact integers)
            last_u = -(-(int(cum[j]) << 64) // C)
            assert abs((last_u - first_u) * C - (int(P[j]) << 64)) <= C
