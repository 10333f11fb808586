"""Pins of the oracle's energy-distribution overlap and its bisection (the
adaptive temperature step, Sec. 3): alpha(0) = 1; the per-replica form
(1/R) sum_j min(1, tau_j), tau_j = R w_j / sum w, evaluated in extended
precision from the energies; a two-level population in closed form, and the
step the bisection must return for it; the limit of a large step; and
monotonicity in the step."""
import numpy as np
import pytest

import oracle


def _tau_overlap(E, dbeta):
    x = -np.longdouble(dbeta) * E.astype(np.longdouble)
    w = np.exp(x - x.max())
    tau = len(E) * w / w.sum()
    return float(np.minimum(np.longdouble(1), tau).sum() / len(E))


def _two_level(h0, h1, L=4):
    """h0 all-up ground states (E = -2N) and h1 states with one spin flipped
    (E = -2N + 8)."""
    s = np.ones((h0 + h1, L, L), np.int8)
    s[h0:, 1, 2] = -1
    p = oracle.OraclePA(L, h0 + h1, seed=2)
    p.set_population(s)
    return p


def _alpha_two_level(h0, h1, dbeta):
    e = np.exp(-8.0 * np.longdouble(dbeta))
    return float(np.longdouble(h0) / (h0 + h1) + h1 * e / (h0 + h1 * e))


@pytest.fixture(scope="module")
def spread():
    """A population at beta = 0 (energies spread over many levels)."""
    p = oracle.OraclePA(8, 3000, seed=11)
    E = p.population()[1].copy()
    yield p, E
    p.close()


def test_zero_step_overlaps_fully(spread):
    p, _ = spread
    assert abs(p.overlap(0.0) - 1.0) < 1e-14


@pytest.mark.parametrize("dbeta", [1e-4, 0.01, 0.05, 0.2, 1.0, 5.0])
def test_overlap_equals_the_per_replica_form(spread, dbeta):
    p, E = spread
    assert p.overlap(dbeta) == pytest.approx(_tau_overlap(E, dbeta),
                                             rel=1e-12)


def test_overlap_is_monotone_and_tends_to_the_lowest_level(spread):
    p, E = spread
    grid = np.linspace(0.0, 3.0, 61)
    a = np.array([p.overlap(d) for d in grid])
    assert np.all(np.diff(a) <= 1e-15)
    lowest = np.mean(E == E.min())
    assert p.overlap(200.0) == pytest.approx(lowest, rel=1e-12)


@pytest.mark.parametrize("h0,h1", [(300, 700), (50, 950), (900, 100)])
def test_two_level_overlap_in_closed_form(h0, h1):
    p = _two_level(h0, h1)
    for d in (0.0, 0.01, 0.1, 0.4, 2.0):
        assert p.overlap(d) == pytest.approx(_alpha_two_level(h0, h1, d),
                                             rel=1e-13)
    p.close()


@pytest.mark.parametrize("h0,h1,target", [(300, 700, 0.85), (300, 700, 0.5),
                                          (50, 950, 0.9), (900, 100, 0.95)])
def test_bisection_inverts_the_two_level_overlap(h0, h1, target):
    """alpha = a + h1 e / (h0 + h1 e), a = h0 / R, e = exp(-8 dbeta): the
    step with alpha = target is e* = u h0 / (h1 (1 - u)), u = target - a."""
    p = _two_level(h0, h1)
    a = h0 / (h0 + h1)
    u = target - a
    d_star = -np.log(u * h0 / (h1 * (1.0 - u))) / 8.0
    beta_f = 10.0
    d = p.bisect_dbeta(target, beta_f)
    assert d == pytest.approx(d_star, rel=1e-9)
    assert p.overlap(d) >= target
    # a target the whole span meets returns the span
    assert p.bisect_dbeta(_alpha_two_level(h0, h1, 0.05) - 1e-9, 0.05) == 0.05
    p.close()
