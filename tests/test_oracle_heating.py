"""Pins of the oracle's heating protocol (Sec. 2: the population starts near
zero temperature in the ground states and beta decreases): the start state
and its free energy, and ln Z along a heating run against enumeration and
Kaufman's exact solution."""
import numpy as np
import pytest

import exact_ising as X
import exact_potts as XP
import oracle


def test_ground_state_start():
    L, R, beta0 = 8, 3000, 3.0
    p = oracle.OraclePA(L, R, seed=5)
    p.start_heating(beta0)
    s, E, M = p.population()
    N = L * L
    assert np.all(E == -2 * N) and np.all(np.abs(M) == N)
    assert np.all(s.reshape(R, -1) == np.sign(M)[:, None])
    up = (M > 0).mean()
    assert abs(up - 0.5) < 5 * np.sqrt(0.25 / R)
    # Kaufman's finite-torus ln Z; what the start leaves out is of order
    # N exp(-16 beta0) = 1e-19 here, far below the rounding of ln Z
    exact = float(X.kaufman_lnZ(L, beta0))
    assert abs(p.free_energy()[0] - exact) <= 4e-16 * exact
    assert p.beta == beta0
    # ground states are a fresh ferromagnet's only
    q = oracle.OraclePA(L, 10, seed=5, J=np.ones((2, L, L), np.int8))
    try:
        q.start_heating(beta0)
        raise AssertionError("heating start accepted couplings")
    except RuntimeError:
        pass


@pytest.mark.parametrize("beta0", [1.0, 1.5, 2.0, 2.5, 3.0, 4.0])
def test_start_lnZ_ising_L4_within_the_expansion_bound(beta0):
    """The start's ln Z against enumeration of all 2^16 states.  With
    y = exp(-2 beta0) per broken bond, the first neglected term of ln Z is
    of order N y^8 (two distant flipped spins, straight and bent triples,
    2x2 squares), so the difference must stay below a few N exp(-16 beta0);
    that bound is 14 times smaller than the dimer term 2 N exp(-12 beta0)
    at beta0 = 1 and shrinks faster with beta0."""
    L = 4
    N = L * L
    p = oracle.OraclePA(L, 10, seed=3)
    p.start_heating(beta0)
    exact = X.brute_thermo(L, beta0)["lnZ"]
    bound = 8.0 * N * np.exp(-16.0 * beta0) + 4e-16 * exact
    assert abs(p.free_energy()[0] - exact) <= bound


@pytest.mark.parametrize("beta0", [2.0, 3.0, 4.0, 5.0, 6.0])
def test_start_lnZ_potts_q3_L4_within_the_expansion_bound(beta0):
    """The q = 3 Potts start against the transfer-matrix density of states.
    One broken bond costs exp(-beta0); the first neglected terms have eight
    broken bonds, so the difference stays below a few N exp(-8 beta0), which
    is below the two-different-neighbours term 2 N (q-1)(q-2) exp(-7 beta0)
    from beta0 = 2 on."""
    L, q = 4, 3
    N = L * L
    p = oracle.OraclePA(L, 10, seed=3, q=q)
    p.start_heating(beta0)
    exact = XP.thermo(L, q, beta0)["lnZ"]
    bound = 12.0 * N * np.exp(-8.0 * beta0) + 4e-16 * exact
    assert abs(p.free_energy()[0] - exact) <= bound


def _heat(L, R, beta0, beta_f, K, theta, seed):
    p = oracle.OraclePA(L, R, seed=seed)
    p.start_heating(beta0)
    for i in range(1, K + 1):
        b = beta0 + ((beta_f - beta0) * i) / K
        p.resample(b)
        p.sweep(theta)
    return p


def test_heating_lnZ_L4_matches_enumeration():
    L, beta0, beta_f = 4, 4.0, 0.3
    exact = X.brute_thermo(L, beta_f)["lnZ"]
    z = np.array([_heat(L, 400, beta0, beta_f, 30, 3, seed).free_energy()[0]
                  for seed in range(1, 31)])
    assert abs(z.mean() - exact) < 4 * z.std(ddof=1) / np.sqrt(len(z)) + 2e-3


def test_heating_to_infinite_temperature_recovers_N_ln2():
    """Heating all the way to beta = 0 must end at ln Z(0) = N ln 2."""
    L = 4
    z = np.array([_heat(L, 600, 3.0, 0.0, 40, 3, seed).free_energy()[0]
                  for seed in range(1, 21)])
    want = L * L * np.log(2.0)
    assert abs(z.mean() - want) < 4 * z.std(ddof=1) / np.sqrt(len(z)) + 2e-3


def test_heating_lnZ_L16_matches_kaufman():
    L, beta0, beta_f = 16, 2.0, 0.5
    exact = float(X.kaufman_lnZ(L, beta_f))
    z = np.array([_heat(L, 1000, beta0, beta_f, 60, 4, seed).free_energy()[0]
                  for seed in range(1, 7)])
    assert abs(z.mean() - exact) < 5 * z.std(ddof=1) / np.sqrt(len(z)) + 0.05
