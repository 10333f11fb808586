"""Pins of the oracle's heating protocol (Sec. 2: the population starts near
zero temperature in the ground states and beta decreases): the start state
and its free energy, and ln Z along a heating run against enumeration and
Kaufman's exact solution."""
import numpy as np

import exact_ising as X
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
    assert p.free_energy()[0] == np.log(2.0) + 2.0 * N * beta0
    assert p.beta == beta0
    # ground states are a fresh ferromagnet's only
    q = oracle.OraclePA(L, 10, seed=5, J=np.ones((2, L, L), np.int8))
    try:
        q.start_heating(beta0)
        raise AssertionError("heating start accepted couplings")
    except RuntimeError:
        pass


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
