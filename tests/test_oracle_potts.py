"""Pins of the oracle's q-state Potts model (Sec. 2 names it with the heating
protocol): the exact density of states of the q = 3, L = 4 torus, the
Boltzmann distribution its Metropolis sweeps sample, free energies along
cooling and heating runs, and the identity of the q = 2 model with the
Ising model at half the coupling (Kaufman's solution)."""
import numpy as np
from scipy import stats

import exact_ising as X
import exact_potts as XP
import oracle


def test_density_of_states_closed_forms():
    g = XP.density_of_states(4, 3)
    assert g.sum() == 3 ** 16
    assert g[32] == 3                      # ground states
    assert g[31] == 0 and g[30] == 0        # one site out breaks 4 bonds
    assert g[28] == 3 * 16 * 2              # one site in another state
    gi = XP.density_of_states(4, 2)         # q = 2 is the Ising model
    E_ising, _ = X.enumerate_states(4)
    counts = np.bincount((E_ising + 32) // 2, minlength=33)
    # E_Potts = -N + E_Ising / 2, i.e. m = N - E_Ising / 2 satisfied bonds
    m = 16 - np.arange(-32, 33, 2) // 2
    ref = np.zeros(33)
    ref[m] = counts
    assert np.array_equal(gi, ref)


def test_energy_and_start_state():
    L, q, R = 8, 5, 4000
    p = oracle.OraclePA(L, R, seed=2, q=q)
    s, E, M = p.population()
    N = L * L
    assert s.min() >= 0 and s.max() < q
    Er, Mr = np.empty(R, np.int32), np.empty(R, np.int32)
    right = (s == np.roll(s, -1, axis=2)).sum(axis=(1, 2))
    down = (s == np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    assert np.array_equal(E, -(right + down))
    assert np.array_equal(M, q * (s == 0).sum(axis=(1, 2)) - N)
    # bond indicators are pairwise independent at beta = 0
    assert abs(E.mean() + 2 * N / q) < 5 * np.sqrt(2 * N / q / R)
    var = 2 * N * (1 / q) * (1 - 1 / q)
    assert abs(E.var() / var - 1) < 0.1
    assert p.free_energy()[0] == N * np.log(q)


def test_metropolis_samples_boltzmann_q3_L4():
    L, q, beta, R = 4, 3, 0.9, 6000
    p = oracle.OraclePA(L, R, seed=3, q=q)
    p.resample(beta)
    p.sweep(60)
    E, _ = p.energies()
    ex = XP.thermo(L, q, beta)["p"]
    obs = np.bincount(-E, minlength=len(ex)).astype(np.float64)
    exp = R * ex
    keep = exp > 5
    chi2 = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert chi2 < stats.chi2.ppf(0.999, keep.sum() - 1), chi2
    assert obs[~keep].sum() < 5 * max(1.0, exp[~keep].sum()) + 10


def _lnZ_runs(L, q, beta_f, K, theta, seeds, R, heat_from=None):
    z = []
    for seed in seeds:
        p = oracle.OraclePA(L, R, seed=seed, q=q)
        b0 = 0.0
        if heat_from is not None:
            p.start_heating(heat_from)
            b0 = heat_from
        for i in range(1, K + 1):
            p.resample(b0 + ((beta_f - b0) * i) / K)
            p.sweep(theta)
        z.append(p.free_energy()[0])
        p.close()
    return np.array(z)


def test_cooling_and_heating_lnZ_q3_L4_match_exact():
    L, q, beta = 4, 3, 1.2
    exact = XP.thermo(L, q, beta)["lnZ"]
    zc = _lnZ_runs(L, q, beta, 30, 3, range(1, 25), 500)
    zh = _lnZ_runs(L, q, beta, 30, 3, range(1, 25), 500, heat_from=4.0)
    for z in (zc, zh):
        assert abs(z.mean() - exact) < 4 * z.std(ddof=1) / np.sqrt(len(z)) + 2e-3


def test_q2_is_the_ising_model_at_half_coupling():
    """ln Z_Potts(beta) = beta N + ln Z_Ising(beta / 2) on the L = 16 torus."""
    L, beta = 16, 1.0
    N = L * L
    exact = beta * N + float(X.kaufman_lnZ(L, beta / 2))
    z = _lnZ_runs(L, 2, beta, 50, 4, range(1, 7), 1000)
    assert abs(z.mean() - exact) < 5 * z.std(ddof=1) / np.sqrt(len(z)) + 0.05


def test_single_replica_sweep_follows_the_population_sweep():
    """The single-replica Potts sweep (used to check sampled replicas at
    large populations) takes each replica through the same sweeps as the
    population sweep, from the same state, step and slot; and its returned
    E and M equal the energy and magnetisation of the state it returns."""
    L, q, R = 6, 4, 12
    p = oracle.OraclePA(L, R, seed=5, pop=2, q=q)
    p.resample(0.3)
    s0, E0, M0 = p.population()
    p.sweep(3)
    s1, E1, M1 = p.population()
    for j in range(R):
        s, e, m = oracle.sweep_potts_replica(s0[j], E0[j], M0[j], p.beta, q,
                                             5, 2, p.step, 0, 3, j)
        assert np.array_equal(s, s1[j]) and (e, m) == (E1[j], M1[j])
        # H = -(number of equal nearest-neighbour pairs), M = q n_0 - N
        ee = -int((s == np.roll(s, 1, 0)).sum() + (s == np.roll(s, 1, 1)).sum())
        assert (e, m) == (ee, q * int((s == 0).sum()) - L * L)
    p.close()
