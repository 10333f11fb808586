"""Pins of the oracle's model, initial state and Metropolis sweep against
enumeration, closed forms and invariants (none of them re-types the oracle's
own formulas)."""
import numpy as np
import pytest

import exact_ising as X
import oracle


def _np_energy(s, J=None):
    s = s.astype(np.int64)
    L = s.shape[-1]
    Jr = np.ones((L, L), np.int64) if J is None else J[0].astype(np.int64)
    Jd = np.ones((L, L), np.int64) if J is None else J[1].astype(np.int64)
    right = np.roll(s, -1, axis=-1)
    down = np.roll(s, -1, axis=-2)
    E = -(Jr * s * right).sum(axis=(-1, -2)) - (Jd * s * down).sum(
        axis=(-1, -2))
    return E, s.sum(axis=(-1, -2))


def _rand_J(L, seed):
    rng = np.random.default_rng(seed)
    return (2 * rng.integers(0, 2, (2, L, L)) - 1).astype(np.int8)


@pytest.mark.parametrize("L", [4, 6, 16])
@pytest.mark.parametrize("glass", [False, True])
def test_energy_matches_bond_sum(L, glass):
    rng = np.random.default_rng(L)
    J = _rand_J(L, 3) if glass else None
    for _ in range(20):
        s = (2 * rng.integers(0, 2, (L, L)) - 1).astype(np.int8)
        E, M = oracle.energy(s, J)
        e2, m2 = _np_energy(s, J)
        assert (E, M) == (int(e2), int(m2))


def test_density_of_states_L4(oracle_lib):
    """All 2^16 states of L=4 through the oracle's energy function."""
    L = 4
    g = X.density_of_states(L)
    # closed forms: two ground states at -2N, 2N single flips at -2N+8,
    # no state at -2N+4, 2^N states in total, symmetric under E -> -E
    N = L * L
    assert g[-2 * N] == 2 and g[-2 * N + 8] == 2 * N
    assert (-2 * N + 4) not in g and sum(g.values()) == 2 ** N
    assert all(g[e] == g[-e] for e in g)
    # Z(beta) = sum g e^{-beta E} agrees with Kaufman's torus formula
    for b in (0.1, 0.44, 0.9):
        lz = np.log(sum(c * np.exp(-b * e) for e, c in g.items()))
        assert abs(lz - float(X.kaufman_lnZ(L, b))) < 1e-12
    # the oracle's energies of every state reproduce g(E)
    idx = np.arange(1 << N, dtype=np.int64)
    s = (2 * ((idx[:, None] >> np.arange(N)) & 1) - 1).astype(np.int8)
    p = oracle.OraclePA(L, 1 << N, seed=1, capacity=1 << N)
    p.set_population(s.reshape(-1, L, L))
    E, M = p.energies()
    vals, cnt = np.unique(E, return_counts=True)
    assert dict(zip(vals.tolist(), cnt.tolist())) == g


def test_initial_population_is_uniform():
    """beta_0 = 0: <E> = 0 and Var(E) = 2N (the 2N bond products are
    pairwise independent), spins are fair coins."""
    L, R = 16, 4000
    N = L * L
    p = oracle.OraclePA(L, R, seed=11)
    s, E, M = p.population()
    assert abs(E.mean()) < 5 * np.sqrt(2 * N / R)
    assert abs(E.var() / (2 * N) - 1) < 5 * np.sqrt(2 / R)
    up = (s == 1).mean()
    assert abs(up - 0.5) < 5 * np.sqrt(0.25 / (R * N))
    e2, m2 = _np_energy(s)
    assert np.array_equal(E, e2) and np.array_equal(M, m2)
    # different seeds and population ids give different populations
    s2, _, _ = oracle.OraclePA(L, 10, seed=12).population()
    s3, _, _ = oracle.OraclePA(L, 10, seed=11, pop=1).population()
    assert not np.array_equal(s[:10], s2) and not np.array_equal(s[:10], s3)


@pytest.mark.parametrize("glass", [False, True])
def test_metropolis_samples_boltzmann_L4(glass):
    """After resampling to beta and sweeping, every replica's energy follows
    g(E) e^{-beta E} / Z (chi^2 over the energy levels)."""
    L, R, beta = 4, 20000, 0.45
    J = _rand_J(L, 5) if glass else None
    p = oracle.OraclePA(L, R, seed=21, J=J)
    p.resample(beta)
    p.sweep(60)
    E, M = p.energies()
    g = X.density_of_states(L, J)
    levels = sorted(g)
    w = np.array([g[e] * np.exp(-beta * e) for e in levels])
    prob = w / w.sum()
    obs = np.array([(E == e).sum() for e in levels])
    n = len(E)
    exp_cnt = prob * n
    keep = exp_cnt > 5
    chi2 = ((obs[keep] - exp_cnt[keep]) ** 2 / exp_cnt[keep]).sum()
    dof = keep.sum() - 1
    assert chi2 < dof + 6 * np.sqrt(2 * dof), (chi2, dof)
    assert obs[~keep].sum() < max(25, 5 * exp_cnt[~keep].sum())


@pytest.mark.parametrize("L", [6, 8, 12])
def test_order_within_colour_is_irrelevant(L):
    """Same-colour sites share no bond, so visiting them in any order gives
    the same configuration bit for bit."""
    a = oracle.OraclePA(L, 50, seed=3)
    b = oracle.OraclePA(L, 50, seed=3)
    b.set_visit_shuffle(987654321)
    for beta in (0.2, 0.5):
        a.resample(beta)
        b.resample(beta)
        a.sweep(3)
        b.sweep(3)
    sa, Ea, Ma = a.population()
    sb, Eb, Mb = b.population()
    assert np.array_equal(sa, sb) and np.array_equal(Ea, Eb)
    assert np.array_equal(Ma, Mb)


@pytest.mark.parametrize("L", [4, 6, 10])
def test_infinite_temperature_sweep_flips_every_spin(L):
    """At beta = 0 every proposal is accepted: one sweep flips each spin once
    (colour 0, then colour 1), so the result is the mirrored state."""
    rng = np.random.default_rng(L)
    s = (2 * rng.integers(0, 2, (L, L)) - 1).astype(np.int8)
    E, M = oracle.energy(s)
    s1, E1, M1 = oracle.sweep_replica(s, E, M, 0.0, 1, 0, 1, 0, 1, 0)
    assert np.array_equal(s1, -s) and E1 == E and M1 == -M


@pytest.mark.parametrize("glass", [False, True])
def test_zero_temperature_sweep_never_raises_energy(glass):
    L = 12
    J = _rand_J(L, 8) if glass else None
    rng = np.random.default_rng(2)
    s = (2 * rng.integers(0, 2, (L, L)) - 1).astype(np.int8)
    E, M = oracle.energy(s, J)
    for t in range(6):
        s, E2, M2 = oracle.sweep_replica(s, E, M, 40.0, 1, 0, 1, t, 1, 0, J)
        assert E2 <= E
        assert (E2, M2) == oracle.energy(s, J)
        E, M = E2, M2


def test_tracked_energy_equals_recomputed_after_annealing():
    L = 8
    for J in (None, _rand_J(L, 4)):
        p = oracle.OraclePA(L, 300, seed=5, J=J)
        for i in range(1, 11):
            p.resample(0.1 * i)
            p.sweep(2)
        s, E, M = p.population()
        for j in range(len(E)):
            assert (E[j], M[j]) == oracle.energy(s[j], J)


def test_threaded_sweep_equals_single_thread():
    """The replica-parallel sweep (used to time the oracle on all host
    cores) gives the single-threaded result bit for bit."""
    import oracle as O
    import pa_workloads as W
    a = O.OraclePA(8, 333, seed=5)
    b = O.OraclePA(8, 333, seed=5)
    for beta in W.linear_schedule(0.6, 4):
        assert a.resample(beta) == b.resample(beta)
        a.sweep(3)
        b.sweep(3, threads=7)
    sa, Ea, Ma = a.population()
    sb, Eb, Mb = b.population()
    assert np.array_equal(sa, sb) and np.array_equal(Ea, Eb)
    assert np.array_equal(Ma, Mb)
    assert a.free_energy() == b.free_energy()
