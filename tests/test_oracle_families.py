"""Pins of the oracle's family bookkeeping (the descendants of each replica
of the founding population, the population-annealing diagnostic that goes
with weighted averaging): families are the parent map composed over the
resamplings (numpy repeat of the copy counts), and the family statistics
against closed forms and their definition in extended precision."""
import numpy as np
import pytest

import oracle


def _definition(fam, n0):
    c = np.bincount(np.asarray(fam, np.int64), minlength=n0)
    R = c.sum()
    nu = c[c > 0].astype(np.longdouble) / R
    return {"families": int((c > 0).sum()), "largest": int(c.max()),
            "rho_t": float(R * (nu * nu).sum()),
            "rho_s": float(R * np.exp((nu * np.log(nu)).sum()))}


def test_every_replica_founds_a_family():
    p = oracle.OraclePA(6, 400, seed=4)
    f, n0 = p.families()
    assert n0 == 400 and np.array_equal(f, np.arange(400))
    assert oracle.family_stats(f, n0) == {"families": 400, "largest": 1,
                                          "rho_t": 1.0, "rho_s": 1.0}
    p.close()


def test_families_compose_over_resamplings():
    """After each resampling the family of new slot k is the family of its
    parent; the parents are numpy's repeat of the slots by the copy counts
    that the (separately pinned) count step gives on the energies."""
    L, R = 8, 600
    p = oracle.OraclePA(L, R, seed=7, pop=2)
    fam = np.arange(R)
    for i, b in enumerate((0.2, 0.35, 0.5, 0.6), start=1):
        E = p.population()[1]
        n, Rn, _ = oracle.counts(L * L, E, R, b - p.beta, 7, 2, i)
        fam = fam[np.repeat(np.arange(len(E)), n)]
        assert p.resample(b) == Rn
        f, n0 = p.families()
        assert n0 == R and np.array_equal(f, fam), i
        p.sweep(2)
    p.close()


def test_zero_step_keeps_every_family():
    p = oracle.OraclePA(6, 500, seed=5)
    p.resample(0.0)
    f, _ = p.families()
    assert np.array_equal(f, np.arange(500))
    p.close()


def test_family_stats_closed_forms():
    # one family holding everything: rho_t = rho_s = R
    s = oracle.family_stats(np.full(300, 7, np.uint32), 10)
    assert s["families"] == 1 and s["largest"] == 300
    assert s["rho_t"] == pytest.approx(300, rel=1e-14)
    assert s["rho_s"] == pytest.approx(300, rel=1e-14)
    # k equal families of m members: rho_t = rho_s = m
    for k, m in ((5, 40), (17, 3), (1, 1)):
        fam = np.repeat(np.arange(0, 2 * k, 2), m).astype(np.uint32)
        s = oracle.family_stats(fam, 2 * k)
        assert s["families"] == k and s["largest"] == m
        assert s["rho_t"] == pytest.approx(m, rel=1e-14)
        assert s["rho_s"] == pytest.approx(m, rel=1e-13)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_family_stats_match_the_definition(seed):
    rng = np.random.default_rng(seed)
    n0 = 500
    fam = rng.zipf(1.6, 3000) % n0
    s = oracle.family_stats(fam.astype(np.uint32), n0)
    d = _definition(fam, n0)
    assert (s["families"], s["largest"]) == (d["families"], d["largest"])
    assert s["rho_t"] == pytest.approx(d["rho_t"], rel=1e-12)
    assert s["rho_s"] == pytest.approx(d["rho_s"], rel=1e-12)
    assert s["rho_t"] >= s["rho_s"]      # exp of Renyi entropies: H1 >= H2
    with pytest.raises(RuntimeError):
        oracle.family_stats(np.array([0, n0], np.uint32), n0)


def test_set_population_and_heating_found_new_families():
    L, R = 6, 300
    p = oracle.OraclePA(L, R, seed=6)
    p.resample(0.4)
    p.set_population(p.population()[0][:250])
    f, n0 = p.families()
    assert n0 == 250 and np.array_equal(f, np.arange(250))
    h = oracle.OraclePA(L, R, seed=6)
    h.start_heating(2.0)
    f, n0 = h.families()
    assert n0 == R and np.array_equal(f, np.arange(R))
    p.close()
    h.close()
