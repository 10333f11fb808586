"""Pins of the whole oracle PA run against exact physics: brute-force
enumeration at L=4, Kaufman's torus partition function at L=16, the
unbiasedness of the partition-function estimate, the +-M symmetry and the
gauge symmetry of the +-J model."""
import numpy as np
import pytest

import exact_ising as X
import oracle
import pa_workloads as W


def _run(L, R, K, theta, beta_f, seed, J=None, pop=0):
    p = oracle.OraclePA(L, R, seed=seed, J=J, pop=pop)
    traj = []
    for i in range(1, K + 1):
        b = (beta_f * i) / K
        p.resample(b)
        p.sweep(theta)
        o = p.observables()
        z, q = p.free_energy()
        traj.append((b, z, o["e"], o["abs_m"], p.R))
    return p, traj


def test_lnZ_and_Zhat_unbiased_L4():
    """Over independent runs, exp(ln Z_hat) is an unbiased estimate of Z
    (the paper's recursion is a product of unbiased ratio estimates), and
    ln Z_hat is within statistical error of the enumerated value."""
    L, beta_f = 4, 1.0
    exact = X.brute_thermo(L, beta_f)["lnZ"]
    z = []
    for seed in range(1, 41):
        p, tr = _run(L, 400, 20, 3, beta_f, seed)
        z.append(tr[-1][1])
    z = np.array(z)
    ratio = np.exp(z - exact)
    se = ratio.std(ddof=1) / np.sqrt(len(z))
    assert abs(ratio.mean() - 1.0) < 4 * se + 2e-3
    assert abs(z.mean() - exact) < 4 * z.std(ddof=1) / np.sqrt(len(z)) + 2e-3


def test_observables_L4_match_enumeration():
    """Energy, |m|, m^2 and specific heat of equilibrated L = 4 populations
    against their exact Boltzmann averages (the specific heat from the
    population's energy variance, as the oracle defines it)."""
    L, beta = 4, 0.5
    ex = X.brute_thermo(L, beta)
    e, am, m2, cv = [], [], [], []
    for seed in range(1, 9):
        p, tr = _run(L, 2000, 10, 5, beta, seed)
        o = p.observables()
        e.append(o["e"])
        am.append(o["abs_m"])
        m2.append(o["m2"])
        cv.append(o["C"])
    for vals, want in ((e, ex["e"]), (am, ex["abs_m"]), (m2, ex["m2"]),
                       (cv, ex["C"])):
        vals = np.array(vals)
        se = vals.std(ddof=1) / np.sqrt(len(vals))
        assert abs(vals.mean() - want) < 5 * se + 1e-3, (vals.mean(), want)


@pytest.mark.slow
def test_lnZ_and_energy_L16_match_kaufman():
    """The C1-shape workload (L=16, beta 0 -> 1), shortened to 50 steps."""
    L = 16
    zs, es = [], []
    for seed in range(1, 5):
        p, tr = _run(L, 1000, 50, 5, 1.0, seed)
        zs.append(tr[-1][1])
        es.append(tr[-1][2])
    z_ex = float(X.kaufman_lnZ(L, 1.0))
    e_ex = X.kaufman_energy(L, 1.0)
    zs, es = np.array(zs), np.array(es)
    # ln Z_hat has a small negative bias of order Var/2; allow it plus 5 se
    se_z = zs.std(ddof=1) / np.sqrt(len(zs))
    assert -0.25 - 5 * se_z < zs.mean() - z_ex < 5 * se_z + 0.02, (zs, z_ex)
    se_e = es.std(ddof=1) / np.sqrt(len(es))
    assert abs(es.mean() - e_ex) < 5 * se_e + 2e-3, (es, e_ex)
    # at beta = 0.5 on the way (the trajectory passes the critical region)
    p, tr = _run(L, 1000, 50, 5, 1.0, 9)
    b, z, e, am, R = tr[24]
    assert abs(b - 0.5) < 1e-12
    assert abs(z - float(X.kaufman_lnZ(L, 0.5))) < 0.3
    assert abs(e - X.kaufman_energy(L, 0.5)) < 0.05


def test_global_flip_symmetry():
    """Flipping every spin of the initial population changes nothing but the
    sign of M: same energies, same copy counts, same ln Z, bit for bit."""
    L, R = 8, 300
    a = oracle.OraclePA(L, R, seed=5)
    b = oracle.OraclePA(L, R, seed=5)
    s, _, _ = a.population()
    b.set_population(-s)
    for i in range(1, 8):
        R_old = a.R
        Ra = a.resample(0.12 * i)
        Rb = b.resample(0.12 * i)
        assert Ra == Rb
        assert np.array_equal(a.counts(R_old), b.counts(R_old))
        a.sweep(2)
        b.sweep(2)
        sa, Ea, Ma = a.population()
        sb, Eb, Mb = b.population()
        assert np.array_equal(sa, -sb)
        assert np.array_equal(Ea, Eb) and np.array_equal(Ma, -Mb)
        assert a.free_energy() == b.free_energy()


def test_gauge_symmetry_of_pmJ_model():
    """With couplings J_xy = eps_x eps_y and spins eps*sigma, the +-J model is
    the ferromagnet in disguise: identical energies, copy counts and ln Z,
    spins related by eps, bit for bit."""
    L, R = 8, 300
    rng = np.random.default_rng(77)
    eps = (2 * rng.integers(0, 2, (L, L)) - 1).astype(np.int8)
    J = np.empty((2, L, L), np.int8)
    J[0] = eps * np.roll(eps, -1, axis=1)
    J[1] = eps * np.roll(eps, -1, axis=0)
    f = oracle.OraclePA(L, R, seed=6)
    g = oracle.OraclePA(L, R, seed=6, J=J)
    s, E, M = f.population()
    g.set_population(s * eps[None])
    for i in range(1, 8):
        Rf_old = f.R
        assert f.resample(0.15 * i) == g.resample(0.15 * i)
        assert np.array_equal(f.counts(Rf_old), g.counts(Rf_old))
        f.sweep(2)
        g.sweep(2)
        sf, Ef, _ = f.population()
        sg, Eg, _ = g.population()
        assert np.array_equal(sf * eps[None], sg)
        assert np.array_equal(Ef, Eg)
        assert f.free_energy() == g.free_energy()


def test_glass_L4_lnZ_matches_enumeration():
    L = 4
    rng = np.random.default_rng(3)
    J = (2 * rng.integers(0, 2, (2, L, L)) - 1).astype(np.int8)
    exact = X.brute_thermo(L, 1.5, J)["lnZ"]
    z = []
    for seed in range(1, 25):
        p, tr = _run(L, 400, 30, 3, 1.5, seed, J=J)
        z.append(tr[-1][1])
    z = np.array(z)
    assert abs(z.mean() - exact) < 4 * z.std(ddof=1) / np.sqrt(len(z)) + 5e-3


def test_lnZ_bias_and_variance_shrink_as_one_over_R():
    """The paper's error claims for the free-energy estimate (Sec. 4): over
    3000 independent L = 4 runs per size, Var(ln Z_hat) and the systematic
    error E[ln Z_hat] - ln Z both scale as 1/R (R = 8 against R = 32: ratios
    near 4), and the bias is -Var/2 to first order (ln of an unbiased
    estimate of Z)."""
    L, beta_f, K, theta = 4, 1.0, 10, 2
    ex = X.brute_thermo(L, beta_f)["lnZ"]
    stats = {}
    for R in (8, 32):
        d = []
        for s in range(1, 3001):
            p = oracle.OraclePA(L, R, seed=s)
            for b in W.linear_schedule(beta_f, K):
                p.resample(b)
                p.sweep(theta)
            d.append(p.free_energy()[0] - ex)
            p.close()
        d = np.array(d)
        stats[R] = (d.mean(), d.std(ddof=1) / np.sqrt(len(d)), d.var())
    (b8, se8, v8), (b32, se32, v32) = stats[8], stats[32]
    assert b8 < -10 * se8 and b32 < -5 * se32          # biased low
    assert 2.5 < b8 / b32 < 5.5                        # ~ 1/R
    assert 3.0 < v8 / v32 < 5.0
    for b, se, v in (stats[8], stats[32]):
        assert abs(b + v / 2) < 5 * se + 0.15 * abs(b)
