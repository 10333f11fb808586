"""Pins of the oracle's bit-plane random numbers (ORC_RNG_PLANES): a site's
32-bit number r = B 2^24 + floor(w / 2^8), B a byte of bit planes shared out
of one Philox block per 16 colour sites, w the site's default word.  The
Metropolis rule r < T is unchanged, so the sweep must keep sampling the
Boltzmann distribution and the run must keep estimating ln Z without bias;
the planes of different sites must be different bits (independent), and
every bit of r must be a fair coin."""
import numpy as np
import pytest

import exact_ising as X
import oracle


def _draws(mode, L, n_slots, hs=3, step=7, seed=11, pop=2):
    """r of every site of colour hs mod 2 of every row for n_slots replica
    slots: array [n_slots][L][L/2], index k = x/2."""
    out = np.zeros((n_slots, L, L // 2), np.uint64)
    for j in range(n_slots):
        for y in range(L):
            for k in range(L // 2):
                x = 2 * k + ((hs + y) & 1)
                out[j, y, k] = oracle.site_draw(mode, L, seed, pop, step, hs, j,
                                                y, x)
    return out


def test_plane_draws_are_fair_and_independent():
    L = 64
    r = _draws(oracle.RNG_PLANES, L, 24)
    flat = r.reshape(-1)
    n = flat.size
    # every bit of r is a fair coin (6 sigma)
    for b in range(32):
        ones = int(((flat >> np.uint64(b)) & np.uint64(1)).sum())
        assert abs(ones - n / 2) < 6 * np.sqrt(n / 4), (b, ones, n)
    # the top byte (the plane byte) is uniform over its 256 values
    top = (flat >> np.uint64(24)).astype(np.int64)
    cnt = np.bincount(top, minlength=256)
    e = n / 256.0
    chi2 = ((cnt - e) ** 2 / e).sum()
    assert chi2 < 255 + 6 * np.sqrt(2 * 255), chi2
    # neighbouring colour sites of one plane group draw different bits:
    # their plane bytes agree about 1 time in 256, and the bytes of sites k
    # and k + 1 are uncorrelated
    a = (r[:, :, 0::2] >> np.uint64(24)).astype(np.float64).reshape(-1)
    b = (r[:, :, 1::2] >> np.uint64(24)).astype(np.float64).reshape(-1)
    same = float((a == b).mean())
    assert same < 4.0 / 256, same
    corr = np.corrcoef(a, b)[0, 1]
    assert abs(corr) < 6 / np.sqrt(len(a)), corr
    # the low 24 bits are the high 24 bits of the default word of the site
    w = _draws(oracle.RNG_WORD, L, 2)
    assert np.array_equal(r[:2] & np.uint64(0xFFFFFF), w >> np.uint64(8))


def test_plane_draws_of_a_site_change_with_the_half_sweep_and_slot():
    L = 16
    a = _draws(oracle.RNG_PLANES, L, 2, hs=0)
    b = _draws(oracle.RNG_PLANES, L, 2, hs=1)
    assert (a != b).mean() > 0.99
    assert (a[0] != a[1]).mean() > 0.99


@pytest.mark.parametrize("glass", [False, True])
def test_planes_metropolis_samples_boltzmann_L4(glass):
    """The sweep with bit-plane numbers samples g(E) e^{-beta E} / Z (chi^2
    over the energy levels of every replica), at a beta where the ties of
    the plane byte with the threshold's top byte matter."""
    L, R, beta = 4, 20000, 0.45
    J = None
    if glass:
        rng = np.random.default_rng(5)
        J = np.where(rng.random((2, L, L)) < 0.5, -1, 1).astype(np.int8)
    p = oracle.OraclePA(L, R, seed=21, J=J, rng_mode=oracle.RNG_PLANES)
    p.resample(beta)
    p.sweep(60)
    E, _ = p.energies()
    g = X.density_of_states(L, J)
    levels = sorted(g)
    w = np.array([g[e] * np.exp(-beta * e) for e in levels])
    prob = w / w.sum()
    obs = np.array([(E == e).sum() for e in levels])
    exp_cnt = prob * len(E)
    keep = exp_cnt > 5
    chi2 = ((obs[keep] - exp_cnt[keep]) ** 2 / exp_cnt[keep]).sum()
    dof = keep.sum() - 1
    assert chi2 < dof + 6 * np.sqrt(2 * dof), (chi2, dof)
    assert obs[~keep].sum() < max(25, 5 * exp_cnt[~keep].sum())


def test_planes_lnZ_unbiased_L4():
    """Over independent runs with bit-plane numbers, exp(ln Z_hat) is an
    unbiased estimate of the enumerated Z."""
    L, beta_f, K = 4, 1.0, 20
    exact = X.brute_thermo(L, beta_f)["lnZ"]
    z = []
    for seed in range(1, 41):
        p = oracle.OraclePA(L, 400, seed=seed, rng_mode=oracle.RNG_PLANES)
        for i in range(1, K + 1):
            p.resample((beta_f * i) / K)
            p.sweep(3)
        z.append(p.free_energy()[0])
    z = np.array(z)
    ratio = np.exp(z - exact)
    se = ratio.std(ddof=1) / np.sqrt(len(z))
    assert abs(ratio.mean() - 1.0) < 4 * se + 2e-3
    assert abs(z.mean() - exact) < 4 * z.std(ddof=1) / np.sqrt(len(z)) + 2e-3


def test_planes_mode_changes_only_the_numbers():
    """Same population, same schedule: the two modes give different spins
    (different random numbers) but the same initial state and the same
    rule; beta = 0 flips every spin in either mode."""
    a = oracle.OraclePA(8, 100, seed=4)
    b = oracle.OraclePA(8, 100, seed=4, rng_mode=oracle.RNG_PLANES)
    assert np.array_equal(a.population()[0], b.population()[0])
    a.resample(0.0)
    b.resample(0.0)
    a.sweep(1)
    b.sweep(1)
    assert np.array_equal(a.population()[0], b.population()[0])
    for x in (a, b):
        x.resample(0.4)
        x.sweep(2)
    assert not np.array_equal(a.population()[0], b.population()[0])
