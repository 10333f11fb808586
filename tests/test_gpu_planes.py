"""Parity of the bit-plane random-number mode of the sweep (PA_RNG_PLANES)
with the oracle's plane mode: spins, energies, magnetisations, copy counts
bit for bit and ln Z to 1e-12, over lattice sizes, both spin layouts, every
launch shape, ferromagnets and +-J glasses, and the threshold edge cases
(T = 2^32 for one energy step only, top bytes of 0 and 255, low
temperatures where most draws tie on a zero byte)."""
import os

import numpy as np
import pytest

import oracle
import pa_workloads as W

pytestmark = pytest.mark.gpu

REL = 1e-12


@pytest.fixture(scope="module")
def pa():
    if not os.path.exists("/dev/kfd"):
        pytest.skip("no GPU")
    from paper_2006_00561_amd import binding
    binding.lib()
    return binding


def _close(a, b):
    return abs(a - b) <= REL * max(1.0, abs(a), abs(b))


def _cmp(g, o, tag):
    sg, Eg, Mg = g.population()
    so, Eo, Mo = o.population()
    assert len(Eg) == len(Eo), tag
    assert np.array_equal(Eg, Eo), tag
    assert np.array_equal(Mg, Mo), tag
    assert np.array_equal(sg, so), tag
    zg, qg = g.free_energy()
    zo, qo = o.free_energy()
    assert _close(zg, zo) and _close(qg, qo), (tag, zg, zo)
    og, oo = g.observables(), o.observables()
    for k in ("R", "sumE", "sumE2", "sumAbsM", "sumM2", "Emin", "Emax"):
        assert og[k] == oo[k], (tag, k)


def _run(pa, L, R, betas, theta, seed=1, pop=0, J=None, layout=0, rpl=0,
         sweep_at_zero=0):
    print("planes L=%d R=%d steps=%d theta=%d layout=%d rpl=%d J=%s"
          % (L, R, len(betas), theta, layout, rpl, J is not None), flush=True)
    g = pa.Population(L, R, seed=seed, population_id=pop, J=J, layout=layout,
                      rows_per_lane=rpl, rng_mode=pa.PA_RNG_PLANES)
    o = oracle.OraclePA(L, R, seed=seed, pop=pop, J=J,
                        rng_mode=oracle.RNG_PLANES)
    if sweep_at_zero:
        g.sweep(0.0, sweep_at_zero)
        o.sweep(sweep_at_zero)
        _cmp(g, o, "beta 0")
    for i, b in enumerate(betas, start=1):
        R_old = g.R
        assert g.resample(b) == o.resample(b), i
        assert np.array_equal(g.counts(), o.counts(R_old)), i
        g.sweep(b, theta)
        o.sweep(theta)
        _cmp(g, o, "step %d" % i)
    g.close()
    o.close()


SHAPES = [
    # L, R, layout, rows per lane, glass
    (4, 37, 0, 0, False), (4, 37, 1, 4, True), (6, 300, 1, 2, True),
    (8, 257, 0, 0, True), (10, 129, 1, 0, False), (12, 100, 0, 4, False),
    (16, 700, 1, 2, False), (24, 333, 0, 0, True), (32, 300, 1, 4, True),
    (40, 65, 0, 2, False), (48, 90, 1, 0, True), (64, 129, 0, 0, False),
    (64, 129, 1, 1, False), (64, 70, 1, 2, True), (64, 70, 0, 4, False),
    (66, 20, 0, 0, False), (96, 30, 1, 3, True), (100, 12, 0, 4, False),
    (128, 24, 1, 0, False), (128, 20, 0, 4, True), (12, 250, 1, 3, False),
    (64, 129, 0, 2, False), (64, 67, 0, 2, True),
]


@pytest.mark.parametrize("L,R,layout,rpl,glass", SHAPES)
def test_plane_mode_shapes_and_layouts(pa, L, R, layout, rpl, glass):
    J = W.pmj_couplings(L, 300 + L) if glass else None
    _run(pa, L, R, W.linear_schedule(1.2, 5), 2, seed=5 + L, pop=L, J=J,
         layout=layout, rpl=rpl)


def test_plane_mode_threshold_edges(pa):
    """beta = 0 sweeps (T = 2^32 for both steps), beta = 1e-17 (T = 2^32 for
    dE = 4 only, top byte 255 for dE = 8), then cold temperatures where the
    top bytes are 0 and every positive step ties on a zero byte with
    probability 1/256."""
    betas = [1e-17, 0.05, 0.3, 1.0, 2.0, 3.5, 5.0]
    for layout in (0, 1):
        _run(pa, 16, 400, betas, 3, seed=21, layout=layout, sweep_at_zero=2)
        _run(pa, 32, 150, betas, 2, seed=22, layout=layout,
             J=W.pmj_couplings(32, 77))


def test_plane_mode_C1_trajectory(pa):
    c = W.CONFIGS["C1"]
    _run(pa, c["L"], c["R"], W.linear_schedule(c["beta_f"], c["K"]),
         c["theta"], seed=c["seed"])


def test_plane_mode_survives_save_and_load(pa, tmp_path):
    L, R = 24, 300
    g = pa.Population(L, R, seed=4, rng_mode=pa.PA_RNG_PLANES)
    o = oracle.OraclePA(L, R, seed=4, rng_mode=oracle.RNG_PLANES)
    sched = W.linear_schedule(0.9, 6)
    for b in sched[:3]:
        g.resample(b)
        g.sweep(b, 2)
        o.resample(b)
        o.sweep(2)
    path = str(tmp_path / "planes.pa")
    g.save(path)
    g.close()
    g = pa.Population.load(path)
    for b in sched[3:]:
        g.resample(b)
        g.sweep(b, 2)
        o.resample(b)
        o.sweep(2)
    _cmp(g, o, "resumed")
    g.close()
    o.close()


def test_plane_mode_differs_from_word_mode_but_not_its_law(pa):
    """The two modes draw different numbers (so their trajectories part),
    while the first sweep at beta = 0 accepts every flip in both."""
    L, R = 16, 200
    a = pa.Population(L, R, seed=8)
    b = pa.Population(L, R, seed=8, rng_mode=pa.PA_RNG_PLANES)
    a.sweep(0.0, 1)
    b.sweep(0.0, 1)
    for x, y in zip(a.population(), b.population()):
        assert np.array_equal(x, y)
    for p in (a, b):
        p.resample(0.5)
        p.sweep(0.5, 3)
    assert not np.array_equal(a.population()[0], b.population()[0])
    a.close()
    b.close()


def test_plane_mode_refused_where_unsupported(pa):
    with pytest.raises(pa.PAError):
        pa.Population(16, 100, q=4, rng_mode=pa.PA_RNG_PLANES)
    with pytest.raises(pa.PAError):
        pa.Population(16, 100, rng_mode=7)
