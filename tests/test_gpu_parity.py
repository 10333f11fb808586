"""Parity of the HIP path (through the C ABI) with the oracle.

Spins, energies, magnetisations, copy counts and population sizes must be
bit-exact; ln Z, ln Q and observables within 1e-12 relative (both sides
compute them in the same double-precision operation order, so they are in
fact expected to be identical).  At the full benchmark sizes the oracle
checks every copy count and ln Q exactly and a sample of replicas through
their sweeps."""
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


def _cmp_obs(og, oo):
    for k in ("R", "sumE", "sumE2", "sumAbsM", "sumM2", "Emin", "Emax"):
        assert og[k] == oo[k], k
    for k in ("beta", "e", "abs_m", "m2", "C"):
        assert _close(og[k], oo[k]), (k, og[k], oo[k])


def _cmp_state(g, o, tag):
    sg, Eg, Mg = g.population()
    so, Eo, Mo = o.population()
    assert len(Eg) == len(Eo), tag
    assert np.array_equal(Eg, Eo), tag
    assert np.array_equal(Mg, Mo), tag
    assert np.array_equal(sg, so), tag
    zg, qg = g.free_energy()
    zo, qo = o.free_energy()
    assert _close(zg, zo) and _close(qg, qo), (tag, zg, zo, qg, qo)
    # families: bit-exact, and their statistics to the floating-point bar
    fg, n0g = g.families()
    fo, n0o = o.families()
    assert n0g == n0o and np.array_equal(fg, fo), tag
    sg_, so_ = g.family_stats(), oracle.family_stats(fo, n0o)
    assert (sg_["families"], sg_["largest"]) == (so_["families"],
                                                 so_["largest"]), tag
    assert _close(sg_["rho_t"], so_["rho_t"]), tag
    assert _close(sg_["rho_s"], so_["rho_s"]), tag


def _parity_run(pa, L, R, steps, theta, beta_f, seed=1, pop=0, J=None,
                layout=0, rpl=0, check_every=1, law=0, q=0):
    print("parity L=%d R=%d steps=%d theta=%d layout=%d rpl=%d J=%s law=%d "
          "q=%d" % (L, R, steps, theta, layout, rpl, J is not None, law, q),
          flush=True)
    g = pa.Population(L, R, seed=seed, population_id=pop, J=J, layout=layout,
                      rows_per_lane=rpl, resampling=law, q=q)
    o = oracle.OraclePA(L, R, seed=seed, pop=pop, J=J, law=law, q=q)
    _cmp_state(g, o, "init")
    for i, b in enumerate(W.linear_schedule(beta_f, steps), start=1):
        R_old = g.R
        rg = g.resample(b)
        ro = o.resample(b)
        assert rg == ro, (i, rg, ro)
        assert np.array_equal(g.counts(), o.counts(R_old)), i
        g.sweep(b, theta)
        o.sweep(theta)
        if i % check_every == 0 or i == steps:
            _cmp_state(g, o, "step %d" % i)
            _cmp_obs(g.observables(), o.observables())
    g.close()
    o.close()


def test_C1_full_trajectory(pa):
    """L=16, R=1000, beta 0 -> 1 in 100 steps, theta=5, seed 1: every step."""
    c = W.CONFIGS["C1"]
    _parity_run(pa, c["L"], c["R"], c["K"], c["theta"], c["beta_f"],
                seed=c["seed"])


SHAPES = [
    # L, R, layout, rows per lane, glass
    (4, 37, 0, 0, False), (4, 37, 1, 4, True), (6, 300, 0, 0, False),
    (6, 300, 1, 2, True), (8, 257, 0, 0, True), (10, 129, 1, 0, False),
    (12, 513, 0, 0, True), (12, 100, 0, 4, False), (16, 700, 1, 2, False),
    (24, 333, 0, 0, True), (24, 200, 1, 4, True), (32, 300, 0, 1, False),
    (32, 300, 1, 4, True), (40, 65, 0, 2, False), (48, 90, 1, 0, True),
    (64, 129, 0, 0, False), (64, 70, 1, 2, True), (64, 70, 0, 4, False),
    (66, 20, 0, 0, False), (96, 30, 1, 0, True), (100, 12, 0, 4, False),
    (128, 24, 1, 0, False), (128, 20, 0, 4, True),
    (12, 250, 1, 3, False), (24, 300, 0, 3, True), (48, 90, 0, 3, False),
    (96, 30, 1, 3, True),
    # int8 L = 64 at two rows per lane: two replicas per wave moved as
    # whole kilobytes; an odd R leaves the last wave one replica
    (64, 129, 0, 2, False), (64, 67, 0, 2, True),
]


@pytest.mark.parametrize("L,R,layout,rpl,glass", SHAPES)
def test_shapes_and_layouts(pa, L, R, layout, rpl, glass):
    J = W.pmj_couplings(L, 100 + L) if glass else None
    _parity_run(pa, L, R, 5, 2, 0.8, seed=3 + L, pop=L, J=J, layout=layout,
                rpl=rpl)


def test_launch_shape_and_layout_do_not_change_results(pa):
    for L in (24, 32, 64):
        runs = []
        for layout in (0, 1):
            for rpl in ((1, 2, 3, 4) if L % 3 == 0 else (1, 2, 4)):
                g = pa.Population(L, 500, seed=9, layout=layout,
                                  rows_per_lane=rpl)
                for b in W.linear_schedule(0.7, 6):
                    g.resample(b)
                    g.sweep(b, 3)
                runs.append(g.population())
                g.close()
        for r in runs[1:]:
            for a, b in zip(runs[0], r):
                assert np.array_equal(a, b)


def test_zero_step_is_identity(pa):
    g = pa.Population(16, 400, seed=5)
    s0, E0, M0 = g.population()
    z0, _ = g.free_energy()
    assert g.resample(0.0) == 400
    assert np.all(g.counts() == 1)
    s1, E1, M1 = g.population()
    assert np.array_equal(s0, s1) and np.array_equal(E0, E1)
    z1, q1 = g.free_energy()
    assert q1 == 0.0 and z1 == z0


def test_capacity_overflow_leaves_population_untouched(pa):
    for seed in range(1, 40):
        g = pa.Population(6, 1000, seed=seed, capacity=1000)
        s0, E0, M0 = g.population()
        rc, Rn = g.resample_rc(0.3)
        if rc == pa.PA_OK:
            continue
        assert rc == pa.PA_ECAPACITY and Rn > 1000
        assert g.state() == (1000, 0.0, 0)
        s, E, M = g.population()
        assert np.array_equal(s, s0) and np.array_equal(E, E0)
        # the context still works afterwards
        o = oracle.OraclePA(6, 1000, seed=seed, capacity=1000)
        assert o.resample_rc(0.3) == (oracle.ECAPACITY, Rn)
        return
    raise AssertionError("no seed overflowed")


def test_state_errors(pa):
    g = pa.Population(8, 50, seed=1)
    with pytest.raises(pa.PAError) as e:
        g.sweep(0.5, 1)            # not the current beta
    assert e.value.code == pa.PA_ESTATE
    g.resample(0.2)
    with pytest.raises(pa.PAError) as e:
        g.resample(-0.1)           # beta stays >= 0
    assert e.value.code == pa.PA_EINVAL
    with pytest.raises(pa.PAError) as e:
        g.start_heating(2.0)       # only before the first resampling
    assert e.value.code == pa.PA_ESTATE
    with pytest.raises(pa.PAError):
        g.set_population(np.zeros((3, 8, 8), np.int8))


def test_set_population_and_global_flip(pa):
    L, R = 16, 300
    g = pa.Population(L, R, seed=5)
    o = oracle.OraclePA(L, R, seed=5)
    s, _, _ = o.population()
    g.set_population(-s)
    o.set_population(-s)
    _cmp_state(g, o, "flipped")
    for b in W.linear_schedule(0.8, 5):
        assert g.resample(b) == o.resample(b)
        g.sweep(b, 3)
        o.sweep(3)
    _cmp_state(g, o, "after")


def test_gauge_transformed_glass_matches_ferromagnet(pa):
    L, R = 24, 400
    J, eps = W.gauge_couplings(L, 31)
    f = pa.Population(L, R, seed=6)
    g = pa.Population(L, R, seed=6, J=J)
    s, _, _ = f.population()
    g.set_population(s * eps[None])
    for b in W.linear_schedule(1.0, 8):
        assert f.resample(b) == g.resample(b)
        f.sweep(b, 2)
        g.sweep(b, 2)
    sf, Ef, _ = f.population()
    sg, Eg, _ = g.population()
    assert np.array_equal(sf * eps[None], sg) and np.array_equal(Ef, Eg)
    assert f.free_energy() == g.free_energy()


def test_overlap_and_bisection_match_oracle(pa):
    L, R = 16, 2000
    g = pa.Population(L, R, seed=8)
    o = oracle.OraclePA(L, R, seed=8)
    for b in W.linear_schedule(0.4, 4):
        g.resample(b)
        o.resample(b)
        g.sweep(b, 2)
        o.sweep(2)
    for d in (0.0, 0.01, 0.1, 0.5):
        assert g.overlap(d) == o.overlap(d)
    assert g.bisect_dbeta(0.85, 3.0) == o.bisect_dbeta(0.85, 3.0)
    hg, st = g.histogram()
    ho = o.histogram()
    assert np.array_equal(hg, ho[::st])


def test_timing_counters(pa):
    g = pa.Population(32, 1000, seed=2)
    g.set_timing(True)
    for b in W.linear_schedule(0.5, 3):
        g.resample(b)
        g.sweep(b, 4)
    t = g.timing()
    assert t["sweep"]["launches"] == 3 and t["sweep"]["ms"] > 0
    # the sweeps made the resampling copies: no gather of its own
    assert t["gather"]["launches"] == 0 and t["hist"]["launches"] == 3
    assert t["attempts"] > 3 * 4 * 32 * 32 * 900
    # a read of the population before the sweep needs the gather
    g.resample(0.6)
    g.energies()
    g.sweep(0.6, 1)
    t = g.timing()
    assert t["gather"]["launches"] == 1 and t["sweep"]["launches"] == 4
    # timing of the sweeps alone
    g.set_timing(True, classes=("sweep",))
    g.resample(0.7, wait=False)
    g.sweep(0.7, 2)
    g.observables()
    t = g.timing()
    assert t["sweep"]["launches"] == 1 and t["sweep"]["ms"] > 0
    assert t["attempts"] == g.R * 32 * 32 * 2
    for k in ("hist", "counts", "scatter", "gather"):
        assert t[k]["launches"] == 0 and t[k]["ms"] == 0.0


@pytest.mark.parametrize("name,start,steps,sample,rng", [
    ("C2", 1, 3, 48, 0), ("C3a", 1, 2, 24, 0), ("C3b", 1, 2, 16, 0),
    ("CQ10", 1, 2, 24, 0),
    # the steps nearest the critical point beta_c = ln(1 + sqrt 2)/2 = 0.4407
    # (beta = 0.44 at step 88 of both schedules), where the copy counts
    # spread widest
    ("C2", 88, 2, 48, 0), ("C3a", 88, 2, 24, 0),
    # the bit-plane random numbers at the paper's scale
    ("C3a", 1, 2, 24, 1), ("C3a", 88, 2, 24, 1)])
def test_full_size_sampled(pa, name, start, steps, sample, rng):
    """At the benchmark sizes and in the benchmark's launch configuration
    (the capacity at which no resampling waits for its new size, resampling
    without waiting, the copies made by the next sweep from the parents):
    the population first runs unchecked on the device up to step start - 1;
    then, for `steps` steps, every copy count, R_new and ln Q exactly from
    the oracle's count step on the device energies; a sample of new
    replicas through theta sweeps with the oracle's single-replica sweep,
    started from their parents' states read before the resampling;
    observables from the full E and M arrays."""
    c = W.CONFIGS[name]
    L, R, theta, q = c["L"], c["R"], c["theta"], c.get("q", 0)
    layout = 1 if c["layout"] == "bits" else 0
    print("full-size parity %s L=%d R=%d layout=%d q=%d start=%d rng=%d"
          % (name, L, R, layout, q, start, rng), flush=True)
    g = pa.Population(L, R, seed=c["seed"], layout=layout, q=q,
                      capacity=W.deferral_capacity(R), rng_mode=rng)
    rng_o = oracle.RNG_PLANES if rng else oracle.RNG_WORD
    gen = np.random.default_rng(start)
    sched = W.linear_schedule(c["beta_f"], c["K"])
    if start == 1:
        # initial state: sampled replicas against the oracle's init
        o = oracle.OraclePA(L, 8, seed=c["seed"], q=q)
        so, Eo, Mo = o.population()
        sg, Eg, Mg = g.replicas(np.arange(8))
        assert np.array_equal(sg, so) and np.array_equal(Eg, Eo)
        assert np.array_equal(Mg, Mo)
        o.close()
        fam, n0 = g.families()
        assert n0 == R and np.array_equal(fam, np.arange(R))
    else:
        for b in sched[:start - 1]:
            g.resample(b, wait=False)
            g.sweep(b, theta)
        fam, n0 = g.families()
    zlast = g.free_energy()[0]
    for i in range(start, start + steps):
        b = sched[i - 1]
        E, M = g.energies()
        n_o, Rn_o, lnQ_o = oracle.counts(L * L, E, R, b - g.beta, c["seed"],
                                         0, i)
        parent = np.repeat(np.arange(len(E)), n_o)
        fam = fam[parent]  # every copy joins its parent's family
        slots = np.sort(gen.choice(Rn_o, size=sample, replace=False))
        s_pre, E_pre, M_pre = g.replicas(parent[slots])
        g.resample(b, wait=False)
        g.sweep(b, theta)
        assert g.state()[0] == Rn_o
        assert np.array_equal(g.counts(), n_o)
        assert np.array_equal(g.families()[0], fam)
        z, dq = g.free_energy()
        assert _close(dq, lnQ_o) and _close(z, zlast + lnQ_o)
        zlast = z
        s_post, E_post, M_post = g.replicas(slots)
        for k, j in enumerate(slots):
            if q:
                so, eo, mo = oracle.sweep_potts_replica(
                    s_pre[k], E_pre[k], M_pre[k], b, q, c["seed"], 0, i, 0,
                    theta, int(j))
            else:
                so, eo, mo = oracle.sweep_replica(s_pre[k], E_pre[k],
                                                  M_pre[k], b, c["seed"], 0,
                                                  i, 0, theta, int(j),
                                                  rng_mode=rng_o)
            assert np.array_equal(s_post[k], so), (name, i, j)
            assert (E_post[k], M_post[k]) == (eo, mo)
        E2, M2 = g.energies()
        ob = g.observables()
        assert ob["sumE"] == int(E2.astype(np.int64).sum())
        assert ob["sumAbsM"] == int(np.abs(M2.astype(np.int64)).sum())
        assert ob["sumM2"] == int((M2.astype(np.int64) ** 2).sum())
    g.close()


@pytest.mark.parametrize("layout,glass", [(0, False), (1, True)])
def test_resampling_copies_in_every_call_order(pa, layout, glass):
    """The copies of a resampling are made by the next sweep or, before any
    other read of the population, by a plain gather: every order of calls
    after a resampling must give the oracle's population."""
    L, R = 12, 600
    J = W.pmj_couplings(L, 77) if glass else None
    g = pa.Population(L, R, seed=4, population_id=3, J=J, layout=layout)
    o = oracle.OraclePA(L, R, seed=4, pop=3, J=J)
    betas = iter(W.linear_schedule(1.4, 14))

    def step():
        b = next(betas)
        assert g.resample(b) == o.resample(b)
        return b

    # resample, then sweep (copies fused into the sweep)
    b = step()
    g.sweep(b, 3)
    o.sweep(3)
    _cmp_state(g, o, "fused")
    # resample, energies only, then sweep
    b = step()
    Eg, Mg = g.energies()
    Eo, Mo = o.energies()
    assert np.array_equal(Eg, Eo) and np.array_equal(Mg, Mo)
    g.sweep(b, 2)
    o.sweep(2)
    _cmp_state(g, o, "energies first")
    # two resamplings in a row, then a sweep
    step()
    b = step()
    g.sweep(b, 2)
    o.sweep(2)
    _cmp_state(g, o, "back to back")
    # resample, zero sweeps, observables, then sweeps
    b = step()
    g.sweep(b, 0)
    o.sweep(0)
    _cmp_obs(g.observables(), o.observables())
    g.sweep(b, 2)
    o.sweep(2)
    _cmp_state(g, o, "zero sweeps")
    # resample, single replicas, overlap and histogram, then sweep
    b = step()
    slots = [0, g.R // 2, g.R - 1]
    s1, E1, M1 = g.replicas(slots)
    so, Eo, Mo = o.population()
    assert np.array_equal(s1, so[slots]) and np.array_equal(E1, Eo[slots])
    hg, st = g.histogram()
    assert np.array_equal(hg, o.histogram()[::st])
    assert g.overlap(0.05) == o.overlap(0.05)
    g.sweep(b, 1)
    o.sweep(1)
    _cmp_state(g, o, "replicas first")
    # resample, then a new population replaces the resampled one
    step()
    spins = o.population()[0][:300].copy()
    spins[:, 0, 0] *= -1
    g.set_population(spins)
    o.set_population(spins)
    _cmp_state(g, o, "replaced")
    b = step()
    g.sweep(b, 2)
    o.sweep(2)
    _cmp_state(g, o, "after replacement")
    g.close()
    o.close()


@pytest.mark.parametrize("layout,glass", [(0, False), (1, True)])
def test_deferred_population_size_matches_waiting_path(pa, layout, glass):
    """Resampling without waiting for the new size (the kernels read it on
    the device) against the waiting path and the oracle: same populations,
    sizes, ln Z, and the same timing totals."""
    L, R, theta = 16, 900, 3
    J = W.pmj_couplings(L, 21) if glass else None
    fast = pa.Population(L, R, seed=6, population_id=1, J=J, layout=layout)
    slow = pa.Population(L, R, seed=6, population_id=1, J=J, layout=layout)
    o = oracle.OraclePA(L, R, seed=6, pop=1, J=J)
    fast.set_timing(True)
    slow.set_timing(True)
    sizes = [R]
    for i, b in enumerate(W.linear_schedule(1.2, 12), start=1):
        assert fast.resample(b, wait=False) is None
        rs = slow.resample(b)
        ro = o.resample(b)
        assert rs == ro
        sizes.append(ro)
        fast.sweep(b, theta)
        slow.sweep(b, theta)
        o.sweep(theta)
        if i % 4 == 0:
            assert fast.R == ro               # synchronises
        oo = o.observables()
        _cmp_obs(fast.observables(), oo)
        _cmp_obs(slow.observables(), oo)
    _cmp_state(fast, o, "deferred")
    _cmp_state(slow, o, "waiting")
    tf, ts = fast.timing(), slow.timing()
    for k in ("sweep", "hist", "counts", "scatter"):
        print(k, "deferred", tf[k]["launches"], tf[k]["bytes"],
              "waiting", ts[k]["launches"], ts[k]["bytes"])
    print("sizes", sizes, "sum", sum(sizes))
    assert tf["attempts"] == ts["attempts"] == sum(sizes[1:]) * L * L * theta
    # one histogram per step and one before the first resampling
    assert tf["hist"]["launches"] == len(sizes)
    assert tf["hist"]["bytes"] == ts["hist"]["bytes"] == 8 * sum(sizes)
    for k in ("sweep", "hist", "counts", "scatter"):
        assert tf[k]["launches"] == ts[k]["launches"], k
        assert tf[k]["bytes"] == ts[k]["bytes"], k
    # a deferred resampling followed directly by reads of the population
    b = 1.3
    fast.resample(b, wait=False)
    o.resample(b)
    _cmp_state(fast, o, "deferred, read before the sweep")
    fast.close()
    slow.close()
    o.close()


@pytest.mark.parametrize("layout,glass,pending,law", [(0, False, False, 0),
                                                      (1, True, True, 0),
                                                      (0, True, False, 1)])
def test_save_and_load_resume_bit_for_bit(pa, tmp_path, layout, glass,
                                          pending, law):
    """A run saved halfway and continued from the file equals the
    uninterrupted run and the oracle, bit for bit (the saved state can sit
    between a resampling and its sweep)."""
    L, R, theta = 12, 700, 2
    J = W.pmj_couplings(L, 31) if glass else None
    betas = W.linear_schedule(1.1, 10)
    a = pa.Population(L, R, seed=9, population_id=4, J=J, layout=layout,
                      resampling=law)
    o = oracle.OraclePA(L, R, seed=9, pop=4, J=J, law=law)
    path = str(tmp_path / "half.pa")
    b = None
    for i, beta in enumerate(betas):
        a.resample(beta, wait=False)
        o.resample(beta)
        if b is not None:
            b.resample(beta, wait=False)
        if pending and i == 5:        # saved between resampling and sweep
            a.save(path)
            b = pa.Population.load(path)
        a.sweep(beta, theta)
        o.sweep(theta)
        if b is not None:
            b.sweep(beta, theta)
        if not pending and i == 4:    # saved after a complete step
            a.save(path)
            b = pa.Population.load(path)
    for g in (a, b):
        _cmp_state(g, o, "resumed")
        assert g.state() == (o.R, o.beta, o.step)
        _cmp_obs(g.observables(), o.observables())
    a.close()
    b.close()


@pytest.mark.parametrize("L,R,layout,glass", [(16, 1000, 0, False),
                                              (12, 700, 1, True)])
def test_poisson_resampling_matches_oracle(pa, L, R, layout, glass):
    """The Poisson law (Sec. 2): copy counts, populations, ln Z and
    observables after every step equal the oracle's."""
    J = W.pmj_couplings(L, 61) if glass else None
    _parity_run(pa, L, R, 40, 3, 1.2, seed=5, pop=2, J=J, layout=layout,
                law=oracle.POISSON)


def test_poisson_resampling_with_large_means(pa):
    """One resampling from beta = 0 straight to beta = 2: the lowest levels
    get means in the hundreds (long threshold lists), the rest almost none."""
    L, R = 16, 400
    g = pa.Population(L, R, seed=3, resampling=pa.PA_POISSON)
    o = oracle.OraclePA(L, R, seed=3, law=oracle.POISSON)
    R_old = g.R
    assert g.resample(2.0) == o.resample(2.0)
    n = g.counts()
    assert np.array_equal(n, o.counts(R_old))
    assert n.max() > 50
    g.sweep(2.0, 2)
    o.sweep(2)
    _cmp_state(g, o, "large means")
    g.close()
    o.close()


@pytest.mark.parametrize("L,R,layout,law", [(16, 800, 0, 0), (12, 600, 1, 1)])
def test_heating_matches_oracle(pa, L, R, layout, law):
    """Heating protocol (Sec. 2): ground states at beta0 = 2.5, then beta
    down to 0.2; every step bit-exact with the oracle."""
    beta0, beta_f, K, theta = 2.5, 0.2, 30, 3
    g = pa.Population(L, R, seed=12, population_id=1, layout=layout,
                      resampling=law)
    o = oracle.OraclePA(L, R, seed=12, pop=1, law=law)
    g.start_heating(beta0)
    o.start_heating(beta0)
    _cmp_state(g, o, "ground states")
    for i in range(1, K + 1):
        b = beta0 + ((beta_f - beta0) * i) / K
        R_old = g.R
        assert g.resample(b) == o.resample(b)
        assert np.array_equal(g.counts(), o.counts(R_old)), i
        g.sweep(b, theta)
        o.sweep(theta)
        _cmp_state(g, o, "heating step %d" % i)
        _cmp_obs(g.observables(), o.observables())
    with pytest.raises(pa.PAError):
        g.start_heating(1.0)                  # only before any resampling
    g.close()
    o.close()


@pytest.mark.parametrize("L,R,q,beta_f,law", [(16, 600, 3, 1.2, 0),
                                               (12, 500, 10, 1.8, 1),
                                               (6, 300, 16, 2.0, 0),
                                               (32, 150, 7, 1.5, 0),
                                               (8, 700, 2, 0.9, 1),
                                               (128, 40, 4, 1.1, 0)])
def test_potts_matches_oracle(pa, L, R, q, beta_f, law):
    """q-state Potts populations (Sec. 2 names the model): every step
    bit-exact with the oracle, including q = 10 across its first-order
    transition and the largest lattice.  L = 8, 16, 32, 128 take the
    four-sites-per-word pass, L = 6 and 12 the generic one."""
    _parity_run(pa, L, R, 30, 3, beta_f, seed=8, pop=5, law=law, q=q)


def test_potts_heating_and_resume(pa, tmp_path):
    """Potts heating from ground states, saved and resumed halfway."""
    L, R, q, beta0, beta_f, K = 10, 400, 10, 3.0, 0.8, 20
    g = pa.Population(L, R, seed=21, q=q)
    o = oracle.OraclePA(L, R, seed=21, q=q)
    g.start_heating(beta0)
    o.start_heating(beta0)
    _cmp_state(g, o, "potts ground states")
    path = str(tmp_path / "potts.pa")
    for i in range(1, K + 1):
        b = beta0 + ((beta_f - beta0) * i) / K
        g.resample(b, wait=False)
        o.resample(b)
        g.sweep(b, 2)
        o.sweep(2)
        if i == K // 2:
            g.save(path)
            g.close()
            g = pa.Population.load(path)
        _cmp_state(g, o, "potts heating step %d" % i)
    _cmp_obs(g.observables(), o.observables())
    g.close()
    o.close()


@pytest.mark.parametrize("L,R,layout,glass,q,law", [
    (16, 1000, 0, False, 0, 2), (12, 700, 1, True, 0, 2),
    (8, 500, 0, False, 5, 2), (16, 900, 0, False, 0, 3),
    (12, 600, 1, True, 0, 3), (16, 800, 0, False, 0, 4),
    (10, 500, 1, True, 0, 4)])
def test_systematic_resampling_matches_oracle(pa, L, R, layout, glass, q,
                                              law):
    """Systematic, residual and multinomial resampling: copy counts,
    populations and ln Z equal the oracle's at every step; the size stays
    within one of the target (exactly the target for the residual and
    multinomial laws)."""
    J = W.pmj_couplings(L, 71) if glass else None
    _parity_run(pa, L, R, 30, 3, 1.2, seed=6, pop=3, J=J, layout=layout,
                law=law, q=q)
    g = pa.Population(L, R, seed=6, J=J, layout=layout, q=q,
                      resampling=law)
    for b in W.linear_schedule(1.2, 10):
        Rn = g.resample(b)
        assert (Rn == R) if law in (3, 4) else (R - 1 <= Rn <= R)
        g.sweep(b, 1)
    g.close()


def test_empty_resampling_leaves_population_untouched(pa):
    """Three replicas with a target of one: each keeps a copy with
    probability about 1/3, so some seeds draw no copy at all.  Both sides
    report PA_EEMPTY, and nothing changes."""
    L = 4
    rng = np.random.default_rng(0)
    spins = np.where(rng.random((3, L, L)) < 0.5, 1, -1).astype(np.int8)
    for seed in range(1, 60):
        g = pa.Population(L, 1, seed=seed, capacity=8)
        o = oracle.OraclePA(L, 1, seed=seed, capacity=8)
        g.set_population(spins)
        o.set_population(spins)
        rc, Rn = g.resample_rc(0.1)
        assert (rc, Rn) == o.resample_rc(0.1)
        if rc == pa.PA_OK:
            g.close()
            continue
        assert rc == pa.PA_EEMPTY and Rn == 0
        assert g.state() == (3, 0.0, 0)
        s, E, M = g.population()
        assert np.array_equal(s, spins)
        assert g.free_energy() == o.free_energy()
        g.close()
        return
    raise AssertionError("no seed drew an empty population")


def test_impossible_population_reports_enomem(pa):
    """A population whose buffers cannot fit in device memory (2^31 - 1
    replicas of 16 KB, twice) is refused with PA_ENOMEM and no context;
    what was allocated is released, and a normal context works after it."""
    import ctypes as C
    lib = pa.lib()
    cfg = pa.pa_config()
    cfg.L, cfg.R_target, cfg.model = 128, (1 << 31) - 1, pa.PA_FERRO
    cfg.rows_per_lane = 2
    h = C.c_void_p()
    assert lib.pa_init(C.byref(cfg), C.byref(h)) == pa.PA_ENOMEM
    assert not h.value
    g = pa.Population(16, 200, seed=2)
    o = oracle.OraclePA(16, 200, seed=2)
    g.resample(0.3)
    o.resample(0.3)
    _cmp_state(g, o, "after ENOMEM")
    g.close()
    o.close()


def _hip_runtime():
    """The HIP runtime the library already loaded (no second copy)."""
    import ctypes
    for name in ("libamdhip64.so.7", "libamdhip64.so.6", "libamdhip64.so"):
        try:
            return ctypes.CDLL(name, mode=os.RTLD_NOLOAD)
        except OSError:
            continue
    pytest.skip("the library's HIP runtime is not visible to ctypes")


def test_results_do_not_depend_on_the_stream(pa):
    """The same run on the null stream and on a stream of its own (default
    priority, made by the library's HIP runtime) and, for a batch, on its
    private stream and on that stream: identical populations, ln Z and
    families."""
    import ctypes
    pa.lib()
    hip = _hip_runtime()
    side = ctypes.c_void_p()
    assert hip.hipStreamCreate(ctypes.byref(side)) == 0
    runs = []
    for st in (None, side.value):
        g = pa.Population(24, 700, seed=12, layout=1, stream=st,
                          J=W.pmj_couplings(24, 5))
        for b in W.linear_schedule(1.1, 9):
            g.resample(b, wait=False)
            g.sweep(b, 3)
        runs.append((g.population(), g.free_energy(), g.families()[0]))
        g.close()
    (s0, z0, f0), (s1, z1, f1) = runs
    assert all(np.array_equal(a, b) for a, b in zip(s0, s1))
    assert z0 == z1 and np.array_equal(f0, f1)
    pops = [dict(L=16, R=400, seed=3, population_id=0),
            dict(L=32, R=300, q=7, seed=4, population_id=1)]
    betas = np.array(W.linear_schedule(1.0, 6))
    out = []
    for st in (None, side.value):
        b = pa.Batch(pops, stream=st)
        b.run(betas, 2, use_graph=True)
        out.append([(b.population(p), b.state(p)[3]) for p in range(2)])
        b.close()
    for (pa_, za), (pb, zb) in zip(out[0], out[1]):
        assert all(np.array_equal(a, b) for a, b in zip(pa_, pb))
        assert za == zb
    assert hip.hipStreamSynchronize(side) == 0
    assert hip.hipStreamDestroy(side) == 0


@pytest.mark.parametrize("law", [1, 2, 3, 4])
def test_full_size_every_law(pa, law):
    """The 64 x 64, 65536-replica workload under the Poisson, systematic,
    residual and multinomial laws, in the benchmark's launch configuration
    (no wait for the new size, copies made by the sweep): every copy count,
    the new size and ln Q exactly from the oracle's count step on the device
    energies; a sample of new replicas through their sweeps."""
    c = W.CONFIGS["C2"]
    L, R, theta = c["L"], c["R"], c["theta"]
    print("full-size law %d" % law, flush=True)
    g = pa.Population(L, R, seed=c["seed"], resampling=law,
                      capacity=W.deferral_capacity(R))
    rng = np.random.default_rng(law)
    sched = W.linear_schedule(c["beta_f"], c["K"])
    zlast = g.free_energy()[0]
    for i in (1, 2):
        b = sched[i - 1]
        E, M = g.energies()
        n_o, Rn_o, lnQ_o = oracle.counts(L * L, E, R, b - g.beta, c["seed"],
                                         0, i, law=law)
        parent = np.repeat(np.arange(len(E)), n_o)
        slots = np.sort(rng.choice(Rn_o, size=16, replace=False))
        s_pre, E_pre, M_pre = g.replicas(parent[slots])
        g.resample(b, wait=False)
        g.sweep(b, theta)
        assert g.state()[0] == Rn_o
        assert np.array_equal(g.counts(), n_o)
        z, dq = g.free_energy()
        assert _close(dq, lnQ_o) and _close(z, zlast + lnQ_o)
        zlast = z
        s_post, E_post, M_post = g.replicas(slots)
        for k, j in enumerate(slots):
            so, eo, mo = oracle.sweep_replica(s_pre[k], E_pre[k], M_pre[k], b,
                                              c["seed"], 0, i, 0, theta,
                                              int(j))
            assert np.array_equal(s_post[k], so), (law, i, j)
            assert (E_post[k], M_post[k]) == (eo, mo)
    g.close()
