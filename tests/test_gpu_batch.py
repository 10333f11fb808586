"""Batched populations: every population of a batch must be bit for bit the
oracle's run of the same configuration (spins, energies, ln Z, observables
after every step); the graph-captured step must reproduce the eager one on
every replay; the batch must equal the single-population path; the
adaptive schedule must make the oracle's bisection choices."""
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


MIXED = [  # L, R, glass, layout
    (4, 50, False, 0), (6, 300, True, 0), (8, 257, True, 0),
    (12, 513, True, 0), (16, 700, False, 1), (24, 333, True, 0),
    (32, 300, False, 0), (64, 70, True, 0), (128, 20, False, 1),
]


def _mixed_pops():
    pops = []
    for k, (L, R, glass, layout) in enumerate(MIXED):
        pops.append(dict(L=L, R=R, J=W.pmj_couplings(L, 50 + k) if glass
                         else None, seed=7, population_id=k, layout=layout))
    return pops


def _oracle_run(pop, betas, theta):
    o = oracle.OraclePA(pop["L"], pop["R"], seed=pop["seed"],
                        pop=pop["population_id"], J=pop["J"],
                        rng_mode=pop.get("rng_mode", 0))
    traj = []
    for b in betas:
        o.resample(b)
        o.sweep(theta)
        traj.append((o.observables(), o.free_energy()[0]))
    return o, traj


def _check_pop(batch, p, o, traj_o):
    s, E, M = batch.population(p)
    so, Eo, Mo = o.population()
    assert np.array_equal(E, Eo) and np.array_equal(M, Mo), p
    assert np.array_equal(s, so), p
    R, beta, step, lnZ = batch.state(p)
    assert R == o.R and beta == o.beta and step == o.step
    assert _close(lnZ, o.free_energy()[0])
    obs, lnZs = batch.trajectory(p)
    assert len(obs) == len(traj_o)
    for (og, zg), (oo, zo) in zip(zip(obs, lnZs), traj_o):
        for k in ("R", "sumE", "sumE2", "sumAbsM", "sumM2", "Emin", "Emax"):
            assert og[k] == oo[k], (p, k)
        for k in ("beta", "e", "abs_m", "m2", "C"):
            assert _close(og[k], oo[k]), (p, k)
        assert _close(zg, zo)


@pytest.mark.parametrize("use_graph", [False, True])
def test_mixed_batch_matches_oracle(pa, use_graph):
    pops = _mixed_pops()
    betas = W.linear_schedule(1.2, 6)
    theta = 3
    print("batch parity graph=%s" % use_graph, flush=True)
    b = pa.Batch(pops)
    b.run(np.array(betas), theta, use_graph=use_graph)
    for p, pop in enumerate(pops):
        o, traj = _oracle_run(pop, betas, theta)
        _check_pop(b, p, o, traj)
    b.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_plane_stream_batch_matches_oracle(pa, use_graph):
    """Populations in the bit-plane random-number stream beside populations
    in the word stream, in one batch (both persistent sweep classes in one
    step): every population equals the oracle's run in its own stream."""
    pops = _mixed_pops()
    for k, p in enumerate(pops):
        p["rng_mode"] = pa.PA_RNG_PLANES if k % 3 != 1 else pa.PA_RNG_WORD
    betas = W.linear_schedule(1.4, 6)
    theta = 3
    print("plane-stream batch parity graph=%s" % use_graph, flush=True)
    b = pa.Batch(pops, autotune=use_graph)
    b.run(np.array(betas), theta, use_graph=use_graph)
    for p, pop in enumerate(pops):
        o, traj = _oracle_run(pop, betas, theta)
        _check_pop(b, p, o, traj)
    b.close()


def test_two_replicas_per_wave_int8_batch_matches_oracle(pa):
    """int8 L = 64 populations at two rows per lane in the persistent sweep
    (two replicas per wave moved as whole kilobytes), an odd R leaving the
    last wave one replica, in both random-number streams and with +-J
    bonds: every population equals the oracle's run."""
    pops = []
    for k, (R, glass, rng) in enumerate([(129, False, 1), (67, True, 1),
                                         (131, True, 0), (64, False, 0)]):
        pops.append(dict(L=64, R=R, J=W.pmj_couplings(64, 70 + k) if glass
                         else None, seed=9, population_id=k, layout=0,
                         rows_per_lane=2, rng_mode=rng))
    betas = W.linear_schedule(1.0, 5)
    theta = 2
    b = pa.Batch(pops)
    b.run(np.array(betas), theta, use_graph=True)
    for p, pop in enumerate(pops):
        o, traj = _oracle_run(pop, betas, theta)
        _check_pop(b, p, o, traj)
    b.close()


def test_graph_replays_match_eager_across_runs(pa):
    """Two graph runs of 4 steps each, with host reads in between, against
    one eager run of 8 steps: identical populations and ln Z."""
    pops = _mixed_pops()
    betas = np.array(W.linear_schedule(1.6, 8))
    g = pa.Batch(pops)
    e = pa.Batch(pops)
    g.run(betas[:4], 2, use_graph=True)
    mid = [g.state(p) for p in range(len(pops))]
    g.run(betas[4:], 2, use_graph=True)
    e.run(betas[:4], 2, use_graph=False)
    assert [e.state(p) for p in range(len(pops))] == mid
    e.run(betas[4:], 2, use_graph=False)
    for p in range(len(pops)):
        assert g.state(p) == e.state(p)
        for a, c in zip(g.population(p), e.population(p)):
            assert np.array_equal(a, c)


def test_batch_equals_single_population_path(pa):
    """The batched glass workload (64 instances, L in {8..32}, R up to 2^16),
    first 12 steps of its schedule, against each instance run alone through
    pa_init / pa_resample / pa_sweep: populations, ln Z and families."""
    inst = W.batched_glass_instances()
    betas = np.array(W.linear_schedule(3.0, 300)[:12])
    theta = 10
    b = pa.Batch(inst, autotune=True)
    b.run(betas, theta, use_graph=True)
    for p, c in enumerate(inst):
        g = pa.Population(c["L"], c["R"], seed=c["seed"],
                          population_id=c["population_id"], J=c["J"])
        for beta in betas:
            g.resample(beta)
            g.sweep(beta, theta)
        sg, Eg, Mg = g.population()
        sb, Eb, Mb = b.population(p)
        assert np.array_equal(Eg, Eb) and np.array_equal(sg, sb), p
        assert g.free_energy()[0] == b.state(p)[3]
        fg, n0g = g.families()
        fb, n0b = b.families(p)
        assert n0g == n0b and np.array_equal(fg, fb), p
        g.close()
    b.close()


def test_adaptive_schedule_matches_oracle_bisection(pa):
    pops = [dict(L=L, R=R, J=W.pmj_couplings(L, 90 + k) if k % 2 else None,
                 seed=3, population_id=k)
            for k, (L, R) in enumerate([(8, 400), (12, 300), (16, 500),
                                        (24, 200)])]
    target, beta_f, theta = 0.85, 2.0, 2
    b = pa.Batch(pops)
    steps = b.run_adaptive(target, beta_f, 200, theta, use_graph=True)
    assert steps < 200
    for p, pop in enumerate(pops):
        o = oracle.OraclePA(pop["L"], pop["R"], seed=3, pop=p, J=pop["J"])
        traj = []
        while o.beta < beta_f:
            span = beta_f - o.beta
            d = o.bisect_dbeta(target, beta_f)
            nb = beta_f if d == span else o.beta + d
            if not nb > o.beta:
                nb = beta_f
            if d < span:
                # the bisection step honours the overlap target
                assert o.overlap(d) >= target
            o.resample(nb)
            o.sweep(theta)
            traj.append((o.observables(), o.free_energy()[0]))
        _check_pop(b, p, o, traj)
    b.close()


def test_autotuner_reports_valid_shapes(pa):
    for L, valid in ((16, (1, 2, 4)), (24, (1, 2, 3, 4)), (64, (1, 2, 4)),
                     (96, (2, 3, 4)), (128, (2, 4))):
        best, ms = pa.tune_rows_per_lane(L, R=2048, theta=2)
        assert best in valid
        for rpl, t in zip((1, 2, 3, 4), ms):
            assert (t > 0) == (rpl in valid)


def test_sweep_launch_shape_does_not_change_results(pa):
    """Workgroups and work items per queue atomic of the persistent sweep
    change only the schedule, never a bit of the populations."""
    pops = _mixed_pops()
    betas = np.array(W.linear_schedule(1.2, 5))
    ref = pa.Batch(pops)
    ref.run(betas, 3)
    for blocks, chunk in ((1, 1), (37, 3), (4096, 16)):
        b = pa.Batch(pops)
        b.set_sweep_blocks(blocks, chunk)
        b.run(betas, 3)
        for p in range(len(pops)):
            assert b.state(p) == ref.state(p), (blocks, chunk, p)
            for x, y in zip(b.population(p), ref.population(p)):
                assert np.array_equal(x, y), (blocks, chunk, p)
        b.close()
    ref.close()


def test_weighted_average_of_independent_populations_is_exact(pa):
    """Many independent ferromagnet populations combined by weighted
    averaging: the energy per spin and ln Z at beta_f agree with the exact
    finite-torus results within the statistical error."""
    import exact_ising
    L, R, M, beta_f = 16, 400, 48, 0.6
    pops = [dict(L=L, R=R, seed=500 + m, population_id=m) for m in range(M)]
    b = pa.Batch(pops)
    b.run(np.array(W.linear_schedule(beta_f, 60)), 4)
    lnZ = np.array([b.state(p)[3] for p in range(M)])
    obs = [b.trajectory(p)[0][-1] for p in range(M)]
    assert all(o["beta"] == beta_f for o in obs)
    comb = pa.combine_observables(lnZ, obs, L * L)
    e = np.array([o["e"] for o in obs])
    e_exact = float(exact_ising.kaufman_energy(L, beta_f))  # per spin
    z_exact = float(exact_ising.kaufman_lnZ(L, beta_f))
    assert abs(comb["e"] - e_exact) < 5 * e.std(ddof=1) / np.sqrt(M) + 1e-4
    assert abs(comb["lnZ"] - z_exact) < 5 * lnZ.std(ddof=1) / np.sqrt(M) + 0.05
    b.close()


def test_potts_populations_in_a_batch_equal_their_single_runs(pa):
    """q-state Potts populations of every four-sites-per-word size, batched
    with a ferromagnet and a +-J glass: every population's states, E, M,
    ln Z and families equal its run alone through the single-population
    path, for a linear schedule through the q = 10 transition region and
    for the adaptive schedule (to beta = 0.9, below the Potts transitions,
    where overlap-targeted steps stay few)."""
    pops = [dict(L=8, R=700, q=3, seed=5, population_id=0),
            dict(L=16, R=900, q=10, seed=5, population_id=1),
            dict(L=32, R=300, q=16, seed=6, population_id=2),
            dict(L=64, R=200, q=10, seed=7, population_id=3),
            dict(L=128, R=40, q=4, seed=8, population_id=4),
            dict(L=16, R=500, seed=9, population_id=5),
            dict(L=24, R=400, J=W.pmj_couplings(24, 77), seed=9,
                 population_id=6)]
    betas = np.array(W.linear_schedule(1.6, 14))
    theta = 3
    for adaptive in (False, True):
        b = pa.Batch(pops)
        if adaptive:
            steps = b.run_adaptive(0.8, 0.9, 2000, theta, use_graph=True)
            assert steps < 2000
        else:
            b.run(betas, theta, use_graph=True)
        for p, c in enumerate(pops):
            g = pa.Population(c["L"], c["R"], seed=c["seed"],
                              population_id=c["population_id"], J=c.get("J"),
                              q=c.get("q", 0))
            if adaptive:
                traj, _ = b.trajectory(p)
                sched = [o["beta"] for o in traj]
            else:
                sched = betas
            for beta in sched:
                g.resample(beta)
                g.sweep(beta, theta)
            sg, Eg, Mg = g.population()
            sb, Eb, Mb = b.population(p)
            tag = (adaptive, p)
            assert np.array_equal(Eg, Eb) and np.array_equal(Mg, Mb), tag
            assert np.array_equal(sg, sb), tag
            assert g.free_energy()[0] == b.state(p)[3], tag
            fg, _ = g.families()
            fb, _ = b.families(p)
            assert np.array_equal(fg, fb), tag
            g.close()
        b.close()


def test_batch_refuses_theta_beyond_the_counter(pa):
    """theta above 32767 would overflow the 16 half-sweep bits of the
    random counter: the run is refused, and the batch still runs."""
    b = pa.Batch([dict(L=8, R=100, seed=1, population_id=0)])
    with pytest.raises(pa.PAError) as e:
        b.run(np.array([0.1]), 40000)
    assert e.value.code == pa.PA_EINVAL
    b.run(np.array([0.1, 0.2]), 2)
    assert b.state(0)[2] == 2
    b.close()


def test_rows_per_lane_tuner_keeps_results(pa):
    """PA_BATCH_AUTOTUNE times rows per lane with the batch's own sweep on
    scratch batches; the tuned batch equals the untuned one (default rows
    per lane) bit for bit, and a population that sets its rows per lane
    keeps it."""
    pops = _mixed_pops()
    pops[0] = dict(pops[0], rows_per_lane=2)  # L = 4: two lanes per replica
    betas = np.array(W.linear_schedule(1.0, 4))
    t = pa.Batch(pops, autotune=True)
    d = pa.Batch(pops)
    t.run(betas, 3)
    d.run(betas, 3)
    for p in range(len(pops)):
        assert t.state(p) == d.state(p), p
        for a, b in zip(t.population(p), d.population(p)):
            assert np.array_equal(a, b), p
    t.close()
    d.close()


def test_sweep_shape_tuner_keeps_results(pa):
    """PA_BATCH_TUNE_SWEEP times the persistent sweep's launch shapes on a
    scratch batch; the tuned batch's results equal the default batch's bit
    for bit, and the chosen shape is one of the candidates."""
    pops = _mixed_pops()
    betas = np.array(W.linear_schedule(1.0, 4))
    t = pa.Batch(pops, autotune=True, tune_sweep=True)
    d = pa.Batch(pops, autotune=True)
    assert t.sweep_blocks() in [(1024, 4), (512, 4), (2048, 4), (1024, 8),
                                (2048, 8), (1024, 2)]
    assert d.sweep_blocks() == (1024, 4)
    t.run(betas, 3)
    d.run(betas, 3)
    for p in range(len(pops)):
        assert t.state(p) == d.state(p)
        for a, b in zip(t.population(p), d.population(p)):
            assert np.array_equal(a, b)
    t.close()
    # every candidate shape, and a ragged one, gives the same populations
    for blocks, chunk in [(512, 4), (2048, 4), (1024, 8), (2048, 8),
                          (1024, 2), (37, 3)]:
        c = pa.Batch(pops, autotune=True)
        c.set_sweep_blocks(blocks, chunk)
        assert c.sweep_blocks() == (blocks, chunk)
        c.run(betas, 3)
        for p in range(len(pops)):
            assert c.state(p) == d.state(p), (blocks, chunk, p)
            for a, b in zip(c.population(p), d.population(p)):
                assert np.array_equal(a, b), (blocks, chunk, p)
        c.close()
    d.close()
