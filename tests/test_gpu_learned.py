"""The temperature-step network: FP32 kernels against the FP64 reference,
training on the GPU, and the learned schedule against the oracle (schedule
replay parity and the overlap criterion), with its gain over the exact
bisection measured in exact overlap evaluations."""
import os

import numpy as np
import pytest

import oracle
import pa_workloads as W
from oracle import mlp_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pa():
    if not os.path.exists("/dev/kfd"):
        pytest.skip("no GPU")
    from paper_2006_00561_amd import binding
    binding.lib()
    return binding


def test_gradients_match_fp64_reference(pa):
    rng = np.random.default_rng(3)
    mlp = pa.MLP(8, 64, 3, seed=5)
    p = mlp.params().astype(np.float64)
    X = rng.normal(0, 1.2, (96, 8)).astype(np.float32)
    T = rng.normal(-5, 1.0, 96).astype(np.float32)
    mu = rng.normal(0, 0.5, 8).astype(np.float32)
    sd = rng.uniform(0.5, 2.0, 8).astype(np.float32)
    mlp.set_norm(mu, sd, -5.0, 1.5)
    loss, g = mlp.loss_grad(X, T)
    lref, gref = mlp_ref.loss_and_grad(p, X.astype(np.float64),
                                       T.astype(np.float64), 8, 64, 3, mu, sd,
                                       -5.0, 1.5)
    assert abs(loss - lref) <= 1e-4 * max(1.0, lref)
    scale = np.abs(gref).max()
    assert np.max(np.abs(g - gref)) <= 1e-4 * scale
    y = mlp.forward(X)
    z, _ = mlp_ref.forward(p, X.astype(np.float64), 8, 64, 3, mu, sd)
    assert np.max(np.abs(y - (-5.0 + 1.5 * z))) <= 1e-4 * 5


def test_training_fits_a_smooth_target(pa):
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, (4096, 8)).astype(np.float32)
    T = (np.sin(2 * X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] - 4.0).astype(np.float32)
    mlp = pa.MLP(8, 64, 3, seed=9)
    mlp.set_norm(np.zeros(8), np.ones(8), -4.0, 1.0)
    l0, _ = mlp.loss_grad(X[:512], T[:512])
    mlp.train(X, T, batch=256, iters=1500, lr=2e-3, seed=3)
    l1, _ = mlp.loss_grad(X[:512], T[:512])
    assert l1 < 0.05 * l0


def _ferro_pops(specs, seed0, id0=0):
    return [dict(L=L, R=R, seed=seed0 + k, population_id=id0 + k)
            for k, (L, R) in enumerate(specs)]


def test_learned_schedule_replays_on_the_oracle_and_saves_bisections(pa):
    from paper_2006_00561_amd import learned
    # training data: exact schedules of small ferromagnets and glasses whose
    # sizes and population sizes bracket the held-out ones
    train_pops = _ferro_pops([(8, 600), (12, 2000), (16, 1000), (16, 500),
                              (24, 1500), (24, 700), (12, 900)], 100)
    train_pops += [dict(L=L, R=R, J=W.pmj_couplings(L, 300 + k), seed=5,
                        population_id=10 + k)
                   for k, (L, R) in enumerate([(8, 1200), (12, 600),
                                               (16, 1600)])]
    X, T = learned.generate(train_pops, [0.8, 0.85, 0.9], 1.5, 2)
    assert len(X) > 500
    mlp, loss = learned.train(X, T, iters=4000, lr=2e-3, seed=11)
    fit = np.sqrt(np.mean((mlp.forward(X) - T) ** 2))
    print("pairs %d  loss %.4f  rms log-dbeta error %.4f" % (len(X), loss, fit))
    assert fit < 0.2
    # held-out populations
    test_pops = _ferro_pops([(12, 800), (16, 1200), (20, 800)], 500)
    target, tol, beta_f, theta = 0.85, 0.02, 1.5, 2
    b = pa.Batch(test_pops)
    steps, src = b.run_learned(mlp, target, tol, beta_f, 1000, theta)
    stats = b.host_stats()
    # the proposal inside the run is the network on the device summaries
    for p in range(len(test_pops)):
        f, db, srcs, prop = b.decisions(p, with_proposals=True)
        net = srcs != learned.SRC_REST
        assert np.allclose(prop[net], mlp.forward(f[net]), atol=1e-4)
    print("sources", list(src), "overlap evals", stats["overlap_evals"])
    assert src[2] > 0.6 * (src[2] + src[3])           # mostly accepted
    ref = pa.Batch(test_pops)
    ref.run_adaptive(target, beta_f, 1000, theta)
    ref_stats = ref.host_stats()
    assert stats["overlap_evals"] < 0.3 * ref_stats["overlap_evals"]
    # the learned schedule replayed on the oracle: same populations, and
    # every accepted proposal meets the overlap criterion exactly
    for p, pop in enumerate(test_pops):
        obs, lnZ = b.trajectory(p)
        f, db, srcs = b.decisions(p)
        o = oracle.OraclePA(pop["L"], pop["R"], seed=pop["seed"],
                            pop=pop["population_id"])
        for k, ob in enumerate(obs):
            if srcs[k] == 2:
                a = o.overlap(ob["beta"] - o.beta)
                assert abs(a - target) <= tol + 1e-12
            o.resample(ob["beta"])
            o.sweep(theta)
            assert o.free_energy()[0] == lnZ[k]
        s, E, M = b.population(p)
        so, Eo, Mo = o.population()
        assert np.array_equal(s, so) and np.array_equal(E, Eo)
        assert o.beta == beta_f


def test_device_summaries_match_numpy(pa):
    """The 8 histogram summaries the device computes before a step, against
    numpy on the population's energies."""
    pops = [dict(L=L, R=R, J=W.pmj_couplings(L, 7) if g else None, seed=2,
                 population_id=k)
            for k, (L, R, g) in enumerate([(16, 700, False), (12, 500, True),
                                           (32, 300, False)])]
    b = pa.Batch(pops)
    b.run(np.array([[0.3, 0.3, 0.3]]), 2)       # move away from beta = 0
    E = [b.population(p)[1].astype(np.float64) for p in range(3)]
    b.run_adaptive(0.85, 1.0, 1, 2)              # one decision per population
    for p, pop in enumerate(pops):
        f, db, src = b.decisions(p)
        e = E[p]
        N = pop["L"] ** 2
        mean, var = e.mean(), e.var()
        sd = np.sqrt(max(var, 1e-3))
        want = [mean / N, np.log(sd), ((e - mean) ** 3).mean() / var ** 1.5,
                (e.min() - mean) / sd, 0.3, np.log(N), np.log(len(e)), 0.85]
        assert np.allclose(f[0], want, rtol=1e-5, atol=1e-5), (p, f[0], want)


def test_graph_follows_network_scratch_and_scale_changes(pa):
    """A batch whose graph captured the network's inference, then the
    network's scratch regrown (a larger forward batch) and its output scale
    changed: the next graph run must use the new scratch and scale."""
    pops = _ferro_pops([(8, 300), (12, 200), (16, 250)], 40)
    mlp = pa.MLP(8, 32, 2, seed=3)
    mu = np.array([-1, 3, 0, -2, 0.5, 5, 6, 0.85], np.float32)
    mlp.set_norm(mu, np.ones(8, np.float32), -4.0, 1.0)
    b = pa.Batch(pops)
    for k in range(2):
        b.run_learned(mlp, 0.85, 0.02, 1.5, 3, 2, use_graph=True)
        for p in range(len(pops)):
            f, db, srcs, prop = b.decisions(p, with_proposals=True)
            assert len(f) == 3
            assert np.allclose(prop, mlp.forward(f), atol=1e-4), (k, p)
        big = np.random.default_rng(k).normal(0, 1, (4096, 8))
        mlp.forward(big.astype(np.float32))              # regrows scratch
        mlp.set_norm(mu, np.ones(8, np.float32), -3.0 - k, 0.5)


@pytest.mark.parametrize("corruption", ["huge", "nan"])
def test_corrupted_network_falls_back_to_the_exact_schedule(pa, corruption):
    """A network whose weights are wrecked (a huge constant, or NaN)
    proposes steps that never meet the overlap criterion: every step falls
    back to the exact bisection, so the learned run's schedule and
    populations equal those of the pure bisection run bit for bit."""
    from paper_2006_00561_amd import learned
    pops = _ferro_pops([(12, 600), (16, 400)], 40)
    target, tol, beta_f, theta = 0.85, 0.02, 1.0, 2
    mlp = pa.MLP(seed=3)
    p = mlp.params()
    p[:] = 1e6 if corruption == "huge" else np.nan
    mlp.set_params(p)
    b = pa.Batch(pops)
    steps, src = b.run_learned(mlp, target, tol, beta_f, 1000, theta)
    assert src[learned.SRC_NET] == 0
    assert src[learned.SRC_FALLBACK] > 0
    ref = pa.Batch(pops)
    ref.run_adaptive(target, beta_f, 1000, theta)
    for k in range(len(pops)):
        obs, lnZ = b.trajectory(k)
        obs_r, lnZ_r = ref.trajectory(k)
        assert [o["beta"] for o in obs] == [o["beta"] for o in obs_r], k
        assert np.array_equal(lnZ, lnZ_r), k
        s, E, M = b.population(k)
        sr, Er, Mr = ref.population(k)
        assert np.array_equal(s, sr) and np.array_equal(E, Er), k
    b.close()
    ref.close()
    mlp.close()


def _replay_on_oracle(b, pops, theta, target, tol, n_steps=None):
    """Replays each population's schedule of the batch on the oracle: equal
    ln Z after every replayed step and equal populations at the end; every
    step that came from a bisection or the network meets the overlap test
    exactly.  n_steps limits the replay to the first steps."""
    from paper_2006_00561_amd import learned
    for p, pop in enumerate(pops):
        obs, lnZ = b.trajectory(p)
        f, db, srcs = b.decisions(p)
        o = oracle.OraclePA(pop["L"], pop["R"], seed=pop["seed"],
                            pop=pop["population_id"])
        last = len(obs) if n_steps is None else min(n_steps, len(obs))
        for k in range(last):
            beta = obs[k]["beta"]
            if srcs[k] in (learned.SRC_NET, learned.SRC_BISECT):
                a = o.overlap(beta - o.beta)
                assert abs(a - target) <= tol + 1e-12, (p, k, a)
            o.resample(beta)
            o.sweep(theta)
            assert o.free_energy()[0] == lnZ[k], (p, k)
        if last == len(obs):
            s, E, M = b.population(p)
            so, Eo, Mo = o.population()
            assert np.array_equal(s, so) and np.array_equal(E, Eo)
        o.close()


def test_tolerance_bisection_meets_the_network_test_and_replays(pa):
    """The bisection stopped at the first step within tol of the target
    (the baseline of the learned schedule): every bisection step passes the
    network's acceptance test on the oracle, the run replays bit for bit,
    and it needs fewer exact overlap evaluations than the 64 halvings."""
    pops = _ferro_pops([(12, 700), (16, 500), (20, 400)], 800, id0=50)
    target, tol, beta_f, theta = 0.85, 0.02, 1.2, 2
    b = pa.Batch(pops)
    b.run_adaptive(target, beta_f, 1000, theta, tol=tol)
    ev_tol = b.host_stats()["overlap_evals"]
    _replay_on_oracle(b, pops, theta, target, tol)
    ref = pa.Batch(pops)
    ref.run_adaptive(target, beta_f, 1000, theta)
    ev_exact = ref.host_stats()["overlap_evals"]
    print("overlap evaluations: tol-stopped %d, exact %d" % (ev_tol, ev_exact))
    assert ev_tol < 0.5 * ev_exact
    b.close()
    ref.close()


def test_learned_schedule_at_L64_replays_on_the_oracle(pa):
    """A network trained on exact schedules of L = 32..64 ferromagnets runs
    an L = 64 population (the benchmark's lattice): the first steps of its
    schedule, replayed on the oracle, give the same ln Z, and each accepted
    proposal meets the overlap test exactly."""
    from paper_2006_00561_amd import learned
    train = _ferro_pops([(32, 1500), (48, 1000), (64, 800), (64, 1600)],
                        900, id0=60)
    target, tol, beta_f, theta = 0.85, 0.02, 1.0, 10
    X, T = learned.generate(train, [0.8, 0.85, 0.9], beta_f, theta)
    mlp, loss = learned.train(X, T, iters=3000, lr=2e-3, seed=21)
    pops = _ferro_pops([(64, 300)], 990, id0=70)
    b = pa.Batch(pops)
    steps, src = b.run_learned(mlp, target, tol, beta_f, 1000, theta)
    print("L=64 learned schedule: %d steps, sources %s" % (steps, list(src)))
    assert src[learned.SRC_NET] > 0
    _replay_on_oracle(b, pops, theta, target, tol, n_steps=6)
    mlp.close()
    b.close()
