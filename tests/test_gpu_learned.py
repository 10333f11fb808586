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


def _ferro_pops(Ls, R, seed0):
    return [dict(L=L, R=R, seed=seed0 + k, population_id=k)
            for k, L in enumerate(Ls)]


def test_learned_schedule_replays_on_the_oracle_and_saves_bisections(pa):
    from paper_2006_00561_amd import learned
    # training data: exact schedules of a few small ferromagnets and glasses
    train_pops = _ferro_pops([8, 12, 16, 16, 24], 1500, 100)
    train_pops += [dict(L=L, R=1200, J=W.pmj_couplings(L, 300 + k), seed=5,
                        population_id=10 + k)
                   for k, L in enumerate([8, 12, 16])]
    X, T = learned.generate(train_pops, [0.8, 0.85, 0.9], 1.5, 2)
    assert len(X) > 500
    mlp, loss = learned.train(X, T, iters=2000, lr=2e-3, seed=11)
    assert loss < 0.2
    # held-out populations
    test_pops = _ferro_pops([12, 16, 20], 800, 500)
    target, tol, beta_f, theta = 0.85, 0.02, 1.5, 2
    b = pa.Batch(test_pops)
    steps, src = b.run_learned(mlp, target, tol, beta_f, 1000, theta)
    stats = b.host_stats()
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
        o = oracle.OraclePA(pop["L"], pop["R"], seed=pop["seed"], pop=p)
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
