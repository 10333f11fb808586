"""Pins of the double-precision reference network: its gradient against
central finite differences, and its forward pass against a per-sample loop
written from the formula."""
import numpy as np

from oracle import mlp_ref as M


def _setup(seed=0, n_in=8, width=16, depth=3, B=12):
    rng = np.random.default_rng(seed)
    n = M.n_params(n_in, width, depth)
    params = rng.normal(0, 0.4, n)
    X = rng.normal(0, 1.5, (B, n_in))
    T = rng.normal(-5, 1, B)
    mu = rng.normal(0, 1, n_in)
    sigma = rng.uniform(0.5, 2, n_in)
    return params, X, T, mu, sigma


def test_parameter_count_of_the_default_network():
    # 8 -> 64 -> 64 -> 64 -> 1
    assert M.n_params(8, 64, 3) == 8 * 64 + 64 + 2 * (64 * 64 + 64) + 64 + 1


def test_forward_matches_per_sample_loop():
    params, X, T, mu, sigma = _setup()
    z, _ = M.forward(params, X, 8, 16, 3, mu, sigma)
    layers = M.unpack(params, 8, 16, 3)
    for s in range(len(X)):
        h = [(X[s, i] - mu[i]) / sigma[i] for i in range(8)]
        for W, b in layers[:-1]:
            h = [np.tanh(sum(W[o, i] * h[i] for i in range(len(h))) + b[o])
                 for o in range(W.shape[0])]
        W, b = layers[-1]
        zs = sum(W[0, i] * h[i] for i in range(len(h))) + b[0]
        assert abs(zs - z[s]) < 1e-12


def test_gradient_matches_central_differences():
    params, X, T, mu, sigma = _setup(seed=1)
    args = (X, T, 8, 16, 3, mu, sigma, -5.0, 1.3)
    loss, g = M.loss_and_grad(params, *args)
    eps = 1e-6
    rng = np.random.default_rng(2)
    idx = rng.choice(len(params), 60, replace=False)
    for k in idx:
        p1 = params.copy()
        p2 = params.copy()
        p1[k] += eps
        p2[k] -= eps
        fd = (M.loss_and_grad(p1, *args)[0] - M.loss_and_grad(p2, *args)[0]) / (
            2 * eps)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])
