"""Double-precision reference of the temperature-step network (test
infrastructure only: gradient checks of the FP32 HIP kernels).

The network maps histogram summaries of a population to log(dbeta):
  u   = (x - mu) / sigma                      input standardisation
  h_1 = tanh(W_1 u + b_1), ..., h_d = tanh(W_d h_{d-1} + b_d)
  z   = w_out . h_d + b_out                   (standardised output)
  loss = mean_s (z_s - (t_s - mu_y) / sigma_y)^2
Parameters are one flat vector: for each layer W (out x in, row-major) then
b (out); the last layer has one output.  Written directly from these
formulas with numpy; the gradient is plain reverse-mode differentiation of
them and is pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np


def layer_shapes(n_in: int, width: int, depth: int):
    shapes = []
    prev = n_in
    for _ in range(depth):
        shapes.append((width, prev))
        prev = width
    shapes.append((1, prev))
    return shapes


def n_params(n_in: int, width: int, depth: int) -> int:
    return sum(o * i + o for o, i in layer_shapes(n_in, width, depth))


def unpack(params, n_in, width, depth):
    p = np.asarray(params, dtype=np.float64)
    out, k = [], 0
    for o, i in layer_shapes(n_in, width, depth):
        W = p[k:k + o * i].reshape(o, i)
        k += o * i
        b = p[k:k + o]
        k += o
        out.append((W, b))
    assert k == len(p)
    return out


def forward(params, X, n_in, width, depth, mu, sigma):
    """Standardised outputs z (shape [B]) and the activations."""
    layers = unpack(params, n_in, width, depth)
    u = (np.asarray(X, np.float64) - np.asarray(mu, np.float64)) / np.asarray(
        sigma, np.float64)
    acts = [u]
    h = u
    for W, b in layers[:-1]:
        h = np.tanh(h @ W.T + b)
        acts.append(h)
    W, b = layers[-1]
    z = (h @ W.T + b)[:, 0]
    return z, acts


def loss_and_grad(params, X, T, n_in, width, depth, mu, sigma, mu_y, sigma_y):
    """Mean squared error on standardised targets and its gradient."""
    layers = unpack(params, n_in, width, depth)
    z, acts = forward(params, X, n_in, width, depth, mu, sigma)
    t = (np.asarray(T, np.float64) - mu_y) / sigma_y
    B = len(z)
    r = z - t
    loss = float(np.mean(r * r))
    grads = [None] * len(layers)
    dz = (2.0 / B) * r[:, None]               # d loss / d z, [B, 1]
    W, b = layers[-1]
    grads[-1] = (dz.T @ acts[-1], dz.sum(axis=0))
    dh = dz @ W                                # [B, width]
    for l in range(len(layers) - 2, -1, -1):
        h = acts[l + 1]
        da = dh * (1.0 - h * h)                # through tanh
        grads[l] = (da.T @ acts[l], da.sum(axis=0))
        dh = da @ layers[l][0]
    flat = np.concatenate([np.concatenate([g[0].ravel(), g[1].ravel()])
                           for g in grads])
    return loss, flat
