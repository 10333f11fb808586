"""Learned temperature steps: training data from the exact adaptive schedule,
training of the network on the GPU, and the learned schedule itself.

The exact schedule picks, for each population and step, the largest dbeta
whose energy-distribution overlap is at least the target (bisection on the
histogram, in double precision).  Each such decision, with the 8 histogram
summaries the device computed before it, is one training pair
(features, log dbeta).  The network (``binding.MLP``) is trained on these
pairs by the library's FP32 forward, backward and Adam kernels.  In the
learned schedule (``Batch.run_learned``) its proposal is accepted only when
the exact overlap at the proposed step is within a tolerance of the target;
otherwise the bisection runs.  Reweighting is exact either way, so the
network changes which temperatures are visited, never the weights.
"""
from __future__ import annotations

import numpy as np

from . import binding as B

FEATURES = ("mean E / N", "ln sd(E)", "skewness of E", "(Emin - mean) / sd",
            "beta", "ln N", "ln R", "overlap target")
# sources of a step (see pa_batch_decisions)
SRC_SCHEDULE, SRC_BISECT, SRC_NET, SRC_FALLBACK, SRC_REST = 0, 1, 2, 3, 4


def collect_pairs(batch, n_pops, sources=(SRC_BISECT, SRC_FALLBACK)):
    """(features, log dbeta) of every bisection decision of the last run."""
    X, T = [], []
    for p in range(n_pops):
        f, db, src = batch.decisions(p)
        keep = np.isin(src, sources) & (db > 0.0)
        X.append(f[keep])
        T.append(np.log(db[keep]))
    return (np.concatenate(X).astype(np.float32),
            np.concatenate(T).astype(np.float32))


def generate(populations, targets, beta_f, theta, max_steps=2000,
             stream=None):
    """Run the exact adaptive schedule once per target on a batch of the
    given populations and return all (features, log dbeta) pairs."""
    Xs, Ts = [], []
    for target in targets:
        b = B.Batch(populations, stream=stream)
        b.run_adaptive(target, beta_f, max_steps, theta, use_graph=True)
        X, T = collect_pairs(b, len(populations))
        Xs.append(X)
        Ts.append(T)
        b.close()
    return np.concatenate(Xs), np.concatenate(Ts)


def fit_norm(X, T):
    """Per-feature standardisation (constant features keep scale 1)."""
    mu = X.mean(axis=0).astype(np.float32)
    sd = X.std(axis=0).astype(np.float32)
    sd[sd < 1e-3] = 1.0
    return mu, sd, float(T.mean()), float(max(T.std(), 1e-3))


def train(X, T, width=64, depth=3, iters=3000, batch=256, lr=1e-3, seed=1,
          stream=None):
    """A network fitted to (X, T) on the GPU; returns (mlp, final loss)."""
    mlp = B.MLP(n_in=X.shape[1], width=width, depth=depth, seed=seed,
                stream=stream)
    mlp.set_norm(*fit_norm(X, T))
    loss = mlp.train(X, T, batch=batch, iters=iters, lr=lr, seed=seed + 1)
    return mlp, loss
