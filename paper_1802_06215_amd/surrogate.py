"""Rollout-value surrogate: training pairs from expansions, and fitting.

A leaf expanded with full rollouts and per-pair outputs holds, for every
(action, scenario), the stepped state s' and the discounted value of the
rollout from it (the default-policy lower bound of Eq. 13).  The features
of s' at depth + 1 and that value make one training pair.  fit() runs the
library's own forward, backward and Adam kernels over shuffled minibatches;
the shuffling gather and the bookkeeping here are plain tensor plumbing.
"""
from __future__ import annotations

import math

import torch

from . import hdx as H

FLOPS_FWD = 2 * (H.MLP_IN * H.MLP_HIDDEN + 2 * H.MLP_HIDDEN * H.MLP_HIDDEN + H.MLP_HIDDEN)
FLOPS_TRAIN = 3 * FLOPS_FWD  # forward, and the backward's two products per layer


def leaf_pairs(ctx: "H.Context", model: "H.Model", out: "H.LeafBuffers", depth: int, horizon: int):
    """(features [A*n, 64] BF16 bits, values [A*n] f32) of one leaf expanded
    with per-pair outputs (LeafBuffers(per_pair=True)); row a*n + k is the
    pair (action a, scenario k)."""
    n, A = out.n, model.n_actions
    if n == 0:
        return (torch.empty((0, H.MLP_IN), dtype=torch.int16, device=out.L.device),
                torch.empty(0, dtype=torch.float32, device=out.L.device))
    depths = torch.full((A * n,), depth + 1, dtype=torch.int32, device=out.L.device)
    X = H.features(ctx, model, out.sprime, depths, horizon)
    return X, out.L[:, :n].reshape(-1).contiguous()


def fit(mlp: "H.Mlp", X: torch.Tensor, t: torch.Tensor, epochs: int, batch: int = 4096, lr: float = 1e-3,
        seed: int = 0, lr_final: float | None = None) -> list:
    """Adam on mean squared error over `epochs` passes of shuffled
    minibatches of `batch` rows (a multiple of 64; a ragged last batch is
    dropped); with lr_final the rate follows a cosine from lr down to
    lr_final over the epochs.  Returns the mean training loss of each epoch."""
    if batch % 64 or batch <= 0:
        raise ValueError("batch must be a positive multiple of 64")
    N = X.shape[0]
    steps = N // batch
    if steps == 0:
        raise ValueError("fewer rows than one batch")
    g = torch.Generator(device=X.device)
    g.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=X.device)
    acc = torch.zeros(1, dtype=torch.float32, device=X.device)
    hist = []
    for e in range(epochs):
        rate = lr
        if lr_final is not None and epochs > 1:
            rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * e / (epochs - 1)))
        perm = torch.randperm(N, generator=g, device=X.device)
        Xs, ts = X[perm], t[perm]
        acc.zero_()
        for i in range(steps):
            mlp.train_step(Xs[i * batch:(i + 1) * batch], ts[i * batch:(i + 1) * batch], rate, loss)
            acc += loss
        hist.append(float(acc) / steps)
    return hist


def predict(mlp: "H.Mlp", X: torch.Tensor) -> torch.Tensor:
    return mlp.forward(X)
