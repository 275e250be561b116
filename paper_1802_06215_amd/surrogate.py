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

import numpy as np
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


def _cat_states(parts: list) -> dict:
    """Concatenate state dicts along the scenario axis (the last one)."""
    return {k: torch.cat([p[k] for p in parts], dim=-1).contiguous() for k in parts[0]}


def planner_pairs(ctx: "H.Context", model: "H.Model", root_states, K: int, cfg: "H.RolloutCfg",
                  seeds, levels: int, nodes_per_level: int, horizon: int, ref_keys: int,
                  ref_seed: int = 1 << 21):
    """Training pairs from the planner's own trees: for each seed, a root of
    K scenarios (`root_states(seed)`) is expanded, then up to
    `nodes_per_level` of the children reached at each depth (drawn from the
    seed) are expanded in turn, down to `levels` levels; every (action,
    scenario) pair of every expanded node contributes its stepped state at
    its depth, with the mean of `ref_keys` independent default-policy
    rollouts from it as the target.  Returns (features [N, 64] BF16 bits,
    targets [N] f32)."""
    A = model.n_actions
    feats, targets = [], []
    for seed in seeds:
        gen = np.random.default_rng(np.random.SeedSequence([0x504C4E, seed]))
        root = root_states(seed)
        dev = root[next(iter(root))].device
        ids = torch.arange(K, dtype=torch.int32, device=dev)
        level = [(root, ids, torch.arange(K, dtype=torch.int16, device=dev), 0, -1)]
        keep = []
        for _ in range(levels):
            outs = [H.LeafBuffers(model, int(idx.numel()), per_pair=True) for _, _, idx, _, _ in level]
            ctx.expand_leaf([H.make_leaf(model, par, pid, idx, d, la, o, seed, 0, cfg)
                             for (par, pid, idx, d, la), o in zip(level, outs)])
            torch.cuda.synchronize()
            front = _cat_states([{k: v[..., :A * o.n] for k, v in o.sprime.items()} for o in outs])
            fids = torch.cat([o.ids[:o.n].repeat(A) for o in outs])
            depths = torch.cat([torch.full((A * o.n,), d + 1, dtype=torch.int32, device=dev)
                                for (_, _, _, d, _), o in zip(level, outs)])
            acc = torch.zeros(fids.numel(), dtype=torch.float64, device=dev)
            for r in range(ref_keys):
                _, L, _ = ctx.rollout_bounds(model, cfg, front, fids, depths, ref_seed + 1000 * seed + r, 0)
                acc += L.double()
            feats.append(H.features(ctx, model, front, depths, horizon))
            targets.append((acc / ref_keys).float())
            # next level: children with at least one scenario, a random subset
            cands = []
            for (_, _, _, d, _), o in zip(level, outs):
                nc, off, cn = o.n_children.cpu().numpy(), o.child_off.cpu().numpy(), o.child_n.cpu().numpy()
                for a in range(A):
                    for c in range(int(nc[a])):
                        if cn[a, c] > 0:
                            cands.append((o, a, int(off[a, c]), int(cn[a, c]), d + 1))
            if not cands:
                break
            pick = gen.choice(len(cands), size=min(nodes_per_level, len(cands)), replace=False)
            level = []
            for i in sorted(pick):
                o, a, off, cn, d = cands[i]
                states = {k: v[..., :o.n].contiguous() for k, v in o.states.items()}
                level.append((states, o.ids[:o.n], o.perm[a, off:off + cn].contiguous(), d, a))
            keep.append(outs)
    if not feats:
        return (torch.empty((0, H.MLP_IN), dtype=torch.int16, device="cuda"),
                torch.empty(0, dtype=torch.float32, device="cuda"))
    return torch.cat(feats), torch.cat(targets)
