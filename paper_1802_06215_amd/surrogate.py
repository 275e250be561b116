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


def root_values_same_tree(ctx: "H.Context", model: "H.Model", gamma: float, root: dict, K: int,
                          cfg: "H.RolloutCfg", key: int, mlp: "H.Mlp", horizon: int,
                          ref_keys: int = 32, ref_seed: int = 1 << 20) -> dict:
    """Root lower bound of one two-level DESPOT tree with its frontier valued
    three ways: single default-policy rollouts (the plain method), the mean
    of `ref_keys` independent rollouts per scenario (the reference), and the
    surrogate.  The root (K scenarios `root`, ids 0..K-1) and every child it
    reaches are expanded by the library's kernels under random-number key
    `key` (that fixes the tree); the grandchildren at depth 2 form the
    frontier; child lower bounds are frontier means over each child's
    scenarios (Eq. 13) and the root value is the Eq. 4 backup of the
    library's host tree.  Returns the three root values, and two readings of
    how large a root error is: the root values of the two halves of the
    reference's rollouts (its own sampling spread), and of frontier values
    that keep a fraction s of the surrogate's error (reference + s (surrogate
    - reference))."""
    dev = root[next(iter(root))].device
    A = model.n_actions
    ids = torch.arange(K, dtype=torch.int32, device=dev)
    idx = torch.arange(K, dtype=torch.int16, device=dev)
    out0 = H.LeafBuffers(model, K)
    ctx.expand_leaf([H.make_leaf(model, root, ids, idx, 0, -1, out0, key, 0, cfg)])
    torch.cuda.synchronize()
    nc0, off0, cn0 = out0.n_children.cpu().numpy(), out0.child_off.cpu().numpy(), out0.child_n.cpu().numpy()
    perm0 = out0.perm.cpu().numpy()
    nodes, keep, leaves = [], [], []
    for a in range(A):
        for c in range(int(nc0[a])):
            seg = torch.from_numpy(perm0[a, off0[a, c]:off0[a, c] + cn0[a, c]].astype(np.int16)).to(dev)
            out = H.LeafBuffers(model, int(cn0[a, c]), per_pair=True)
            leaves.append(H.make_leaf(model, root, ids, seg, 1, a, out, key, 0, cfg))
            nodes.append(out)
            keep.append(seg)
    ctx.expand_leaf(leaves)
    torch.cuda.synchronize()
    # frontier: every (action, scenario) pair of every depth-1 node, at depth 2
    front = _cat_states([{k: v[..., :A * o.n] for k, v in o.sprime.items()} for o in nodes])
    fids = torch.cat([o.ids[:o.n].repeat(A) for o in nodes])
    depths = torch.full((fids.numel(),), 2, dtype=torch.int32, device=dev)
    v_one = torch.cat([o.L[:, :o.n].reshape(-1) for o in nodes])
    half = ref_keys // 2
    acc = [torch.zeros_like(v_one, dtype=torch.float64) for _ in range(2)]
    for r in range(ref_keys):
        _, L, _ = ctx.rollout_bounds(model, cfg, front, fids, depths, ref_seed + r, 0)
        acc[0 if r < half else 1] += L.double()
    v_ref = (acc[0] + acc[1]) / ref_keys
    v_sur = mlp.forward(H.features(ctx, model, front, depths, horizon))
    torch.cuda.synchronize()
    host = [dict(n=o.n, nc=o.n_children.cpu().numpy(), z=o.child_z.cpu().numpy().view(np.uint64),
                 cn=o.child_n.cpu().numpy(), off=o.child_off.cpu().numpy(), perm=o.perm.cpu().numpy(),
                 u0=o.child_u0.cpu().numpy(), r=o.r_mean.cpu().numpy(), cap=o.cap) for o in nodes]
    root_host = [out0.n_children.cpu().numpy(), out0.child_z.cpu().numpy().view(np.uint64), cn0,
                 out0.child_u0.cpu().numpy(), out0.child_l0.cpu().numpy(), out0.r_mean.cpu().numpy()]

    def root_value(values: np.ndarray) -> float:
        tree = H.Tree(A, gamma, K, 0.0, 0.0)
        first = tree.add_children(0, *root_host, out0.cap)
        o = 0
        for i, h in enumerate(host):
            v = values[o:o + A * h["n"]].reshape(A, h["n"])
            o += A * h["n"]
            l0 = np.zeros_like(h["u0"])
            for a in range(A):
                for c in range(int(h["nc"][a])):
                    seg = h["perm"][a, h["off"][a, c]:h["off"][a, c] + h["cn"][a, c]]
                    l0[a, c] = v[a, seg].mean()
            tree.add_children(first + i, h["nc"], h["z"], h["cn"], h["u0"], l0, h["r"], h["cap"])
            tree.backup(first + i)
        return tree.bounds(0)[1]

    ref = v_ref.cpu().numpy()
    sur = v_sur.cpu().numpy().astype(np.float64)
    one = v_one.cpu().numpy().astype(np.float64)
    halves = [(a / max(h, 1)).cpu().numpy() for a, h in ((acc[0], half), (acc[1], ref_keys - half))]
    scaled = {s_: root_value(ref + s_ * (sur - ref)) for s_ in (0.5, 0.25, 0.1, 0.05)}
    return dict(rollout=root_value(one), reference=root_value(ref), surrogate=root_value(sur),
                reference_halves=[root_value(h) for h in halves], surrogate_error_scaled=scaled,
                depth1_nodes=len(nodes), frontier_pairs=int(fids.numel()),
                frontier_mean_reference=float(ref.mean()), frontier_bias_surrogate=float((sur - ref).mean()),
                frontier_mae_surrogate=float(np.abs(sur - ref).mean()),
                frontier_mae_rollout=float(np.abs(one - ref).mean()))


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
