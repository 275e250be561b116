"""Helpers that grow a DESPOT tree with the oracle (for the tests only)."""
import numpy as np

import oracle


def grow(desc, rc, parent, parent_ids, idx, depth, last_action, seed, step, horizon, node=None):
    """Expand a leaf, then every child, down to ``horizon``; back up (Eq. 4)."""
    res = oracle.expand_leaf(desc, rc, parent, parent_ids, idx, depth, last_action, seed, step)
    if node is None:
        node = oracle.Node(None, len(idx), 0.0, 0.0)
    oracle.attach_children(desc, node, res)
    if depth + 1 < horizon:
        for a, (r_mean, kids) in enumerate(node.actions):
            for c, kid in enumerate(kids):
                off, cnt = res["child_off"][a, c], res["child_n"][a, c]
                grow(desc, rc, res["states"], res["ids"], res["perm"][a, off:off + cnt],
                     depth + 1, a, seed, step, horizon, kid)
    node.u = oracle.node_value(node, desc["gamma"], "u")
    node.l = oracle.node_value(node, desc["gamma"], "l")
    return node


def brute_force(desc, rc, st, ids, depth, h, seed, step, which):
    """Scenario-determinised expectimax, grouping by a dictionary."""
    n = len(ids)
    if h == 0:
        U, L, _ = oracle.rollout_bounds(desc, rc, st, ids, depth, seed, step)
        return float(np.mean(U if which == "u" else L))
    best = -np.inf
    for a in range(desc["n_actions"]):
        nxt, r, z = oracle.step(desc, st, ids, a, depth, seed, step)
        groups = {}
        for k in range(n):
            groups.setdefault(int(z[k]), []).append(k)
        q = float(np.sum(r.astype(np.float64))) / n
        for zz, ks in groups.items():
            sub = oracle.take_states(desc, nxt, ks)
            q += desc["gamma"] * len(ks) / n * brute_force(desc, rc, sub, ids[ks], depth + 1, h - 1,
                                                           seed, step, which)
        best = max(best, q)
    return best
