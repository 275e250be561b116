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
