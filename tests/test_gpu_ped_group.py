"""Element-level expansion of small driving leaves (one lane per pedestrian).

A one-leaf call launches through the kernel arguments; when every scenario
of the leaf gets a group of lanes (n times the pedestrian count rounded up
to a power of two is at most 64), its gather, update step, expansion step
(with the observation hash chained over the group's lanes), upper bound
and rollout run element by element.  They must give the oracle's states,
rewards and observations bit for bit and its values within the usual FP
tolerance, and the one-lane path's results bit for bit: the stand-alone
bounds call (one lane per state) on the leaf's stepped states, ids and
depth, and a staged batched launch of the same leaf on one lane per
scenario (a larger leaf in the same dispatch keeps it off the
element-level instance), field by field.  Batches of small leaves take the
element-level instance of the staged kernel: they must match the oracle
and the one-leaf calls bit for bit, under both launch plans and in a
graph."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import cfg_pair, collect, compare_leaf, gpu_leaf_desc, host, ids_dev, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1802_06215_amd import Context
    c = Context(0)
    yield c
    c.close()


CASES = [(peds, n, pol) for peds, n in ((0, 3), (3, 9), (6, 8), (6, 5), (16, 1), (16, 4), (20, 2), (32, 2), (16, 5))
         for pol in (0, 2)] + [(16, 3, 1)]


@pytest.mark.parametrize("peds,n,policy", CASES)
def test_small_leaf_group_rollout(ctx, peds, n, policy):
    from paper_1802_06215_amd import Batch
    from paper_1802_06215_amd import hdx as H
    desc = W.pednav_model(peds, 5, 2)
    m = ctx.upload_model(desc)
    lf = W.pednav_leaf(desc, 40, n, 7 + n + peds, p_term=0.1)
    ocfg, hcfg = cfg_pair(policy, 50, -1, const_action=1)
    par_np = oracle.parent_states(desc, lf)
    par, pids = to_dev(par_np), ids_dev(lf["ids"])
    print("ped group leaf peds=%d n=%d policy=%d" % (peds, n, policy), flush=True)
    leaf, out, idx = gpu_leaf_desc(m, par, pids, lf["idx"], lf["depth"], lf["last_action"], 11, 2, hcfg, True)
    ctx.expand_leaf([leaf])
    torch.cuda.synchronize()
    got = collect(m, out)
    ref = oracle.expand_leaf(desc, ocfg, par_np, lf["ids"].astype(np.uint32), lf["idx"], lf["depth"],
                             lf["last_action"], 11, 2, per_pair=True)
    compare_leaf(desc, got, ref, n)
    # bit for bit against one lane per state on the same stepped states
    A = desc["n_actions"]
    sp = {k: v[..., :A * n].contiguous() for k, v in out.sprime.items()}
    ids = out.ids[:n].repeat(A).contiguous()
    depths = torch.full((A * n,), lf["depth"] + 1, dtype=torch.int32, device="cuda")
    _, L1, steps1 = ctx.rollout_bounds(m, hcfg, sp, ids, depths, 11, 2)
    torch.cuda.synchronize()
    assert np.array_equal(host(L1).view(np.uint32), got["L"].reshape(-1).view(np.uint32))
    assert np.array_equal(host(steps1).reshape(A, n).sum(1), got["steps"][:, 1])
    # and against the batched launch (one lane per scenario), field by field
    for t in [out.L, out.U, out.r, out.z, out.child_l0, out.child_u0, out.child_z, out.child_n, out.child_off,
              out.perm, out.child_of, out.steps, out.r_mean, out.n_children, out.ids]:
        t.fill_(-5)
    for d in (out.states, out.sprime):
        for t in d.values():
            t.fill_(7)
    # one dispatch whose largest leaf (100 scenarios) keeps it on one lane
    # per scenario
    big = W.pednav_leaf(desc, 200, 100, 5 + peds, p_term=0.1)
    bpar, bpids = to_dev(oracle.parent_states(desc, big)), ids_dev(big["ids"])
    bleaf, bout, bidx = gpu_leaf_desc(m, bpar, bpids, big["idx"], big["depth"], big["last_action"], 11, 2, hcfg, True)
    b = Batch(ctx, 2, 2 * A)
    b.set_split(False)
    b.set_leaves([leaf, bleaf])
    b.launch()
    torch.cuda.synchronize()
    got2 = collect(m, out)
    for key in ("L", "U", "r", "z", "perm", "child_of", "steps", "r_mean", "n_children", "ids"):
        a1, a2 = np.asarray(got[key]), np.asarray(got2[key])
        if a1.dtype == np.float32:
            a1, a2 = a1.view(np.uint32), a2.view(np.uint32)
        assert np.array_equal(a1, a2), key
    for d in ("states", "sprime"):
        for k in got[d]:
            assert np.array_equal(np.asarray(got[d][k]).view(np.uint8), np.asarray(got2[d][k]).view(np.uint8)), (d, k)
    for a_, nc in enumerate(got["n_children"]):  # slots past a child count are not written
        for key in ("child_l0", "child_u0", "child_z", "child_n", "child_off"):
            a1, a2 = got[key][a_, :nc], got2[key][a_, :nc]
            if a1.dtype == np.float32:
                a1, a2 = a1.view(np.uint32), a2.view(np.uint32)
            assert np.array_equal(a1, a2), key
    b.close()


@pytest.mark.parametrize("split,graph", [(True, False), (False, False), (False, True)])
def test_batched_small_leaves_element_level(ctx, split, graph):
    """Small driving leaves of three pedestrian bounds (8, 16, 32) in one
    batch: every dispatch's largest leaf fits its wavefront with a lane per
    pedestrian, so the staged kernel's element-level instance runs.  Each
    leaf matches the oracle and its own one-leaf call bit for bit."""
    from paper_1802_06215_amd import Batch
    from paper_1802_06215_amd import hdx as H
    ocfg, hcfg = cfg_pair(0, 50, -1)
    items = []
    for peds, ns in ((6, (1, 5, 8)), (16, (1, 2, 3, 4, 4, 3, 2, 1)), (20, (1, 2))):
        desc = W.pednav_model(peds, 5, 3)
        m = ctx.upload_model(desc)
        for j, n in enumerate(ns):
            lf = W.pednav_leaf(desc, 30, n, 40 + 7 * peds + j, p_term=0.1)
            par_np = oracle.parent_states(desc, lf)
            par, pids = to_dev(par_np), ids_dev(lf["ids"])
            leaf, out, idx = gpu_leaf_desc(m, par, pids, lf["idx"], lf["depth"], lf["last_action"], 13, 1, hcfg,
                                           True)
            items.append((desc, m, lf, par_np, par, pids, leaf, out, idx))
    print("batched element-level leaves", len(items), "split", split, "graph", graph, flush=True)
    single = []
    for desc, m, lf, par_np, par, pids, leaf, out, idx in items:
        ctx.expand_leaf([leaf])
        torch.cuda.synchronize()
        single.append(collect(m, out))
    if split and not graph:
        # more leaves than one kernel-argument pack: hdx_expand_leaf stages
        # them and launches the element-level instance per model
        assert len(items) > 11
        for it in items:
            it[7].L.fill_(-3)
            it[7].perm.fill_(-3)
        ctx.expand_leaf([it[6] for it in items])
        torch.cuda.synchronize()
        for (desc, m, lf, par_np, par, pids, leaf, out, idx), one in zip(items, single):
            got = collect(m, out)
            for key in ("L", "U", "r", "z", "perm", "child_of", "steps", "r_mean", "n_children", "ids"):
                a1, a2 = np.asarray(one[key]), np.asarray(got[key])
                if a1.dtype == np.float32:
                    a1, a2 = a1.view(np.uint32), a2.view(np.uint32)
                assert np.array_equal(a1, a2), ("staged call", key, desc["n_peds"])
    tiles = sum(it[0]["n_actions"] for it in items)
    b = Batch(ctx, len(items), tiles)
    b.set_split(split)
    b.set_leaves([it[6] for it in items])
    if graph:
        b.use_graph(True)
    for rep in range(2 if graph else 1):
        for it in items:
            for t in (it[7].L, it[7].perm, it[7].child_l0, it[7].steps, it[7].n_children):
                t.fill_(-3)
        b.launch()
        torch.cuda.synchronize()
        for (desc, m, lf, par_np, par, pids, leaf, out, idx), one in zip(items, single):
            got = collect(m, out)
            n = len(lf["idx"])
            ref = oracle.expand_leaf(desc, ocfg, par_np, lf["ids"].astype(np.uint32), lf["idx"], lf["depth"],
                                     lf["last_action"], 13, 1, per_pair=True)
            compare_leaf(desc, got, ref, n)
            for key in ("L", "U", "r", "z", "perm", "child_of", "steps", "r_mean", "n_children", "ids"):
                a1, a2 = np.asarray(one[key]), np.asarray(got[key])
                if a1.dtype == np.float32:
                    a1, a2 = a1.view(np.uint32), a2.view(np.uint32)
                assert np.array_equal(a1, a2), (key, desc["n_peds"], n)
    b.close()
