"""Element-level expansion of small driving leaves (one lane per pedestrian).

A one-leaf call launches through the kernel arguments; when every scenario
of the leaf gets a group of lanes (n times the pedestrian count rounded up
to a power of two is at most 64), its gather, update step, expansion step
(with the observation hash chained over the group's lanes), upper bound
and rollout run element by element.  They must give the oracle's states,
rewards and observations bit for bit and its values within the usual FP
tolerance, and the one-lane path's results bit for bit: the stand-alone
bounds call (one lane per state) on the leaf's stepped states, ids and
depth, and the staged batched launch of the same leaf (which never uses
the element-level path), field by field."""
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
    b = Batch(ctx, 1, A)
    b.set_leaves([leaf])
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
