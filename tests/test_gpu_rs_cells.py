"""GPU parity of RockSample leaves whose scenarios stand on different cells.

Robot motion is deterministic, so the scenarios of a node reached from one
root share the robot's cell, and the kernels tabulate the upper bound of
Eq. 12 once per cell for a whole wavefront.  Any states are valid inputs of
an expansion, though: here the parent's scenarios draw their own cells
(every wavefront takes the per-lane bound), or alternate 64-scenario runs of
one shared cell and of scattered cells (a wavefront switches between the
table and the per-lane sum from one chunk to the next).  Single-leaf calls
and the batched launch under both plans are compared with the oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import cfg_pair, collect, compare_leaf, gpu_leaf_desc, ids_dev, run_gpu_leaf, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1802_06215_amd import Context
    c = Context(0)
    yield c
    c.close()


def mixed_leaf(desc, n_parent, n_leaf, seed, pattern, depth=None):
    lf = W.rocksample_leaf(desc, n_parent, n_leaf, seed, p_term=0.05, depth=depth, shared_cell=False)
    if pattern == "runs":
        # leaf positions in 64-runs: even runs on one cell, odd runs scattered
        x, y = np.array(lf["x"]), np.array(lf["y"])
        pos = np.asarray(lf["idx"])
        for j, k in enumerate(pos):
            if (j // 64) % 2 == 0:
                x[k], y[k] = 3, 2
        lf["x"], lf["y"] = x, y
    return lf


def oracle_leaf(desc, ocfg, lf, seed, step):
    return oracle.expand_leaf(desc, ocfg, oracle.parent_states(desc, lf), lf["ids"].astype(np.uint32), lf["idx"],
                              lf["depth"], lf["last_action"], seed, step, per_pair=True)


@pytest.mark.parametrize("pattern", ["scattered", "runs"])
@pytest.mark.parametrize("grid,rocks,n_parent,n_leaf,policy", [
    (7, 8, 100, 100, 0), (7, 8, 500, 437, 0), (15, 15, 500, 500, 0), (15, 15, 2048, 2048, 0),
    (15, 15, 700, 513, 2), (20, 20, 2048, 1999, 0)])
def test_mixed_cell_leaf(ctx, pattern, grid, rocks, n_parent, n_leaf, policy):
    desc = W.rocksample_model(grid, rocks, 4)
    m = ctx.upload_model(desc)
    lf = mixed_leaf(desc, n_parent, n_leaf, 31 + n_leaf, pattern)
    ocfg, hcfg = cfg_pair(policy, 1 << 30, 90) if grid > 7 else cfg_pair(policy, 30)
    print("mixed-cell leaf grid=%d n=%d pattern=%s policy=%d" % (grid, n_leaf, pattern, policy), flush=True)
    par = oracle.parent_states(desc, lf)
    gpu = run_gpu_leaf(ctx, m, par, lf["ids"], lf["idx"], lf["depth"], lf["last_action"], 5, 2, hcfg)
    ref = oracle_leaf(desc, ocfg, lf, 5, 2)
    compare_leaf(desc, gpu, ref, n_leaf)
    # the leaf's scenarios really do stand on several cells
    w = ref["states"]["w"]
    assert len(np.unique(w & 0x3FF)) > 1


def test_mixed_cell_batch_both_plans(ctx):
    """Mixed-cell and shared-cell leaves of several sizes in one batch: both
    plans and several schedules give the single-leaf results bit for bit,
    and every leaf matches the oracle."""
    from paper_1802_06215_amd import Batch
    desc = W.rocksample_model(15, 15, 6)
    m = ctx.upload_model(desc)
    ocfg, hcfg = cfg_pair(0, 1 << 30, 90)
    items = []
    for i, (n, pattern) in enumerate(((500, "scattered"), (2048, "runs"), (250, "shared"), (125, "runs"),
                                      (31, "scattered"), (1, "scattered"), (700, "scattered"))):
        if pattern == "shared":
            lf = W.rocksample_leaf(desc, 500, n, 70 + i, p_term=0.05)
        else:
            lf = mixed_leaf(desc, max(n, 500), n, 70 + i, pattern)
        par_np = oracle.parent_states(desc, lf)
        par, pids = to_dev(par_np), ids_dev(lf["ids"])
        leaf, out, idx = gpu_leaf_desc(m, par, pids, lf["idx"], lf["depth"], lf["last_action"], 40 + i, 1, hcfg,
                                       True)
        items.append(dict(lf=lf, leaf=leaf, out=out, keep=(par, pids, idx)))
    for it in items:
        ctx.expand_leaf([it["leaf"]])
    torch.cuda.synchronize()
    single = [collect(m, it["out"]) for it in items]
    for it, got in zip(items, single):
        lf = it["lf"]
        compare_leaf(desc, got, oracle_leaf(desc, ocfg, lf, it["leaf"].seed, 1), len(lf["idx"]))
    b = Batch(ctx, len(items), len(items) * desc["n_actions"])
    b.set_leaves([it["leaf"] for it in items])
    for split, threads, persistent, xcd in ((False, 64, 0, 1), (False, 256, 0, 0), (True, 128, 0, 1)):
        print("mixed-cell batch split=%d threads=%d" % (split, threads), flush=True)
        for it in items:
            for t in (it["out"].perm, it["out"].child_l0, it["out"].child_u0, it["out"].U, it["out"].L):
                t.fill_(-7)
        b.set_split(split)
        b.set_schedule(threads, persistent, xcd)
        b.launch()
        torch.cuda.synchronize()
        for it, want in zip(items, single):
            got = collect(m, it["out"])
            assert np.array_equal(got["perm"], want["perm"])
            assert np.array_equal(got["steps"], want["steps"])
            for key in ("U", "L"):
                assert np.array_equal(got[key].view(np.uint32), want[key].view(np.uint32)), key
            for a, nc in enumerate(want["n_children"]):
                for key in ("child_u0", "child_l0"):
                    assert np.array_equal(got[key][a, :nc].view(np.uint32), want[key][a, :nc].view(np.uint32))
    b.close()
