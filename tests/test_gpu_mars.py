"""GPU parity for multi-agent RockSample (Sec. IV-A; |A| = (5+m)^2 up to 625).

The HIP path through the C ABI against the oracle on the same seeded
inputs: sampling, leaves of the paper's three sizes (11,11), (15,15),
(20,20) with chunks, ragged tails, the empty and one-scenario leaf, leaves
whose scenarios share the robots' cells (the wavefront-shared bound) and
leaves where they do not, the default and uniform-random policies, the
stand-alone bounds call, batches mixing every model in one call and in the
batch API (bit-identical to one-leaf calls, graph replays included), and
the search driver on (20,20)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import (assert_states_equal, cfg_pair, collect, compare_leaf, gpu_leaf_desc, host, ids_dev,
                      run_gpu_leaf, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1802_06215_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("K", [1, 500, 777])
def test_sample_scenarios_mars(ctx, K):
    from paper_1802_06215_amd import hdx as H
    desc = W.mars_model(20, 20, 2)
    m = ctx.upload_model(desc)
    b = W.mars_belief(desc, 0.5)
    out = H.empty_states(m, K)
    ctx.sample_scenarios(m, b, K, 9, 4, out)
    torch.cuda.synchronize()
    ref = oracle.sample_scenarios(desc, b, K, 9, 4)
    assert np.array_equal(host(out["w"]), ref["w"])


CASES = [
    # (n, m, n_parent, n_leaf, shared cells, policy, seed)
    (11, 11, 100, 1, True, 0, 1),
    (11, 11, 100, 37, False, 0, 2),
    (11, 11, 200, 130, True, 2, 3),
    (15, 15, 500, 64, False, 2, 4),
    (15, 15, 500, 333, True, 0, 5),
    (20, 20, 500, 500, True, 0, 6),
    (20, 20, 500, 257, False, 0, 7),
    (20, 20, 300, 129, True, 2, 8),
]


@pytest.mark.parametrize("case", CASES)
def test_leaf_parity(ctx, case):
    n, m_rocks, n_par, n_leaf, shared, policy, seed = case
    desc = W.mars_model(n, m_rocks, seed)
    m = ctx.upload_model(desc)
    lf = W.mars_leaf(desc, n_par, n_leaf, seed, shared_cells=shared, p_term=0.05)
    cfgs = cfg_pair(policy, 1 << 30, 90) if policy == 2 else cfg_pair(0, 1 << 30, 90)
    par = oracle.parent_states(desc, lf)
    print("mars leaf n=%d m=%d leaf=%d shared=%d policy=%d" % (n, m_rocks, n_leaf, shared, policy), flush=True)
    gpu = run_gpu_leaf(ctx, m, par, lf["ids"], lf["idx"], lf["depth"], lf["last_action"], 31 + seed, 2, cfgs[1])
    ref = oracle.expand_leaf(desc, cfgs[0], par, lf["ids"].astype(np.uint32), lf["idx"], lf["depth"],
                             lf["last_action"], 31 + seed, 2, per_pair=True)
    compare_leaf(desc, gpu, ref, n_leaf)


def test_root_and_degenerate_leaves(ctx):
    desc = W.mars_model(20, 20, 1)
    m = ctx.upload_model(desc)
    K = 500
    st = oracle.sample_scenarios(desc, W.mars_belief(desc), K, 3, 0)
    ids = np.arange(K)
    cfgs = cfg_pair(0, 1 << 30, 90)
    # the root: every child's lower bound is the closed-form exit value
    gpu = run_gpu_leaf(ctx, m, st, ids, ids, 0, -1, 3, 0, cfgs[1])
    ref = oracle.expand_leaf(desc, cfgs[0], st, ids.astype(np.uint32), ids, 0, -1, 3, 0, per_pair=True)
    compare_leaf(desc, gpu, ref, K)
    assert int(gpu["steps"][:, 1].sum()) == K * (19 + 624 * 20)
    # empty leaf
    gpu = run_gpu_leaf(ctx, m, st, ids, np.zeros(0, np.int32), 1, 7, 3, 0, cfgs[1])
    assert np.all(gpu["n_children"] == 0) and np.all(gpu["r_mean"] == 0.0)
    # every scenario terminal: one child per action, no steps
    lf = W.mars_leaf(desc, 200, 150, 9, p_term=1.0)
    par = oracle.parent_states(desc, lf)
    gpu = run_gpu_leaf(ctx, m, par, lf["ids"], lf["idx"], 2, -1, 5, 0, cfgs[1])
    ref = oracle.expand_leaf(desc, cfgs[0], par, lf["ids"].astype(np.uint32), lf["idx"], 2, -1, 5, 0,
                             per_pair=True)
    compare_leaf(desc, gpu, ref, 150)
    assert np.all(gpu["n_children"] == 1) and int(gpu["steps"].sum()) == 0


def test_rollout_bounds_mars(ctx):
    from paper_1802_06215_amd import hdx as H
    desc = W.mars_model(15, 15, 3)
    m = ctx.upload_model(desc)
    lf = W.mars_leaf(desc, 3000, 10, 4, shared_cells=False, p_term=0.05)
    st = oracle.parent_states(desc, lf)
    n = 3000
    depths = (np.arange(n) % 40).astype(np.int32)
    for policy in (0, 2):
        ocfg, hcfg = cfg_pair(policy, 1 << 30, 90)
        U, L, steps = ctx.rollout_bounds(m, hcfg, to_dev(st), ids_dev(lf["ids"]),
                                         torch.from_numpy(depths).cuda(), 12, 1)
        torch.cuda.synchronize()
        rU, rL, rs, rabs = oracle.rollout_bounds(desc, ocfg, st, lf["ids"], depths, 12, 1, with_abs=True)
        assert np.array_equal(host(steps), rs)
        assert np.all(np.abs(host(U) - rU) <= 1e-5 * np.abs(rU) + 1e-30)
        assert np.all(np.abs(host(L) - rL) <= 1e-5 * np.maximum(np.abs(rL), rabs) + 1e-30)


def mixed_items(ctx, seed, per_pair=False):
    """Leaves of all three models, multi-agent ones of each size."""
    items = []
    specs = [("mars", 11, 11, 100), ("rs", 15, 15, 500), ("mars", 20, 20, 500), ("ped", 16, 5, 500),
             ("mars", 15, 15, 300), ("rs", 7, 8, 100), ("mars", 20, 20, 64)]
    for i, (kind, a, b, K) in enumerate(specs):
        if kind == "mars":
            desc = W.mars_model(a, b, seed + i)
            lf = W.mars_leaf(desc, K, K - (i * 17) % (K // 2), seed + i, shared_cells=i % 2 == 0)
            cfgs = cfg_pair(0, 1 << 30, 90)
        elif kind == "rs":
            desc = W.rocksample_model(a, b, seed + i)
            lf = W.rocksample_leaf(desc, K, K - (i * 13) % (K // 2), seed + i)
            cfgs = cfg_pair(0, 1 << 30, 90)
        else:
            desc = W.pednav_model(a, b, seed + i)
            lf = W.pednav_leaf(desc, K, K - (i * 13) % (K // 2), seed + i)
            cfgs = cfg_pair(0, 50)
        m = ctx.upload_model(desc)
        par_np = oracle.parent_states(desc, lf)
        par, pids = to_dev(par_np), ids_dev(lf["ids"])
        leaf, out, idx = gpu_leaf_desc(m, par, pids, lf["idx"], lf["depth"], lf["last_action"], seed + i, 1,
                                       cfgs[1], per_pair)
        items.append(dict(desc=desc, m=m, lf=lf, par_np=par_np, leaf=leaf, out=out, cfgs=cfgs,
                          keep=(par, pids, idx)))
    return items


def same(a, b):
    for x, y in zip(a, b):
        for key in ("n_children", "perm", "steps", "ids"):
            assert np.array_equal(x[key], y[key]), key
        assert np.array_equal(x["r_mean"].view(np.uint32), y["r_mean"].view(np.uint32))
        for k in x["states"]:
            assert np.array_equal(x["states"][k], y["states"][k])
        for a_, nc in enumerate(y["n_children"]):
            for key in ("child_z", "child_n", "child_off", "child_u0", "child_l0"):
                u, v = x[key][a_, :nc], y[key][a_, :nc]
                if u.dtype == np.float32:
                    u, v = u.view(np.uint32), v.view(np.uint32)
                assert np.array_equal(u, v), key


def wipe(items):
    for it in items:
        o = it["out"]
        for t in (o.child_u0, o.child_l0, o.r_mean, o.perm, o.n_children, o.steps):
            t.fill_(-7)
    torch.cuda.synchronize()


def test_mixed_calls_and_batches_match_single_leaves(ctx):
    from paper_1802_06215_amd import Batch
    items = mixed_items(ctx, 50)
    for it in items:
        ctx.expand_leaf([it["leaf"]])
    torch.cuda.synchronize()
    ref = [collect(it["m"], it["out"]) for it in items]
    # one call with every model (staged descriptors, one dispatch per variant)
    wipe(items)
    ctx.expand_leaf([it["leaf"] for it in items])
    torch.cuda.synchronize()
    same([collect(it["m"], it["out"]) for it in items], ref)
    # a few leaves mixing the multi-agent model with another: not a single
    # kernel-argument launch, yet the same results
    wipe(items)
    ctx.expand_leaf([items[0]["leaf"], items[1]["leaf"], items[4]["leaf"]])
    torch.cuda.synchronize()
    got = [collect(items[i]["m"], items[i]["out"]) for i in (0, 1, 4)]
    same(got, [ref[0], ref[1], ref[4]])
    # the batch API under both plans and several schedules, and a graph
    b = Batch(ctx, len(items), sum(it["desc"]["n_actions"] for it in items))
    b.set_leaves([it["leaf"] for it in items])
    torch.cuda.synchronize()
    for split, threads, persistent, xcd in ((False, 64, 0, 0), (False, 256, 0, 1), (True, 64, 0, 1),
                                            (True, 128, 2, 0)):
        print("mixed batch split=%d schedule" % split, threads, persistent, xcd, flush=True)
        wipe(items)
        b.set_split(split)
        b.set_schedule(threads, persistent, xcd)
        b.launch()
        torch.cuda.synchronize()
        same([collect(it["m"], it["out"]) for it in items], ref)
    b.set_split(False)
    b.set_schedule(64, 0, 0)
    b.use_graph(True)
    stream = torch.cuda.Stream()
    for rep in range(3):
        wipe(items)
        with torch.cuda.stream(stream):
            b.set_leaves([it["leaf"] for it in items], stream)
            b.launch(stream)
            junk = torch.randn(1 << 16, device="cuda").sum()
        stream.synchronize()
        assert torch.isfinite(junk)
        same([collect(it["m"], it["out"]) for it in items], ref)
    b.close()


def test_batch_matches_oracle(ctx):
    from paper_1802_06215_amd import Batch
    items = mixed_items(ctx, 60, per_pair=True)
    b = Batch(ctx, len(items), sum(it["desc"]["n_actions"] for it in items))
    b.set_leaves([it["leaf"] for it in items])
    b.launch()
    torch.cuda.synchronize()
    for it in items:
        if it["desc"]["kind"] != W.MARS:
            continue
        lf, desc = it["lf"], it["desc"]
        ref = oracle.expand_leaf(desc, it["cfgs"][0], it["par_np"], lf["ids"].astype(np.uint32), lf["idx"],
                                 lf["depth"], lf["last_action"], it["leaf"].seed, 1, per_pair=True)
        compare_leaf(desc, collect(it["m"], it["out"]), ref, len(lf["idx"]))
    b.close()


@pytest.mark.parametrize("threads,batch", [(1, 0), (8, 8)])
def test_mars20_search(ctx, threads, batch):
    from paper_1802_06215_amd import hdx as H
    desc = W.mars_model(20, 20, 1)
    m = ctx.upload_model(desc)
    res = ctx.search(m, W.mars_belief(desc), K=500, n_threads=threads, max_depth=90, batch_leaves=batch,
                     time_budget_s=0.5, rollout=H.rollout_cfg(0, 1 << 30, 90), arena_bytes=4 << 30)
    print(threads, batch, {k: res[k] for k in ("trials", "expansions", "nodes", "launches", "u_root", "l_root")},
          flush=True)
    assert res["trials"] > 0 and res["expansions"] > 0
    tol = 1e-4 * max(1.0, abs(res["u0_root"]))
    assert res["l0_root"] - tol <= res["l_root"] <= res["u_root"] + tol <= res["u0_root"] + 2 * tol
    # both robots moving east is worth the two exit rewards, so the root's
    # lower bound is at least that once the root is expanded
    assert res["l_root"] >= 2 * 10 * 0.95 ** 19 - tol
    assert res["best_action"] == int(np.argmax(res["action_l"]))
    assert len(res["action_l"]) == 625


def test_surrogate_rejects_mars(ctx):
    from paper_1802_06215_amd import HdxError
    from paper_1802_06215_amd import hdx as H
    desc = W.mars_model(7, 8, 1)
    m = ctx.upload_model(desc)
    st = H.empty_states(m, 4)
    with pytest.raises(HdxError) as e:
        H.features(ctx, m, st, torch.zeros(4, dtype=torch.int32, device="cuda"), 90)
    assert e.value.code == -6


def test_no_rocks_search_finds_both_exits(ctx):
    """No rocks and no rollouts: expansions and Eq. 4 backups alone must find
    the two robots' exit value 10 gamma^(n-1-x1) + 10 gamma^(n-1-x2), and the
    first joint action moves both robots east."""
    from paper_1802_06215_amd import hdx as H
    n = 3
    desc = dict(kind=2, n=n, m=0, rock_x=np.zeros(0, np.int32), rock_y=np.zeros(0, np.int32), gamma=0.95,
                start=(0, 1, 0, 0), n_actions=25)
    m = ctx.upload_model(desc)
    belief = dict(pos=(0, 1, 1, 0, 0, 0), p=np.zeros(0))
    res = ctx.search(m, belief, K=4, n_threads=1, max_depth=6, time_budget_s=20.0, max_trials=4000,
                     gap_epsilon=1e-9, rollout=H.rollout_cfg(0, 0), arena_bytes=256 << 20)
    exact = 10 * 0.95 ** 2 + 10 * 0.95 ** 1
    assert abs(res["u0_root"] - exact) < 1e-5 and res["l0_root"] == 0.0
    assert abs(res["l_root"] - exact) < 1e-5 and abs(res["u_root"] - exact) < 1e-5
    assert res["best_action"] == 2 * 5 + 2
