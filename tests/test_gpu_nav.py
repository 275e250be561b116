"""GPU parity for navigation in a partially known map (Sec. IV-A).

The HIP path through the C ABI against the oracle on the same seeded inputs:
sampling from the prior, leaves of the paper's 13 x 13 map (124 unknown
cells) at several sizes up to the largest a tile takes (5120 scenarios:
the paper's scenario counts reach 5000), with scenarios
spread over neighbouring cells or sharing one, both rollout policies, the
empty and all-terminal leaves, the stand-alone bounds call, a batch mixing
navigation with the other models (bit-identical to one-leaf calls, both
plans, a graph), and the search driver."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import cfg_pair, collect, compare_leaf, gpu_leaf_desc, host, ids_dev, run_gpu_leaf, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1802_06215_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("K", [1, 500, 2048, 5000])
def test_sample_scenarios_nav(ctx, K):
    from paper_1802_06215_amd import hdx as H
    desc = W.nav_model(1)
    m = ctx.upload_model(desc)
    b = W.nav_belief(desc)
    out = H.empty_states(m, K)
    ctx.sample_scenarios(m, b, K, 9, 4, out)
    torch.cuda.synchronize()
    ref = oracle.sample_scenarios(desc, b, K, 9, 4)
    assert np.array_equal(host(out["w"]), ref["w"])


CASES = [
    # (n_parent, n_leaf, shared cell, policy, seed)
    (100, 1, False, 0, 1),
    (100, 63, False, 0, 2),
    (300, 257, True, 0, 3),
    (500, 500, False, 2, 4),
    (800, 333, False, 0, 5),
    (2048, 2048, False, 0, 6),
    (2048, 1500, True, 2, 7),
    (3000, 3000, False, 0, 8),
    (5000, 5000, False, 2, 9),
    (5120, 4097, True, 0, 10),  # one scenario past 64 full chunks
    (5120, 5120, False, 0, 11),  # the largest leaf
]


@pytest.mark.parametrize("case", CASES)
def test_leaf_parity(ctx, case):
    n_par, n_leaf, shared, policy, seed = case
    desc = W.nav_model(seed % 3)
    m = ctx.upload_model(desc)
    lf = W.nav_leaf(desc, n_par, n_leaf, seed, shared_cell=shared, p_term=0.05)
    cfgs = cfg_pair(policy, 1 << 30, 90)
    par = oracle.parent_states(desc, lf)
    print("nav leaf parent=%d leaf=%d shared=%d policy=%d" % (n_par, n_leaf, shared, policy), flush=True)
    gpu = run_gpu_leaf(ctx, m, par, lf["ids"], lf["idx"], lf["depth"], lf["last_action"], 41 + seed, 3, cfgs[1])
    ref = oracle.expand_leaf(desc, cfgs[0], par, lf["ids"].astype(np.uint32), lf["idx"], lf["depth"],
                             lf["last_action"], 41 + seed, 3, per_pair=True)
    compare_leaf(desc, gpu, ref, n_leaf)


SMALL = [(n, pol) for n in (1, 2, 3, 5, 8, 12, 16) for pol in (0, 2)] + [(4, 1)]


@pytest.mark.parametrize("n,policy", SMALL)
def test_small_leaf_argument_launch_matches_staged_launch(ctx, n, policy):
    """A one-leaf call of at most 16 scenarios (a search thread's typical
    expansion) travels in the kernel arguments; its values and step counts
    must be the oracle's, and every output the bits of the staged batched
    launch of the same leaf."""
    from paper_1802_06215_amd import Batch
    desc = W.nav_model(n % 3)
    m = ctx.upload_model(desc)
    lf = W.nav_leaf(desc, 40, n, 30 + n + policy, p_term=0.05)
    ocfg, hcfg = cfg_pair(policy, 1 << 30, 90, const_action=3)
    par_np = oracle.parent_states(desc, lf)
    par, pids = to_dev(par_np), ids_dev(lf["ids"])
    print("nav small leaf n=%d policy=%d" % (n, policy), flush=True)
    leaf, out, keep = gpu_leaf_desc(m, par, pids, lf["idx"], lf["depth"], lf["last_action"], 13, 4, hcfg, True)
    ctx.expand_leaf([leaf])
    torch.cuda.synchronize()
    got = collect(m, out)
    ref = oracle.expand_leaf(desc, ocfg, par_np, lf["ids"].astype(np.uint32), lf["idx"], lf["depth"],
                             lf["last_action"], 13, 4, per_pair=True)
    compare_leaf(desc, got, ref, n)
    wipe([dict(out=out)])
    for t in (out.L, out.U):
        t.fill_(-5)
    b = Batch(ctx, 1, desc["n_actions"])
    b.set_leaves([leaf])
    b.launch()
    torch.cuda.synchronize()
    got2 = collect(m, out)
    same([got2], [got])
    for key in ("L", "U"):
        assert np.array_equal(got2[key].view(np.uint32), got[key].view(np.uint32)), key
    b.close()


def test_root_and_degenerate_leaves(ctx):
    desc = W.nav_model(1)
    m = ctx.upload_model(desc)
    K = 1000
    st = oracle.sample_scenarios(desc, W.nav_belief(desc), K, 3, 0)
    ids = np.arange(K)
    cfgs = cfg_pair(0, 1 << 30, 90)
    gpu = run_gpu_leaf(ctx, m, st, ids, ids, 0, -1, 3, 0, cfgs[1])
    ref = oracle.expand_leaf(desc, cfgs[0], st, ids.astype(np.uint32), ids, 0, -1, 3, 0, per_pair=True)
    compare_leaf(desc, gpu, ref, K)
    gpu = run_gpu_leaf(ctx, m, st, ids, np.zeros(0, np.int32), 1, 4, 3, 0, cfgs[1])
    assert np.all(gpu["n_children"] == 0) and np.all(gpu["r_mean"] == 0.0)
    lf = W.nav_leaf(desc, 200, 150, 9, p_term=1.0)
    par = oracle.parent_states(desc, lf)
    gpu = run_gpu_leaf(ctx, m, par, lf["ids"], lf["idx"], 2, -1, 5, 0, cfgs[1])
    ref = oracle.expand_leaf(desc, cfgs[0], par, lf["ids"].astype(np.uint32), lf["idx"], 2, -1, 5, 0,
                             per_pair=True)
    compare_leaf(desc, gpu, ref, 150)
    assert np.all(gpu["n_children"] == 1) and int(gpu["steps"].sum()) == 0
    assert np.all(gpu["child_z"][:, 0] == 256)


def test_large_leaf_is_independent_of_the_schedule(ctx):
    """A 5000-scenario leaf: every workgroup width splits its 79 chunks
    into different runs per wavefront, and the results stay bit-identical."""
    from paper_1802_06215_amd import Batch
    desc = W.nav_model(2)
    m = ctx.upload_model(desc)
    lf = W.nav_leaf(desc, 5000, 5000, 12, p_term=0.05)
    par, pids = to_dev(oracle.parent_states(desc, lf)), ids_dev(lf["ids"])
    leaf, out, keep = gpu_leaf_desc(m, par, pids, lf["idx"], lf["depth"], lf["last_action"], 5, 2,
                                    cfg_pair(0, 1 << 30, 90)[1], per_pair=False)
    ctx.expand_leaf([leaf])
    torch.cuda.synchronize()
    ref = collect(m, out)
    b = Batch(ctx, 1, desc["n_actions"])
    b.set_leaves([leaf])
    for threads, persistent, xcd in ((64, 0, 0), (192, 0, 1), (320, 2, 0), (1024, 0, 0)):
        print("nav 5000 schedule", threads, persistent, xcd, flush=True)
        wipe([dict(out=out)])
        b.set_schedule(threads, persistent, xcd)
        b.launch()
        torch.cuda.synchronize()
        same([collect(m, out)], [ref])
    b.close()


def test_leaf_and_search_size_limits(ctx):
    from paper_1802_06215_amd import HdxError
    from paper_1802_06215_amd import hdx as H
    for desc, n_ok, lf_fn in ((W.nav_model(1), H.MAX_NAV_LEAF_SCENARIOS, W.nav_leaf),
                              (W.rocksample_model(7, 8, 1), H.MAX_LEAF_SCENARIOS, W.rocksample_leaf)):
        m = ctx.upload_model(desc)
        lf = lf_fn(desc, n_ok + 1, n_ok + 1, 3)
        par, pids = to_dev(oracle.parent_states(desc, lf)), ids_dev(lf["ids"])
        leaf, out, keep = gpu_leaf_desc(m, par, pids, lf["idx"], lf["depth"], lf["last_action"], 1, 0,
                                        cfg_pair(0, 1 << 30, 90)[1], per_pair=False)
        with pytest.raises(HdxError) as e:
            ctx.expand_leaf([leaf])
        assert e.value.code == -4
        belief = W.nav_belief(desc) if desc["kind"] == W.NAV else W.rocksample_belief(desc)
        with pytest.raises(HdxError) as e:
            ctx.search(m, belief, K=n_ok + 1, n_threads=1, max_depth=10, time_budget_s=0.1,
                       rollout=H.rollout_cfg(0, 10), arena_bytes=256 << 20)
        assert e.value.code == -1
        res = ctx.search(m, belief, K=n_ok, n_threads=1, max_depth=10, time_budget_s=0.1, max_trials=2,
                         rollout=H.rollout_cfg(0, 10), arena_bytes=256 << 20)
        assert res["trials"] >= 1


def test_rollout_bounds_nav(ctx):
    desc = W.nav_model(2)
    m = ctx.upload_model(desc)
    lf = W.nav_leaf(desc, 4000, 10, 4, p_term=0.05)
    st = oracle.parent_states(desc, lf)
    n = 4000
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
    items = []
    specs = [("nav", 500), ("rs", 500), ("mars", 300), ("nav", 2000), ("ped", 500), ("nav", 64)]
    for i, (kind, K) in enumerate(specs):
        if kind == "nav":
            desc = W.nav_model(seed + i)
            lf = W.nav_leaf(desc, K, K - (i * 17) % (K // 2), seed + i, shared_cell=i % 2 == 1)
            cfgs = cfg_pair(0, 1 << 30, 90)
        elif kind == "rs":
            desc = W.rocksample_model(15, 15, seed + i)
            lf = W.rocksample_leaf(desc, K, K - (i * 13) % (K // 2), seed + i)
            cfgs = cfg_pair(0, 1 << 30, 90)
        elif kind == "mars":
            desc = W.mars_model(11, 11, seed + i)
            lf = W.mars_leaf(desc, K, K - (i * 13) % (K // 2), seed + i)
            cfgs = cfg_pair(0, 1 << 30, 90)
        else:
            desc = W.pednav_model(16, 5, seed + i)
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


def test_mixed_batches_match_single_leaves_and_oracle(ctx):
    from paper_1802_06215_amd import Batch
    items = mixed_items(ctx, 70, per_pair=True)
    for it in items:
        ctx.expand_leaf([it["leaf"]])
    torch.cuda.synchronize()
    ref = [collect(it["m"], it["out"]) for it in items]
    wipe(items)
    ctx.expand_leaf([it["leaf"] for it in items])
    torch.cuda.synchronize()
    same([collect(it["m"], it["out"]) for it in items], ref)
    wipe(items)
    ctx.expand_leaf([items[0]["leaf"], items[5]["leaf"]])  # two navigation leaves: kernel arguments
    torch.cuda.synchronize()
    same([collect(items[i]["m"], items[i]["out"]) for i in (0, 5)], [ref[0], ref[5]])
    b = Batch(ctx, len(items), sum(it["desc"]["n_actions"] for it in items))
    b.set_leaves([it["leaf"] for it in items])
    torch.cuda.synchronize()
    for split, threads, persistent, xcd in ((False, 256, 0, 0), (False, 1024, 0, 0), (True, 64, 0, 1),
                                            (True, 512, 2, 0)):
        print("mixed batch split=%d schedule" % split, threads, persistent, xcd, flush=True)
        wipe(items)
        b.set_split(split)
        b.set_schedule(threads, persistent, xcd)
        b.launch()
        torch.cuda.synchronize()
        same([collect(it["m"], it["out"]) for it in items], ref)
    b.set_split(False)
    b.set_schedule(256, 0, 0)
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
    for it in items:
        if it["desc"]["kind"] != W.NAV:
            continue
        lf, desc = it["lf"], it["desc"]
        want = oracle.expand_leaf(desc, it["cfgs"][0], it["par_np"], lf["ids"].astype(np.uint32), lf["idx"],
                                  lf["depth"], lf["last_action"], it["leaf"].seed, 1, per_pair=True)
        compare_leaf(desc, collect(it["m"], it["out"]), want, len(lf["idx"]))


@pytest.mark.parametrize("threads,batch,K", [(1, 0, 500), (8, 8, 2000), (32, 16, 5000), (64, 8, 1000)])
def test_nav_search(ctx, threads, batch, K):
    from paper_1802_06215_amd import hdx as H
    desc = W.nav_model(1)
    m = ctx.upload_model(desc)
    res = ctx.search(m, W.nav_belief(desc), K=K, n_threads=threads, max_depth=90, batch_leaves=batch,
                     time_budget_s=0.5, rollout=H.rollout_cfg(0, 1 << 30, 90), arena_bytes=8 << 30)
    print(threads, batch, K, {k: res[k] for k in ("trials", "expansions", "nodes", "u_root", "l_root")},
          flush=True)
    assert res["trials"] > 0 and res["expansions"] > 0
    tol = 1e-4 * max(1.0, abs(res["u0_root"]))
    assert res["l0_root"] - tol <= res["l_root"] <= res["u_root"] + tol <= res["u0_root"] + 2 * tol
    assert res["best_action"] == int(np.argmax(res["action_l"]))
    assert max(res["action_l"]) == res["l_root"] and max(res["action_u"]) == res["u_root"]


def test_upload_rejects_bad_maps(ctx):
    from paper_1802_06215_amd import HdxError
    good = W.nav_model(1)
    ctx.upload_model(good)
    bad = []
    d = dict(good, cell=good["cell"].copy())
    d["cell"][good["wall"], good["gate_x"][0]] = -2  # a gate that is not unknown cell 0
    bad.append((d, -1))
    d = dict(good, cell=good["cell"].copy())
    d["cell"][12, good["goal_x"]] = -2  # the goal on a wall
    bad.append((d, -1))
    d = dict(good, cell=good["cell"].copy())
    ys, xs = np.nonzero(d["cell"] >= 2)
    d["cell"][ys[1], xs[1]] = d["cell"][ys[0], xs[0]]  # one unknown index used twice
    bad.append((d, -1))
    bad.append((dict(good, p_err=1.0), -1))
    bad.append((dict(good, n=4, cell=np.full((4, 4), -1)), -4))  # grids of 5..16 only
    for desc, code in bad:
        with pytest.raises(HdxError) as e:
            ctx.upload_model(desc)
        assert e.value.code == code
    with pytest.raises(HdxError) as e:
        ctx.upload_model(dict(W.mars_model(7, 8, 1), n=1))  # two robots need a grid of 2 or more
    assert e.value.code == -4
