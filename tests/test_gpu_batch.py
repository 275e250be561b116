"""GPU tests of the batched form: many independent planner instances of
uneven K and |A| (RockSample and crowd driving mixed) in one launch, under
every launch schedule the autotuner can pick and through a replayed HIP
graph; outputs must be bit-identical to per-instance launches, and sampled
leaves must match the oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import cfg_pair, collect, compare_leaf, gpu_leaf_desc, ids_dev, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1802_06215_amd import Context
    c = Context(0)
    yield c
    c.close()


def build_instances(ctx, count, seed, per_pair=False):
    inst = W.mixed_instances(count, seed)
    items = []
    for i, it in enumerate(inst):
        desc, K = it["model"], it["K"]
        m = ctx.upload_model(desc)
        if desc["kind"] == 0:
            lf = W.rocksample_leaf(desc, K, K - (i * 13) % (K // 2), seed + i)
            cfgs = cfg_pair(0, 1 << 30, 90)
        else:
            lf = W.pednav_leaf(desc, K, K - (i * 13) % (K // 2), seed + i)
            cfgs = cfg_pair(0, 50)
        par_np = oracle.parent_states(desc, lf)
        par, pids = to_dev(par_np), ids_dev(lf["ids"])
        leaf, out, idx = gpu_leaf_desc(ctx_model := m, par, pids, lf["idx"], lf["depth"], lf["last_action"],
                                       seed + i, 1, cfgs[1], per_pair)
        items.append(dict(desc=desc, m=ctx_model, lf=lf, par_np=par_np, leaf=leaf, out=out, cfgs=cfgs,
                          keep=(par, pids, idx)))
    return items


def snapshot(items):
    return [collect(it["m"], it["out"]) for it in items]


def assert_same(a, b):
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


def clear(items):
    for it in items:
        o = it["out"]
        for t in (o.child_u0, o.child_l0, o.r_mean, o.perm, o.n_children, o.steps):
            t.fill_(-7)
    torch.cuda.synchronize()


def test_batch_equals_per_instance_under_every_schedule(ctx):
    from paper_1802_06215_amd import Batch
    items = build_instances(ctx, 64, 42)
    print("64 instances, %d tiles" % sum(it["desc"]["n_actions"] for it in items), flush=True)
    for it in items:
        ctx.expand_leaf([it["leaf"]])
    torch.cuda.synchronize()
    ref = snapshot(items)
    b = Batch(ctx, 64, 64 * 25)
    b.set_leaves([it["leaf"] for it in items])
    torch.cuda.synchronize()
    for split in (False, True):
        b.set_split(split)
        assert b.split() == split
        for threads in (64, 128, 256):
            for persistent, xcd in ((0, 0), (0, 1), (1, 0), (3, 0), (8, 0)):
                print("plan split=%d schedule" % split, threads, persistent, xcd, flush=True)
                clear(items)
                b.set_schedule(threads, persistent, xcd)
                b.launch()
                torch.cuda.synchronize()
                assert_same(snapshot(items), ref)
    b.close()


def test_batch_matches_oracle_on_sampled_leaves(ctx):
    from paper_1802_06215_amd import Batch
    items = build_instances(ctx, 16, 7, per_pair=True)
    b = Batch(ctx, 16, 16 * 25)
    b.set_leaves([it["leaf"] for it in items])
    b.launch()
    torch.cuda.synchronize()
    for it in items[::3]:
        lf, desc = it["lf"], it["desc"]
        ref = oracle.expand_leaf(desc, it["cfgs"][0], it["par_np"], lf["ids"].astype(np.uint32), lf["idx"],
                                 lf["depth"], lf["last_action"], it["leaf"].seed, 1, per_pair=True)
        compare_leaf(desc, collect(it["m"], it["out"]), ref, len(lf["idx"]))
    b.close()


def test_graph_replays_match_eager(ctx):
    from paper_1802_06215_amd import Batch
    items_a = build_instances(ctx, 24, 11)
    items_b = build_instances(ctx, 24, 12)
    # eager references
    for it in items_a + items_b:
        ctx.expand_leaf([it["leaf"]])
    torch.cuda.synchronize()
    ref_a, ref_b = snapshot(items_a), snapshot(items_b)
    stream = torch.cuda.Stream()
    b = Batch(ctx, 64, 64 * 25)
    b.set_schedule(256, 2, 0)
    b.use_graph(True)
    for rep in range(4):
        items, ref = (items_a, ref_a) if rep % 2 == 0 else (items_b, ref_b)
        clear(items)
        with torch.cuda.stream(stream):
            b.set_leaves([it["leaf"] for it in items], stream)
            b.launch(stream)
            # some eager work of the program between replays
            junk = torch.randn(1 << 16, device="cuda").sum()
        stream.synchronize()
        assert torch.isfinite(junk)
        assert_same(snapshot(items), ref)
    b.close()


def test_autotune_keeps_results(ctx):
    from paper_1802_06215_amd import Batch
    items = build_instances(ctx, 32, 5)
    for it in items:
        ctx.expand_leaf([it["leaf"]])
    torch.cuda.synchronize()
    ref = snapshot(items)
    b = Batch(ctx, 32, 32 * 25)
    b.set_leaves([it["leaf"] for it in items])
    ms = b.autotune(2)
    assert ms > 0
    threads, persistent, xcd = b.schedule()
    assert threads in (64, 128, 256, 512)
    clear(items)
    b.launch()
    torch.cuda.synchronize()
    assert_same(snapshot(items), ref)
    b.close()


def test_batch_capacity_error(ctx):
    from paper_1802_06215_amd import Batch, HdxError
    items = build_instances(ctx, 4, 3)
    b = Batch(ctx, 2, 1000)
    with pytest.raises(HdxError) as e:
        b.set_leaves([it["leaf"] for it in items])
    assert e.value.code == -5
    b.close()


def test_rocksample_plans_match_single_leaf_calls(ctx):
    """RockSample leaves of every size class (terminal scenarios, a sense
    action before the leaf) in one batch: under the unsplit plan (all sizes
    in one dispatch, largest first, one wavefront or more per tile) and the
    split plan, every output, per-pair ones included, must equal one-leaf
    calls, and sampled leaves must match the oracle."""
    from paper_1802_06215_amd import Batch
    desc = W.rocksample_model(15, 15, 3)
    m = ctx.upload_model(desc)
    items = []
    for i, n in enumerate((500, 250, 125, 62, 31, 7, 1, 300, 499, 64, 65, 200)):
        lf = W.rocksample_leaf(desc, 500, n, 900 + i, p_term=0.1, depth=1 + (7 * i) % 40)
        # a sense action before the leaf exercises the update step's no-draw path
        if i % 3 == 0:
            lf["last_action"] = 5 + i % desc["m"]
        par_np = oracle.parent_states(desc, lf)
        par, pids = to_dev(par_np), ids_dev(lf["ids"])
        cfgs = cfg_pair(0, 1 << 30, 90)
        leaf, out, idx = gpu_leaf_desc(m, par, pids, lf["idx"], lf["depth"], lf["last_action"], 77 + i, 3,
                                       cfgs[1], True)
        items.append(dict(desc=desc, m=m, lf=lf, par_np=par_np, leaf=leaf, out=out, cfgs=cfgs,
                          keep=(par, pids, idx)))
    for it in items:  # one leaf per call: one tile per workgroup, no cache
        ctx.expand_leaf([it["leaf"]])
    torch.cuda.synchronize()
    ref = snapshot(items)
    b = Batch(ctx, len(items), len(items) * desc["n_actions"])
    b.set_leaves([it["leaf"] for it in items])
    torch.cuda.synchronize()
    for split, threads, persistent, xcd in ((False, 64, 0, 0), (False, 64, 0, 1), (False, 256, 0, 0),
                                            (False, 512, 2, 0), (True, 64, 0, 1), (True, 128, 1, 0)):
        print("plan split=%d schedule" % split, threads, persistent, xcd, flush=True)
        clear(items)
        for it in items:
            for t in (it["out"].r, it["out"].z, it["out"].U, it["out"].L):
                t.fill_(-3)
        b.set_split(split)
        b.set_schedule(threads, persistent, xcd)
        b.launch()
        torch.cuda.synchronize()
        got = snapshot(items)
        assert_same(got, ref)
        for x, y in zip(got, ref):
            for key in ("r", "U", "L"):
                assert np.array_equal(x[key].view(np.uint32), y[key].view(np.uint32)), key
            assert np.array_equal(x["z"], y["z"])
            assert np.array_equal(x["sprime"]["w"], y["sprime"]["w"])
    b.close()
    for it in items[::4]:
        lf = it["lf"]
        want = oracle.expand_leaf(desc, it["cfgs"][0], it["par_np"], lf["ids"].astype(np.uint32), lf["idx"],
                                  lf["depth"], lf["last_action"], it["leaf"].seed, 3, per_pair=True)
        compare_leaf(desc, collect(m, it["out"]), want, len(lf["idx"]))
