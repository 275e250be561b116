"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Sizes span several 64-scenario chunks and ragged tails, every model, the
paper's workload shapes (RockSample 7x7/8 rocks K=100, 15x15/15 rocks K=500
with horizon 90, crowd driving with 16 pedestrians K=500 and rollouts of 50
steps) and the degenerate cases (empty and one-scenario leaves, all-terminal
leaves, the largest leaf a tile takes)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import (assert_states_equal, cfg_pair, collect, compare_leaf, gpu_leaf_desc, host,
                      ids_dev, run_gpu_leaf, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1802_06215_amd import Context
    c = Context(0)
    yield c
    c.close()


def models(ctx, desc):
    return ctx.upload_model(desc)


def oracle_leaf(desc, ocfg, parent, pids, idx, depth, last_action, seed, step):
    return oracle.expand_leaf(desc, ocfg, parent, np.asarray(pids, np.uint32), idx, depth, last_action,
                              seed, step, per_pair=True)


def check_leaf(ctx, desc, parent, pids, idx, depth, last_action, seed, step, cfgs):
    m = models(ctx, desc)
    ocfg, hcfg = cfgs
    print("leaf: kind=%d n=%d depth=%d a=%d seed=%d" % (desc["kind"], len(idx), depth, last_action, seed),
          flush=True)
    gpu = run_gpu_leaf(ctx, m, parent, pids, idx, depth, last_action, seed, step, hcfg)
    ref = oracle_leaf(desc, ocfg, parent, pids, idx, depth, last_action, seed, step)
    compare_leaf(desc, gpu, ref, len(idx))
    return gpu, ref


def test_philox_matches_oracle(ctx):
    rng = np.random.default_rng(7)
    ctr = rng.integers(0, 2**32, size=(1 << 20, 4), dtype=np.uint64).astype(np.uint32)
    dev = torch.from_numpy(ctr.view(np.int32)).cuda()
    for key in [(0, 0), (123, 456), (0xFFFFFFFF, 0xFFFFFFFF)]:
        out = host(ctx.philox(dev, *key)).view(np.uint32)
        assert np.array_equal(out, oracle.philox(ctr, key))


@pytest.mark.parametrize("K", [1, 100, 500, 777])
def test_sample_scenarios_rocksample(ctx, K):
    desc = W.rocksample_model(15, 15, 2)
    b = W.rocksample_belief(desc, 0.5)
    b["p"] = np.linspace(0.0, 1.0, 15)
    m = models(ctx, desc)
    g = ctx.sample_scenarios(m, b, K, 9, 4)
    torch.cuda.synchronize()
    ref = oracle.sample_scenarios(desc, b, K, 9, 4)
    assert_states_equal({k: host(v) for k, v in g.items()}, ref)


@pytest.mark.parametrize("K", [1, 500, 1000])
def test_sample_scenarios_pednav(ctx, K):
    desc = W.pednav_model(16, 5, 3)
    gp = np.random.default_rng(1).dirichlet(np.ones(5), 16)
    b = W.pednav_belief(desc, gp, s=1.5, level=2)
    m = models(ctx, desc)
    g = ctx.sample_scenarios(m, b, K, 5, 1)
    torch.cuda.synchronize()
    ref = oracle.sample_scenarios(desc, b, K, 5, 1)
    assert_states_equal({k: host(v) for k, v in g.items()}, ref)


@pytest.mark.parametrize("model_seed", [1, 2, 3])
def test_rs7_root_parity_and_closed_form(ctx, model_seed):
    desc = W.rocksample_model(7, 8, model_seed)
    st = oracle.sample_scenarios(desc, W.rocksample_belief(desc), 100, model_seed, 0)
    ids = np.arange(100)
    gpu, ref = check_leaf(ctx, desc, st, ids, ids, 0, -1, model_seed, 0, cfg_pair(0, 30))
    for a in range(desc["n_actions"]):
        want = 10 * 0.95 ** 5 if a == 2 else 10 * 0.95 ** 6
        nc = gpu["n_children"][a]
        assert np.allclose(gpu["child_l0"][a, :nc], want, rtol=1e-6)
    assert int(gpu["steps"][:, 1].sum()) == 9000
    assert gpu["steps"].tolist() == [[100, 600] if a == 2 else [100, 700] for a in range(desc["n_actions"])]


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
@pytest.mark.parametrize("n_parent,n_leaf", [(100, 100), (100, 37), (130, 129), (65, 1)])
def test_rs7_corpus_leaves(ctx, seed, n_parent, n_leaf):
    desc = W.rocksample_model(7, 8, seed)
    lf = W.rocksample_leaf(desc, n_parent, n_leaf, seed, k_root=max(100, n_parent), p_term=0.05)
    check_leaf(ctx, desc, oracle.parent_states(desc, lf), lf["ids"], lf["idx"], lf["depth"],
               lf["last_action"], seed, 0, cfg_pair(0, 30))


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("n_leaf", [500, 333, 64])
def test_rs15_leaves_horizon_90(ctx, seed, n_leaf):
    desc = W.rocksample_model(15, 15, seed)
    lf = W.rocksample_leaf(desc, 500, n_leaf, seed, p_term=0.03, depth=int(seed * 27))
    check_leaf(ctx, desc, oracle.parent_states(desc, lf), lf["ids"], lf["idx"], lf["depth"],
               lf["last_action"], seed, 3, cfg_pair(0, 1 << 30, 90))


@pytest.mark.parametrize("seed", [1, 2])
def test_rs15_random_rollout_policy(ctx, seed):
    desc = W.rocksample_model(15, 15, seed)
    lf = W.rocksample_leaf(desc, 500, 500, seed, depth=5)
    check_leaf(ctx, desc, oracle.parent_states(desc, lf), lf["ids"], lf["idx"], lf["depth"],
               lf["last_action"], seed, 0, cfg_pair(2, 1 << 30, 90))


@pytest.mark.parametrize("seed", [1, 2])
def test_ped16_root(ctx, seed):
    desc = W.pednav_model(16, 5, seed)
    st = oracle.sample_scenarios(desc, W.pednav_belief(desc), 500, seed, 0)
    ids = np.arange(500)
    check_leaf(ctx, desc, st, ids, ids, 0, -1, seed, 0, cfg_pair(0, 50))


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("n_parent,n_leaf", [(500, 500), (500, 211), (90, 17)])
def test_ped16_corpus_leaves(ctx, seed, n_parent, n_leaf):
    desc = W.pednav_model(16, 5, seed)
    lf = W.pednav_leaf(desc, n_parent, n_leaf, seed, k_root=500, p_term=0.05)
    check_leaf(ctx, desc, oracle.parent_states(desc, lf), lf["ids"], lf["idx"], lf["depth"],
               lf["last_action"], seed, 2, cfg_pair(0, 50))


@pytest.mark.parametrize("n_peds", [0, 1, 6, 12, 20, 32])
def test_ped_pedestrian_counts(ctx, n_peds):
    desc = W.pednav_model(n_peds, 5, 4)
    lf = W.pednav_leaf(desc, 200, 150, 4, p_term=0.05)
    check_leaf(ctx, desc, oracle.parent_states(desc, lf), lf["ids"], lf["idx"], lf["depth"],
               lf["last_action"], 4, 0, cfg_pair(0, 20))


def test_ped_maintain_policy(ctx):
    desc = W.pednav_model(16, 5, 5)
    lf = W.pednav_leaf(desc, 300, 300, 5)
    check_leaf(ctx, desc, oracle.parent_states(desc, lf), lf["ids"], lf["idx"], lf["depth"],
               lf["last_action"], 5, 0, cfg_pair(1, 50, -1, 1))


def test_empty_single_and_terminal_leaves(ctx):
    desc = W.rocksample_model(7, 8, 1)
    lf = W.rocksample_leaf(desc, 100, 100, 1)
    par = oracle.parent_states(desc, lf)
    for idx in (np.array([], np.int32), np.array([42], np.int32)):
        check_leaf(ctx, desc, par, lf["ids"], idx, 3, 2, 1, 0, cfg_pair(0, 30))
    lf_t = W.rocksample_leaf(desc, 100, 100, 2, p_term=1.0)
    check_leaf(ctx, desc, oracle.parent_states(desc, lf_t), lf_t["ids"], lf_t["idx"], 4, -1, 2, 0,
               cfg_pair(0, 30))
    dp = W.pednav_model(16, 5, 1)
    lp = W.pednav_leaf(dp, 100, 100, 3, p_term=1.0)
    check_leaf(ctx, dp, oracle.parent_states(dp, lp), lp["ids"], lp["idx"], 4, -1, 2, 0,
               cfg_pair(0, 50))


@pytest.mark.parametrize("kind", [0, 1])
def test_largest_leaf(ctx, kind):
    # 2048 scenarios: the crowd-driving case has more distinct observations
    # than the chunk table holds and takes the LDS bitonic path
    if kind == 0:
        desc = W.rocksample_model(20, 20, 6)
        lf = W.rocksample_leaf(desc, 2048, 2048, 6, k_root=4096)
        cfgs = cfg_pair(0, 1 << 30, 90)
    else:
        desc = W.pednav_model(16, 5, 6)
        lf = W.pednav_leaf(desc, 2048, 2048, 6, k_root=4096)
        cfgs = cfg_pair(0, 10)
    check_leaf(ctx, desc, oracle.parent_states(desc, lf), lf["ids"], lf["idx"], lf["depth"],
               lf["last_action"], 6, 0, cfgs)


def test_rollout_bounds_parity(ctx):
    from paper_1802_06215_amd import hdx as H
    for desc, lf, cfgs in [
        (W.rocksample_model(15, 15, 1), None, cfg_pair(2, 1 << 30, 90)),
        (W.pednav_model(16, 5, 1), None, cfg_pair(0, 50)),
    ]:
        if desc["kind"] == 0:
            lf = W.rocksample_leaf(desc, 1000, 10, 3)
        else:
            lf = W.pednav_leaf(desc, 1000, 10, 3)
        st = oracle.parent_states(desc, lf)
        depths = np.random.default_rng(0).integers(0, 60, 1000).astype(np.int32)
        U, L, steps, Labs = oracle.rollout_bounds(desc, cfgs[0], st, lf["ids"], depths, 8, 1, with_abs=True)
        m = models(ctx, desc)
        gU, gL, gs = ctx.rollout_bounds(m, cfgs[1], to_dev(st), ids_dev(lf["ids"]),
                                        torch.from_numpy(depths).cuda(), 8, 1)
        torch.cuda.synchronize()
        assert np.array_equal(host(gs), steps)
        from gpu_util import close
        close(host(gU), U, 0.0, "U")
        close(host(gL), L, Labs, "L")


def test_batched_mixed_instances_equal_single_launches(ctx):
    # independent planner instances of uneven size in one launch: every
    # output is bit-identical to expanding each leaf on its own
    from paper_1802_06215_amd import hdx as H
    inst = W.mixed_instances(24, 42)
    leaves, outs, keep = [], [], []
    singles = []
    for i, it in enumerate(inst):
        desc, K = it["model"], it["K"]
        m = models(ctx, desc)
        if desc["kind"] == 0:
            lf = W.rocksample_leaf(desc, K, K - i % 7, i)
            cfgs = cfg_pair(0, 1 << 30, 90)
        else:
            lf = W.pednav_leaf(desc, K, K - i % 7, i)
            cfgs = cfg_pair(0, 50)
        par = to_dev(oracle.parent_states(desc, lf))
        pids = ids_dev(lf["ids"])
        leaf, out, idx = gpu_leaf_desc(m, par, pids, lf["idx"], lf["depth"], lf["last_action"], i, 0,
                                       cfgs[1])
        leaves.append(leaf)
        outs.append((m, out))
        keep += [par, pids, idx]
        g1 = run_gpu_leaf(ctx, m, oracle.parent_states(desc, lf), lf["ids"], lf["idx"], lf["depth"],
                          lf["last_action"], i, 0, cfgs[1])
        singles.append(g1)
    ctx.expand_leaf(leaves)
    torch.cuda.synchronize()
    for (m, out), g1 in zip(outs, singles):
        gb = collect(m, out)
        for key in ("n_children", "perm", "steps", "ids", "r", "z", "child_of"):
            assert np.array_equal(gb[key], g1[key]), key
        for key in ("r_mean", "U", "L"):
            assert np.array_equal(gb[key].view(np.uint32), g1[key].view(np.uint32)), key
        for a, nc in enumerate(g1["n_children"]):
            for key in ("child_z", "child_n", "child_off", "child_u0", "child_l0"):
                x, y = gb[key][a, :nc], g1[key][a, :nc]
                assert np.array_equal(x.view(np.uint32) if x.dtype == np.float32 else x,
                                      y.view(np.uint32) if y.dtype == np.float32 else y), key
        assert_states_equal(gb["states"], g1["states"])
        assert_states_equal(gb["sprime"], g1["sprime"])


def test_repeat_runs_are_bit_identical(ctx):
    desc = W.pednav_model(16, 5, 9)
    lf = W.pednav_leaf(desc, 500, 500, 9)
    m = models(ctx, desc)
    ocfg, hcfg = cfg_pair(0, 50)
    a = run_gpu_leaf(ctx, m, oracle.parent_states(desc, lf), lf["ids"], lf["idx"], lf["depth"],
                     lf["last_action"], 9, 0, hcfg)
    b = run_gpu_leaf(ctx, m, oracle.parent_states(desc, lf), lf["ids"], lf["idx"], lf["depth"],
                     lf["last_action"], 9, 0, hcfg)
    for k in ("child_u0", "child_l0", "r_mean", "perm", "child_z"):
        assert np.array_equal(a[k], b[k]), k


def test_argument_errors(ctx):
    from paper_1802_06215_amd import hdx as H
    desc = W.rocksample_model(7, 8, 1)
    m = models(ctx, desc)
    lf = W.rocksample_leaf(desc, 100, 100, 1)
    par = to_dev(oracle.parent_states(desc, lf))
    pids = ids_dev(lf["ids"])
    leaf, out, idx = gpu_leaf_desc(m, par, pids, lf["idx"], 3, 1, 1, 0, H.rollout_cfg(0, 30))
    leaf.cap = 2  # RockSample needs 3 child slots per action
    with pytest.raises(H.HdxError) as e:
        ctx.expand_leaf([leaf])
    assert e.value.code == -5
    leaf.cap = 3
    leaf.n = 2049
    with pytest.raises(H.HdxError) as e:
        ctx.expand_leaf([leaf])
    assert e.value.code == -4
    leaf.n = 100
    leaf.last_action = 13
    with pytest.raises(H.HdxError) as e:
        ctx.expand_leaf([leaf])
    assert e.value.code == -1
    leaf.last_action = 1
    leaf.rollout = H.rollout_cfg(0, 5000)
    with pytest.raises(H.HdxError) as e:
        ctx.expand_leaf([leaf])
    assert e.value.code == -4


def test_fp32_rounding_selftest(ctx):
    # sqrt and division correctly rounded, products and sums rounded
    # separately (no fused multiply-add), denormals kept: numpy's float32
    # arithmetic is the IEEE-754 reference
    from paper_1802_06215_amd import hdx as H
    rng = np.random.default_rng(11)
    n = 1 << 20
    a = (rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))).astype(np.float32)
    b = (rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))).astype(np.float32)
    c = (rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))).astype(np.float32)
    a[:1000] = (np.arange(1000) * np.float32(1e-42)).astype(np.float32)  # denormals
    b[b == 0] = 1.0
    dev = [torch.from_numpy(v).cuda() for v in (a, b, c)]
    out = host(H.fp32_selftest(ctx, *dev))
    with np.errstate(all="ignore"):
        want = [np.sqrt(np.abs(a)), a / b, a * b + c, np.floor(a)]
    for i, w in enumerate(want):
        assert np.array_equal(out[i].view(np.uint32), w.astype(np.float32).view(np.uint32)), i


@pytest.mark.parametrize("which", ["rs", "ped", "mars", "nav"])
def test_expand_out_bytes_covers_the_required_outputs(ctx, which):
    from paper_1802_06215_amd import hdx as H
    desc = dict(rs=lambda: W.rocksample_model(15, 15, 1), ped=lambda: W.pednav_model(16, 5, 1),
                mars=lambda: W.mars_model(11, 11, 1), nav=lambda: W.nav_model(1))[which]()
    m = ctx.upload_model(desc)
    r = lambda b: (b + 255) // 256 * 256
    for K in (1, 100, 500, 2048):
        out = H.LeafBuffers(m, K)
        tensors = list(out.states.values()) + [out.ids, out.perm, out.n_children, out.child_z, out.child_n,
                                               out.child_off, out.child_u0, out.child_l0, out.r_mean, out.steps]
        want = sum(r(t.numel() * t.element_size()) for t in tensors)
        assert m.out_bytes(K) == want, (which, K)
        assert m.out_bytes(K, 7) == 7 * want
    assert m.out_bytes(-1) == 0
