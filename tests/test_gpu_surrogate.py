"""GPU tests of leaf expansion with the surrogate in place of the rollouts.

Everything but the lower bounds must equal the plain expansion and the
oracle bit for bit (states, groupings, rewards, observations, upper bounds);
no rollout steps are taken; the per-scenario value is the MLP at the
features of the stepped state (depth + 1), matched against the FP64
reference of the network fed the same BF16 weights and features (2e-2 of
the output scale); each child's l0 is the mean of its scenarios' values
(1e-5 relative)."""
import time

import numpy as np
import pytest
import torch

import bench
import oracle
import workloads as W
from gpu_util import cfg_pair, collect, gpu_leaf_desc, ids_dev, to_dev, assert_states_equal, bits
from oracle import mlp as ref

pytestmark = pytest.mark.gpu

HORIZON = 90


@pytest.fixture(scope="module")
def ctx():
    from paper_1802_06215_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def net(ctx):
    from paper_1802_06215_amd import Mlp
    m = Mlp(ctx, seed=11)
    yield m
    m.close()


def reference_values(desc, net, sprime, depth):
    """MLP(features(s')) over every (action, scenario), FP64 with BF16 weights."""
    A = desc["n_actions"]
    if desc["kind"] == W.ROCKSAMPLE:
        n = sprime["w"].shape[1]
        f = ref.rocksample_features(desc, sprime["w"].reshape(-1), np.full(A * n, depth + 1), HORIZON)
    else:
        n = sprime["s"].shape[1]
        st = dict(s=sprime["s"].reshape(-1), car=sprime["car"].reshape(-1),
                  px=sprime["px"].reshape(-1, A * n), py=sprime["py"].reshape(-1, A * n),
                  goal=sprime["goal"].reshape(-1, A * n))
        f = ref.pednav_features(desc, st, np.full(A * n, depth + 1), HORIZON)
    w = ref.unpack(net.params().astype(np.float64))
    for k in ("W1", "W2", "W3", "w4"):
        w[k] = ref.bf16_round(w[k].astype(np.float32)).astype(np.float64)
    return ref.forward(ref.pack(w), ref.bf16_round(f), bf16=True).reshape(A, n)


def run_surrogate(ctx, net, m, lf, seed, step, hcfg):
    parent = to_dev(oracle.parent_states(m.desc, lf))
    pids = ids_dev(lf["ids"])
    leaf, out, keep = gpu_leaf_desc(m, parent, pids, lf["idx"], lf["depth"], lf["last_action"], seed, step, hcfg)
    ctx.expand_leaf_surrogate([leaf], net, HORIZON)
    torch.cuda.synchronize()
    return collect(m, out), out


def check(ctx, net, desc, lf, seed, step, cfgs):
    ocfg, hcfg = cfgs
    m = ctx.upload_model(desc)
    n = len(lf["idx"])
    print("surrogate leaf: kind=%d n=%d depth=%d seed=%d" % (desc["kind"], n, lf["depth"], seed), flush=True)
    gpu, out = run_surrogate(ctx, net, m, lf, seed, step, hcfg)
    want = oracle.expand_leaf(desc, ocfg, oracle.parent_states(desc, lf), np.asarray(lf["ids"], np.uint32),
                              lf["idx"], lf["depth"], lf["last_action"], seed, step, per_pair=True)
    A = desc["n_actions"]
    assert_states_equal(gpu["states"], want["states"])
    assert_states_equal(gpu["sprime"], want["sprime"])
    for f in ("n_children", "perm", "child_of"):
        assert np.array_equal(gpu[f], want[f]), f
    assert np.array_equal(bits(gpu["r"]), bits(want["r"]))
    assert np.array_equal(gpu["z"], want["z"])
    assert np.array_equal(gpu["steps"][:, 0], want["steps"][:, 0])
    assert np.all(gpu["steps"][:, 1] == 0)
    if n:
        # the forward that forms features from the states equals the features
        # kernel followed by the forward, bit for bit
        from paper_1802_06215_amd import hdx as H
        sp = {k: v[..., :A * n].contiguous() for k, v in out.sprime.items()}
        depths = torch.full((A * n,), lf["depth"] + 1, dtype=torch.int32, device="cuda")
        y = net.forward(H.features(ctx, m, sp, depths, HORIZON))
        assert np.array_equal(bits(gpu["L"].reshape(-1)), bits(y.cpu().numpy()))
    vals = reference_values(desc, net, want["sprime"], lf["depth"])
    scale = (np.abs(vals).mean() if n else 0.0) + 1e-3
    err = np.max(np.abs(gpu["L"] - vals)) if n else 0.0
    assert err <= 2e-2 * scale + 1e-3, (err, scale)
    for a in range(A):
        nc = int(want["n_children"][a])
        for f in ("child_z", "child_n", "child_off"):
            assert np.array_equal(gpu[f][a, :nc], want[f][a, :nc]), (f, a)
        assert np.allclose(gpu["child_u0"][a, :nc], want["child_u0"][a, :nc], rtol=1e-5, atol=0)
        for c in range(nc):
            off, cnt = want["child_off"][a, c], want["child_n"][a, c]
            seg = want["perm"][a, off:off + cnt]
            mean = gpu["L"][a, seg].astype(np.float64).mean()
            tol = 1e-5 * max(abs(mean), np.abs(gpu["L"][a, seg]).mean()) + 1e-30
            assert abs(gpu["child_l0"][a, c] - mean) <= tol, (a, c, gpu["child_l0"][a, c], mean)
    return gpu


@pytest.mark.parametrize("n_leaf", [1, 63, 500, 777])
def test_surrogate_expansion_rocksample(ctx, net, n_leaf):
    desc = W.rocksample_model(15, 15, 2)
    lf = W.rocksample_leaf(desc, max(n_leaf, 500), n_leaf, 4, p_term=0.05, depth=7)
    check(ctx, net, desc, lf, 4, 1, cfg_pair(0, 1 << 30, HORIZON))


@pytest.mark.parametrize("n_peds", [0, 6, 16, 32])
def test_surrogate_expansion_pednav(ctx, net, n_peds):
    desc = W.pednav_model(n_peds, 5, 3)
    lf = W.pednav_leaf(desc, 500, 300, 6, p_term=0.05)
    check(ctx, net, desc, lf, 6, 2, cfg_pair(0, 50))


def test_surrogate_empty_leaf(ctx, net):
    desc = W.rocksample_model(7, 8, 1)
    lf = W.rocksample_leaf(desc, 100, 0, 1)
    gpu = check(ctx, net, desc, lf, 1, 0, cfg_pair(0, 30))
    assert np.all(gpu["n_children"] == 0)


def test_surrogate_batch_matches_single_calls(ctx, net):
    """Several leaves (both models, one empty) in one call give the same
    bits as one call per leaf: a row's MLP value does not depend on its
    neighbours."""
    from paper_1802_06215_amd import hdx as H
    specs = [(W.rocksample_model(15, 15, 2), 400), (W.pednav_model(16, 5, 3), 250),
             (W.rocksample_model(7, 8, 1), 0), (W.rocksample_model(11, 11, 1), 130)]
    leaves, outs, keep = [], [], []
    singles = []
    for i, (desc, n) in enumerate(specs):
        m = ctx.upload_model(desc)
        gen = W.rocksample_leaf if desc["kind"] == W.ROCKSAMPLE else W.pednav_leaf
        lf = gen(desc, 500, n, 10 + i, p_term=0.05)
        hcfg = H.rollout_cfg(0, 1 << 30, HORIZON)
        singles.append(run_surrogate(ctx, net, m, lf, 10 + i, 3, hcfg)[0])
        parent = to_dev(oracle.parent_states(desc, lf))
        pids = ids_dev(lf["ids"])
        leaf, out, k = gpu_leaf_desc(m, parent, pids, lf["idx"], lf["depth"], lf["last_action"], 10 + i, 3, hcfg)
        leaves.append(leaf)
        outs.append((m, out))
        keep += [parent, pids, k]
    ctx.expand_leaf_surrogate(leaves, net, HORIZON)
    torch.cuda.synchronize()
    for (m, out), one in zip(outs, singles):
        got = collect(m, out)
        assert np.array_equal(got["n_children"], one["n_children"])
        assert np.array_equal(got["perm"], one["perm"])
        assert np.array_equal(bits(got["L"]), bits(one["L"]))
        for a, nc in enumerate(one["n_children"]):
            for f in ("child_n", "child_off", "child_z", "child_l0", "child_u0"):
                assert np.array_equal(bits(got[f][a, :nc]), bits(one[f][a, :nc])), (f, a)


def expand_with_rollouts(ctx, m, desc, leaves_spec, hcfg):
    """Expand leaves with full rollouts and per-pair outputs (one call)."""
    from paper_1802_06215_amd import hdx as H
    descs, outs, keep = [], [], []
    for seed, n, depth in leaves_spec:
        lf = W.rocksample_leaf(desc, 500, n, seed, depth=depth)
        par = H.rocksample_states(lf["x"], lf["y"], lf["rocks"], lf["term"])
        pids = torch.from_numpy(lf["ids"].astype(np.int32)).cuda()
        idx = H.positions(lf["idx"])
        out = H.LeafBuffers(m, n, per_pair=True)
        descs.append(H.make_leaf(m, par, pids, idx, lf["depth"], lf["last_action"], out, seed, 0, hcfg))
        outs.append((out, lf["depth"]))
        keep += [par, pids, idx]
    ctx.expand_leaf(descs)
    torch.cuda.synchronize()
    return descs, outs, keep


def test_surrogate_training_beats_constant(ctx):
    """Fit the surrogate to random-policy depth-90 RockSample 15x15 rollout
    values and check it generalises to held-out leaves: pair-level error
    below the targets' variance and child-level l0 closer to the rollout
    l0 than the best constant."""
    from paper_1802_06215_amd import Mlp, hdx as H
    from paper_1802_06215_amd import surrogate as S
    desc = W.rocksample_model(15, 15, 1)
    m = ctx.upload_model(desc)
    hcfg = H.rollout_cfg(H.POLICY_RANDOM, 1 << 30, HORIZON)
    # many small leaves: the value depends on the robot's cell, the rocks
    # and the remaining depth, so breadth over leaves is what generalises
    spec = [(2000 + i, 100, 1 + (7 * i) % 60) for i in range(640)]
    _, outs, keep = expand_with_rollouts(ctx, m, desc, spec, hcfg)
    Xs, ts = zip(*(S.leaf_pairs(ctx, m, o, d, HORIZON) for o, d in outs))
    X, t = torch.cat(Xs), torch.cat(ts)
    print("training pairs %d, target mean %.4f var %.4f" % (len(t), float(t.mean()), float(t.var())), flush=True)
    net = Mlp(ctx, seed=2)
    t0 = time.perf_counter()
    hist = S.fit(net, X, t, epochs=3, batch=4096, lr=1e-3)
    torch.cuda.synchronize()
    print("fit: %.2f s" % (time.perf_counter() - t0), flush=True)
    print("epoch losses", ["%.4f" % h for h in hist], flush=True)
    assert hist[-1] < hist[0]
    # held-out leaves
    spec = [(9000 + i, 500 >> (i % 3), 1 + (11 * i) % 60) for i in range(24)]
    descs, outs, keep2 = expand_with_rollouts(ctx, m, desc, spec, hcfg)
    Xh, th = zip(*(S.leaf_pairs(ctx, m, o, d, HORIZON) for o, d in outs))
    Xh, th = torch.cat(Xh), torch.cat(th)
    mse = float(((net.forward(Xh) - th) ** 2).mean())
    var = float(th.var())
    print("held-out pair mse %.4f vs target variance %.4f" % (mse, var), flush=True)
    assert mse < var
    full = [out.child_l0.cpu().numpy().copy() for out, _ in outs]
    nch = [out.n_children.cpu().numpy().copy() for out, _ in outs]
    ctx.expand_leaf_surrogate(descs, net, HORIZON)
    torch.cuda.synchronize()
    e_sur, e_const = [], []
    vals = np.concatenate([f[a, :nc[a]] for f, nc in zip(full, nch) for a in range(len(nc))])
    c = vals.mean()
    for (out, _), f, nc in zip(outs, full, nch):
        sur = out.child_l0.cpu().numpy()
        for a in range(len(nc)):
            e_sur.append(np.abs(sur[a, :nc[a]] - f[a, :nc[a]]))
            e_const.append(np.abs(c - f[a, :nc[a]]))
    e_sur, e_const = np.concatenate(e_sur).mean(), np.concatenate(e_const).mean()
    print("child l0 mean abs error: surrogate %.4f, constant %.4f" % (e_sur, e_const), flush=True)
    assert e_sur < e_const
    net.close()


@pytest.mark.parametrize("threads,batch", [(4, 0), (8, 8)])
def test_search_with_surrogate(ctx, net, threads, batch):
    from paper_1802_06215_amd import hdx as H
    desc = W.rocksample_model(15, 15, 1)
    m = ctx.upload_model(desc)
    b = W.rocksample_belief(desc)
    print("search: threads=%d batch=%d" % (threads, batch), flush=True)
    r = ctx.search(m, b, K=500, n_threads=threads, batch_leaves=batch, time_budget_s=0.3, max_depth=HORIZON,
                   rollout=H.rollout_cfg(H.POLICY_RANDOM, 1 << 30, HORIZON), surrogate=net,
                   surrogate_horizon=HORIZON, seed=5, arena_bytes=2 << 30)
    print(r["trials"], r["expansions"], r["l_root"], r["u_root"], flush=True)
    assert r["expansions"] > 0 and r["trials"] >= r["expansions"]
    assert 0 <= r["best_action"] < desc["n_actions"]
    assert np.isfinite(r["l_root"]) and np.isfinite(r["u_root"])


@pytest.mark.parametrize("threads,batch", [(4, 0), (8, 8)])
def test_search_surrogate_judge_and_fallback(ctx, net, threads, batch):
    """Every 4th surrogate expansion is judged against rollouts; with a zero
    error bound the monitor never switches, with a tiny one it falls back to
    rollouts once 8 leaves are judged."""
    from paper_1802_06215_amd import hdx as H
    desc = W.rocksample_model(15, 15, 1)
    m = ctx.upload_model(desc)
    b = W.rocksample_belief(desc)
    common = dict(K=500, n_threads=threads, batch_leaves=batch, time_budget_s=0.3, max_depth=HORIZON,
                  rollout=H.rollout_cfg(H.POLICY_RANDOM, 1 << 30, HORIZON), surrogate=net,
                  surrogate_horizon=HORIZON, surrogate_judge_every=4, seed=5, arena_bytes=2 << 30)
    print("judge: threads=%d batch=%d" % (threads, batch), flush=True)
    r = ctx.search(m, b, surrogate_max_rel_err=0.0, **common)
    print(r["judged_leaves"], r["judged_children"], r["judge_mae"], r["judge_rel_err"], flush=True)
    assert r["judged_leaves"] > 0 and r["judged_children"] >= r["judged_leaves"]
    assert r["surrogate_off"] == 0
    assert np.isfinite(r["judge_mae"]) and r["judge_rel_err"] >= 0
    r = ctx.search(m, b, surrogate_max_rel_err=1e-12, **common)
    print(r["judged_leaves"], r["judge_rel_err"], r["surrogate_off"], flush=True)
    assert r["judged_leaves"] >= 8
    assert r["surrogate_off"] == (1 if r["judge_rel_err"] > 1e-12 else 0)
    # bias correction: the judged children's mean signed difference, bounded
    # by their mean absolute one; the tree's bounds stay ordered
    r = ctx.search(m, b, surrogate_bias_correct=True, **common)
    print("bias", r["judged_leaves"], r["judge_bias"], r["judge_mae"], flush=True)
    assert r["judged_leaves"] > 0 and np.isfinite(r["judge_bias"])
    assert abs(r["judge_bias"]) <= r["judge_mae"] + 1e-12
    assert r["l_root"] <= r["u_root"] + 1e-4 * max(1.0, abs(r["u_root"]))


def _oracle_two_level_root(desc, ocfg, root_np, K, key):
    """Root lower bound of the two-level tree, every node expanded by the
    oracle (FP64) and backed up by the oracle's Eq. 4."""
    ids = np.arange(K, dtype=np.uint32)
    res0 = oracle.expand_leaf(desc, ocfg, root_np, ids, np.arange(K, dtype=np.int32), 0, -1, key, 0)
    root = oracle.Node(None, K, 0.0, 0.0)
    oracle.attach_children(desc, root, res0)
    for a in range(desc["n_actions"]):
        for c in range(int(res0["n_children"][a])):
            off, n = int(res0["child_off"][a, c]), int(res0["child_n"][a, c])
            res = oracle.expand_leaf(desc, ocfg, root_np, ids, res0["perm"][a, off:off + n], 1, a, key, 0)
            node = root.actions[a][1][c]
            oracle.attach_children(desc, node, res)
            oracle.backup(node, desc["gamma"])
    return root.l


def test_same_tree_root_values_match_oracle(ctx, net):
    """The plain-rollout root value of the two-level comparison tree equals
    the oracle's tree built from its own expansions (1e-5 relative); the
    reference and surrogate variants are finite; the frontier holds every
    (action, scenario) pair of every depth-1 node."""
    from paper_1802_06215_amd import hdx as H
    desc = W.rocksample_model(7, 8, 1)
    m = ctx.upload_model(desc)
    K = 48
    cfg = H.rollout_cfg(H.POLICY_RANDOM, 1 << 30, 30)
    for key in (1, 2):
        root = ctx.sample_scenarios(m, W.rocksample_belief(desc), K, 10 + key, 0)
        torch.cuda.synchronize()
        root_np = dict(w=root["w"].cpu().numpy().astype(np.int32))
        got = bench.root_values_same_tree(ctx, m, desc["gamma"], root, K, cfg, key, net, 30, ref_keys=2)
        want = _oracle_two_level_root(desc, oracle.cfg(2, 1 << 30, 30), root_np, K, key)
        print("key", key, got, want, flush=True)
        assert abs(got["rollout"] - want) <= 1e-5 * max(1.0, abs(want)), (got["rollout"], want)
        assert np.isfinite(got["reference"]) and np.isfinite(got["surrogate"])
        # every depth-1 node holds a share of the K scenarios per action
        assert got["frontier_pairs"] == desc["n_actions"] * desc["n_actions"] * K


def test_planner_pairs_first_level(ctx):
    """Training pairs from planner trees: the first level is the root's
    expansion, rows a*K + k in order; its targets are the mean of the
    rollout values under the reference keys, recomputed here from an
    independent expansion of the same root."""
    from paper_1802_06215_amd import hdx as H, surrogate as S
    desc = W.rocksample_model(7, 8, 1)
    m = ctx.upload_model(desc)
    K, A, R = 64, desc["n_actions"], 3
    cfg = H.rollout_cfg(H.POLICY_RANDOM, 1 << 30, 30)
    root_of = lambda sd: ctx.sample_scenarios(m, W.rocksample_belief(desc), K, sd, 0)
    X, t = S.planner_pairs(ctx, m, root_of, K, cfg, [5], levels=3, nodes_per_level=4, horizon=30, ref_keys=R,
                           ref_seed=777)
    assert X.shape[1] == 64 and X.shape[0] == t.shape[0] and X.shape[0] > A * K
    assert torch.isfinite(t).all()
    root = root_of(5)
    out = H.LeafBuffers(m, K, per_pair=True)
    ids = torch.arange(K, dtype=torch.int32, device="cuda")
    ctx.expand_leaf([H.make_leaf(m, root, ids, H.positions(np.arange(K)), 0, -1, out, 5, 0, cfg)])
    sp = {k: v[..., :A * K].contiguous() for k, v in out.sprime.items()}
    fids = out.ids[:K].repeat(A)
    depths = torch.ones(A * K, dtype=torch.int32, device="cuda")
    acc = torch.zeros(A * K, dtype=torch.float64, device="cuda")
    for r in range(R):
        _, L, _ = ctx.rollout_bounds(m, cfg, sp, fids, depths, 777 + 1000 * 5 + r, 0)
        acc += L.double()
    assert torch.equal(t[:A * K], (acc / R).float())
    assert torch.equal(X[:A * K], H.features(ctx, m, sp, depths, 30))


def _keyed_leaves(ctx, m, desc, spec, hcfg):
    """Leaves of `spec` with per-pair outputs, and a function that re-keys
    them: the same leaves and buffers under another random-number key."""
    from paper_1802_06215_amd import hdx as H
    built = []
    for seed, n, depth in spec:
        lf = W.rocksample_leaf(desc, 500, n, seed, depth=depth)
        par = H.rocksample_states(lf["x"], lf["y"], lf["rocks"], lf["term"])
        pids = torch.from_numpy(lf["ids"].astype(np.int32)).cuda()
        idx = H.positions(lf["idx"])
        out = H.LeafBuffers(m, n, per_pair=True)
        built.append((par, pids, idx, lf, out))

    def keyed(key=None):
        return [H.make_leaf(m, par, pids, idx, lf["depth"], lf["last_action"], out,
                            lf_seed if key is None else key, 0, hcfg)
                for (par, pids, idx, lf, out), (lf_seed, _, _) in zip(built, spec)]
    return built, keyed


def test_surrogate_gains_over_single_rollouts(ctx):
    """What the trained network gains over the method without it (plain
    default-policy rollouts in Eq. 13), RockSample 15x15 with uniform-random
    rollouts of depth 90.  On held-out leaves of 31 and 62 scenarios with
    fixed keys, each child's l0 from the surrogate is closer to the child's
    value -- the mean over 16 independent rollouts per (action, scenario)
    pair -- than the l0 from the single rollouts it replaces; and at equal
    planning time the search with the surrogate completes more trials per
    second."""
    from paper_1802_06215_amd import Mlp, hdx as H
    from paper_1802_06215_amd import surrogate as S
    desc = W.rocksample_model(15, 15, 1)
    m = ctx.upload_model(desc)
    hcfg = H.rollout_cfg(H.POLICY_RANDOM, 1 << 30, HORIZON)
    # training pairs: stepped states of synthetic leaves, each target the mean
    # of 4 rollouts (the stepped states do not depend on the key)
    spec = [(3000 + i, 100, 1 + (7 * i) % 60) for i in range(640)]
    built, keyed = _keyed_leaves(ctx, m, desc, spec, hcfg)
    ctx.expand_leaf(keyed())
    torch.cuda.synchronize()
    X = torch.cat([S.leaf_pairs(ctx, m, out, lf["depth"], HORIZON)[0] for _, _, _, lf, out in built])
    acc = [torch.zeros_like(out.L[:, :out.n]) for *_, out in built]
    for r in range(4):
        ctx.expand_leaf(keyed(600000 + r))
        for a_, (*_, out) in zip(acc, built):
            a_ += out.L[:, :out.n]
    t = torch.cat([(a_ / 4).reshape(-1) for a_ in acc])
    net = Mlp(ctx, seed=3)
    hist = S.fit(net, X, t, epochs=8, batch=4096, lr=2e-3, lr_final=2e-4)
    torch.cuda.synchronize()
    print("gain: %d training pairs, epoch losses %s" % (len(t), ["%.4f" % h for h in hist]), flush=True)
    del built, keyed, X, t, acc

    # held-out leaves of the sizes a search expands below its root (62 and 31
    # scenarios: a sense splits a node's scenarios between two readings); the
    # reference value of a pair is its mean over 16 keys
    spec = [(9100 + i, (62, 31)[i % 2], 1 + (13 * i) % 60) for i in range(64)]
    built, keyed = _keyed_leaves(ctx, m, desc, spec, hcfg)
    ctx.expand_leaf(keyed())
    torch.cuda.synchronize()
    one = [dict(l0=out.child_l0.cpu().numpy().copy(), nc=out.n_children.cpu().numpy().copy(),
                off=out.child_off.cpu().numpy().copy(), cn=out.child_n.cpu().numpy().copy(),
                perm=out.perm.cpu().numpy()[:, :out.n].astype(np.int64)) for *_, out in built]
    ref_sum = [torch.zeros_like(out.L[:, :out.n], dtype=torch.float64) for *_, out in built]
    for r in range(16):
        ctx.expand_leaf(keyed(800000 + r))
        for a_, (*_, out) in zip(ref_sum, built):
            a_ += out.L[:, :out.n].double()
    ctx.expand_leaf_surrogate(keyed(), net, HORIZON)  # the first key's grouping again
    torch.cuda.synchronize()
    e_one, e_sur = [], []
    for h, a_, (*_, out) in zip(one, ref_sum, built):
        truth = (a_ / 16).cpu().numpy()
        sur = out.child_l0.cpu().numpy()
        assert np.array_equal(out.n_children.cpu().numpy(), h["nc"])
        for a in range(len(h["nc"])):
            for c in range(h["nc"][a]):
                v = truth[a, h["perm"][a, h["off"][a, c]:h["off"][a, c] + h["cn"][a, c]]].mean()
                e_one.append(abs(h["l0"][a, c] - v))
                e_sur.append(abs(sur[a, c] - v))
    e_one, e_sur = float(np.mean(e_one)), float(np.mean(e_sur))
    print("gain: child l0 mean abs error vs the 16-rollout mean: surrogate %.4f, one rollout %.4f (%d children)"
          % (e_sur, e_one, sum(int(h["nc"].sum()) for h in one)), flush=True)
    assert e_sur < e_one

    # equal planning time: trials per second with each source of leaf values
    b = W.rocksample_belief(desc)
    common = dict(K=500, n_threads=8, batch_leaves=8, time_budget_s=0.5, max_depth=HORIZON, rollout=hcfg,
                  arena_bytes=4 << 30)
    rate = {"rollouts": [], "surrogate": []}
    for key in (21, 22):
        r = ctx.search(m, b, seed=key, **common)
        rate["rollouts"].append(r["trials"] / r["elapsed_s"])
        r = ctx.search(m, b, seed=key, surrogate=net, surrogate_horizon=HORIZON, **common)
        rate["surrogate"].append(r["trials"] / r["elapsed_s"])
    print("gain: trials/s rollouts %s, surrogate %s" % (rate["rollouts"], rate["surrogate"]), flush=True)
    assert sum(rate["surrogate"]) > sum(rate["rollouts"])
    net.close()
