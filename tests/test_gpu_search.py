"""GPU tests of the parallel DESPOT search driver (hdx_search).

* Closed form: with no rocks and no rollouts the search must discover the
  exit value 10 gamma^(n-1-x) through expansions and Eq. 4 backups alone,
  and pick "east".
* Bounds: the upper-bound heuristic is consistent and the rollouts share the
  scenarios' random numbers with the expansion, so backed-up bounds stay
  inside the initial ones: l0 <= l <= u <= u0 at the root (up to FP32).
* Threads and the leaf batchers run to completion and expand leaves.  The
  tree has no tree-wide lock; once the threads have ended every node must
  agree with its children, so the root's bounds equal the best of its
  action bounds recomputed from its children, bit for bit.
* Anytime: a zero budget returns the initial bounds; a full device arena
  stops the search cleanly.
* One thread without exploration bonuses builds the host DESPOT loop's tree
  (the oracle's trial loop over its own expansion), trial for trial.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1802_06215_amd import Context
    c = Context(0)
    yield c
    c.close()


def test_no_rocks_search_finds_exit_value(ctx):
    from paper_1802_06215_amd import hdx as H
    desc = dict(kind=0, n=5, m=0, rock_x=np.zeros(0, np.int32), rock_y=np.zeros(0, np.int32), gamma=0.95,
                start_x=0, start_y=2, n_actions=5)
    m = ctx.upload_model(desc)
    res = ctx.search(m, dict(x=0, y=2, p=np.zeros(0)), K=8, n_threads=1, max_depth=12, time_budget_s=20.0,
                     max_trials=200, gap_epsilon=1e-9, rollout=H.rollout_cfg(0, 0), arena_bytes=64 << 20)
    exact = 10 * 0.95 ** 4
    assert abs(res["u0_root"] - exact) < 1e-5 and res["l0_root"] == 0.0
    assert abs(res["l_root"] - exact) < 1e-5 and abs(res["u_root"] - exact) < 1e-5
    assert res["best_action"] == 2
    assert res["expansions"] >= 5


@pytest.mark.parametrize("threads,batch", [(1, 0), (4, 0), (8, 0), (16, 0), (8, 8), (16, 16), (33, 11), (48, 16), (48, 8), (64, 16)])
def test_rs15_search_bounds(ctx, threads, batch):
    from paper_1802_06215_amd import hdx as H
    desc = W.rocksample_model(15, 15, 1)
    m = ctx.upload_model(desc)
    res = ctx.search(m, W.rocksample_belief(desc), K=500, n_threads=threads, max_depth=90,
                     batch_leaves=batch, time_budget_s=0.5, rollout=H.rollout_cfg(0, 1 << 30, 90),
                     arena_bytes=4 << 30)
    print(threads, batch, {k: res[k] for k in ("trials", "expansions", "nodes", "launches", "u_root", "l_root")},
          flush=True)
    assert res["trials"] > 0 and res["expansions"] > 0 and res["arena_full"] == 0
    tol = 1e-4 * max(1.0, abs(res["u0_root"]))
    assert res["l0_root"] - tol <= res["l_root"] <= res["u_root"] + tol <= res["u0_root"] + 2 * tol
    assert 0 <= res["best_action"] < desc["n_actions"]
    assert res["best_action"] == int(np.argmax(res["action_l"]))
    assert max(res["action_l"]) == res["l_root"] and max(res["action_u"]) == res["u_root"]
    if batch:
        assert res["launches"] <= res["expansions"]


def test_pednav_search_runs(ctx):
    from paper_1802_06215_amd import hdx as H
    desc = W.pednav_model(16, 5, 1)
    m = ctx.upload_model(desc)
    res = ctx.search(m, W.pednav_belief(desc), K=500, n_threads=4, max_depth=50, batch_leaves=4,
                     time_budget_s=0.5, rollout=H.rollout_cfg(0, 50), arena_bytes=4 << 30)
    assert res["trials"] > 0 and res["expansions"] > 0
    assert res["l_root"] <= res["u_root"] + 1e-3 * max(1.0, abs(res["u_root"]))


def test_zero_budget_and_full_arena(ctx):
    from paper_1802_06215_amd import hdx as H
    desc = W.rocksample_model(7, 8, 1)
    m = ctx.upload_model(desc)
    res = ctx.search(m, W.rocksample_belief(desc), K=100, n_threads=2, max_depth=30, time_budget_s=0.0,
                     rollout=H.rollout_cfg(0, 30))
    assert res["trials"] == 0 and res["u_root"] == res["u0_root"] and res["l_root"] == res["l0_root"]
    res = ctx.search(m, W.rocksample_belief(desc), K=100, n_threads=2, max_depth=30, time_budget_s=5.0,
                     rollout=H.rollout_cfg(0, 30), arena_bytes=1 << 20)
    assert res["arena_full"] == 1 and res["expansions"] >= 1


@pytest.mark.parametrize("n,K,R,D", [(5, 2, 0, 8), (9, 4, 0, 14), (12, 1, 0, 10), (12, 4, 2, 14)])
def test_one_thread_search_makes_the_despot_analogue_choices(ctx, n, K, R, D):
    """hdx_search on one thread with c_a = c_o = 0 takes DESPOT's choices
    (Eq. 5 actions, Eq. 7 observation branches, Eq. 4 backups) and so builds
    the same tree as the host DESPOT loop over the oracle's expansion, trial
    for trial: equal node and expansion counts and root bounds within 1e-5
    after the same number of trials.  RockSample without rocks: every
    choice is decided by more than FP32 resolution or by an exact tie (the
    analogue counts the choices that are not), so the library's FP32 child
    bounds and the oracle's FP64 ones must make the same choices; with
    rollouts shorter than the way out and a depth limit below it (12 x 12,
    depth 10) the lower bound stays 0 and the search ends on its gap."""
    from paper_1802_06215_amd import hdx as H
    desc = W.rocksample_model(n, 0, 1)
    mdl = ctx.upload_model(desc)
    belief = W.rocksample_belief(desc)
    T = 200
    root = oracle.sample_scenarios(desc, belief, K, 3, 0)
    ref = oracle.despot(desc, oracle.cfg(0, R, D), root, K, 3, 0, D, 0.95, 60.0, T)
    print("analogue", ref, flush=True)
    assert ref["near_ties"] == 0
    r = ctx.search(mdl, belief, K=K, n_threads=1, max_depth=D, batch_leaves=0, time_budget_s=60.0, max_trials=T,
                   xi=0.95, c_a=0.0, c_o=0.0, gap_epsilon=0.0, arena_bytes=1 << 28, seed=3, step=0,
                   rollout=H.rollout_cfg(0, R, D))
    print("search", {k: r[k] for k in ("trials", "expansions", "nodes", "u_root", "l_root")}, flush=True)
    assert r["expansions"] == ref["expansions"]
    assert r["nodes"] == ref["nodes"]
    for a, b in ((r["u_root"], ref["u_root"]), (r["l_root"], ref["l_root"])):
        assert abs(a - b) <= 1e-5 * max(abs(b), 1.0)
