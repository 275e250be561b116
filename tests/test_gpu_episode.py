"""Closed-loop RockSample: plan with the search, act in a true environment
stepped by the library, update the belief, replan, until the robot exits."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_rocksample_episode_closed_loop():
    from paper_1802_06215_amd import Context, hdx as H
    from paper_1802_06215_amd import episode as E
    ctx = Context(0)
    desc = W.rocksample_model(7, 8, 1)
    m = ctx.upload_model(desc)
    rocks = np.random.default_rng(5).random(8) < 0.5
    print("true rocks", rocks.astype(int), flush=True)
    res = E.run_rocksample(ctx, m, desc, rocks, max_steps=60, K=100, n_threads=1, max_depth=30,
                           time_budget_s=10.0, max_trials=300, rollout=H.rollout_cfg(0, 1 << 30, 30),
                           seed=3, arena_bytes=1 << 30)
    print(res["actions"], res["discounted_return"], flush=True)
    assert set(res["rewards"]) <= {-10.0, 0.0, 10.0}
    assert res["exited"]
    # at least the value of walking straight east from the start
    move_east = 10.0 * desc["gamma"] ** (desc["n"] - 1 - desc["start_x"])
    assert res["discounted_return"] >= move_east - 1e-9
    ctx.close()
