"""The oracle's host DESPOT trial loop (the baseline of the paper's speedup
metric) against facts it must reproduce: without rocks it finds the exit
value 10 gamma^(n-1-x) exactly and its lower bound never passes its upper
bound; a depth limit below the way out leaves the lower bound at the
rollout-free value 0; a trial budget is honoured."""
import numpy as np
import pytest

import oracle
import workloads as W


@pytest.mark.parametrize("n,K", [(5, 2), (9, 4), (12, 1)])
def test_no_rocks_exit_value(n, K):
    desc = W.rocksample_model(n, 0, 1)
    root = oracle.sample_scenarios(desc, W.rocksample_belief(desc), K, 3, 0)
    r = oracle.despot(desc, oracle.cfg(0, 0, 30), root, K, 3, 0, 30, 0.95, 30.0, 500)
    exact = 10.0 * 0.95 ** (n - 1 - desc["start_x"])
    assert abs(r["l_root"] - exact) < 1e-12 and abs(r["u_root"] - exact) < 1e-12
    assert r["near_ties"] == 0


def test_depth_limit_below_the_exit():
    desc = W.rocksample_model(12, 0, 1)
    root = oracle.sample_scenarios(desc, W.rocksample_belief(desc), 1, 3, 0)
    r = oracle.despot(desc, oracle.cfg(0, 0, 10), root, 1, 3, 0, 10, 0.95, 30.0, 500)
    assert r["l_root"] == 0.0
    assert abs(r["u_root"] - 10.0 * 0.95 ** 11) < 1e-12


def test_bounds_ordered_and_trial_budget():
    desc = W.rocksample_model(6, 2, 1)
    root = oracle.sample_scenarios(desc, W.rocksample_belief(desc), 8, 3, 0)
    U, L, _ = oracle.rollout_bounds(desc, oracle.cfg(0, 1 << 30, 9), root, np.arange(8), np.zeros(8, np.int32), 3, 0)
    for T in (1, 7, 40):
        r = oracle.despot(desc, oracle.cfg(0, 1 << 30, 9), root, 8, 3, 0, 9, 0.95, 30.0, T)
        assert r["trials"] <= T and r["expansions"] <= r["trials"]
        assert L.mean() - 1e-12 <= r["l_root"] <= r["u_root"] <= U.mean() + 1e-12
