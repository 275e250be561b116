"""Pins for the multi-agent RockSample model in the oracle (Sec. IV-A).

* Closed forms: with both robots moving east the rollout value is the sum of
  the two exit rewards, 10 gamma^(n-1-x1) + 10 gamma^(n-1-x2), over
  max(n - x1, n - x2) steps; at the start every child of every joint action
  has that value from the cells the action leads to, and the step counts of
  the root expansion follow.
* Reduction: with robot 2 gone, a joint action is robot 1's own action, so
  step, observation, upper bound and rollout equal the single-robot model
  (pinned on its own in test_oracle_rocksample.py) on robot 1's cell and
  the rocks; with robot 1 gone, robot 2's moves, samples and exits do too.
* Robot 2's sensor: the fraction of correct readings at each distance is
  0.5 + 0.5 2^(-d/20) within 5 sigma, and its readings are independent of
  robot 1's.
* The readings for two robots acting in one step (robot 1 first), by hand.
* Fully known (no rocks): the tree grown to the exit depth backs up (Eq. 4)
  to the closed form, in both bounds.
* Brute force: tiny trees equal the independent determinised recursion.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle_tree_util import brute_force, grow

G = 0.95
EAST, SAMPLE, SENSE0 = 2, 4, 5


def mars(n, rocks):
    rx = np.array([r[0] for r in rocks], np.int32)
    ry = np.array([r[1] for r in rocks], np.int32)
    return dict(kind=2, n=n, m=len(rocks), rock_x=rx, rock_y=ry, gamma=G,
                start=(0, n // 2, 0, n // 2 - 1), n_actions=(5 + len(rocks)) ** 2)


def single(d):
    return dict(kind=0, n=d["n"], m=d["m"], rock_x=d["rock_x"], rock_y=d["rock_y"], gamma=G,
                start_x=0, start_y=d["n"] // 2, n_actions=5 + d["m"])


def exit_value(n, xs):
    return sum(10 * G ** (n - 1 - x) for x in xs)


@pytest.mark.parametrize("x1,x2,g1,g2", [(0, 0, 0, 0), (3, 0, 0, 0), (6, 2, 0, 0), (4, 5, 1, 0), (2, 1, 0, 1)])
def test_move_east_closed_form(x1, x2, g1, g2):
    d = W.mars_model(7, 8, 3)
    K = 16
    rocks = np.random.default_rng(0).random((K, 8)) < 0.5
    st = dict(w=oracle.mars_pack((x1, 2, x2, 5, g1, g2), rocks))
    U, L, steps = oracle.rollout_bounds(d, oracle.cfg(0), st, np.arange(K), 4, 9, 0)
    live = [x for x, g in ((x1, g1), (x2, g2)) if not g]
    assert np.all(np.abs(L - exit_value(7, live)) < 1e-12)
    assert np.all(steps == max(7 - x for x in live))
    assert np.all(U >= L)
    # a depth limit cuts the rollout: only exits within the horizon count
    _, Lc, sc = oracle.rollout_bounds(d, oracle.cfg(0, max_depth=4 + 6 - x1), st, np.arange(K), 4, 9, 0)
    if not g1 and x1 < 6:
        want = sum(10 * G ** (6 - x) for x in live if 7 - x <= 6 - x1)
        assert np.all(np.abs(Lc - want) < 1e-12)


def test_root_children_closed_form():
    n, m, K = 7, 8, 100
    d = W.mars_model(n, m, 1)
    st = oracle.sample_scenarios(d, W.mars_belief(d), K, 5, 0)
    res = oracle.expand_leaf(d, oracle.cfg(0), st, np.arange(K), np.arange(K), 0, -1, 5, 0)
    per = 5 + m
    total = 0
    for a in range(d["n_actions"]):
        xs = [1 if b == EAST else 0 for b in (a // per, a % per)]
        want = exit_value(n, xs)
        nc = res["n_children"][a]
        assert np.all(np.abs(res["child_l0"][a, :nc] - want) < 1e-12)
        assert res["r_mean"][a] == 0.0  # no rock on a start cell, no exit from column 0
        total += K * max(n - x for x in xs)
    assert res["expand_steps"] == K * d["n_actions"]
    assert res["rollout_steps"] == total == K * ((n - 1) + (d["n_actions"] - 1) * n)


def random_states(d, K, seed, gone):
    rng = np.random.default_rng(seed)
    n = d["n"]
    cells = [rng.integers(0, n, K) for _ in range(4)]
    g1 = np.full(K, gone == 1, np.int64)
    g2 = np.full(K, gone == 2, np.int64)
    rocks = rng.random((K, d["m"])) < 0.5
    return cells, rocks, dict(w=oracle.mars_pack((*cells, g1, g2), rocks))


def test_reduces_to_single_robot():
    d = W.mars_model(9, 10, 2)
    s1 = single(d)
    K = 400
    (x1, y1, _, _), rocks, st = random_states(d, K, 1, gone=2)
    ws = oracle.rs_pack(0, 0, rocks, np.zeros(K, bool)) | (x1 | (y1 << 5)).astype(np.int32)
    one = dict(w=ws.astype(np.int32))
    ids = np.random.default_rng(2).choice(1 << 20, K, replace=False)
    per = 5 + d["m"]
    rng = np.random.default_rng(3)
    for b in range(per):
        a = b * per + int(rng.integers(0, per))
        nxt, r, z = oracle.step(d, st, ids, a, 6, 11, 2)
        nxt1, r1, z1 = oracle.step(s1, one, ids, b, 6, 11, 2)
        assert np.array_equal(r, r1)
        assert np.array_equal(z, 3 * z1)
        u = oracle.mars_unpack(nxt["w"])
        u1 = oracle.rs_unpack(nxt1["w"])
        assert np.array_equal(u["rocks"], u1["rocks"])
        assert np.array_equal(u["term"], u1["term"])
        live = u1["term"] == 0
        assert np.array_equal(u["x1"][live], u1["x"][live]) and np.array_equal(u["y1"][live], u1["y"][live])
    # rollouts: the default policy (both east) and constant joint actions
    for b1 in (None, 0, EAST, SAMPLE, SENSE0 + 3):
        rc = oracle.cfg(0, 40) if b1 is None else oracle.cfg(1, 40, const_action=b1 * per + 1)
        rc1 = oracle.cfg(0, 40) if b1 is None else oracle.cfg(1, 40, const_action=b1)
        U, L, sc = oracle.rollout_bounds(d, rc, st, ids, 3, 4, 0)
        U1, L1, sc1 = oracle.rollout_bounds(s1, rc1, one, ids, 3, 4, 0)
        assert np.allclose(U, U1, rtol=1e-14, atol=0) and np.array_equal(L, L1) and np.array_equal(sc, sc1)


def test_robot2_moves_match_single_robot():
    d = W.mars_model(8, 6, 4)
    s1 = single(d)
    K = 300
    (_, _, x2, y2), rocks, st = random_states(d, K, 5, gone=1)
    one = dict(w=(oracle.rs_pack(0, 0, rocks, np.zeros(K, bool)) | (x2 | (y2 << 5)).astype(np.int32)).astype(np.int32))
    ids = np.arange(K)
    per = 5 + d["m"]
    for b in range(SENSE0):
        nxt, r, z = oracle.step(d, st, ids, 7 * per + b, 2, 1, 0)
        nxt1, r1, z1 = oracle.step(s1, one, ids, b, 2, 1, 0)
        assert np.array_equal(r, r1) and np.all(z == 0) and np.all(z1 == 0)
        u, u1 = oracle.mars_unpack(nxt["w"]), oracle.rs_unpack(nxt1["w"])
        assert np.array_equal(u["rocks"], u1["rocks"]) and np.array_equal(u["term"], u1["term"])
        live = u1["term"] == 0
        assert np.array_equal(u["x2"][live], u1["x"][live]) and np.array_equal(u["y2"][live], u1["y"][live])


def test_robot2_sensor_accuracy_and_independence():
    n = 21
    d = mars(n, [(0, 0)])
    K = 60000
    ids = np.arange(K)
    rocks = np.ones((K, 1), bool)
    for dist in (0, 3, 10, 20):
        st = dict(w=oracle.mars_pack((0, dist, 0, dist, 0, 0), rocks))
        # both robots sense rock 0 from the same cell
        _, _, z = oracle.step(d, st, ids, (SENSE0 + 0) * 6 + SENSE0 + 0, 1, 77, 3)
        z1, z2 = z // 3, z % 3
        p = 0.5 + 0.5 * 2.0 ** (-dist / 20.0)
        for zz in (z1, z2):
            frac = np.mean(zz == 1)  # the rock is good: reading 1 is correct
            assert abs(frac - p) <= 5 * np.sqrt(p * (1 - p) / K) + 1e-12
        agree = np.mean(z1 == z2)
        q = p * p + (1 - p) * (1 - p)
        assert abs(agree - q) <= 5 * np.sqrt(q * (1 - q) / K) + 1e-12


def test_two_robots_in_one_step():
    d = mars(5, [(2, 2), (4, 1)])
    per = 7
    both_sample = SAMPLE * per + SAMPLE
    # both on good rock 0: robot 1 takes +10 and the rock turns bad, robot 2 gets -10
    st = dict(w=oracle.mars_pack((2, 2, 2, 2, 0, 0), np.array([[True, True], [False, True]])))
    nxt, r, z = oracle.step(d, st, np.arange(2), both_sample, 1, 1, 0)
    assert list(r) == [0.0, -20.0]
    assert list(oracle.mars_unpack(nxt["w"])["rocks"]) == [2, 2]
    # both leave through the east border in one step: +20 and terminal
    st = dict(w=oracle.mars_pack((4, 0, 4, 3, 0, 0), np.zeros((1, 2), bool)))
    nxt, r, z = oracle.step(d, st, np.arange(1), EAST * per + EAST, 1, 1, 0)
    assert r[0] == 20.0 and oracle.mars_unpack(nxt["w"])["term"][0] == 1
    # terminal states are absorbing and make no step
    nxt2, r2, _ = oracle.step(d, nxt, np.arange(1), EAST * per + SAMPLE, 2, 1, 0)
    assert r2[0] == 0.0 and np.array_equal(nxt2["w"], nxt["w"])
    _, L, sc = oracle.rollout_bounds(d, oracle.cfg(0), nxt, np.arange(1), 2, 1, 0)
    assert L[0] == 0.0 and sc[0] == 0
    # one robot leaves: only it is marked gone, and it does nothing afterwards
    st = dict(w=oracle.mars_pack((4, 0, 1, 3, 0, 0), np.zeros((1, 2), bool)))
    nxt, r, _ = oracle.step(d, st, np.arange(1), EAST * per + 0, 1, 1, 0)
    u = oracle.mars_unpack(nxt["w"])
    assert r[0] == 10.0 and u["gone1"][0] == 1 and u["gone2"][0] == 0 and u["term"][0] == 0
    assert u["y2"][0] == 4
    nxt2, r2, _ = oracle.step(d, nxt, np.arange(1), 3 * per + 1, 2, 1, 0)
    u2 = oracle.mars_unpack(nxt2["w"])
    assert r2[0] == 0.0 and u2["x1"][0] == 4 and u2["y2"][0] == 3
    # the upper bound counts each good rock once, from the nearer robot still in
    st = dict(w=oracle.mars_pack((0, 0, 4, 1, 0, 0), np.array([[True, True]])))
    U, _, _ = oracle.rollout_bounds(d, oracle.cfg(0, 0), st, np.arange(1), 0, 1, 0)
    want = 10 * G ** 3 + 10 * G ** 0 + 10 * G ** 4 + 10 * G ** 0  # rock 0 is 3 cells from robot 2
    assert abs(U[0] - want) < 1e-12


@pytest.mark.parametrize("n,x1,x2", [(2, 0, 0), (3, 1, 2)])
def test_no_rocks_tree_closed_form(n, x1, x2):
    d = mars(n, [])
    K = 2
    st = dict(w=oracle.mars_pack((x1, 0, x2, n - 1, 0, 0), np.zeros((K, 0), bool)))
    rc = oracle.cfg(0, 0)
    need = n - min(x1, x2)
    exact = exit_value(n, [x1, x2])
    deep = grow(d, rc, st, np.arange(K), np.arange(K), 0, -1, 1, 0, need)
    assert abs(deep.l - exact) < 1e-12 and abs(deep.u - exact) < 1e-12
    shallow = grow(d, rc, st, np.arange(K), np.arange(K), 0, -1, 1, 0, need - 1)
    assert shallow.l < exact - 1.0


@pytest.mark.parametrize("case", range(2))
def test_brute_force_tiny_mars(case):
    rng = np.random.default_rng(10 + case)
    n = 3
    cells = [c for c in [(x, y) for x in range(n) for y in range(n)] if c not in ((0, 1), (0, 0))]
    pick = rng.permutation(len(cells))[:1]
    d = mars(n, [cells[i] for i in pick])
    K = 5
    H = 2
    rc = oracle.cfg(0, 3)
    st = oracle.sample_scenarios(d, W.mars_belief(d, 0.5), K, case + 1, 0)
    ids = np.arange(K)
    root = grow(d, rc, st, ids, ids, 0, -1, case + 1, 0, H)
    for which in ("u", "l"):
        want = brute_force(d, rc, st, ids, 0, H, case + 1, 0, which)
        assert abs(getattr(root, which) - want) < 1e-12
    assert root.l <= root.u


def test_leaf_invariants():
    d = W.mars_model(11, 11, 7)
    leaf = W.mars_leaf(d, 60, 40, 3, shared_cells=False, p_term=0.1)
    par = oracle.parent_states(d, leaf)
    res = oracle.expand_leaf(d, oracle.cfg(0, 30), par, leaf["ids"], leaf["idx"], leaf["depth"],
                             leaf["last_action"], 4, 1, per_pair=True)
    A, n = d["n_actions"], 40
    assert A == 256
    for a in range(A):
        nc = res["n_children"][a]
        assert 1 <= nc <= 9 and res["child_n"][a, :nc].sum() == n
        assert np.all(np.diff(res["child_z"][a, :nc].astype(np.int64)) > 0)
        assert np.all(res["child_z"][a, :nc] < 9)
        assert np.all(res["child_l0"][a, :nc] <= res["child_u0"][a, :nc] + 1e-12)
    assert np.all(res["L"] <= res["U"] + 1e-12)
    assert np.array_equal(res["ids"], leaf["ids"][leaf["idx"]])
    # recomputed leaf states equal the parent stepped with the last action
    sub = oracle.take_states(d, par, leaf["idx"])
    st, _, _ = oracle.step(d, sub, leaf["ids"][leaf["idx"]], leaf["last_action"], leaf["depth"] - 1, 4, 1)
    assert np.array_equal(st["w"], res["states"]["w"])
