"""Pins for the navigation model in the oracle (Sec. IV-A, partially known map).

* Closed forms with the noise switched off (no move failures, no sensor
  errors): the default policy's walk through the open gate to the goal on a
  hand-built map, its value sum_j gamma^j r_j with -0.1 per move and +20 on
  entering the goal, its step count, and the upper bound 20 gamma^(d-1).
* The rewards and moves by hand: stay, crash into a known wall, off the map,
  into an unknown occupied cell, into an unknown free one, the goal (+20,
  terminal, observation 256), absorbing terminal states.
* Readings against the true occupancy with the sensor noise off; with the
  paper's 0.03, each neighbour's flip rate and the move-failure rate within
  5 sigma, and the flips independent across neighbours.
* The prior: start column uniform over the top row, exactly one gate open
  (each half the time), other unknown cells occupied at p.
* Brute force on tiny maps against the independent determinised recursion.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle_tree_util import brute_force, grow

G = 0.95


def small_map(p_fail=0.0, p_err=0.0):
    """5 x 5: wall on row 2 with gates at columns 1 (cell 0) and 3 (cell 1);
    unknown cells 2 at (0, 1) and 3 at (4, 3); goal at (2, 4)."""
    n = 5
    cell = np.full((n, n), -1, np.int64)
    cell[2, :] = -2
    cell[2, 1], cell[2, 3] = 0, 1
    cell[1, 0], cell[3, 4] = 2, 3
    return dict(kind=3, n=n, cell=cell, wall=2, gate_x=np.array([1, 3], np.int32), goal_x=2,
                n_unknown=4, p_occ=0.1, gamma=G, p_fail=p_fail, p_err=p_err, n_actions=9)


def state(x, y, cells, term=0):
    return dict(w=oracle.nav_pack(np.array([x]), np.array([y]), np.array([cells], bool), np.array([term])))


def test_default_walk_closed_form():
    d = small_map()
    step = float(np.float32(-0.1))  # reward constants are FP32 values
    # gate 1 (column 3) open, target (3, 2): from (0, 0) SE to (1, 1); SE
    # (2, 2) is wall and S (1, 2) the closed gate, so E to (2, 1); SE through
    # the gate (3, 2); then towards the goal (2, 4): SW (2, 3), S (2, 4).
    # Five moves, the last one pays +20.
    st = state(0, 0, [1, 0, 0, 0])
    U, L, steps = oracle.rollout_bounds(d, oracle.cfg(0, 100), st, np.arange(1), 0, 1, 0)
    want = sum(step * G ** j for j in range(4)) + 20 * G ** 4
    assert abs(L[0] - want) < 1e-12 and steps[0] == 5
    assert abs(U[0] - 20 * G ** 3) < 1e-12  # Chebyshev distance 4 to (2, 4)
    # gate 0 open: (0, 0) -> SE (1, 1) -> S (1, 2) gate -> SE (2, 3) -> S (2, 4)
    st = state(0, 0, [0, 1, 0, 0])
    _, L, steps = oracle.rollout_bounds(d, oracle.cfg(0, 100), st, np.arange(1), 0, 1, 0)
    assert abs(L[0] - (sum(step * G ** j for j in range(3)) + 20 * G ** 3)) < 1e-12 and steps[0] == 4


def test_moves_rewards_by_hand():
    d = small_map()
    ids = np.arange(1)
    # stay
    nxt, r, z = oracle.step(d, state(2, 0, [1, 0, 0, 0]), ids, 0, 0, 1, 0)
    assert r[0] == np.float32(-0.2) and oracle.nav_unpack(nxt["w"])["x"][0] == 2
    # crash into the known wall below (2, 1) -> (2, 2)
    nxt, r, _ = oracle.step(d, state(2, 1, [1, 0, 0, 0]), ids, 5, 0, 1, 0)
    u = oracle.nav_unpack(nxt["w"])
    assert r[0] == np.float32(-1.0) and (u["x"][0], u["y"][0]) == (2, 1)
    # off the map (north from row 0)
    nxt, r, _ = oracle.step(d, state(2, 0, [1, 0, 0, 0]), ids, 1, 0, 1, 0)
    assert r[0] == np.float32(-1.0)
    # into unknown cell 2 at (0, 1): occupied -> crash, free -> move
    nxt, r, _ = oracle.step(d, state(0, 0, [1, 0, 1, 0]), ids, 5, 0, 1, 0)
    assert r[0] == np.float32(-1.0)
    nxt, r, _ = oracle.step(d, state(0, 0, [1, 0, 0, 0]), ids, 5, 0, 1, 0)
    u = oracle.nav_unpack(nxt["w"])
    assert r[0] == np.float32(-0.1) and (u["x"][0], u["y"][0]) == (0, 1)
    # the closed gate is a crash, the open one a move
    nxt, r, _ = oracle.step(d, state(1, 1, [1, 0, 0, 0]), ids, 5, 0, 1, 0)
    assert r[0] == np.float32(-1.0)
    nxt, r, _ = oracle.step(d, state(1, 1, [0, 1, 0, 0]), ids, 5, 0, 1, 0)
    assert r[0] == np.float32(-0.1) and oracle.nav_unpack(nxt["w"])["y"][0] == 2
    # the goal: +20, terminal, the terminal reading, then absorbing
    nxt, r, z = oracle.step(d, state(2, 3, [1, 0, 0, 0]), ids, 5, 0, 1, 0)
    assert r[0] == 20.0 and oracle.nav_unpack(nxt["w"])["term"][0] == 1 and z[0] == 256
    nxt2, r2, z2 = oracle.step(d, nxt, ids, 3, 1, 1, 0)
    assert r2[0] == 0.0 and np.array_equal(nxt2["w"], nxt["w"]) and z2[0] == 256
    _, L, sc = oracle.rollout_bounds(d, oracle.cfg(0, 10), nxt, ids, 1, 1, 0)
    assert L[0] == 0.0 and sc[0] == 0


def test_reading_without_noise():
    d = small_map()
    # at (1, 1): neighbours N (1,0) free, NE (2,0) free, E (2,1) free,
    # SE (2,2) wall, S (1,2) gate 0, SW (0,2) wall, W (0,1) cell 2, NW (0,0) free
    for g0, c2 in ((1, 0), (0, 1), (1, 1)):
        _, _, z = oracle.step(d, state(1, 1, [g0, 1 - g0, c2, 0]), np.arange(1), 0, 0, 1, 0)
        want = (1 << 3) | (g0 << 4) | (1 << 5) | (c2 << 6)
        assert z[0] == want
    # corner (4, 0): N, NE, E, SE off the map read occupied; S (4,1) free,
    # SW (3,1) free, W (3,0) free, NW off the map
    _, _, z = oracle.step(d, state(4, 0, [1, 0, 0, 0]), np.arange(1), 0, 0, 1, 0)
    assert z[0] == (1 | 2 | 4 | 8 | 128)


def test_noise_rates():
    d = small_map(p_fail=0.03, p_err=0.03)
    K = 100000
    ids = np.arange(K)
    cells = np.zeros((K, 4), bool)
    cells[:, 0] = True
    st = dict(w=oracle.nav_pack(np.full(K, 2), np.full(K, 0), cells, np.zeros(K)))
    # move east from (2, 0): failures leave the robot in place
    nxt, r, z = oracle.step(d, st, ids, 3, 4, 9, 2)
    u = oracle.nav_unpack(nxt["w"])
    fail = np.mean(u["x"] == 2)
    assert abs(fail - 0.03) <= 5 * np.sqrt(0.03 * 0.97 / K)
    assert np.all(r[u["x"] == 2] == np.float32(-0.1))
    # readings at (2, 0) with stay: true pattern N, NE, NW off the map
    _, _, z = oracle.step(d, st, ids, 0, 4, 9, 2)
    truth = 1 | 2 | 128
    flips = np.stack([((z.astype(np.int64) ^ truth) >> j) & 1 for j in range(8)], axis=1)
    for j in range(8):
        assert abs(flips[:, j].mean() - 0.03) <= 5 * np.sqrt(0.03 * 0.97 / K)
    both = np.mean(flips[:, 0] & flips[:, 5])
    assert abs(both - 0.03 ** 2) <= 5 * np.sqrt(0.03 ** 2 / K) + 1e-12


def test_prior_sampling():
    d = W.nav_model(2)
    K = 40000
    st = oracle.sample_scenarios(d, W.nav_belief(d), K, 3, 0)
    u = oracle.nav_unpack(st["w"])
    assert np.all(u["y"] == 0) and np.all(u["term"] == 0)
    counts = np.bincount(u["x"], minlength=13)
    assert counts.shape[0] == 13
    p = 1 / 13
    assert np.all(np.abs(counts / K - p) <= 5 * np.sqrt(p * (1 - p) / K))
    c = u["cells"]
    assert np.all(c[:, 0] ^ c[:, 1])
    assert abs(np.mean(~c[:, 0]) - 0.5) <= 5 * np.sqrt(0.25 / K)
    frac = c[:, 2:d["n_unknown"]].mean()
    assert abs(frac - 0.1) <= 5 * np.sqrt(0.09 / (K * (d["n_unknown"] - 2)))
    assert not c[:, d["n_unknown"]:].any()


@pytest.mark.parametrize("case", range(2))
def test_brute_force_tiny_nav(case):
    d = small_map(p_fail=0.03 * case, p_err=0.03)
    K = 4
    H = 2
    rc = oracle.cfg(0, 6)
    rng = np.random.default_rng(case)
    cells = rng.random((K, 4)) < 0.3
    cells[:, 1] = ~cells[:, 0]
    st = dict(w=oracle.nav_pack(np.array([1, 1, 2, 3]), np.zeros(K, np.int64), cells, np.zeros(K)))
    ids = np.arange(K)
    root = grow(d, rc, st, ids, ids, 0, -1, case + 5, 0, H)
    for which in ("u", "l"):
        want = brute_force(d, rc, st, ids, 0, H, case + 5, 0, which)
        assert abs(getattr(root, which) - want) < 1e-12
    assert root.l <= root.u


def test_leaf_invariants():
    d = W.nav_model(4)
    leaf = W.nav_leaf(d, 80, 50, 2, p_term=0.1)
    par = oracle.parent_states(d, leaf)
    res = oracle.expand_leaf(d, oracle.cfg(0, 1 << 30, 90), par, leaf["ids"], leaf["idx"], leaf["depth"],
                             leaf["last_action"], 4, 1, per_pair=True)
    n = 50
    for a in range(9):
        nc = res["n_children"][a]
        assert res["child_n"][a, :nc].sum() == n
        assert np.all(np.diff(res["child_z"][a, :nc].astype(np.int64)) > 0)
        assert np.all(res["child_z"][a, :nc] <= 256)
        assert np.all(res["child_l0"][a, :nc] <= res["child_u0"][a, :nc] + 1e-12)
    assert np.all(res["L"] <= res["U"] + 1e-12)
    sub = oracle.take_states(d, par, leaf["idx"])
    st, _, _ = oracle.step(d, sub, leaf["ids"][leaf["idx"]], leaf["last_action"], leaf["depth"] - 1, 4, 1)
    assert np.array_equal(st["w"], res["states"]["w"])


@pytest.mark.parametrize("x,y,d", [(2, 3, 1), (1, 3, 1), (4, 3, 2), (0, 1, 3), (2, 0, 4), (4, 0, 4)])
def test_upper_bound_by_distance(x, y, d):
    """One move per cell of Chebyshev distance d to the goal (2, 4); the
    bound collects +20 on the d-th move, discounted d - 1 times."""
    dm = small_map()
    U, _, _ = oracle.rollout_bounds(dm, oracle.cfg(0, 100), state(x, y, [1, 0, 0, 0]), np.arange(1), 0, 1, 0)
    assert abs(U[0] - 20 * G ** (d - 1)) < 1e-12


def test_upper_bound_terminal_is_zero():
    dm = small_map()
    U, L, _ = oracle.rollout_bounds(dm, oracle.cfg(0, 100), state(2, 4, [1, 0, 0, 0], term=1), np.arange(1), 0, 1, 0)
    assert U[0] == 0.0 and L[0] == 0.0


def test_upper_bound_on_the_goal_cell():
    """A robot standing on the goal without the episode having ended (no step
    produces it: entering the goal is terminal) collects +20 soonest by
    leaving and re-entering, two moves: the bound is 20 gamma.  It must be
    admissible -- at least the best return, which with the noise off is
    -0.1 (leave) + gamma 20 (re-enter) -- and consistent, u(s) >= r + gamma u(s')
    for every action."""
    dm = small_map()
    on_goal = state(2, 4, [1, 0, 0, 0])
    U, _, _ = oracle.rollout_bounds(dm, oracle.cfg(0, 100), on_goal, np.arange(1), 0, 1, 0)
    assert abs(U[0] - 20 * G) < 1e-12
    best = float(np.float32(-0.1)) + G * 20.0
    assert U[0] >= best
    for a in range(9):
        nxt, r, _ = oracle.step(dm, on_goal, np.arange(1), a, 0, 1, 0)
        Un, _, _ = oracle.rollout_bounds(dm, oracle.cfg(0, 100), nxt, np.arange(1), 1, 1, 0)
        assert U[0] >= float(r[0]) + G * Un[0] - 1e-12, a
    # the brute-force optimum over three steps from the goal cell is the
    # leave-and-re-enter return, and the bound is above it
    v = brute_force(dm, oracle.cfg(1, 0), on_goal, np.arange(1), 0, 3, 1, 0, "l")
    assert abs(v - best) < 1e-6 and U[0] >= v
