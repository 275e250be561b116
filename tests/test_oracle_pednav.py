"""Pins for the oracle's crowd-driving model (Sec. IV-A, driving in a crowd).

Closed forms for degenerate cases (no pedestrians, a static pedestrian on the
path), geometric facts of the pedestrian update (step length, heading
rotation preserving length), the Gaussian heading noise recovered from the
motion and compared with the Irwin-Hall draw it was built from, the action
failure rate, and the belief's goal prior as frequencies.
"""
import numpy as np
import pytest

import oracle
import workloads as W

ALL_ONES = np.uint64(0xFFFFFFFFFFFFFFFF)


def model(n_peds=0, goals=((20.0, 0.0),), sigma_h=0.3, p_fail=0.01, gamma=0.98):
    d = W.pednav_model(max(n_peds, 1), len(goals), 0, gamma=gamma)
    d.update(n_peds=n_peds, n_goals=len(goals), sigma_h=sigma_h, p_fail=p_fail,
             goal_x=np.array([g[0] for g in goals], np.float32),
             goal_y=np.array([g[1] for g in goals], np.float32))
    return d


def states(d, K, s, level, px=(), py=(), goal=(), term=False):
    P = d["n_peds"]
    return dict(s=np.full(K, s, np.float32),
                car=np.full(K, level | (0x100 if term else 0), np.int32),
                px=np.tile(np.array(px, np.float32).reshape(P, 1), (1, K)),
                py=np.tile(np.array(py, np.float32).reshape(P, 1), (1, K)),
                goal=np.tile(np.array(goal, np.uint8).reshape(P, 1), (1, K)))


def discounted(rewards, g):
    return sum(r * g ** j for j, r in enumerate(rewards))


@pytest.mark.parametrize("s0,level", [(3.0, 3), (0.0, 1), (12.25, 4), (39.5, 2)])
def test_maintain_without_pedestrians_closed_form(s0, level):
    d = model(n_peds=0)
    v = 0.5 * level
    T = int(np.ceil((40.0 - s0) / (v * 0.5)))
    want = discounted([-0.1] * T, 0.98) + 100 * 0.98 ** (T - 1)
    st = states(d, 1, s0, level)
    U, L, steps = oracle.rollout_bounds(d, oracle.cfg(1, 1000, const_action=1), st, [0], 2, 1, 0)
    assert steps[0] == T
    assert abs(L[0] - want) <= 1e-7 * (abs(want) + 0.1 * T)
    # the upper bound uses the earliest arrival at top speed (1 m per step)
    Tu = max(1, int(np.ceil(40.0 - s0)))
    assert np.isclose(U[0], 100 * 0.98 ** (Tu - 1), rtol=1e-12)
    assert L[0] <= U[0]


def test_static_pedestrian_collision_closed_form():
    # a pedestrian whose goal is its own spot stays there; the car at 1 m/s
    # moves 0.5 m per step and collides once within 1 m of it
    d = model(n_peds=1, goals=((10.3, 0.0),))
    st = states(d, 1, 0.0, 2, px=[10.3], py=[0.0], goal=[0])
    U, L, steps = oracle.rollout_bounds(d, oracle.cfg(1, 1000, const_action=1), st, [0], 0, 1, 0)
    T = 19  # first s' = 0.5 k with (10.3 - s')^2 < 1 is s' = 9.5
    want = discounted([-0.1] * (T - 1) + [-1000.1], 0.98)
    assert steps[0] == T
    assert abs(L[0] - want) <= 1e-7 * 1100


def test_default_policy_brakes_for_pedestrian_ahead():
    # pedestrian 2.5 m ahead on the path: the default policy brakes to a stop
    # and then waits (no collision at zero speed), earning -0.1 per step
    d = model(n_peds=1, goals=((12.5, 0.0),), p_fail=0.0)
    st = states(d, 1, 10.0, 1, px=[12.5], py=[0.0], goal=[0])
    R = 40
    U, L, steps = oracle.rollout_bounds(d, oracle.cfg(0, R), st, [0], 0, 1, 0)
    assert steps[0] == R
    assert abs(L[0] - discounted([-0.1] * R, 0.98)) < 1e-7
    # off the corridor (|py| >= 1.5) it accelerates to the goal at top speed
    d2 = model(n_peds=1, goals=((36.0, 3.0),), p_fail=0.0)
    st2 = states(d2, 1, 35.0, 4, px=[36.0], py=[3.0], goal=[0])
    U, L, steps = oracle.rollout_bounds(d2, oracle.cfg(0, R), st2, [0], 0, 1, 0)
    assert steps[0] == 5
    assert abs(L[0] - (discounted([-0.1] * 5, 0.98) + 100 * 0.98 ** 4)) < 1e-5


def test_pedestrian_moves_one_step_length_towards_goal_without_noise():
    d = model(n_peds=1, goals=((30.0, 4.0),), sigma_h=0.0)
    K = 64
    rng = np.random.default_rng(0)
    px = rng.uniform(5, 25, K).astype(np.float32)
    py = rng.uniform(-6, 6, K).astype(np.float32)
    st = dict(s=np.zeros(K, np.float32), car=np.zeros(K, np.int32), px=px[None].copy(),
              py=py[None].copy(), goal=np.zeros((1, K), np.uint8))
    out, r, z = oracle.step(d, st, np.arange(K), 1, 0, 1, 0)
    dx = out["px"][0].astype(np.float64) - px
    dy = out["py"][0].astype(np.float64) - py
    # exact up to the rounding of the stored FP32 positions (a few ulp)
    ulp = np.spacing(np.abs(out["px"][0])).astype(np.float64) + np.spacing(np.abs(out["py"][0]))
    assert np.all(np.abs(np.hypot(dx, dy) - 0.6) <= 4 * ulp)
    gx, gy = 30.0 - px.astype(np.float64), 4.0 - py.astype(np.float64)
    cross = dx * gy - dy * gx
    assert np.all(np.abs(cross / np.hypot(gx, gy)) <= 4 * ulp)  # heading straight at the goal


def test_pedestrian_snaps_to_goal_within_one_step():
    d = model(n_peds=1, goals=((20.0, 1.0),))
    st = states(d, 4, 0.0, 0, px=[20.3], py=[1.2], goal=[0])
    out, r, z = oracle.step(d, st, np.arange(4), 1, 0, 1, 0)
    assert np.all(out["px"] == np.float32(20.0)) and np.all(out["py"] == np.float32(1.0))


def test_heading_noise_is_the_irwin_hall_gaussian():
    d = model(n_peds=2, goals=((38.0, 5.0), (6.0, -5.0)), sigma_h=0.3)
    K = 50000
    st = states(d, K, 0.0, 0, px=[20.0, 20.0], py=[0.0, 0.0], goal=[0, 1])
    depth, seed, step_idx = 4, 21, 2
    out, r, z = oracle.step(d, st, np.arange(K), 1, depth, seed, step_idx)
    for j, (gx, gy) in enumerate([(38.0, 5.0), (6.0, -5.0)]):
        dx = out["px"][j].astype(np.float64) - 20.0
        dy = out["py"][j].astype(np.float64) - 0.0
        # the rotation keeps the step length
        ulp = np.spacing(np.float32(20.0)).astype(np.float64)
        assert np.all(np.abs(np.hypot(dx, dy) - 0.6) <= 4 * ulp)
        ux, uy = gx - 20.0, gy - 0.0
        theta = np.arctan2(ux * dy - uy * dx, ux * dx + uy * dy)
        noise = np.tan(theta / 2) / 0.15  # tangent of the half angle = 0.5 sigma n
        # pedestrian j reads block j+1 of its (id, depth) STEP counter
        ctr = np.stack([np.arange(K), np.full(K, depth), np.full(K, j + 1), np.zeros(K)], 1)
        w = oracle.philox(ctr, (seed, step_idx)).astype(np.int64)
        ih = ((w >> 8).sum(1) - 33554430) * np.sqrt(3.0) / 2 ** 24
        assert np.max(np.abs(noise - ih)) < 2e-3
        assert abs(noise.mean()) < 5 / np.sqrt(K)
        assert abs(noise.var() - 1.0) < 5 * np.sqrt(0.8 / K)  # Irwin-Hall-4 excess kurtosis -0.3
        assert np.max(np.abs(noise)) <= 2 * np.sqrt(3.0) + 1e-3


def test_action_failure_rate_and_level_clamps():
    d = model(n_peds=0)
    K = 200000
    out, r, z = oracle.step(d, states(d, K, 0.0, 2), np.arange(K), 0, 3, 9, 0)
    lvl = out["car"] & 0xFF
    fail = np.mean(lvl == 2)
    assert set(np.unique(lvl)) <= {2, 3}
    assert abs(fail - 0.01) < 5 * np.sqrt(0.01 * 0.99 / K)
    ctr = np.stack([np.arange(K), np.full(K, 3), np.zeros(K), np.zeros(K)], 1)
    w0 = oracle.philox(ctr, (9, 0))[:, 0].astype(np.int64)
    assert np.array_equal(lvl == 2, w0 < int(np.floor(0.01 * 2 ** 32)))
    out, r, z = oracle.step(d, states(d, 100, 0.0, 4), np.arange(100), 0, 0, 1, 0)
    assert np.all(out["car"] & 0xFF == 4)
    out, r, z = oracle.step(d, states(d, 100, 0.0, 0), np.arange(100), 2, 0, 1, 0)
    assert np.all(out["car"] & 0xFF == 0)
    out, r, z = oracle.step(d, states(d, 100, 0.0, 3), np.arange(100), 1, 0, 1, 0)
    assert np.all(out["car"] & 0xFF == 3) and np.all(out["s"] == np.float32(0.75))


def test_goal_terminal_and_absorbing():
    d = model(n_peds=0)
    out, r, z = oracle.step(d, states(d, 3, 39.25, 4), np.arange(3), 1, 0, 1, 0)
    assert np.all(r == np.float32(-0.1) + np.float32(100.0))
    assert np.all(out["car"] >> 8 == 1) and np.all(z == ALL_ONES)
    out2, r2, z2 = oracle.step(d, out, np.arange(3), 0, 1, 1, 0)
    assert np.all(r2 == 0) and np.all(z2 == ALL_ONES)
    assert np.array_equal(out2["s"], out["s"]) and np.array_equal(out2["car"], out["car"])


def test_observation_is_speed_and_floored_positions():
    d = model(n_peds=2, goals=((30.0, 0.0),), sigma_h=0.0)
    # same level and the same floored pedestrian cells, different car
    # positions and sub-metre offsets: same observation
    a = dict(s=np.array([1.0, 7.5], np.float32), car=np.array([2, 2], np.int32),
             px=np.array([[10.1, 10.3], [15.0, 15.2]], np.float32),
             py=np.array([[2.1, 2.3], [-3.5, -3.4]], np.float32), goal=np.zeros((2, 2), np.uint8))
    out, r, z = oracle.step(d, a, np.array([0, 1]), 1, 0, 1, 0)
    assert np.array_equal(np.floor(out["px"][:, 0]), np.floor(out["px"][:, 1]))
    assert z[0] == z[1] and z[0] != ALL_ONES
    b = dict(a)
    b["px"] = np.array([[10.1, 11.3], [15.0, 15.2]], np.float32)
    out, r, z = oracle.step(d, b, np.array([0, 1]), 1, 0, 1, 0)
    assert z[0] != z[1]


def test_sample_scenarios_goal_prior():
    d = W.pednav_model(4, 3, 2)
    gp = np.array([[1, 0, 0], [0.2, 0.3, 0.5], [0, 0, 1], [0.5, 0.5, 0]], np.float64)
    K = 100000
    b = W.pednav_belief(d, gp, s=2.5, level=3)
    st = oracle.sample_scenarios(d, b, K, 4, 1)
    assert np.all(st["s"] == np.float32(2.5)) and np.all(st["car"] == 3)
    assert np.array_equal(st["px"][:, 0], d["ped_x0"])
    for j in range(4):
        freq = np.bincount(st["goal"][j], minlength=3) / K
        sd = np.sqrt(gp[j] * (1 - gp[j]) / K) + 1e-12
        assert np.all(np.abs(freq - gp[j]) <= 5 * sd)


def test_observation_mixer_is_splitmix64():
    """The observation hash's mixing step is splitmix64's output function:
    driven as the generator (state += the golden-ratio increment), it gives
    the generator's published first outputs from state 0."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "splitmix64_seed0.json")))
    inc, st = int(g["increment"], 16), 0
    for want in g["outputs"]:
        st = (st + inc) & 0xFFFFFFFFFFFFFFFF
        assert oracle.mix64(st) == int(want, 16)
