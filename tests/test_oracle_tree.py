"""Pins for leaf expansion, grouping and backup in the oracle.

* Closed form (fully observed, no rocks): growing the tree deep enough and
  backing up with Eq. 4 recovers the exit value 10 gamma^(n-1-x).
* Brute force: an independently written recursion over the
  scenario-determinised tree, V_H(Phi) = max_a [ mean r + gamma sum_z
  |Phi_z|/|Phi| V_{H-1}(Phi_z) ] with grouping by dictionary, equals the
  oracle's expand + attach + backup.
* Invariants of Eq. 11-13: each scenario in exactly one child per action,
  child counts sum to the parent's, canonical child and scenario order,
  per-scenario L <= U hence l0 <= u0, ids carried along, terminal states
  absorbing, recomputed leaf states equal to the stepped states.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle_tree_util import brute_force, grow


def rs_model(n, rocks):
    rx = np.array([r[0] for r in rocks], np.int32)
    ry = np.array([r[1] for r in rocks], np.int32)
    return dict(kind=0, n=n, m=len(rocks), rock_x=rx, rock_y=ry, gamma=0.95,
                start_x=0, start_y=n // 2, n_actions=5 + len(rocks))


@pytest.mark.parametrize("n,x0", [(4, 0), (3, 1), (5, 2)])
def test_no_rocks_depth_closed_form(n, x0):
    d = rs_model(n, [])
    K = 3
    st = dict(w=oracle.rs_pack(x0, 1, np.zeros((K, 0), bool), np.zeros(K, bool)))
    rc = oracle.cfg(0, 0)  # no rollouts: lower bounds at the fringe are 0
    need = n - x0  # east moves to leave the grid
    exact = 10 * 0.95 ** (n - 1 - x0)
    shallow = grow(d, rc, st, np.arange(K), np.arange(K), 0, -1, 1, 0, need - 1)
    assert shallow.l == 0.0
    deep = grow(d, rc, st, np.arange(K), np.arange(K), 0, -1, 1, 0, need)
    assert abs(deep.l - exact) < 1e-12
    assert abs(deep.u - exact) < 1e-12  # the heuristic is tight with no rocks


@pytest.mark.parametrize("case", range(4))
def test_brute_force_tiny_rocksample(case):
    rng = np.random.default_rng(case)
    n = int(rng.integers(2, 4))
    m = int(rng.integers(0, 3))
    cells = rng.permutation([(x, y) for x in range(n) for y in range(n) if (x, y) != (0, n // 2)])
    d = rs_model(n, [tuple(c) for c in cells[:m]])
    K = int(rng.integers(3, 9))
    H = 3
    rc = oracle.cfg(0, 4)
    st = oracle.sample_scenarios(d, W.rocksample_belief(d, 0.5), K, case + 1, 0)
    ids = np.arange(K)
    root = grow(d, rc, st, ids, ids, 0, -1, case + 1, 0, H)
    for which in ("u", "l"):
        want = brute_force(d, rc, st, ids, 0, H, case + 1, 0, which)
        assert abs(getattr(root, which) - want) < 1e-12


def test_brute_force_tiny_pednav():
    d = W.pednav_model(2, 2, 3)
    d["n_levels"] = 5
    K = 5
    rc = oracle.cfg(0, 6)
    st = oracle.sample_scenarios(d, W.pednav_belief(d), K, 2, 0)
    ids = np.arange(K)
    root = grow(d, rc, st, ids, ids, 0, -1, 2, 0, 2)
    for which in ("u", "l"):
        want = brute_force(d, rc, st, ids, 0, 2, 2, 0, which)
        assert abs(getattr(root, which) - want) < 1e-9


def _leaf(kind, seed, n_parent=200, n_leaf=150):
    if kind == 0:
        d = W.rocksample_model(11, 12, seed)
        lf = W.rocksample_leaf(d, n_parent, n_leaf, seed, p_term=0.1)
        rc = oracle.cfg(0, 30)
    else:
        d = W.pednav_model(16, 5, seed)
        lf = W.pednav_leaf(d, n_parent, n_leaf, seed, p_term=0.1)
        rc = oracle.cfg(0, 20)
    return d, lf, rc


def _action_states(d, sp, a):
    if d["kind"] == 0:
        return dict(w=np.ascontiguousarray(sp["w"][a]))
    return {f: np.ascontiguousarray(sp[f][a] if f in ("s", "car") else sp[f][:, a]) for f in sp}


@pytest.mark.parametrize("kind,seed", [(0, 1), (0, 2), (1, 1), (1, 2)])
def test_expansion_invariants(kind, seed):
    d, lf, rc = _leaf(kind, seed)
    par = oracle.parent_states(d, lf)
    res = oracle.expand_leaf(d, rc, par, lf["ids"], lf["idx"], lf["depth"], lf["last_action"], 7, 1,
                             per_pair=True)
    n = len(lf["idx"])
    A = d["n_actions"]
    assert np.array_equal(res["ids"], lf["ids"][lf["idx"]])
    for a in range(A):
        nc = res["n_children"][a]
        assert nc >= 1
        assert res["child_n"][a, :nc].sum() == n
        assert np.all(np.diff(res["child_z"][a, :nc].astype(object)) > 0) if nc > 1 else True
        perm = res["perm"][a]
        assert sorted(perm.tolist()) == list(range(n))
        for c in range(nc):
            off, cnt = res["child_off"][a, c], res["child_n"][a, c]
            seg = perm[off:off + cnt]
            assert np.all(np.diff(seg) > 0)
            assert np.all(res["child_of"][a, seg] == c)
            assert np.all(res["z"][a, seg] == res["child_z"][a, c])
            assert np.isclose(res["child_u0"][a, c], res["U"][a, seg].mean(), rtol=1e-12, atol=1e-12)
            assert np.isclose(res["child_l0"][a, c], res["L"][a, seg].mean(), rtol=1e-12, atol=1e-12)
            assert res["child_l0"][a, c] <= res["child_u0"][a, c] + 1e-9
        assert np.all(res["L"][a] <= res["U"][a] + 1e-9)
        assert np.isclose(res["r_mean"][a], res["r"][a].astype(np.float64).mean(), rtol=1e-12, atol=1e-12)
    # terminal leaf scenarios are absorbing
    if d["kind"] == 0:
        term = (res["states"]["w"] >> 30) & 1
        for a in range(A):
            assert np.all(res["sprime"]["w"][a][term == 1] == res["states"]["w"][term == 1])
    else:
        term = res["states"]["car"] >> 8
        for a in range(A):
            assert np.all(res["sprime"]["s"][a][term == 1] == res["states"]["s"][term == 1])
    for a in range(A):
        assert np.all(res["r"][a][term == 1] == 0)
    # expansion steps count the non-terminal scenarios once per action
    assert res["expand_steps"] == A * int((term == 0).sum())
    assert np.all(res["steps"][:, 0] == int((term == 0).sum()))
    # each action's rollout steps are those of rollouts from its own stepped
    # states at depth + 1 (a count credited to another action fails here)
    for a in range(A):
        sp_a = _action_states(d, res["sprime"], a)
        _, _, st = oracle.rollout_bounds(d, rc, sp_a, res["ids"], lf["depth"] + 1, 7, 1)
        assert res["steps"][a, 1] == int(np.sum(st))
    assert res["steps"][:, 1].sum() == res["rollout_steps"]


@pytest.mark.parametrize("kind", [0, 1])
def test_recomputed_child_states_equal_stepped_states(kind):
    d, lf, rc = _leaf(kind, 5)
    par = oracle.parent_states(d, lf)
    res = oracle.expand_leaf(d, rc, par, lf["ids"], lf["idx"], lf["depth"], lf["last_action"], 3, 0,
                             per_pair=True)
    for a in range(d["n_actions"]):
        for c in range(res["n_children"][a]):
            off, cnt = res["child_off"][a, c], res["child_n"][a, c]
            pos = res["perm"][a, off:off + cnt]
            kid = oracle.expand_leaf(d, rc, res["states"], res["ids"], pos, lf["depth"] + 1, a, 3, 0)
            if d["kind"] == 0:
                assert np.array_equal(kid["states"]["w"], res["sprime"]["w"][a][pos])
            else:
                for f in ("s", "car"):
                    assert np.array_equal(kid["states"][f], res["sprime"][f][a][pos])
                for f in ("px", "py", "goal"):
                    assert np.array_equal(kid["states"][f], res["sprime"][f][:, a][:, pos])
            assert np.array_equal(kid["ids"], res["ids"][pos])


def test_empty_and_single_scenario_leaves():
    d = W.rocksample_model(7, 8, 1)
    st = oracle.sample_scenarios(d, W.rocksample_belief(d), 10, 1, 0)
    res = oracle.expand_leaf(d, oracle.cfg(0, 30), st, np.arange(10), np.array([], np.int32), 3, 2, 1, 0)
    assert np.all(res["n_children"] == 0) and res["expand_steps"] == 0
    res = oracle.expand_leaf(d, oracle.cfg(0, 30), st, np.arange(10), np.array([4]), 3, 2, 1, 0)
    assert np.all(res["n_children"] == 1) and np.all(res["child_n"][:, 0] == 1)
