"""The synthetic inputs follow the shapes the paper describes (Sec. IV-A).

* Navigation: a 13x13 map whose top and bottom rows are known free, a
  middle wall whose only openings are the two gates (unknown cells 0 and
  1), and 124 unknown cells in all: the paper's 169 x 2^124 states; the goal
  on the bottom row; leaves never put a robot inside a wall or an occupied
  cell, and exactly one gate is open in every scenario.
* Multi-agent RockSample: (5 + m)^2 joint actions (256, 400, 625 for the
  paper's three sizes), rocks on distinct cells off both start cells.
"""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("seed", range(4))
def test_nav_map_matches_the_paper(seed):
    d = W.nav_model(seed)
    cell, n = d["cell"], d["n"]
    assert n == 13 and d["n_actions"] == 9
    assert d["n_unknown"] == 124
    unknown = cell[cell >= 0]
    assert sorted(unknown.tolist()) == list(range(124))
    assert np.all(cell[0] == -1) and np.all(cell[n - 1] == -1)
    wall = cell[d["wall"]]
    assert sorted(np.nonzero(wall != -2)[0].tolist()) == sorted(d["gate_x"].tolist())
    assert wall[d["gate_x"][0]] == 0 and wall[d["gate_x"][1]] == 1
    assert cell[n - 1, d["goal_x"]] == -1
    assert (cell == -2).sum() == (n - 2) + 8  # the wall row minus its gates, and 8 landmarks
    b = W.nav_belief(d)
    assert b["p"].shape == (124,) and np.all(b["p"][:2] == 0.5) and np.all(b["p"][2:] == 0.1)


def test_nav_leaves_are_valid_states():
    d = W.nav_model(1)
    for shared in (False, True):
        lf = W.nav_leaf(d, 300, 100, 5, shared_cell=shared)
        x, y, cells = lf["x"], lf["y"], lf["cells"]
        assert np.all(cells[:, 0] ^ cells[:, 1])  # exactly one gate open
        for k in range(300):
            c = d["cell"][y[k], x[k]]
            assert c != -2
            if c >= 0:
                assert not cells[k, c]
        assert np.all(np.diff(lf["idx"]) > 0) and np.all(np.diff(lf["ids"]) > 0)


@pytest.mark.parametrize("size,actions", [(11, 256), (15, 400), (20, 625)])
def test_mars_sizes(size, actions):
    d = W.mars_model(size, size, 3)
    assert d["n_actions"] == actions
    rocks = set(zip(d["rock_x"].tolist(), d["rock_y"].tolist()))
    assert len(rocks) == size
    s = d["start"]
    assert (s[0], s[1]) not in rocks and (s[2], s[3]) not in rocks and (s[0], s[1]) != (s[2], s[3])
    lf = W.mars_leaf(d, 200, 50, 1)
    g1, g2 = lf["pos"][4], lf["pos"][5]
    term = lf["term"].astype(bool)
    assert np.all((g1 & g2).astype(bool) == term)  # both robots gone exactly when terminal
