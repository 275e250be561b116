"""The belief update of the closed-loop RockSample driver (Eq. 3, through
the C ABI's hdx_belief_update, host only), against Bayes' rule worked by
hand."""
import numpy as np
import pytest

from paper_1802_06215_amd import hdx as H


def desc():
    return dict(kind=H.ROCKSAMPLE, n=7, m=2, rock_x=np.array([2, 5]), rock_y=np.array([3, 3]), gamma=0.95,
                n_actions=7)


def acc(d):
    return 0.5 + 0.5 * 2.0 ** (-d / 20.0)


def test_sense_updates_by_bayes():
    b = dict(x=2, y=0, p=np.array([0.5, 0.3]))
    a0 = acc(3.0)  # rock 0 at distance 3
    good, term = H.belief_update(desc(), b, 5, 1)
    assert not term
    assert abs(good["p"][0] - 0.5 * a0 / (0.5 * a0 + 0.5 * (1 - a0))) < 1e-15
    assert good["p"][1] == 0.3
    bad, _ = H.belief_update(desc(), b, 5, 2)
    assert abs(bad["p"][0] - 0.5 * (1 - a0) / (0.5 * (1 - a0) + 0.5 * a0)) < 1e-15
    # a reading of the other rock, at distance sqrt(9 + 9)
    a1 = acc(np.sqrt(18.0))
    r1, _ = H.belief_update(desc(), dict(x=2, y=0, p=np.array([0.5, 0.3])), 6, 1)
    assert abs(r1["p"][1] - 0.3 * a1 / (0.3 * a1 + 0.7 * (1 - a1))) < 1e-15
    # on the rock's own cell the reading is always right
    on, _ = H.belief_update(desc(), dict(x=2, y=3, p=np.array([0.5, 0.3])), 5, 2)
    assert on["p"][0] == 0.0


def test_sample_moves_and_exit():
    b = dict(x=5, y=3, p=np.array([0.5, 0.9]))
    s, _ = H.belief_update(desc(), b, 4, 0)  # sample at rock 1's cell
    assert s["p"][1] == 0.0 and s["p"][0] == 0.5
    m, term = H.belief_update(desc(), b, 2, 0)  # move east
    assert (m["x"], m["y"]) == (6, 3) and np.array_equal(m["p"], b["p"]) and not term
    n_, _ = H.belief_update(desc(), b, 0, 0)
    s_, _ = H.belief_update(desc(), b, 1, 0)
    w_, _ = H.belief_update(desc(), b, 3, 0)
    assert [(n_["x"], n_["y"]), (s_["x"], s_["y"]), (w_["x"], w_["y"])] == [(5, 4), (5, 2), (4, 3)]
    # walls: north of the top row and west of column 0 are no-ops
    top, _ = H.belief_update(desc(), dict(x=0, y=6, p=b["p"]), 0, 0)
    left, _ = H.belief_update(desc(), dict(x=0, y=6, p=b["p"]), 3, 0)
    assert (top["x"], top["y"]) == (0, 6) and (left["x"], left["y"]) == (0, 6)
    # leaving through the east border ends the episode
    e, term = H.belief_update(desc(), dict(x=6, y=1, p=b["p"]), 2, 0)
    assert term and (e["x"], e["y"]) == (6, 1)
    # a certain rock stays certain under any reading
    c, _ = H.belief_update(desc(), dict(x=2, y=0, p=np.array([1.0, 0.0])), 5, 2)
    assert c["p"][0] == 1.0


def test_invalid_arguments():
    b = dict(x=2, y=0, p=np.array([0.5, 0.3]))
    with pytest.raises(H.HdxError):
        H.belief_update(desc(), b, 7, 1)  # no such action
    with pytest.raises(H.HdxError):
        H.belief_update(desc(), b, 5, 0)  # a reading is good or bad
    with pytest.raises(H.HdxError):
        H.belief_update(desc(), dict(x=9, y=0, p=b["p"]), 2, 0)
