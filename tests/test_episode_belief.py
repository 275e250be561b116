"""Host-side belief update of the closed-loop RockSample driver, against
Bayes' rule worked by hand."""
import numpy as np

from paper_1802_06215_amd import episode as E


def desc():
    return dict(n=7, m=2, rock_x=np.array([2, 5]), rock_y=np.array([3, 3]), gamma=0.95)


def test_sensor_accuracy_law():
    assert E.sensor_accuracy(0.0) == 1.0
    assert abs(E.sensor_accuracy(20.0) - 0.75) < 1e-15
    assert abs(E.sensor_accuracy(40.0) - 0.625) < 1e-15


def test_sense_updates_by_bayes():
    b = dict(x=2, y=0, p=np.array([0.5, 0.3]))
    acc = 0.5 + 0.5 * 2 ** (-3.0 / 20.0)  # rock 0 at distance 3
    good = E.update_belief(desc(), b, 5, 1, 2, 0)
    assert abs(good["p"][0] - 0.5 * acc / (0.5 * acc + 0.5 * (1 - acc))) < 1e-15
    assert good["p"][1] == 0.3
    bad = E.update_belief(desc(), b, 5, 2, 2, 0)
    assert abs(bad["p"][0] - 0.5 * (1 - acc) / (0.5 * (1 - acc) + 0.5 * acc)) < 1e-15
    # a reading of the other rock, at distance sqrt(9 + 9)
    acc1 = 0.5 + 0.5 * 2 ** (-np.sqrt(18.0) / 20.0)
    r1 = E.update_belief(desc(), dict(x=2, y=0, p=np.array([0.5, 0.3])), 6, 1, 2, 0)
    assert abs(r1["p"][1] - 0.3 * acc1 / (0.3 * acc1 + 0.7 * (1 - acc1))) < 1e-15


def test_sample_and_moves():
    b = dict(x=5, y=3, p=np.array([0.5, 0.9]))
    s = E.update_belief(desc(), b, 4, 0, 5, 3)  # sample at rock 1's cell
    assert s["p"][1] == 0.0 and s["p"][0] == 0.5
    m = E.update_belief(desc(), b, 2, 0, 6, 3)  # move east
    assert (m["x"], m["y"]) == (6, 3) and np.array_equal(m["p"], b["p"])
    # a certain rock stays certain under any reading
    c = E.update_belief(desc(), dict(x=2, y=3, p=np.array([1.0, 0.0])), 5, 2, 2, 3)
    assert c["p"][0] == 1.0
