"""Pin: the scenario-determinised model against the true POMDP (Sec. II).

For fixed conditional plans on a tiny RockSample, the exact expected
discounted return follows from the POMDP's probabilities (prior p, sensor
accuracy 0.5 + 0.5 2^(-d/20), Bayes rule of Eq. 3).  The mean over K
sampled scenarios (Sec. III-A) of the same plan, run through the oracle's
step function, is an unbiased estimate of it and must lie within 4
standard errors.  This ties prior sampling, sensor noise, per-depth random
numbers, rewards and dynamics to the model's definition.
"""
import numpy as np
import pytest

import oracle

G = 0.95
N, ROCK = 3, (1, 0)
START = (0, 1)


def model():
    return dict(kind=0, n=N, m=1, rock_x=np.array([ROCK[0]], np.int32),
                rock_y=np.array([ROCK[1]], np.int32), gamma=G, start_x=0, start_y=1, n_actions=6)


def accuracy(cell):
    d = np.hypot(cell[0] - ROCK[0], cell[1] - ROCK[1])
    return 0.5 + 0.5 * 2 ** (-d / 20)


def run_plan(plan, K, p, seed):
    """Run a plan (function of the observation history) on K scenarios."""
    d = model()
    st = oracle.sample_scenarios(d, dict(x=START[0], y=START[1], p=np.array([p])), K, seed, 0)
    ids = np.arange(K)
    ret = np.zeros(K)
    hist = [[] for _ in range(K)]
    for t in range(12):
        acts = np.array([plan(h) for h in hist])
        nxt = dict(w=st["w"].copy())
        for a in np.unique(acts):
            sel = np.nonzero(acts == a)[0]
            sub = oracle.take_states(d, st, sel)
            o, r, z = oracle.step(d, sub, ids[sel], int(a), t, seed, 0)
            nxt["w"][sel] = o["w"]
            ret[sel] += G ** t * r.astype(np.float64)
            for k, zz in zip(sel, z):
                hist[k].append(int(zz))
        st = nxt
    return ret


E, S, SAMPLE, SENSE = 2, 1, 4, 5


def plan_sense_once(h):
    # sense from the start; on "good" walk to the rock, sample, leave east
    if len(h) == 0:
        return SENSE
    if h[0] == 1:
        return [E, S, SAMPLE, E, E, E][min(len(h) - 1, 5)]
    return E


def exact_sense_once(p):
    acc = accuracy(START)
    p_good_obs = p * acc + (1 - p) * (1 - acc)
    sample = 10 * (p * acc) - 10 * ((1 - p) * (1 - acc))  # joint good/bad with a "good" reading
    return G ** 3 * sample + p_good_obs * G ** 5 * 10 + (1 - p_good_obs) * G ** 3 * 10


def plan_sense_twice(h):
    # two readings at different depths; sample only on two "good" readings
    if len(h) < 2:
        return SENSE
    if h[0] == 1 and h[1] == 1:
        return [E, S, SAMPLE, E, E, E][min(len(h) - 2, 5)]
    return E


def exact_sense_twice(p):
    acc = accuracy(START)
    gg = p * acc ** 2 + (1 - p) * (1 - acc) ** 2
    sample = 10 * p * acc ** 2 - 10 * (1 - p) * (1 - acc) ** 2
    return G ** 4 * sample + gg * G ** 6 * 10 + (1 - gg) * G ** 4 * 10


@pytest.mark.parametrize("p", [0.5, 0.3, 0.8])
@pytest.mark.parametrize("plan,exact", [(plan_sense_once, exact_sense_once),
                                        (plan_sense_twice, exact_sense_twice)])
def test_plan_value_matches_pomdp(plan, exact, p):
    K = 60000
    ret = run_plan(plan, K, p, seed=17)
    se = ret.std(ddof=1) / np.sqrt(K)
    assert abs(ret.mean() - exact(p)) < 4 * se + 1e-12
