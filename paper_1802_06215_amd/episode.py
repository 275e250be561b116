"""Closed-loop planning on RockSample (the online loop of Sec. III-A).

At every step the planner runs hdx_search from the current belief, the best
action is executed in a true environment, and the belief is updated from the
observation.  The true environment is stepped by the library's own
expansion kernel (a one-scenario leaf whose parent is the true state, with a
random-number key of its own), so the environment and the planner share one
model definition.  The belief is the robot cell (observed) and each rock's
probability of being good, updated by Bayes' rule on a sensor reading: a
reading is correct with probability 0.5 + 0.5 * 2^(-d/20) at Euclidean
distance d; a sampled rock is known to be bad afterwards.
"""
from __future__ import annotations

import numpy as np
import torch

from . import hdx as H


def sensor_accuracy(d: float) -> float:
    return 0.5 + 0.5 * 2.0 ** (-d / 20.0)


class RockSampleEnv:
    """The true state of one episode, stepped on the device."""

    def __init__(self, ctx: "H.Context", model: "H.Model", x: int, y: int, rocks, seed: int):
        self.ctx, self.model = ctx, model
        self.rocks = np.asarray(rocks, dtype=bool).copy()
        self.x, self.y, self.term = int(x), int(y), False
        self.seed = seed
        self.t = 0
        self._ids = torch.zeros(1, dtype=torch.int32, device="cuda")
        self._idx = torch.zeros(1, dtype=torch.int32, device="cuda")
        self._out = H.LeafBuffers(model, 1, per_pair=True)
        self._cfg = H.rollout_cfg(H.POLICY_CONST, 0, -1, 0)  # no rollouts: only the step

    def step(self, action: int):
        """Execute `action`; returns (reward, observation)."""
        par = H.rocksample_states(self.x, self.y, self.rocks[None, :], [self.term])
        leaf = H.make_leaf(self.model, par, self._ids, self._idx, self.t, -1, self._out, self.seed, 0, self._cfg)
        self.ctx.expand_leaf([leaf])
        torch.cuda.synchronize()
        w = int(self._out.sprime["w"][action].item())
        r = float(self._out.r[action, 0].item())
        z = int(self._out.z[action, 0].item())
        self.x, self.y = w & 31, (w >> 5) & 31
        self.rocks = np.array([(w >> (10 + i)) & 1 for i in range(self.rocks.shape[0])], dtype=bool)
        self.term = bool((w >> 30) & 1)
        self.t += 1
        return r, z


def update_belief(desc: dict, belief: dict, action: int, z: int, x: int, y: int) -> dict:
    """Belief after `action` with observation z, the robot now at (x, y)."""
    p = np.asarray(belief["p"], dtype=np.float64).copy()
    rx, ry = np.asarray(desc["rock_x"]), np.asarray(desc["rock_y"])
    if action == 4:  # sampling leaves the rock under the robot bad
        for i in range(desc["m"]):
            if rx[i] == belief["x"] and ry[i] == belief["y"]:
                p[i] = 0.0
    elif action >= 5:
        i = action - 5
        acc = sensor_accuracy(float(np.hypot(belief["x"] - rx[i], belief["y"] - ry[i])))
        lg, lb = (acc, 1.0 - acc) if z == 1 else (1.0 - acc, acc)
        den = p[i] * lg + (1.0 - p[i]) * lb
        p[i] = p[i] * lg / den if den > 0 else p[i]
    return dict(x=int(x), y=int(y), p=p)


def run_rocksample(ctx: "H.Context", model: "H.Model", desc: dict, true_rocks, max_steps: int,
                   env_seed: int = 12345, **search_kwargs) -> dict:
    """One episode: plan, act, observe, update, until the robot exits or
    max_steps.  search_kwargs go to Context.search (K, n_threads, time
    budget, ...); its step key is the time step."""
    x0, y0 = int(desc["start_x"]), int(desc["start_y"])
    belief = dict(x=x0, y=y0, p=np.full(desc["m"], 0.5))
    env = RockSampleEnv(ctx, model, x0, y0, true_rocks, env_seed)
    gamma, disc, total = desc["gamma"], 1.0, 0.0
    actions, rewards, trials = [], [], []
    for t in range(max_steps):
        res = ctx.search(model, belief, step=t, **search_kwargs)
        a = int(res["best_action"])
        r, z = env.step(a)
        actions.append(a)
        rewards.append(r)
        trials.append(res["trials"])
        total += disc * r
        disc *= gamma
        if env.term:
            break
        belief = update_belief(desc, belief, a, z, env.x, env.y)
    return dict(actions=actions, rewards=rewards, discounted_return=total, steps=len(actions),
                exited=env.term, trials=trials)
