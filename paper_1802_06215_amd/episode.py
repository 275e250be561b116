"""Closed-loop planning on RockSample (the online loop of Sec. III-A).

At every step the planner runs hdx_search from the current belief, the best
action is executed in a true environment, and the belief is updated from the
observation.  The true environment is stepped by the library's own
expansion kernel (a one-scenario leaf whose parent is the true state, with a
random-number key of its own), so the environment and the planner share one
model definition.  The belief (the robot cell and each rock's probability
of being good) is updated by the library's hdx_belief_update (Eq. 3).  This
module is a driver of the library's calls and holds none of the method's
arithmetic.
"""
from __future__ import annotations

import numpy as np
import torch

from . import hdx as H


class RockSampleEnv:
    """The true state of one episode, stepped on the device."""

    def __init__(self, ctx: "H.Context", model: "H.Model", x: int, y: int, rocks, seed: int):
        self.ctx, self.model = ctx, model
        self.rocks = np.asarray(rocks, dtype=bool).copy()
        self.x, self.y, self.term = int(x), int(y), False
        self.seed = seed
        self.t = 0
        self._ids = torch.zeros(1, dtype=torch.int32, device="cuda")
        self._idx = torch.zeros(1, dtype=torch.int16, device="cuda")
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


def run_rocksample(ctx: "H.Context", model: "H.Model", desc: dict, true_rocks, max_steps: int,
                   env_seed: int = 12345, on_step=None, **search_kwargs) -> dict:
    """One episode: plan, act, observe, update, until the robot exits or
    max_steps.  search_kwargs go to Context.search (K, n_threads, time
    budget, ...); its step key is the time step.  on_step(t, action,
    reward, search_result), when given, is called after every step."""
    x0, y0 = int(desc["start_x"]), int(desc["start_y"])
    belief = dict(x=x0, y=y0, p=np.full(desc["m"], 0.5))
    env = RockSampleEnv(ctx, model, x0, y0, true_rocks, env_seed)
    gamma, disc, total = desc["gamma"], 1.0, 0.0
    actions, rewards, trials, plan_s = [], [], [], []
    for t in range(max_steps):
        res = ctx.search(model, belief, step=t, **search_kwargs)
        plan_s.append(res["elapsed_s"])
        a = int(res["best_action"])
        r, z = env.step(a)
        actions.append(a)
        rewards.append(r)
        trials.append(res["trials"])
        if on_step is not None:
            on_step(t, a, r, res)
        total += disc * r
        disc *= gamma
        if env.term:
            break
        belief, _ = H.belief_update(desc, belief, a, z)
        assert (belief["x"], belief["y"]) == (env.x, env.y)
    return dict(actions=actions, rewards=rewards, discounted_return=total, steps=len(actions),
                exited=env.term, trials=trials, planning_s=plan_s)
