"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only draws numbers: model layouts, beliefs and leaf shapes, as
plain numpy arrays of model-level fields (positions, rock qualities, speeds).
It computes nothing of the planning method itself (no step function, no
random stream of the method, no bounds, no grouping), so it can feed both
sides of a parity test without coupling them.

Shapes follow the paper's workloads: RockSample grids with seeded rock
layouts (the canonical benchmark layouts are not used), and a crowd-driving
task with pedestrians, goal points and a straight car path (Sec. IV-A).
"""
from __future__ import annotations

import numpy as np

ROCKSAMPLE = 0
PEDNAV = 1
MARS = 2
NAV = 3


def rocksample_model(n: int, m: int, seed: int, gamma: float = 0.95) -> dict:
    """An n x n RockSample grid with m rocks on distinct seeded cells.

    The robot starts at column 0, row n // 2; no rock is placed on the start
    cell, so a sample there is never rewarded.  Action count is 5 + m
    (four moves, sample, one sense per rock).
    """
    if not (1 <= n <= 31) or not (0 <= m <= 20):
        raise ValueError("need 1 <= n <= 31 and 0 <= m <= 20")
    rng = np.random.default_rng(np.random.SeedSequence([0x525337, n, m, seed]))
    start = (0, n // 2)
    cells = [c for c in range(n * n) if (c % n, c // n) != start]
    if m > len(cells):
        raise ValueError("too many rocks for the grid")
    pick = rng.permutation(len(cells))[:m]
    rx = np.array([cells[i] % n for i in pick], dtype=np.int32)
    ry = np.array([cells[i] // n for i in pick], dtype=np.int32)
    return dict(kind=ROCKSAMPLE, n=n, m=m, rock_x=rx, rock_y=ry, gamma=gamma,
                start_x=start[0], start_y=start[1], n_actions=5 + m)


def rocksample_belief(model: dict, p_good: float = 0.5, x=None, y=None) -> dict:
    """Initial belief: known robot cell, independent rock qualities."""
    m = model["m"]
    return dict(x=model["start_x"] if x is None else x,
                y=model["start_y"] if y is None else y,
                p=np.full(m, p_good, dtype=np.float64))


def mars_model(n: int, m: int, seed: int, gamma: float = 0.95) -> dict:
    """Multi-agent RockSample(n, m): two robots on an n x n grid with m rocks
    on distinct seeded cells (Sec. IV-A).

    Robot 1 starts at column 0, row n // 2, robot 2 at column 0, row
    n // 2 - 1; no rock lies on a start cell.  Each robot has 5 + m actions
    (four moves, sample, one sense per rock), so the joint action count is
    (5 + m)^2: 256, 400 and 625 for (11, 11), (15, 15) and (20, 20).
    """
    if not (2 <= n <= 31) or not (0 <= m <= 20):
        raise ValueError("need 2 <= n <= 31 and 0 <= m <= 20")
    rng = np.random.default_rng(np.random.SeedSequence([0x4D4152, n, m, seed]))
    starts = [(0, n // 2), (0, n // 2 - 1)]
    cells = [c for c in range(n * n) if (c % n, c // n) not in starts]
    if m > len(cells):
        raise ValueError("too many rocks for the grid")
    pick = rng.permutation(len(cells))[:m]
    rx = np.array([cells[i] % n for i in pick], dtype=np.int32)
    ry = np.array([cells[i] // n for i in pick], dtype=np.int32)
    return dict(kind=MARS, n=n, m=m, rock_x=rx, rock_y=ry, gamma=gamma,
                start=(starts[0][0], starts[0][1], starts[1][0], starts[1][1]),
                n_actions=(5 + m) ** 2)


def mars_belief(model: dict, p_good: float = 0.5, pos=None) -> dict:
    """Initial belief: known robot cells (pos = (x1, y1, x2, y2, gone1,
    gone2)), independent rock qualities."""
    if pos is None:
        pos = (*model["start"], 0, 0)
    return dict(pos=tuple(int(v) for v in pos), p=np.full(model["m"], p_good, dtype=np.float64))


def nav_model(seed: int, n: int = 13, n_landmarks: int = 8, p_occ: float = 0.1,
              gamma: float = 0.95) -> dict:
    """Navigation in a partially known n x n map (Sec. IV-A; 13 x 13 in the paper).

    Row 0 (the top border, where the robot starts at a random column) and
    row n-1 (the goal's row, goal column seeded) are known free.  The middle
    row is a known wall except two seeded gate columns, which are unknown
    cells 0 and 1 (exactly one open).  Of the remaining cells, n_landmarks
    seeded ones are known walls and the rest are unknown, each occupied with
    probability p_occ: at n = 13 that is 2 + 122 = 124 unknown cells, the
    paper's 169 x 2^124 states.  Nine actions (stay, eight neighbours).
    """
    if not (5 <= n <= 16):
        raise ValueError("need 5 <= n <= 16")
    rng = np.random.default_rng(np.random.SeedSequence([0x4E4156, n, seed]))
    wall = n // 2
    cell = np.full((n, n), -1, dtype=np.int64)  # [y][x]
    cell[wall, :] = -2
    gates = np.sort(rng.choice(np.arange(1, n - 1), size=2, replace=False))
    for i, gx in enumerate(gates):
        cell[wall, gx] = i
    mid = [(x, y) for y in range(1, n - 1) if y != wall for x in range(n)]
    order = rng.permutation(len(mid))
    for j in order[:n_landmarks]:
        x, y = mid[j]
        cell[y, x] = -2
    u = 2
    for j in np.sort(order[n_landmarks:]):
        x, y = mid[j]
        cell[y, x] = u
        u += 1
    if u > 128:
        raise ValueError("more than 128 unknown cells")
    return dict(kind=NAV, n=n, cell=cell, wall=wall, gate_x=gates.astype(np.int32),
                goal_x=int(rng.integers(0, n)), n_unknown=u, p_occ=p_occ, gamma=gamma,
                p_fail=0.03, p_err=0.03, n_actions=9)


def nav_belief(model: dict) -> dict:
    """Initial belief: robot somewhere on the top row, one gate open (1/2
    each), every other unknown cell occupied with probability p_occ."""
    p = np.full(model["n_unknown"], model["p_occ"], dtype=np.float64)
    p[:2] = 0.5
    return dict(p=p)


def pednav_model(n_peds: int, n_goals: int, seed: int, gamma: float = 0.98,
                 path_len: float = 40.0) -> dict:
    """A car on a straight path from (0, 0) to (path_len, 0) among pedestrians.

    Goal points and the pedestrians' initial positions are seeded in
    [5, path_len] x [-6, 6].  Three actions: accelerate, maintain, decelerate.
    """
    if not (0 <= n_peds <= 32) or not (1 <= n_goals <= 8):
        raise ValueError("need 0 <= n_peds <= 32 and 1 <= n_goals <= 8")
    rng = np.random.default_rng(np.random.SeedSequence([0x504544, n_peds, n_goals, seed]))
    gx = rng.uniform(5.0, path_len, n_goals).astype(np.float32)
    gy = rng.uniform(-6.0, 6.0, n_goals).astype(np.float32)
    px = rng.uniform(5.0, path_len, n_peds).astype(np.float32)
    py = rng.uniform(-6.0, 6.0, n_peds).astype(np.float32)
    return dict(kind=PEDNAV, n_peds=n_peds, n_goals=n_goals, goal_x=gx, goal_y=gy,
                ped_x0=px, ped_y0=py, gamma=gamma, path_len=path_len, dt=0.5,
                ped_speed=1.2, sigma_h=0.3, p_fail=0.01, coll_radius=1.0,
                r_collision=-1000.0, r_step=-0.1, r_goal=100.0, n_levels=5,
                n_actions=3)


def pednav_belief(model: dict, goal_p=None, s: float = 0.0, level: int = 2) -> dict:
    """Initial belief: known car and pedestrian positions, unknown goals."""
    P, G = model["n_peds"], model["n_goals"]
    if goal_p is None:
        goal_p = np.full((P, G), 1.0 / G)
    return dict(s=np.float32(s), level=int(level), px=model["ped_x0"].copy(),
                py=model["ped_y0"].copy(), goal_p=np.asarray(goal_p, dtype=np.float64))


def _sorted_subset(rng, universe: int, size: int) -> np.ndarray:
    return np.sort(rng.choice(universe, size=size, replace=False)).astype(np.int32)


def rocksample_leaf(model: dict, n_parent: int, n_leaf: int, seed: int,
                    k_root: int | None = None, p_term: float = 0.02,
                    depth: int | None = None, shared_cell: bool = True) -> dict:
    """A synthetic RockSample leaf with the shape of one deep in a DESPOT tree.

    The parent holds ``n_parent`` scenarios sharing one robot cell (position
    is deterministic in RockSample), random rock qualities and a few terminal
    scenarios; the leaf is an ascending subset of ``n_leaf`` of them.  With
    shared_cell=False every scenario draws its own cell (states the model
    never produces from one root, but valid inputs of an expansion).
    """
    rng = np.random.default_rng(np.random.SeedSequence([0x4C4541, n_parent, n_leaf, seed]))
    n, m = model["n"], model["m"]
    k_root = max(k_root or n_parent, n_parent)
    leaf = dict(x=int(rng.integers(0, n)), y=int(rng.integers(0, n)),
                rocks=rng.random((n_parent, m)) < 0.5,
                term=rng.random(n_parent) < p_term,
                ids=_sorted_subset(rng, k_root, n_parent),
                idx=_sorted_subset(rng, n_parent, n_leaf),
                depth=int(rng.integers(1, 16)) if depth is None else depth,
                last_action=int(rng.integers(0, model["n_actions"])))
    if not shared_cell:
        leaf["x"] = rng.integers(0, n, n_parent)
        leaf["y"] = rng.integers(0, n, n_parent)
    return leaf


def mars_leaf(model: dict, n_parent: int, n_leaf: int, seed: int,
              k_root: int | None = None, p_term: float = 0.02,
              depth: int | None = None, shared_cells: bool = True) -> dict:
    """A synthetic multi-agent RockSample leaf.

    Robot cells are deterministic in the model, so by default the parent's
    scenarios share both cells (and a robot that has left, with probability
    0.2 each); with shared_cells=False every scenario draws its own cells.
    A few scenarios are terminal (both robots gone).
    """
    rng = np.random.default_rng(np.random.SeedSequence([0x4D4C46, n_parent, n_leaf, seed]))
    n, m = model["n"], model["m"]
    k_root = max(k_root or n_parent, n_parent)
    size = 1 if shared_cells else n_parent
    cells = [rng.integers(0, n, size) for _ in range(4)]
    gone = [(rng.random(size) < 0.2).astype(np.int64) for _ in range(2)]
    both = gone[0] & gone[1]
    gone[1] = gone[1] & ~both  # at most one robot gone unless terminal
    term = rng.random(n_parent) < p_term
    g1 = np.broadcast_to(gone[0], (n_parent,)) | term
    g2 = np.broadcast_to(gone[1], (n_parent,)) | term
    pos = tuple(np.broadcast_to(c, (n_parent,)).astype(np.int64) for c in cells) + (g1.astype(np.int64),
                                                                                   g2.astype(np.int64))
    return dict(pos=pos, rocks=rng.random((n_parent, m)) < 0.5, term=term.astype(np.int64),
                ids=_sorted_subset(rng, k_root, n_parent),
                idx=_sorted_subset(rng, n_parent, n_leaf),
                depth=int(rng.integers(1, 16)) if depth is None else depth,
                last_action=int(rng.integers(0, model["n_actions"])))


def nav_leaf(model: dict, n_parent: int, n_leaf: int, seed: int, k_root: int | None = None,
             p_term: float = 0.02, depth: int | None = None, shared_cell: bool = False) -> dict:
    """A synthetic navigation leaf: robot cells near one another (moves can
    fail, so a node's scenarios spread out), maps drawn from the prior."""
    rng = np.random.default_rng(np.random.SeedSequence([0x4E4C46, n_parent, n_leaf, seed]))
    n, U = model["n"], model["n_unknown"]
    k_root = max(k_root or n_parent, n_parent)
    free = [(x, y) for y in range(n) for x in range(n) if model["cell"][y, x] != -2]
    cx, cy = free[int(rng.integers(0, len(free)))]
    if shared_cell:
        x = np.full(n_parent, cx, np.int64)
        y = np.full(n_parent, cy, np.int64)
    else:
        x = np.clip(cx + rng.integers(-1, 2, n_parent), 0, n - 1)
        y = np.clip(cy + rng.integers(-1, 2, n_parent), 0, n - 1)
    cells = rng.random((n_parent, U)) < model["p_occ"]
    g = rng.random(n_parent) < 0.5
    cells[:, 0], cells[:, 1] = ~g, g
    # a robot never stands in an occupied cell
    for k in range(n_parent):
        c = model["cell"][y[k], x[k]]
        if c == -2:
            x[k], y[k] = cx, cy
            c = model["cell"][cy, cx]
        if c >= 0:
            cells[k, c] = False
    return dict(x=x, y=y, cells=cells, term=rng.random(n_parent) < p_term,
                ids=_sorted_subset(rng, k_root, n_parent),
                idx=_sorted_subset(rng, n_parent, n_leaf),
                depth=int(rng.integers(1, 30)) if depth is None else depth,
                last_action=int(rng.integers(0, 9)))


def pednav_leaf(model: dict, n_parent: int, n_leaf: int, seed: int,
                k_root: int | None = None, p_term: float = 0.02,
                depth: int | None = None) -> dict:
    """A synthetic crowd-driving leaf: per-scenario car and pedestrian fields."""
    rng = np.random.default_rng(np.random.SeedSequence([0x504C46, n_parent, n_leaf, seed]))
    P, G = model["n_peds"], model["n_goals"]
    k_root = max(k_root or n_parent, n_parent)
    s0 = rng.uniform(0.0, model["path_len"] * 0.8)
    jitter = 0.7
    return dict(s=np.float32(s0) + rng.uniform(-1.0, 1.0, n_parent).astype(np.float32),
                level=rng.integers(0, model["n_levels"], n_parent).astype(np.int32),
                term=rng.random(n_parent) < p_term,
                px=(model["ped_x0"][:, None] + rng.uniform(-jitter, jitter, (P, n_parent))).astype(np.float32),
                py=(model["ped_y0"][:, None] + rng.uniform(-jitter, jitter, (P, n_parent))).astype(np.float32),
                goal=rng.integers(0, G, (P, n_parent)).astype(np.uint8),
                ids=_sorted_subset(rng, k_root, n_parent),
                idx=_sorted_subset(rng, n_parent, n_leaf),
                depth=int(rng.integers(1, 12)) if depth is None else depth,
                last_action=int(rng.integers(0, 3)))


def mixed_instances(count: int, seed: int) -> list[dict]:
    """Independent planner instances of uneven size: RockSample with
    probability 0.75 (grid 7..20, rocks 8..20), else crowd driving;
    scenario count K drawn from {100, 200, 500}."""
    rng = np.random.default_rng(np.random.SeedSequence([0x4D4958, count, seed]))
    out = []
    for i in range(count):
        K = int(rng.choice([100, 200, 500]))
        if rng.random() < 0.75:
            n = int(rng.integers(7, 21))
            m = int(rng.integers(8, min(20, n * n - 1) + 1))
            out.append(dict(model=rocksample_model(n, m, seed * 1000 + i), K=K))
        else:
            out.append(dict(model=pednav_model(16, 5, seed * 1000 + i), K=K))
    return out
