"""Sequential CPU oracle for HyP-DESPOT leaf expansion.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The GPU library and its binding
never import it.

The arithmetic lives in ``oracle.c`` (plain loops, FP64 values); this module
marshals numpy arrays to it and holds the Bellman backup of Eq. 4 written out
in Python.  States use the library's documented struct-of-arrays layout:

* RockSample: ``{"w": int32[n]}`` with x in bits 0-4, y in bits 5-9, rock i's
  quality in bit 10+i and the terminal flag in bit 30;
* crowd driving: ``{"s": f32[n], "car": int32[n] (speed level | terminal<<8),
  "px": f32[P, n], "py": f32[P, n], "goal": u8[P, n]}``;
* multi-agent RockSample: ``{"w": int32[2, n]}``, row 0 the robots (robot 1's
  x, y in bits 0-4, 5-9, robot 2's in bits 10-14, 15-19, robot j gone in bit
  20+j, terminal in bit 30), row 1 the rocks (rock i's quality in bit i);
* navigation: ``{"w": int32[5, n]}``, row 0 the robot (x bits 0-3, y bits 4-7,
  terminal bit 30), rows 1-4 the unknown cells' occupancy (cell i in bit i%32
  of row 1 + i//32).

Parity pins for every function here live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain host code, contraction off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Model(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_actions", C.c_int32), ("gamma", C.c_double),
                ("n", C.c_int32), ("m", C.c_int32),
                ("rock_x", C.c_int32 * 20), ("rock_y", C.c_int32 * 20),
                ("n_peds", C.c_int32), ("n_goals", C.c_int32), ("n_levels", C.c_int32),
                ("pad_", C.c_int32),
                ("goal_x", C.c_float * 8), ("goal_y", C.c_float * 8),
                ("path_len", C.c_float), ("dt", C.c_float), ("ped_speed", C.c_float),
                ("sigma_h", C.c_float), ("coll_radius", C.c_float),
                ("r_collision", C.c_float), ("r_step", C.c_float), ("r_goal", C.c_float),
                ("p_fail", C.c_double),
                ("nav_goal_x", C.c_int32), ("nav_wall", C.c_int32), ("nav_gate_x", C.c_int32 * 2),
                ("nav_cell", C.c_int16 * 256), ("p_err", C.c_double)]


class _Cfg(C.Structure):
    _fields_ = [("policy", C.c_int32), ("const_action", C.c_int32),
                ("max_steps", C.c_int32), ("max_depth", C.c_int32)]


class _Soa(C.Structure):
    _fields_ = [("w", C.c_void_p), ("s", C.c_void_p), ("car", C.c_void_p),
                ("px", C.c_void_p), ("py", C.c_void_p), ("goal", C.c_void_p),
                ("stride", C.c_int64)]


class _Out(C.Structure):
    _fields_ = [("states", _Soa), ("ids", C.c_void_p), ("sprime", _Soa),
                ("r", C.c_void_p), ("z", C.c_void_p), ("U", C.c_void_p), ("L", C.c_void_p),
                ("Labs", C.c_void_p), ("child_of", C.c_void_p), ("perm", C.c_void_p), ("n_children", C.c_void_p),
                ("child_z", C.c_void_p), ("child_n", C.c_void_p), ("child_off", C.c_void_p),
                ("child_u0", C.c_void_p), ("child_l0", C.c_void_p), ("r_mean", C.c_void_p),
                ("expand_steps", C.c_void_p), ("rollout_steps", C.c_void_p), ("steps", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.or_philox4x32_10.argtypes = [P, P, P, C.c_int64]
        L.or_step_batch.argtypes = [P, P, P, C.c_int64, C.c_int32, C.c_int32, C.c_uint32,
                                    C.c_uint32, P, P, P]
        L.or_sample_scenarios.argtypes = [P, C.c_int32, C.c_uint32, C.c_uint32, C.c_int32,
                                          C.c_int32, P, C.c_float, C.c_int32, P, P, P, P]
        L.or_rollout_bounds.argtypes = [P, P, C.c_uint32, C.c_uint32, P, P, P, C.c_int64, P, P, P, P]
        L.or_expand_leaf.argtypes = [P, P, C.c_uint32, C.c_uint32, P, P, P, C.c_int32, C.c_int32,
                                     C.c_int32, C.c_int32, P]
        L.or_expand_leaf.restype = C.c_int
        L.or_rs_sense_threshold.argtypes = [C.c_int32]
        L.or_rs_sense_threshold.restype = C.c_uint64
        L.or_mix64.argtypes = [C.c_uint64]
        L.or_mix64.restype = C.c_uint64
        L.or_despot.argtypes = [P, P, C.c_uint32, C.c_uint32, P, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                C.c_int64, P]
        L.or_despot.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


# --------------------------------------------------------------------------
# Philox4x32-10 and the state layout
# --------------------------------------------------------------------------
def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 blocks for counters ``ctr`` (N x 4 uint32), key (2,)."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
    out = np.empty_like(ctr)
    lib().or_philox4x32_10(_ptr(ctr), _ptr(key), _ptr(out), ctr.shape[0])
    return out


def rs_pack(x, y, rocks, term) -> np.ndarray:
    """RockSample state words from fields (rocks: bool [n, m])."""
    rocks = np.asarray(rocks, dtype=bool)
    n = rocks.shape[0]
    w = np.broadcast_to(np.asarray(x, np.int64) | (np.asarray(y, np.int64) << 5), (n,)).copy()
    for i in range(rocks.shape[1]):
        w |= rocks[:, i].astype(np.int64) << (10 + i)
    w |= np.asarray(term, dtype=np.int64) << 30
    return w.astype(np.int32)


def rs_unpack(w) -> dict:
    w = np.asarray(w, dtype=np.int64)
    return dict(x=w & 31, y=(w >> 5) & 31, rocks=(w >> 10) & 0xFFFFF, term=(w >> 30) & 1)


def mars_pack(pos, rocks, term=None) -> np.ndarray:
    """Multi-agent RockSample states [2, n] from fields: pos = (x1, y1, x2,
    y2, gone1, gone2), each a scalar or an [n] array; rocks: bool [n, m];
    term defaults to both robots gone."""
    rocks = np.asarray(rocks, dtype=bool)
    n = rocks.shape[0]
    x1, y1, x2, y2, g1, g2 = (np.broadcast_to(np.asarray(f, dtype=np.int64), (n,)) for f in pos)
    if term is None:
        term = g1 & g2
    row0 = x1 | (y1 << 5) | (x2 << 10) | (y2 << 15) | (g1 << 20) | (g2 << 21)
    row0 = row0 | (np.asarray(term, dtype=np.int64) << 30)
    row1 = np.zeros(n, dtype=np.int64)
    for i in range(rocks.shape[1]):
        row1 |= rocks[:, i].astype(np.int64) << i
    return np.stack([row0, row1]).astype(np.int32)


def mars_unpack(w) -> dict:
    w = np.asarray(w, dtype=np.int64)
    r0 = w[0]
    return dict(x1=r0 & 31, y1=(r0 >> 5) & 31, x2=(r0 >> 10) & 31, y2=(r0 >> 15) & 31,
                gone1=(r0 >> 20) & 1, gone2=(r0 >> 21) & 1, term=(r0 >> 30) & 1, rocks=w[1])


def nav_pack(x, y, cells, term) -> np.ndarray:
    """Navigation states [5, n] from fields: robot x, y (scalars or [n]),
    unknown-cell occupancy bool [n, U] (U <= 128), terminal flags."""
    cells = np.asarray(cells, dtype=bool)
    n = cells.shape[0]
    out = np.zeros((5, n), dtype=np.int64)
    out[0] = (np.broadcast_to(np.asarray(x, np.int64), (n,)) | (np.broadcast_to(np.asarray(y, np.int64), (n,)) << 4)
              | (np.asarray(term, dtype=np.int64) << 30))
    for i in range(cells.shape[1]):
        out[1 + i // 32] |= cells[:, i].astype(np.int64) << (i % 32)
    return out.astype(np.uint32).view(np.int32)


def nav_unpack(w) -> dict:
    w = np.asarray(w).view(np.uint32).astype(np.int64)
    U = 128
    cells = np.stack([(w[1 + i // 32] >> (i % 32)) & 1 for i in range(U)], axis=-1).astype(bool)
    return dict(x=w[0] & 15, y=(w[0] >> 4) & 15, term=(w[0] >> 30) & 1, cells=cells)


def parent_states(desc: dict, leaf: dict) -> dict:
    """States dict for a synthetic leaf's parent (fields from ``workloads``)."""
    if desc["kind"] == 0:
        return dict(w=rs_pack(leaf["x"], leaf["y"], leaf["rocks"], leaf["term"]))
    if desc["kind"] == 2:
        return dict(w=mars_pack(leaf["pos"], leaf["rocks"], leaf["term"]))
    if desc["kind"] == 3:
        return dict(w=nav_pack(leaf["x"], leaf["y"], leaf["cells"], leaf["term"]))
    car = leaf["level"].astype(np.int32) | (leaf["term"].astype(np.int32) << 8)
    return dict(s=np.ascontiguousarray(leaf["s"], dtype=np.float32), car=car.astype(np.int32),
                px=np.ascontiguousarray(leaf["px"], dtype=np.float32),
                py=np.ascontiguousarray(leaf["py"], dtype=np.float32),
                goal=np.ascontiguousarray(leaf["goal"], dtype=np.uint8))


def empty_states(desc: dict, n: int) -> dict:
    if desc["kind"] == 0:
        return dict(w=np.zeros(n, np.int32))
    if desc["kind"] == 2:
        return dict(w=np.zeros((2, n), np.int32))
    if desc["kind"] == 3:
        return dict(w=np.zeros((5, n), np.int32))
    P = desc["n_peds"]
    return dict(s=np.zeros(n, np.float32), car=np.zeros(n, np.int32),
                px=np.zeros((P, n), np.float32), py=np.zeros((P, n), np.float32),
                goal=np.zeros((P, n), np.uint8))


def _soa(desc: dict, st: dict | None, n: int) -> _Soa:
    v = _Soa()
    if st is None:
        return v
    if desc["kind"] in (0, 2, 3):
        v.w = _ptr(st["w"])
    else:
        v.s, v.car = _ptr(st["s"]), _ptr(st["car"])
        v.px, v.py, v.goal = _ptr(st["px"]), _ptr(st["py"]), _ptr(st["goal"])
    v.stride = n
    return v


def _check_states(desc, st):
    if desc["kind"] == 0:
        assert st["w"].dtype == np.int32 and st["w"].flags.c_contiguous
        return st["w"].shape[0]
    if desc["kind"] in (2, 3):
        assert st["w"].dtype == np.int32 and st["w"].flags.c_contiguous
        assert st["w"].shape[0] == (2 if desc["kind"] == 2 else 5)
        return st["w"].shape[1]
    n = st["s"].shape[0]
    P = desc["n_peds"]
    assert st["px"].shape == (P, n) and st["goal"].dtype == np.uint8
    for k in ("s", "car", "px", "py", "goal"):
        assert st[k].flags.c_contiguous
    return n


def model(desc: dict) -> _Model:
    m = _Model()
    m.kind = desc["kind"]
    m.n_actions = desc["n_actions"]
    m.gamma = desc["gamma"]
    if desc["kind"] == 3:
        m.n = desc["n"]
        m.p_fail, m.p_err = desc["p_fail"], desc["p_err"]
        m.nav_goal_x, m.nav_wall = desc["goal_x"], desc["wall"]
        m.nav_gate_x[0], m.nav_gate_x[1] = int(desc["gate_x"][0]), int(desc["gate_x"][1])
        cell = np.asarray(desc["cell"], np.int64).reshape(-1)
        for c in range(cell.shape[0]):
            m.nav_cell[c] = int(cell[c])
    elif desc["kind"] in (0, 2):
        m.n, m.m = desc["n"], desc["m"]
        for i in range(desc["m"]):
            m.rock_x[i] = int(desc["rock_x"][i])
            m.rock_y[i] = int(desc["rock_y"][i])
    else:
        m.n_peds, m.n_goals, m.n_levels = desc["n_peds"], desc["n_goals"], desc["n_levels"]
        for g in range(desc["n_goals"]):
            m.goal_x[g] = float(desc["goal_x"][g])
            m.goal_y[g] = float(desc["goal_y"][g])
        for f in ("path_len", "dt", "ped_speed", "sigma_h", "coll_radius", "r_collision",
                  "r_step", "r_goal"):
            setattr(m, f, float(desc[f]))
        m.p_fail = desc["p_fail"]
    return m


def cfg(policy: int = 0, max_steps: int = 1 << 30, max_depth: int = -1,
        const_action: int = 0) -> _Cfg:
    """Rollout configuration: policy 0 = model default (RockSample: move
    east; multi-agent RockSample: both robots move east; crowd driving: brake
    for a pedestrian ahead, else accelerate),
    1 = constant action, 2 = uniform random action per step."""
    c = _Cfg()
    c.policy, c.const_action, c.max_steps, c.max_depth = policy, const_action, max_steps, max_depth
    return c


# --------------------------------------------------------------------------
# Model entry points
# --------------------------------------------------------------------------
def step(desc, states, ids, action, depth, seed, step_idx):
    """One application of g with a single action to every state."""
    n = _check_states(desc, states)
    out = empty_states(desc, n)
    r = np.zeros(n, np.float32)
    z = np.zeros(n, np.uint64)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    M = model(desc)
    lib().or_step_batch(C.byref(M), C.byref(_soa(desc, states, n)), _ptr(ids), n, action, depth,
                        seed, step_idx, C.byref(_soa(desc, out, n)), _ptr(r), _ptr(z))
    return out, r, z


def sample_scenarios(desc, belief, K, seed, step_idx):
    out = empty_states(desc, K)
    M = model(desc)
    if desc["kind"] == 0:
        p = np.ascontiguousarray(belief["p"], dtype=np.float64)
        lib().or_sample_scenarios(C.byref(M), K, seed, step_idx, belief["x"], belief["y"], _ptr(p),
                                  0.0, 0, None, None, None, C.byref(_soa(desc, out, K)))
    elif desc["kind"] == 3:
        p = np.ascontiguousarray(belief["p"], dtype=np.float64)
        lib().or_sample_scenarios(C.byref(M), K, seed, step_idx, 0, 0, _ptr(p),
                                  0.0, 0, None, None, None, C.byref(_soa(desc, out, K)))
    elif desc["kind"] == 2:
        p = np.ascontiguousarray(belief["p"], dtype=np.float64)
        row0 = int(mars_pack(belief["pos"], np.zeros((1, 0), bool))[0, 0])
        lib().or_sample_scenarios(C.byref(M), K, seed, step_idx, row0, 0, _ptr(p),
                                  0.0, 0, None, None, None, C.byref(_soa(desc, out, K)))
    else:
        px = np.ascontiguousarray(belief["px"], dtype=np.float32)
        py = np.ascontiguousarray(belief["py"], dtype=np.float32)
        gp = np.ascontiguousarray(belief["goal_p"], dtype=np.float64)
        lib().or_sample_scenarios(C.byref(M), K, seed, step_idx, 0, 0, None,
                                  float(belief["s"]), int(belief["level"]), _ptr(px), _ptr(py),
                                  _ptr(gp), C.byref(_soa(desc, out, K)))
    return out


def rollout_bounds(desc, rcfg, states, ids, depths, seed, step_idx, with_abs: bool = False):
    """Upper bound and rollout value per state; with_abs also returns the
    sum of absolute discounted rollout terms (a scale for FP tolerances)."""
    n = _check_states(desc, states)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    depths = np.ascontiguousarray(np.broadcast_to(depths, (n,)), dtype=np.int32)
    U = np.zeros(n)
    L = np.zeros(n)
    Labs = np.zeros(n)
    steps = np.zeros(n, np.int64)
    M = model(desc)
    lib().or_rollout_bounds(C.byref(M), C.byref(rcfg), seed, step_idx,
                            C.byref(_soa(desc, states, n)), _ptr(ids), _ptr(depths), n,
                            _ptr(U), _ptr(L), _ptr(steps), _ptr(Labs))
    if with_abs:
        return U, L, steps, Labs
    return U, L, steps


def max_children(desc: dict, n: int) -> int:
    """Most children one action can have: RockSample observations take 3
    values, multi-agent ones 9; crowd-driving observations are hashes, so up
    to one per scenario."""
    if desc["kind"] == 2:
        return min(n, 9)
    if desc["kind"] == 3:
        return min(n, 257)  # eight neighbour bits, or the terminal reading
    return min(n, 3) if desc["kind"] == 0 else n


def expand_leaf(desc, rcfg, parent, parent_ids, idx, depth, last_action, seed, step_idx,
                per_pair: bool = False, cap: int | None = None) -> dict:
    """Expand one leaf and initialise its children's bounds (Sec. III-D)."""
    n_par = _check_states(desc, parent)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    parent_ids = np.ascontiguousarray(parent_ids, dtype=np.uint32)
    assert parent_ids.shape[0] == n_par
    n = idx.shape[0]
    A = desc["n_actions"]
    cap = max_children(desc, n) if cap is None else cap
    capc = max(cap, 1)
    res = dict(states=empty_states(desc, n), ids=np.zeros(n, np.uint32),
               perm=np.zeros((A, n), np.int32), child_of=np.zeros((A, n), np.int32),
               n_children=np.zeros(A, np.int32), child_z=np.zeros((A, capc), np.uint64),
               child_n=np.zeros((A, capc), np.int32), child_off=np.zeros((A, capc), np.int32),
               child_u0=np.zeros((A, capc)), child_l0=np.zeros((A, capc)),
               r_mean=np.zeros(A), expand_steps=np.zeros(1, np.int64),
               rollout_steps=np.zeros(1, np.int64), steps=np.zeros((A, 2), np.int64))
    o = _Out()
    o.states = _soa(desc, res["states"], n)
    if per_pair:
        res.update(sprime=empty_states(desc, A * n), r=np.zeros((A, n), np.float32),
                   z=np.zeros((A, n), np.uint64), U=np.zeros((A, n)), L=np.zeros((A, n)),
                   Labs=np.zeros((A, n)))
        o.sprime = _soa(desc, res["sprime"], A * n)
        o.r, o.z, o.U, o.L = _ptr(res["r"]), _ptr(res["z"]), _ptr(res["U"]), _ptr(res["L"])
        o.Labs = _ptr(res["Labs"])
    for f in ("ids", "child_of", "perm", "n_children", "child_z", "child_n", "child_off",
              "child_u0", "child_l0", "r_mean", "expand_steps", "rollout_steps", "steps"):
        setattr(o, f, _ptr(res[f]))
    M = model(desc)
    rc = lib().or_expand_leaf(C.byref(M), C.byref(rcfg), seed, step_idx,
                              C.byref(_soa(desc, parent, n_par)), _ptr(parent_ids), _ptr(idx),
                              n, depth, last_action, cap, C.byref(o))
    if rc != 0:
        raise ValueError("child capacity %d exceeded" % cap)
    res["expand_steps"] = int(res["expand_steps"][0])
    res["rollout_steps"] = int(res["rollout_steps"][0])
    if per_pair:
        sp = res["sprime"]
        if desc["kind"] == 0:
            sp["w"] = sp["w"].reshape(A, n)
        elif desc["kind"] in (2, 3):
            sp["w"] = sp["w"].reshape(sp["w"].shape[0], A, n)
        else:
            P = desc["n_peds"]
            sp["s"], sp["car"] = sp["s"].reshape(A, n), sp["car"].reshape(A, n)
            for f in ("px", "py", "goal"):
                sp[f] = sp[f].reshape(P, A, n)
    return res


class _DespotResult(C.Structure):
    _fields_ = [("nodes", C.c_int64), ("trials", C.c_int64), ("expansions", C.c_int64),
                ("scenario_steps", C.c_int64), ("u_root", C.c_double), ("l_root", C.c_double),
                ("elapsed_s", C.c_double), ("max_depth_reached", C.c_int32), ("near_ties", C.c_int32)]


def despot(desc, rcfg, root_states, K, seed, step_idx, max_depth, xi=0.95, seconds=1.0, max_trials=0) -> dict:
    """One planning step of the plain DESPOT trial loop on one host thread
    (Sec. III-A; Eq. 5 and 7 to descend, the oracle's expansion, Eq. 4 back
    up) from the root scenarios `root_states` (ids 0..K-1)."""
    n = _check_states(desc, root_states)
    assert n == K
    res = _DespotResult()
    M = model(desc)
    rc = lib().or_despot(C.byref(M), C.byref(rcfg), seed, step_idx, C.byref(_soa(desc, root_states, K)), K,
                         max_depth, xi, seconds, max_trials, C.byref(res))
    if rc != 0:
        raise MemoryError("or_despot ran out of memory")
    return {f: getattr(res, f) for f, _ in _DespotResult._fields_}


def rs_sense_threshold(d2: int) -> int:
    return int(lib().or_rs_sense_threshold(d2))


def take_states(desc: dict, st: dict, positions) -> dict:
    """Sub-array of states at ``positions`` (for walking down a tree)."""
    positions = np.asarray(positions, dtype=np.int64)
    if desc["kind"] == 0:
        return dict(w=np.ascontiguousarray(st["w"][positions]))
    if desc["kind"] in (2, 3):
        return dict(w=np.ascontiguousarray(st["w"][:, positions]))
    return dict(s=np.ascontiguousarray(st["s"][positions]),
                car=np.ascontiguousarray(st["car"][positions]),
                px=np.ascontiguousarray(st["px"][:, positions]),
                py=np.ascontiguousarray(st["py"][:, positions]),
                goal=np.ascontiguousarray(st["goal"][:, positions]))


# --------------------------------------------------------------------------
# Eq. 4: Bellman backup over a DESPOT tree, FP64
# --------------------------------------------------------------------------
class Node:
    __slots__ = ("parent", "n", "u", "l", "u0", "l0", "actions")

    def __init__(self, parent, n, u0, l0):
        self.parent = parent
        self.n = n
        self.u0, self.l0 = float(u0), float(l0)
        self.u, self.l = float(u0), float(l0)
        self.actions = None  # list of (r_mean, [child nodes])


def attach_children(desc, node: Node, res: dict) -> None:
    """Create the action and observation branches of an expanded node (Eq. 11)."""
    node.actions = []
    for a in range(desc["n_actions"]):
        kids = []
        for c in range(int(res["n_children"][a])):
            kids.append(Node(node, int(res["child_n"][a, c]), res["child_u0"][a, c],
                             res["child_l0"][a, c]))
        node.actions.append((float(res["r_mean"][a]), kids))


def node_value(node: Node, gamma: float, which: str) -> float:
    """V(b) = max_a { R(b,a) + gamma sum_z |Phi_b'|/|Phi_b| V(b') } (Eq. 4)."""
    best = -np.inf
    for r_mean, kids in node.actions:
        q = r_mean + gamma * sum((k.n / node.n) * getattr(k, which) for k in kids)
        best = max(best, q)
    return best


def backup(node: Node, gamma: float) -> None:
    """Update u and l from ``node`` up to the root (Sec. III-A, Backup)."""
    while node is not None:
        if node.actions:
            node.u = node_value(node, gamma, "u")
            node.l = node_value(node, gamma, "l")
        node = node.parent


def mix64(x: int) -> int:
    """The observation hash's 64-bit mixing function (splitmix64's output step)."""
    return int(lib().or_mix64(x & 0xFFFFFFFFFFFFFFFF))
