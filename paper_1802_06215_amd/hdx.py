"""ctypes binding of libhdx.so (the C ABI in include/hdx.h).

Argument marshalling only: every step of leaf expansion runs in the HIP
kernels behind the C ABI.  PyTorch provides device memory (tensors) and
streams.  Importing this module raises if the built library is missing;
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhdx.so")

ROCKSAMPLE, PEDNAV, MARS, NAV = 0, 1, 2, 3
MAX_ACTIONS = 625  # HDX_MAX_ACTIONS
POLICY_DEFAULT, POLICY_CONST, POLICY_RANDOM = 0, 1, 2
SIZE_CLASSES = 6
LAUNCH_GROUPS = 36  # model variant (RockSample; driving <= 8, 16, 32 pedestrians; multi-agent; navigation) x size class
MAX_LEAF_SCENARIOS = 2048
MAX_NAV_LEAF_SCENARIOS = 5120
MAX_HORIZON = 4096
NOALLOC_MAX_LEAVES = 512  # HDX_NOALLOC_MAX_LEAVES
NOALLOC_MAX_TILES = 65536  # HDX_NOALLOC_MAX_TILES

STATUS = {0: "HDX_OK", -1: "HDX_E_INVALID", -2: "HDX_E_DEVICE", -3: "HDX_E_NOMEM", -4: "HDX_E_SHAPE",
          -5: "HDX_E_CAPACITY", -6: "HDX_E_UNSUPPORTED"}


class HdxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class ModelDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_actions", C.c_int32), ("gamma", C.c_double),
                ("grid", C.c_int32), ("n_rocks", C.c_int32),
                ("rock_x", C.c_int32 * 20), ("rock_y", C.c_int32 * 20),
                ("n_peds", C.c_int32), ("n_goals", C.c_int32), ("n_levels", C.c_int32),
                ("reserved", C.c_int32),
                ("goal_x", C.c_float * 8), ("goal_y", C.c_float * 8),
                ("path_len", C.c_float), ("dt", C.c_float), ("ped_speed", C.c_float),
                ("sigma_h", C.c_float), ("coll_radius", C.c_float),
                ("r_collision", C.c_float), ("r_step", C.c_float), ("r_goal", C.c_float),
                ("p_fail", C.c_double),
                ("nav_goal_x", C.c_int32), ("nav_wall", C.c_int32), ("nav_gate_x", C.c_int32 * 2),
                ("nav_cell", C.c_int16 * 256), ("p_err", C.c_double)]


class Belief(C.Structure):
    _fields_ = [("x", C.c_int32), ("y", C.c_int32), ("p_good", C.c_void_p),
                ("s", C.c_float), ("level", C.c_int32), ("px", C.c_void_p), ("py", C.c_void_p),
                ("goal_p", C.c_void_p), ("x2", C.c_int32), ("y2", C.c_int32), ("gone", C.c_int32)]


class RolloutCfg(C.Structure):
    _fields_ = [("policy", C.c_int32), ("const_action", C.c_int32),
                ("max_steps", C.c_int32), ("max_depth", C.c_int32)]


class States(C.Structure):
    _fields_ = [("w", C.c_void_p), ("s", C.c_void_p), ("car", C.c_void_p),
                ("px", C.c_void_p), ("py", C.c_void_p), ("goal", C.c_void_p),
                ("stride", C.c_int64)]


class SearchCfg(C.Structure):
    _fields_ = [("K", C.c_int32), ("n_threads", C.c_int32), ("max_depth", C.c_int32),
                ("batch_leaves", C.c_int32), ("time_budget_s", C.c_double), ("max_trials", C.c_int64),
                ("xi", C.c_double), ("c_a", C.c_double), ("c_o", C.c_double), ("gap_epsilon", C.c_double),
                ("arena_bytes", C.c_int64), ("seed", C.c_uint32), ("step", C.c_uint32),
                ("rollout", RolloutCfg), ("surrogate", C.c_void_p), ("surrogate_horizon", C.c_int32),
                ("surrogate_judge_every", C.c_int32), ("surrogate_max_rel_err", C.c_double),
                ("surrogate_bias_correct", C.c_int32)]


class SearchResult(C.Structure):
    _fields_ = [("best_action", C.c_int32), ("u_root", C.c_double), ("l_root", C.c_double),
                ("u0_root", C.c_double), ("l0_root", C.c_double), ("trials", C.c_int64),
                ("idle_trials", C.c_int64),
                ("expansions", C.c_int64), ("nodes", C.c_int64), ("scenario_steps", C.c_int64),
                ("launches", C.c_int64), ("max_depth_reached", C.c_int32), ("arena_full", C.c_int32),
                ("elapsed_s", C.c_double), ("action_l", C.c_double * MAX_ACTIONS), ("action_u", C.c_double * MAX_ACTIONS),
                ("judged_leaves", C.c_int64), ("judged_children", C.c_int64), ("judge_mae", C.c_double),
                ("judge_rel_err", C.c_double), ("judge_bias", C.c_double), ("surrogate_off", C.c_int32),
                ("time_select_s", C.c_double), ("time_expand_s", C.c_double), ("time_backup_s", C.c_double)]


class Leaf(C.Structure):
    _fields_ = [("model", C.c_void_p), ("seed", C.c_uint32), ("step", C.c_uint32),
                ("rollout", RolloutCfg), ("parent", States), ("parent_ids", C.c_void_p),
                ("idx", C.c_void_p), ("n", C.c_int32), ("depth", C.c_int32),
                ("last_action", C.c_int32), ("cap", C.c_int32), ("states_out", States),
                ("ids_out", C.c_void_p), ("perm", C.c_void_p), ("n_children", C.c_void_p),
                ("child_z", C.c_void_p), ("child_n", C.c_void_p), ("child_off", C.c_void_p),
                ("child_u0", C.c_void_p), ("child_l0", C.c_void_p), ("r_mean", C.c_void_p),
                ("steps", C.c_void_p), ("sprime", States), ("r", C.c_void_p), ("z", C.c_void_p),
                ("U", C.c_void_p), ("L", C.c_void_p), ("child_of", C.c_void_p)]


# every symbol include/hdx.h declares
EXPORTS = ["hdx_version", "hdx_init", "hdx_fini", "hdx_last_error", "hdx_upload_model",
           "hdx_free_model", "hdx_model_actions", "hdx_model_max_children",
           "hdx_sample_scenarios", "hdx_expand_leaf", "hdx_rollout_bounds", "hdx_philox",
           "hdx_fp32_selftest", "hdx_batch_create", "hdx_batch_destroy", "hdx_batch_set_leaves",
           "hdx_batch_set_schedule", "hdx_batch_get_schedule", "hdx_batch_use_graph",
           "hdx_batch_set_split", "hdx_batch_get_split",
           "hdx_batch_set_class_schedule", "hdx_batch_get_class_schedule", "hdx_batch_get_group_schedule",
           "hdx_batch_launch", "hdx_batch_autotune", "hdx_search", "hdx_mlp_create", "hdx_mlp_destroy",
           "hdx_mlp_get_params", "hdx_mlp_set_params", "hdx_mlp_forward", "hdx_mlp_gradients",
           "hdx_mlp_train_step", "hdx_features", "hdx_expand_leaf_surrogate", "hdx_mlp_save", "hdx_mlp_load",
           "hdx_tree_create", "hdx_tree_destroy", "hdx_tree_add_children", "hdx_backup",
           "hdx_tree_bounds", "hdx_tree_size", "hdx_expand_leaf_noalloc", "hdx_expand_out_bytes",
           "hdx_belief_update"]

_lib = None


def load_library():
    """Load libhdx.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhdx.so is not built; run __graft_entry__.build() or "
                          "python paper_1802_06215_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, U32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
    L.hdx_version.restype = C.c_char_p
    L.hdx_init.argtypes = [I32, C.POINTER(P)]
    L.hdx_fini.argtypes = [P]
    L.hdx_last_error.argtypes = [P]
    L.hdx_last_error.restype = C.c_char_p
    L.hdx_upload_model.argtypes = [P, C.POINTER(ModelDesc), C.POINTER(P)]
    L.hdx_free_model.argtypes = [P, P]
    L.hdx_model_actions.argtypes = [P]
    L.hdx_model_max_children.argtypes = [P, I32]
    L.hdx_sample_scenarios.argtypes = [P, P, C.POINTER(Belief), I32, U32, U32, States, P]
    L.hdx_expand_leaf.argtypes = [P, P, I32, P]
    L.hdx_expand_leaf_noalloc.argtypes = [P, P, I32, P]
    L.hdx_expand_out_bytes.argtypes = [P, I32, I32]
    L.hdx_expand_out_bytes.restype = C.c_size_t
    L.hdx_belief_update.argtypes = [C.POINTER(ModelDesc), C.POINTER(Belief), I32, C.c_uint64, C.POINTER(Belief),
                                    P, C.POINTER(I32)]
    L.hdx_rollout_bounds.argtypes = [P, P, C.POINTER(RolloutCfg), U32, U32, States, P, P, I64,
                                     P, P, P, P]
    L.hdx_philox.argtypes = [P, P, I64, U32, U32, P, P]
    L.hdx_fp32_selftest.argtypes = [P, P, P, P, I64, P, P]
    L.hdx_batch_create.argtypes = [P, I32, I64, C.POINTER(P)]
    L.hdx_batch_destroy.argtypes = [P, P]
    L.hdx_batch_set_leaves.argtypes = [P, P, P, I32, P]
    L.hdx_batch_set_split.argtypes = [P, P, I32]
    L.hdx_batch_get_split.argtypes = [P, C.POINTER(I32)]
    L.hdx_batch_set_schedule.argtypes = [P, P, I32, I32, I32]
    L.hdx_batch_get_schedule.argtypes = [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32)]
    L.hdx_batch_set_class_schedule.argtypes = [P, P, I32, I32, I32, I32]
    L.hdx_batch_get_class_schedule.argtypes = [P, I32, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32),
                                               C.POINTER(I64)]
    L.hdx_batch_get_group_schedule.argtypes = [P, I32, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32),
                                               C.POINTER(I64)]
    L.hdx_batch_use_graph.argtypes = [P, P, I32]
    L.hdx_batch_launch.argtypes = [P, P, P]
    L.hdx_batch_autotune.argtypes = [P, P, I32, C.POINTER(C.c_float)]
    L.hdx_search.argtypes = [P, P, C.POINTER(Belief), C.POINTER(SearchCfg), C.POINTER(SearchResult)]
    L.hdx_mlp_create.argtypes = [P, U32, C.POINTER(P)]
    L.hdx_mlp_destroy.argtypes = [P, P]
    L.hdx_mlp_get_params.argtypes = [P, P, P]
    L.hdx_mlp_set_params.argtypes = [P, P, P]
    L.hdx_mlp_forward.argtypes = [P, P, P, I64, P, P]
    L.hdx_mlp_gradients.argtypes = [P, P, P, P, I32, P, P, P]
    L.hdx_mlp_train_step.argtypes = [P, P, P, P, I32, C.c_float, P, P]
    L.hdx_features.argtypes = [P, P, States, P, I64, I32, P, P]
    L.hdx_expand_leaf_surrogate.argtypes = [P, P, I32, P, I32, P]
    L.hdx_mlp_save.argtypes = [P, P, C.c_char_p]
    L.hdx_mlp_load.argtypes = [P, P, C.c_char_p]
    L.hdx_tree_create.argtypes = [I32, C.c_double, I32, C.c_double, C.c_double, C.POINTER(P)]
    L.hdx_tree_destroy.argtypes = [P]
    L.hdx_tree_add_children.argtypes = [P, I64, P, P, P, P, P, P, I32, C.POINTER(I64)]
    L.hdx_backup.argtypes = [P, I64]
    L.hdx_tree_bounds.argtypes = [P, I64, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.hdx_tree_size.argtypes = [P]
    L.hdx_tree_size.restype = I64
    for name in EXPORTS:
        getattr(L, name)
    _lib = L
    return L


def _dp(t):
    return None if t is None else t.data_ptr()


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def model_desc(d: dict) -> ModelDesc:
    m = ModelDesc()
    m.kind = d["kind"]
    m.n_actions = d["n_actions"]
    m.gamma = d["gamma"]
    if d["kind"] == NAV:
        m.grid = d["n"]
        m.nav_goal_x, m.nav_wall = int(d["goal_x"]), int(d["wall"])
        m.nav_gate_x[0], m.nav_gate_x[1] = int(d["gate_x"][0]), int(d["gate_x"][1])
        cell = np.asarray(d["cell"], np.int64).reshape(-1)
        for c in range(cell.shape[0]):
            m.nav_cell[c] = int(cell[c])
        m.p_fail, m.p_err = d["p_fail"], d["p_err"]
    elif d["kind"] in (ROCKSAMPLE, MARS):
        m.grid, m.n_rocks = d["n"], d["m"]
        for i in range(d["m"]):
            m.rock_x[i], m.rock_y[i] = int(d["rock_x"][i]), int(d["rock_y"][i])
    else:
        m.n_peds, m.n_goals, m.n_levels = d["n_peds"], d["n_goals"], d["n_levels"]
        for g in range(d["n_goals"]):
            m.goal_x[g], m.goal_y[g] = float(d["goal_x"][g]), float(d["goal_y"][g])
        for f in ("path_len", "dt", "ped_speed", "sigma_h", "coll_radius", "r_collision", "r_step",
                  "r_goal"):
            setattr(m, f, float(d[f]))
        m.p_fail = d["p_fail"]
    return m


def rollout_cfg(policy=POLICY_DEFAULT, max_steps=1 << 30, max_depth=-1, const_action=0) -> RolloutCfg:
    c = RolloutCfg()
    c.policy, c.const_action, c.max_steps, c.max_depth = policy, const_action, max_steps, max_depth
    return c


class Model:
    def __init__(self, ctx, handle, desc):
        self.ctx, self.handle, self.desc = ctx, handle, desc
        self.kind = desc["kind"]
        self.n_actions = desc["n_actions"]
        self.n_peds = desc.get("n_peds", 0)

    def out_bytes(self, K: int, n_leaves: int = 1) -> int:
        """hdx_expand_out_bytes: device bytes of the required outputs of
        n_leaves leaves of K scenarios."""
        return int(self.ctx.lib.hdx_expand_out_bytes(self.handle, K, n_leaves))

    def max_children(self, n: int) -> int:
        return self.ctx.lib.hdx_model_max_children(self.handle, n)


def states_view(model: Model, st: dict) -> States:
    """hdx_states over a dict of device tensors (library layout)."""
    v = States()
    if model.kind == ROCKSAMPLE:
        v.w = _dp(st["w"])
        v.stride = st["w"].shape[-1]
    elif model.kind in (MARS, NAV):
        # rows of [2, n] (robots, rocks) or [5, n] (robot, four rows of unknown cells)
        assert st["w"].dim() == 2 and st["w"].shape[0] == (2 if model.kind == MARS else 5)
        assert st["w"].stride(1) == 1
        v.w = _dp(st["w"])
        v.stride = st["w"].stride(0)
    else:
        v.s, v.car = _dp(st["s"]), _dp(st["car"])
        if model.n_peds > 0:
            v.px, v.py, v.goal = _dp(st["px"]), _dp(st["py"]), _dp(st["goal"])
            v.stride = st["px"].stride(0) if st["px"].dim() == 2 else st["s"].numel()
        else:
            v.stride = st["s"].numel()
    return v


def empty_states(model: Model, n: int, device="cuda") -> dict:
    if model.kind == ROCKSAMPLE:
        return dict(w=torch.empty(n, dtype=torch.int32, device=device))
    if model.kind in (MARS, NAV):
        return dict(w=torch.empty((2 if model.kind == MARS else 5, n), dtype=torch.int32, device=device))
    P = model.n_peds
    return dict(s=torch.empty(n, dtype=torch.float32, device=device),
                car=torch.empty(n, dtype=torch.int32, device=device),
                px=torch.empty((P, n), dtype=torch.float32, device=device),
                py=torch.empty((P, n), dtype=torch.float32, device=device),
                goal=torch.empty((P, n), dtype=torch.uint8, device=device))


class LeafBuffers:
    """Device outputs of one leaf expansion (allocated once, reusable)."""

    def __init__(self, model: Model, n: int, per_pair: bool = False, device="cuda"):
        A = model.n_actions
        cap = max(model.max_children(n), 1)
        self.n, self.cap, self.A = n, cap, A
        i32, f32 = torch.int32, torch.float32
        self.states = empty_states(model, max(n, 1), device)
        self.ids = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        self.perm = torch.empty((A, max(n, 1)), dtype=torch.int16, device=device)
        self.n_children = torch.empty(A, dtype=i32, device=device)
        self.child_z = torch.empty((A, cap), dtype=torch.int64, device=device)
        self.child_n = torch.empty((A, cap), dtype=i32, device=device)
        self.child_off = torch.empty((A, cap), dtype=i32, device=device)
        self.child_u0 = torch.empty((A, cap), dtype=f32, device=device)
        self.child_l0 = torch.empty((A, cap), dtype=f32, device=device)
        self.r_mean = torch.empty(A, dtype=f32, device=device)
        self.steps = torch.empty((A, 2), dtype=torch.int64, device=device)
        self.per_pair = per_pair
        if per_pair:
            self.sprime = empty_states(model, max(A * n, 1), device)
            self.r = torch.empty((A, max(n, 1)), dtype=f32, device=device)
            self.z = torch.empty((A, max(n, 1)), dtype=torch.int64, device=device)
            self.U = torch.empty((A, max(n, 1)), dtype=f32, device=device)
            self.L = torch.empty((A, max(n, 1)), dtype=f32, device=device)
            self.child_of = torch.empty((A, max(n, 1)), dtype=i32, device=device)


class _SlabLeaf:
    """Per-leaf views into slab tensors (same attributes as LeafBuffers)."""


def leaf_buffer_slab(model: Model, count: int, n_max: int, device="cuda") -> list:
    """Output buffers for `count` leaves of up to n_max scenarios, carved
    from a few large tensors (one allocation per field)."""
    A = model.n_actions
    cap = max(model.max_children(n_max), 1)
    n1 = max(n_max, 1)
    i32, f32 = torch.int32, torch.float32
    slabs = dict(ids=torch.empty((count, n1), dtype=i32, device=device),
                 perm=torch.empty((count, A, n1), dtype=torch.int16, device=device),
                 n_children=torch.empty((count, A), dtype=i32, device=device),
                 child_z=torch.empty((count, A, cap), dtype=torch.int64, device=device),
                 child_n=torch.empty((count, A, cap), dtype=i32, device=device),
                 child_off=torch.empty((count, A, cap), dtype=i32, device=device),
                 child_u0=torch.empty((count, A, cap), dtype=f32, device=device),
                 child_l0=torch.empty((count, A, cap), dtype=f32, device=device),
                 r_mean=torch.empty((count, A), dtype=f32, device=device),
                 steps=torch.empty((count, A, 2), dtype=torch.int64, device=device))
    if model.kind == ROCKSAMPLE:
        st = dict(w=torch.empty((count, n1), dtype=i32, device=device))
    elif model.kind in (MARS, NAV):
        st = dict(w=torch.empty((count, 2 if model.kind == MARS else 5, n1), dtype=i32, device=device))
    else:
        P = model.n_peds
        st = dict(s=torch.empty((count, n1), dtype=f32, device=device),
                  car=torch.empty((count, n1), dtype=i32, device=device),
                  px=torch.empty((count, P, n1), dtype=f32, device=device),
                  py=torch.empty((count, P, n1), dtype=f32, device=device),
                  goal=torch.empty((count, P, n1), dtype=torch.uint8, device=device))
    out = []
    for i in range(count):
        b = _SlabLeaf()
        b.n, b.cap, b.A, b.per_pair = n_max, cap, A, False
        for k, v in slabs.items():
            setattr(b, k, v[i])
        b.states = {k: v[i] for k, v in st.items()}
        out.append(b)
    return out, slabs, st


def rocksample_states(x, y, rocks, term, device="cuda") -> dict:
    """Pack RockSample fields (robot cell, rock qualities [n, m], terminal
    flags) into the library's state word layout, on the device."""
    rocks = np.asarray(rocks, dtype=bool)
    w = np.full(rocks.shape[0], int(x) | (int(y) << 5), dtype=np.int64)
    w |= (rocks.astype(np.int64) << (10 + np.arange(rocks.shape[1]))).sum(1) if rocks.shape[1] else 0
    w |= np.asarray(term, dtype=np.int64) << 30
    return dict(w=torch.from_numpy(w.astype(np.int32)).to(device))


def mars_states(pos, rocks, term, device="cuda") -> dict:
    """Pack multi-agent RockSample fields (pos = (x1, y1, x2, y2, gone1,
    gone2), each a scalar or per scenario; rock qualities [n, m]; terminal
    flags) into the library's two-row layout, on the device."""
    rocks = np.asarray(rocks, dtype=bool)
    n = rocks.shape[0]
    x1, y1, x2, y2, g1, g2 = (np.broadcast_to(np.asarray(f, dtype=np.int64), (n,)) for f in pos)
    row0 = x1 | (y1 << 5) | (x2 << 10) | (y2 << 15) | (g1 << 20) | (g2 << 21)
    row0 = row0 | (np.asarray(term, dtype=np.int64) << 30)
    row1 = (rocks.astype(np.int64) << np.arange(rocks.shape[1])).sum(1) if rocks.shape[1] else np.zeros(n, np.int64)
    w = np.stack([row0, row1]).astype(np.int32)
    return dict(w=torch.from_numpy(w).to(device))


def nav_states(x, y, cells, term, device="cuda") -> dict:
    """Pack navigation fields (robot x, y, scalars or per scenario; unknown
    cells occupied, bool [n, U <= 128]; terminal flags) into the library's
    five-row layout, on the device."""
    cells = np.asarray(cells, dtype=bool)
    n = cells.shape[0]
    w = np.zeros((5, n), dtype=np.int64)
    w[0] = (np.broadcast_to(np.asarray(x, np.int64), (n,)) | (np.broadcast_to(np.asarray(y, np.int64), (n,)) << 4)
            | (np.asarray(term, dtype=np.int64) << 30))
    for i in range(cells.shape[1]):
        w[1 + i // 32] |= cells[:, i].astype(np.int64) << (i % 32)
    return dict(w=torch.from_numpy(w.astype(np.uint32).view(np.int32)).to(device))


def pednav_states(s, level, term, px, py, goal, device="cuda") -> dict:
    """Crowd-driving fields in the library's struct-of-arrays layout."""
    car = np.asarray(level, np.int32) | (np.asarray(term, np.int32) << 8)
    f = lambda a, t: torch.from_numpy(np.ascontiguousarray(a, dtype=t)).to(device)
    return dict(s=f(s, np.float32), car=f(car, np.int32), px=f(px, np.float32), py=f(py, np.float32),
                goal=f(goal, np.uint8))


def positions(idx, device="cuda") -> torch.Tensor:
    """A leaf's positions in its parent's arrays as the int16 device tensor
    hdx_leaf.idx takes."""
    a = np.asarray(idx)
    if a.size and (a.min() < 0 or a.max() >= 1 << 15):
        raise ValueError("positions must lie in [0, 32768)")
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.int16))).to(device)


def belief_update(desc: dict, belief: dict, action: int, z: int):
    """RockSample belief after `action` and observation z (Eq. 3), computed
    by hdx_belief_update; returns (new belief dict, terminal)."""
    lib = load_library()
    md = model_desc(desc)
    p = np.ascontiguousarray(belief["p"], dtype=np.float64)
    b = Belief()
    b.x, b.y, b.p_good = int(belief["x"]), int(belief["y"]), p.ctypes.data
    out = Belief()
    p_out = np.empty_like(p)
    term = C.c_int32(0)
    rc = lib.hdx_belief_update(C.byref(md), C.byref(b), int(action), int(z), C.byref(out),
                               p_out.ctypes.data, C.byref(term))
    if rc != 0:
        raise HdxError(rc, "hdx_belief_update")
    return dict(x=int(out.x), y=int(out.y), p=p_out), bool(term.value)


def make_leaf(model: Model, parent: dict, parent_ids, idx, depth: int, last_action: int,
              out: LeafBuffers, seed: int, step: int, cfg: RolloutCfg) -> Leaf:
    """An hdx_leaf descriptor over device tensors (they must outlive the call).
    idx holds int16 positions (a child's idx is a segment of its parent's
    perm, which the library writes as int16)."""
    if idx.dtype != torch.int16:
        raise TypeError("idx must be an int16 tensor, got %s" % idx.dtype)
    L = Leaf()
    L.model = model.handle
    L.seed, L.step = seed, step
    L.rollout = cfg
    L.parent = states_view(model, parent)
    L.parent_ids = _dp(parent_ids)
    L.idx = _dp(idx)
    L.n = int(idx.numel())
    L.depth, L.last_action, L.cap = depth, last_action, out.cap
    L.states_out = states_view(model, out.states)
    L.ids_out = _dp(out.ids)
    L.perm, L.n_children = _dp(out.perm), _dp(out.n_children)
    L.child_z, L.child_n, L.child_off = _dp(out.child_z), _dp(out.child_n), _dp(out.child_off)
    L.child_u0, L.child_l0 = _dp(out.child_u0), _dp(out.child_l0)
    L.r_mean, L.steps = _dp(out.r_mean), _dp(out.steps)
    if out.per_pair:
        L.sprime = states_view(model, out.sprime)
        L.r, L.z, L.U, L.L = _dp(out.r), _dp(out.z), _dp(out.U), _dp(out.L)
        L.child_of = _dp(out.child_of)
    return L


class Context:
    """An hdx context on one HIP device."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.device = device
        h = C.c_void_p()
        self._check(self.lib.hdx_init(device, C.byref(h)), None)
        self.handle = h

    def _check(self, rc, handle="ctx"):
        if rc != 0:
            msg = ""
            if handle is not None and getattr(self, "handle", None) is not None:
                msg = self.lib.hdx_last_error(self.handle).decode()
            raise HdxError(rc, msg)

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.lib.hdx_fini(self.handle)
            self.handle = None

    def upload_model(self, desc: dict) -> Model:
        h = C.c_void_p()
        md = model_desc(desc)
        self._check(self.lib.hdx_upload_model(self.handle, C.byref(md), C.byref(h)))
        return Model(self, h, desc)

    def sample_scenarios(self, model: Model, belief: dict, K: int, seed: int, step: int,
                         out: dict | None = None, stream=None) -> dict:
        out = empty_states(model, K) if out is None else out
        b, keep = self._belief(model, belief)
        self._check(self.lib.hdx_sample_scenarios(self.handle, model.handle, C.byref(b), K, seed, step,
                                                  states_view(model, out), _stream(stream)))
        return out

    def expand_leaf(self, leaves, stream=None) -> None:
        leaves = list(leaves)
        arr = (Leaf * len(leaves))(*leaves)
        self._check(self.lib.hdx_expand_leaf(self.handle, C.cast(arr, C.c_void_p), len(leaves),
                                             _stream(stream)))

    def expand_leaf_noalloc(self, leaves, stream=None) -> None:
        leaves = list(leaves)
        arr = (Leaf * len(leaves))(*leaves)
        self._check(self.lib.hdx_expand_leaf_noalloc(self.handle, C.cast(arr, C.c_void_p), len(leaves),
                                                     _stream(stream)))

    def expand_leaf_surrogate(self, leaves, mlp: "Mlp", horizon: int, stream=None) -> None:
        leaves = list(leaves)
        arr = (Leaf * len(leaves))(*leaves)
        self._check(self.lib.hdx_expand_leaf_surrogate(self.handle, C.cast(arr, C.c_void_p), len(leaves),
                                                       mlp.handle, horizon, _stream(stream)))

    def rollout_bounds(self, model: Model, cfg: RolloutCfg, states: dict, ids, depths, seed: int,
                       step: int, stream=None):
        n = int(ids.numel())
        U = torch.empty(n, dtype=torch.float32, device=ids.device)
        L = torch.empty(n, dtype=torch.float32, device=ids.device)
        steps = torch.empty(n, dtype=torch.int32, device=ids.device)
        self._check(self.lib.hdx_rollout_bounds(self.handle, model.handle, C.byref(cfg), seed, step,
                                                states_view(model, states), _dp(ids), _dp(depths), n,
                                                _dp(U), _dp(L), _dp(steps), _stream(stream)))
        return U, L, steps

    def search(self, model: Model, belief: dict, K: int = 500, n_threads: int = 8, max_depth: int = 90,
               batch_leaves: int = 0, time_budget_s: float = 1.0, max_trials: int = 0, xi: float = 0.95,
               c_a: float = 0.1, c_o: float = 0.1, gap_epsilon: float = 0.0, arena_bytes: int = 8 << 30,
               seed: int = 1, step: int = 0, rollout: RolloutCfg | None = None,
               surrogate: "Mlp | None" = None, surrogate_horizon: int = 0, surrogate_judge_every: int = 0,
               surrogate_max_rel_err: float = 0.0, surrogate_bias_correct: bool = False) -> dict:
        """hdx_search: one planning step of parallel DESPOT over GPU leaf expansion
        (with `surrogate`, leaf lower bounds come from the MLP instead of rollouts)."""
        b, keep = self._belief(model, belief)
        cfg = SearchCfg(K, n_threads, max_depth, batch_leaves, time_budget_s, max_trials, xi, c_a, c_o,
                        gap_epsilon, arena_bytes, seed, step, rollout or rollout_cfg(),
                        surrogate.handle if surrogate is not None else None, surrogate_horizon,
                        surrogate_judge_every, surrogate_max_rel_err, int(bool(surrogate_bias_correct)))
        res = SearchResult()
        self._check(self.lib.hdx_search(self.handle, model.handle, C.byref(b), C.byref(cfg), C.byref(res)))
        out = {f: getattr(res, f) for f, _ in SearchResult._fields_ if not f.startswith("action_")}
        out["action_l"] = list(res.action_l)[:model.n_actions]
        out["action_u"] = list(res.action_u)[:model.n_actions]
        return out

    def _belief(self, model: Model, belief: dict):
        b = Belief()
        keep = []
        if model.kind == ROCKSAMPLE:
            p = np.ascontiguousarray(belief["p"], dtype=np.float64)
            keep.append(p)
            b.x, b.y, b.p_good = belief["x"], belief["y"], p.ctypes.data
        elif model.kind == NAV:
            p = np.ascontiguousarray(belief["p"], dtype=np.float64)
            keep.append(p)
            b.p_good = p.ctypes.data
        elif model.kind == MARS:
            p = np.ascontiguousarray(belief["p"], dtype=np.float64)
            keep.append(p)
            x1, y1, x2, y2, g1, g2 = (int(v) for v in belief["pos"])
            b.x, b.y, b.x2, b.y2, b.gone, b.p_good = x1, y1, x2, y2, g1 | (g2 << 1), p.ctypes.data
        else:
            px = np.ascontiguousarray(belief["px"], dtype=np.float32)
            py = np.ascontiguousarray(belief["py"], dtype=np.float32)
            gp = np.ascontiguousarray(belief["goal_p"], dtype=np.float64)
            keep += [px, py, gp]
            b.s, b.level = float(belief["s"]), int(belief["level"])
            b.px, b.py, b.goal_p = px.ctypes.data, py.ctypes.data, gp.ctypes.data
        return b, keep

    def philox(self, ctr, k0: int, k1: int, stream=None):
        out = torch.empty_like(ctr)
        self._check(self.lib.hdx_philox(self.handle, _dp(ctr), ctr.shape[0], k0, k1, _dp(out),
                                        _stream(stream)))
        return out


class Batch:
    """hdx_batch: leaves staged in device memory, launched as one kernel (or
    a replayed HIP graph) with an autotuned schedule."""

    def __init__(self, ctx: "Context", max_leaves: int, max_tiles: int):
        self.ctx, self.lib = ctx, ctx.lib
        h = C.c_void_p()
        ctx._check(self.lib.hdx_batch_create(ctx.handle, max_leaves, max_tiles, C.byref(h)))
        self.handle = h
        self._keep = None

    def set_leaves(self, leaves, stream=None):
        leaves = list(leaves)
        arr = (Leaf * max(len(leaves), 1))(*leaves)
        self._keep = arr
        self.ctx._check(self.lib.hdx_batch_set_leaves(self.ctx.handle, self.handle, C.cast(arr, C.c_void_p),
                                                      len(leaves), _stream(stream)))

    def set_split(self, split: bool):
        """One launch group per model variant (False, the default) or per
        model variant and size class (True); re-plans the staged leaves."""
        self.ctx._check(self.lib.hdx_batch_set_split(self.ctx.handle, self.handle, int(split)))

    def split(self) -> bool:
        v = C.c_int32()
        self.ctx._check(self.lib.hdx_batch_get_split(self.handle, C.byref(v)))
        return bool(v.value)

    def set_schedule(self, threads: int, persistent: int, xcd_remap: int):
        self.ctx._check(self.lib.hdx_batch_set_schedule(self.ctx.handle, self.handle, threads, persistent,
                                                        xcd_remap))

    def schedule(self):
        """(threads, persistent, xcd_remap) of the group with the most tiles."""
        t, p, x = C.c_int32(), C.c_int32(), C.c_int32()
        self.ctx._check(self.lib.hdx_batch_get_schedule(self.handle, C.byref(t), C.byref(p), C.byref(x)))
        return t.value, p.value, x.value

    def set_class_schedule(self, size_class: int, threads: int, persistent: int, xcd_remap: int):
        self.ctx._check(self.lib.hdx_batch_set_class_schedule(self.ctx.handle, self.handle, size_class, threads,
                                                              persistent, xcd_remap))

    def class_schedules(self) -> list:
        """[(size_class, threads, persistent, xcd_remap, tiles)] of the non-empty classes."""
        out = []
        for c in range(SIZE_CLASSES):
            t, p, x, n = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
            self.ctx._check(self.lib.hdx_batch_get_class_schedule(self.handle, c, C.byref(t), C.byref(p), C.byref(x),
                                                                  C.byref(n)))
            if n.value:
                out.append((c, t.value, p.value, x.value, n.value))
        return out

    def group_schedules(self) -> list:
        """[(model_variant, size_class, threads, persistent, xcd_remap, tiles)] of the non-empty groups."""
        out = []
        for g in range(LAUNCH_GROUPS):
            t, p, x, n = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
            self.ctx._check(self.lib.hdx_batch_get_group_schedule(self.handle, g, C.byref(t), C.byref(p), C.byref(x),
                                                                  C.byref(n)))
            if n.value:
                out.append((g // SIZE_CLASSES, g % SIZE_CLASSES, t.value, p.value, x.value, n.value))
        return out

    def use_graph(self, enable: bool = True):
        self.ctx._check(self.lib.hdx_batch_use_graph(self.ctx.handle, self.handle, int(enable)))

    def launch(self, stream=None):
        self.ctx._check(self.lib.hdx_batch_launch(self.ctx.handle, self.handle, _stream(stream)))

    def autotune(self, reps: int = 3) -> float:
        ms = C.c_float()
        self.ctx._check(self.lib.hdx_batch_autotune(self.ctx.handle, self.handle, reps, C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.lib.hdx_batch_destroy(self.ctx.handle, self.handle)
            self.handle = None


MLP_IN, MLP_HIDDEN, MLP_PARAMS = 64, 256, 148481


class Mlp:
    """hdx_mlp: the rollout-value surrogate (BF16 MFMA, FP32 master weights)."""

    def __init__(self, ctx: "Context", seed: int = 0):
        self.ctx, self.lib = ctx, ctx.lib
        h = C.c_void_p()
        ctx._check(self.lib.hdx_mlp_create(ctx.handle, seed, C.byref(h)))
        self.handle = h

    def params(self) -> np.ndarray:
        out = np.empty(MLP_PARAMS, np.float32)
        self.ctx._check(self.lib.hdx_mlp_get_params(self.ctx.handle, self.handle, out.ctypes.data))
        return out

    def set_params(self, p) -> None:
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.shape == (MLP_PARAMS,)
        self.ctx._check(self.lib.hdx_mlp_set_params(self.ctx.handle, self.handle, p.ctypes.data))

    def save(self, path: str) -> None:
        self.ctx._check(self.lib.hdx_mlp_save(self.ctx.handle, self.handle, os.fsencode(path)))

    def load(self, path: str) -> None:
        self.ctx._check(self.lib.hdx_mlp_load(self.ctx.handle, self.handle, os.fsencode(path)))

    def forward(self, X: torch.Tensor, stream=None) -> torch.Tensor:
        """X: int16/uint16 BF16 bits [n, 64] on the device."""
        n = X.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=X.device)
        self.ctx._check(self.lib.hdx_mlp_forward(self.ctx.handle, self.handle, _dp(X), n, _dp(y), _stream(stream)))
        return y

    def gradients(self, X, t, stream=None):
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        self.ctx._check(self.lib.hdx_mlp_gradients(self.ctx.handle, self.handle, _dp(X), _dp(t), X.shape[0], _dp(g),
                                                   _dp(loss), _stream(stream)))
        return g, loss

    def train_step(self, X, t, lr: float, loss=None, stream=None):
        self.ctx._check(self.lib.hdx_mlp_train_step(self.ctx.handle, self.handle, _dp(X), _dp(t), X.shape[0], lr,
                                                    _dp(loss), _stream(stream)))

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.lib.hdx_mlp_destroy(self.ctx.handle, self.handle)
            self.handle = None


def features(ctx: "Context", model: Model, states: dict, depths, horizon: int, stream=None) -> torch.Tensor:
    """hdx_features: BF16 surrogate features [n, 64] (as int16 bits)."""
    n = int(depths.numel())
    X = torch.empty((n, MLP_IN), dtype=torch.int16, device=depths.device)
    ctx._check(ctx.lib.hdx_features(ctx.handle, model.handle, states_view(model, states), _dp(depths), n, horizon,
                                    _dp(X), _stream(stream)))
    return X


def fp32_selftest(ctx: "Context", a, b, c, stream=None):
    """Device results of sqrt|a|, a/b, a*b+c (unfused) and floor(a)."""
    n = a.numel()
    out = torch.empty((4, n), dtype=torch.float32, device=a.device)
    ctx._check(ctx.lib.hdx_fp32_selftest(ctx.handle, _dp(a), _dp(b), _dp(c), n, _dp(out), _stream(stream)))
    return out


class Tree:
    """Host DESPOT tree with the Eq. 4 backup (hdx_tree_*)."""

    def __init__(self, n_actions: int, gamma: float, n_root: int, u0: float, l0: float):
        self.lib = load_library()
        h = C.c_void_p()
        rc = self.lib.hdx_tree_create(n_actions, gamma, n_root, u0, l0, C.byref(h))
        if rc != 0:
            raise HdxError(rc, "tree_create")
        self.handle = h
        self.n_actions = n_actions

    def add_children(self, node: int, n_children, child_z, child_n, child_u0, child_l0, r_mean,
                     cap: int) -> int:
        arrs = [np.ascontiguousarray(n_children, np.int32), np.ascontiguousarray(child_z, np.uint64),
                np.ascontiguousarray(child_n, np.int32), np.ascontiguousarray(child_u0, np.float32),
                np.ascontiguousarray(child_l0, np.float32), np.ascontiguousarray(r_mean, np.float32)]
        first = C.c_int64()
        rc = self.lib.hdx_tree_add_children(self.handle, node, *[a.ctypes.data for a in arrs], cap,
                                            C.byref(first))
        if rc != 0:
            raise HdxError(rc, "tree_add_children")
        return first.value

    def backup(self, node: int) -> None:
        rc = self.lib.hdx_backup(self.handle, node)
        if rc != 0:
            raise HdxError(rc, "backup")

    def bounds(self, node: int):
        u, l = C.c_double(), C.c_double()
        rc = self.lib.hdx_tree_bounds(self.handle, node, C.byref(u), C.byref(l))
        if rc != 0:
            raise HdxError(rc, "tree_bounds")
        return u.value, l.value

    def size(self) -> int:
        return self.lib.hdx_tree_size(self.handle)

    def __del__(self):
        if getattr(self, "handle", None) is not None:
            self.lib.hdx_tree_destroy(self.handle)
            self.handle = None
