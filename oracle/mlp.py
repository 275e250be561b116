"""FP64 reference of the rollout-value surrogate (test infrastructure only).

An MLP 64 -> 256 -> 256 -> 256 -> 1 with ReLU, evaluated and
differentiated in FP64 with plain numpy by the chain rule.  Parameters are
one packed vector in the library's documented order: W1[64][256], b1,
W2[256][256], b2, W3[256][256], b3, w4[256], b4 (W[in][out]).  Also the
surrogate's state features, written from their documented definition.

Pinned by central finite differences (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np

IN, HID = 64, 256
SIZES = [("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
         ("W3", (HID, HID)), ("b3", (HID,)), ("w4", (HID,)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SIZES])


def _q(a, on: bool):
    """BF16 rounding point (identity when off)."""
    return bf16_round(np.asarray(a, np.float32)).astype(np.float64) if on else a


def forward(p: np.ndarray, X: np.ndarray, keep: bool = False, bf16: bool = False):
    """MLP output; with bf16=True the hidden activations are rounded to BF16
    after each layer (the library's mixed-precision definition)."""
    w = unpack(p)
    X = np.asarray(X, np.float64)
    z1 = X @ w["W1"] + w["b1"]
    h1 = _q(np.maximum(z1, 0.0), bf16)
    z2 = h1 @ w["W2"] + w["b2"]
    h2 = _q(np.maximum(z2, 0.0), bf16)
    z3 = h2 @ w["W3"] + w["b3"]
    h3 = _q(np.maximum(z3, 0.0), bf16)
    y = h3 @ w["w4"] + w["b4"][0]
    if keep:
        return y, dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3)
    return y


def loss(p: np.ndarray, X: np.ndarray, t: np.ndarray, bf16: bool = False) -> float:
    y = forward(p, X, bf16=bf16)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def gradients(p: np.ndarray, X: np.ndarray, t: np.ndarray, bf16: bool = False) -> np.ndarray:
    """d loss / d p for loss = mean((y - t)^2), by backpropagation; with
    bf16=True the activations and the back-propagated gradients of the
    hidden layers are rounded to BF16 where the library stores them."""
    w = unpack(p)
    y, c = forward(p, X, keep=True, bf16=bf16)
    B = X.shape[0]
    dy = 2.0 * (y - np.asarray(t, np.float64)) / B
    if bf16:
        dy = np.asarray(dy, np.float32).astype(np.float64)
    g = {}
    g["w4"] = c["h3"].T @ dy
    g["b4"] = np.array([dy.sum()])
    dz3 = _q(np.outer(dy, w["w4"]) * (c["h3"] > 0 if bf16 else c["z3"] > 0), bf16)
    g["W3"] = c["h2"].T @ dz3
    g["b3"] = dz3.sum(0)
    dz2 = _q((dz3 @ w["W3"].T) * (c["h2"] > 0 if bf16 else c["z2"] > 0), bf16)
    g["W2"] = c["h1"].T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = _q((dz2 @ w["W2"].T) * (c["h1"] > 0 if bf16 else c["z1"] > 0), bf16)
    g["W1"] = c["X"].T @ dz1
    g["b1"] = dz1.sum(0)
    return pack(g)


def bf16_round(a) -> np.ndarray:
    """Round FP32 values to BF16 (nearest even), returned as float32."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)


def rocksample_features(desc: dict, w: np.ndarray, depths: np.ndarray, horizon: int) -> np.ndarray:
    """Features of RockSample states as FP32 before BF16 rounding: x/n, y/n,
    terminal, (horizon - depth)/100, rock qualities, (rock_x - x)/n,
    (rock_y - y)/n, zeros to 64 columns."""
    w = np.asarray(w, np.int64)
    n, m = desc["n"], desc["m"]
    inv = np.float32(1.0) / np.float32(n)
    x, y = w & 31, (w >> 5) & 31
    f = np.zeros((w.shape[0], IN), np.float32)
    f[:, 0] = x.astype(np.float32) * inv
    f[:, 1] = y.astype(np.float32) * inv
    f[:, 2] = ((w >> 30) & 1).astype(np.float32)
    f[:, 3] = np.maximum(horizon - np.asarray(depths), 0).astype(np.float32) * np.float32(0.01)
    for i in range(m):
        f[:, 4 + i] = ((w >> (10 + i)) & 1).astype(np.float32)
        f[:, 4 + m + i] = (np.float32(desc["rock_x"][i]) - x.astype(np.float32)) * inv
        f[:, 4 + 2 * m + i] = (np.float32(desc["rock_y"][i]) - y.astype(np.float32)) * inv
    return f


def pednav_features(desc: dict, st: dict, depths: np.ndarray, horizon: int) -> np.ndarray:
    """Features of crowd-driving states as FP32 before BF16 rounding: s/path_len,
    speed level/(levels-1), terminal, (horizon - depth)/100, then per
    pedestrian (up to 20): (px - s)/10, py/10, goal index/n_goals."""
    s = np.asarray(st["s"], np.float32)
    car = np.asarray(st["car"], np.int64)
    n = s.shape[0]
    f = np.zeros((n, IN), np.float32)
    f[:, 0] = s / np.float32(desc["path_len"])
    f[:, 1] = (car & 0xFF).astype(np.float32) / np.float32(max(desc["n_levels"] - 1, 1))
    f[:, 2] = ((car >> 8) & 1).astype(np.float32)
    f[:, 3] = np.maximum(horizon - np.asarray(depths), 0).astype(np.float32) * np.float32(0.01)
    P = min(desc["n_peds"], (IN - 4) // 3)
    px, py = np.asarray(st["px"], np.float32), np.asarray(st["py"], np.float32)
    goal = np.asarray(st["goal"], np.int64)
    for j in range(P):
        f[:, 4 + 3 * j] = (px[j] - s) * np.float32(0.1)
        f[:, 5 + 3 * j] = py[j] * np.float32(0.1)
        f[:, 6 + 3 * j] = goal[j].astype(np.float32) / np.float32(desc["n_goals"])
    return f
