"""Pins for the FP64 surrogate reference: gradients against central finite
differences, the forward pass against torch's CPU autograd (an independent
implementation), and BF16 rounding against torch's bfloat16 conversion."""
import numpy as np
import pytest
import torch

from oracle import mlp


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.1, mlp.N_PARAMS)
    X = rng.normal(0, 1, (8, mlp.IN))
    t = rng.normal(0, 1, 8)
    return p, X, t


def test_parameter_count():
    assert mlp.N_PARAMS == 148481


def test_gradients_match_finite_differences(case):
    p, X, t = case
    g = mlp.gradients(p, X, t)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 300, replace=False), np.arange(mlp.N_PARAMS - 257, mlp.N_PARAMS)])
    eps = 1e-6
    for i in idx:
        q = p.copy()
        q[i] += eps
        lp = mlp.loss(q, X, t)
        q[i] -= 2 * eps
        lm = mlp.loss(q, X, t)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, i


def test_forward_and_gradients_match_torch_autograd(case):
    p, X, t = case
    w = mlp.unpack(p)
    T = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in w.items()}
    x = torch.tensor(X)
    h = torch.relu(x @ T["W1"] + T["b1"])
    h = torch.relu(h @ T["W2"] + T["b2"])
    h = torch.relu(h @ T["W3"] + T["b3"])
    y = h @ T["w4"] + T["b4"][0]
    L = torch.mean((y - torch.tensor(t)) ** 2)
    L.backward()
    assert np.allclose(y.detach().numpy(), mlp.forward(p, X), rtol=1e-12, atol=1e-12)
    g = mlp.pack({k: T[k].grad.numpy() for k in T})
    assert np.allclose(g, mlp.gradients(p, X, t), rtol=1e-10, atol=1e-12)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(2)
    a = (rng.standard_normal(100000) * np.exp(rng.uniform(-30, 30, 100000))).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16_round(a).view(np.uint32), ref.view(np.uint32))


def test_rocksample_features_definition():
    desc = dict(n=5, m=2, rock_x=np.array([1, 4]), rock_y=np.array([3, 0]))
    w = np.array([2 | (1 << 5) | (1 << 10), 4 | (4 << 5) | (1 << 11) | (1 << 30)], np.int32)
    f = mlp.rocksample_features(desc, w, np.array([10, 95]), 90)
    assert np.allclose(f[0, :10], [0.4, 0.2, 0, 0.8, 1, 0, -0.2, 0.4, 0.4, -0.2], atol=1e-7)
    assert np.allclose(f[1, :10], [0.8, 0.8, 1, 0, 0, 1, -0.6, 0.0, -0.2, -0.8], atol=1e-7)
    assert np.all(f[:, 10:] == 0)


def test_pednav_features_definition():
    desc = dict(path_len=40.0, n_levels=5, n_peds=2, n_goals=4)
    st = dict(s=np.array([10.0, 20.0], np.float32), car=np.array([2, 4 | (1 << 8)], np.int32),
              px=np.array([[15.0, 18.0], [5.0, 30.0]], np.float32),
              py=np.array([[1.0, -2.0], [3.0, 0.5]], np.float32),
              goal=np.array([[1, 3], [0, 2]], np.uint8))
    f = mlp.pednav_features(desc, st, np.array([0, 100]), 90)
    assert np.allclose(f[0, :10], [0.25, 0.5, 0, 0.9, 0.5, 0.1, 0.25, -0.5, 0.3, 0.0], atol=1e-7)
    assert np.allclose(f[1, :10], [0.5, 1.0, 1, 0, -0.2, -0.2, 0.75, 1.0, 0.05, 0.5], atol=1e-7)
    assert np.all(f[:, 10:] == 0)
