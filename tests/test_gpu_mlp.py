"""GPU tests of the surrogate MLP kernels against the FP64 reference.

The device computes with BF16 weights and activations (FP32 accumulation);
the reference is fed the same BF16-rounded weights and inputs and works in
FP64, so agreement is at BF16 level: forward within 2e-2 of the output
scale, gradients with cosine >= 0.999 and relative L2 <= 2e-2 per block.
Features must match their definition bit for bit after BF16 rounding."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import mlp as ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1802_06215_amd import Context
    c = Context(0)
    yield c
    c.close()


def rounded_params(net):
    return ref.bf16_round(net.params()).astype(np.float64)


def device_bf16(a: np.ndarray) -> torch.Tensor:
    bits = ref.bf16_round(a).view(np.uint32) >> 16
    return torch.from_numpy(bits.astype(np.uint16).view(np.int16)).cuda()


@pytest.mark.parametrize("n", [1, 64, 1000, 4097])
def test_forward_matches_reference(ctx, n):
    from paper_1802_06215_amd import Mlp
    net = Mlp(ctx, seed=3)
    rng = np.random.default_rng(n)
    X = rng.normal(0, 1, (n, 64)).astype(np.float32)
    y = net.forward(device_bf16(X)).cpu().numpy()
    p = net.params().astype(np.float64)
    # biases stay FP32 on the device; weights are BF16
    w = ref.unpack(p)
    for k in ("W1", "W2", "W3", "w4"):
        w[k] = ref.bf16_round(w[k].astype(np.float32)).astype(np.float64)
    want = ref.forward(ref.pack(w), ref.bf16_round(X))
    scale = np.abs(want).mean() + 1e-3
    assert np.max(np.abs(y - want)) <= 2e-2 * scale + 1e-3, (np.max(np.abs(y - want)), scale)
    net.close()


def test_gradients_match_reference(ctx):
    from paper_1802_06215_amd import Mlp
    net = Mlp(ctx, seed=5)
    rng = np.random.default_rng(9)
    B = 512
    X = rng.normal(0, 1, (B, 64)).astype(np.float32)
    t = rng.normal(0, 1, B).astype(np.float32)
    g, loss = net.gradients(device_bf16(X), torch.from_numpy(t).cuda())
    g = g.cpu().numpy().astype(np.float64)
    p = net.params().astype(np.float64)
    w = ref.unpack(p)
    for k in ("W1", "W2", "W3", "w4"):
        w[k] = ref.bf16_round(w[k].astype(np.float32)).astype(np.float64)
    pr = ref.pack(w)
    Xr = ref.bf16_round(X)
    # same rounding points as the device: tight
    gq = ref.gradients(pr, Xr, t, bf16=True)
    # pure FP64: the cost of BF16 activations and gradients, looser
    g64 = ref.gradients(pr, Xr, t)
    assert abs(float(loss.cpu()) - ref.loss(pr, Xr, t, bf16=True)) <= 1e-3 * ref.loss(pr, Xr, t, bf16=True)
    o = 0
    for name, shape in ref.SIZES:
        k = int(np.prod(shape))
        a, b, c = g[o:o + k], gq[o:o + k], g64[o:o + k]
        o += k
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-30)
        rel = np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-30)
        cos64 = a @ c / (np.linalg.norm(a) * np.linalg.norm(c) + 1e-30)
        rel64 = np.linalg.norm(a - c) / (np.linalg.norm(c) + 1e-30)
        print(name, "vs bf16 reference cos %.6f rel %.5f | vs fp64 cos %.6f rel %.4f" % (cos, rel, cos64, rel64),
              flush=True)
        assert cos >= 0.9999 and rel <= 1e-2, name
        assert cos64 >= 0.995 and rel64 <= 0.1, name
    net.close()


def test_adam_step_matches_reference(ctx):
    from paper_1802_06215_amd import Mlp
    net = Mlp(ctx, seed=1)
    rng = np.random.default_rng(4)
    B = 256
    X = device_bf16(rng.normal(0, 1, (B, 64)).astype(np.float32))
    t = torch.from_numpy(rng.normal(0, 1, B).astype(np.float32)).cuda()
    p0 = net.params().astype(np.float64)
    g, _ = net.gradients(X, t)
    g = g.cpu().numpy().astype(np.float64)
    lr = 1e-3
    net.train_step(X, t, lr)
    p1 = net.params().astype(np.float64)
    m = 0.1 * g
    v = 0.001 * g * g
    want = p0 - lr * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
    assert np.max(np.abs(p1 - want)) <= 1e-6 + 1e-5 * lr
    net.close()


def test_training_fits_a_smooth_target(ctx):
    from paper_1802_06215_amd import Mlp
    net = Mlp(ctx, seed=2)
    rng = np.random.default_rng(6)
    N = 65536
    X = rng.uniform(-1, 1, (N, 64)).astype(np.float32)
    t = (np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2] + 0.5 * X[:, 3]).astype(np.float32)
    Xd, td = device_bf16(X), torch.from_numpy(t).cuda()
    loss = torch.zeros(1, device="cuda")
    first = None
    for step in range(300):
        i0 = (step * 1024) % N
        net.train_step(Xd[i0:i0 + 1024], td[i0:i0 + 1024], 2e-3, loss)
        if step == 0:
            first = float(loss.cpu())
    y = net.forward(Xd[:4096]).cpu().numpy()
    mse = float(np.mean((y - t[:4096]) ** 2))
    print("loss first %.4f final mse %.5f" % (first, mse), flush=True)
    assert mse < 0.05 * first
    net.close()


def test_features_match_definition(ctx):
    from paper_1802_06215_amd import features
    import oracle
    desc = W.rocksample_model(15, 15, 3)
    lf = W.rocksample_leaf(desc, 1000, 10, 3, p_term=0.1)
    st = oracle.parent_states(desc, lf)
    m = ctx.upload_model(desc)
    depths = np.random.default_rng(0).integers(0, 100, 1000).astype(np.int32)
    X = features(ctx, m, {"w": torch.from_numpy(st["w"]).cuda()}, torch.from_numpy(depths).cuda(), 90)
    got = X.cpu().numpy().view(np.uint16)
    want = (ref.bf16_round(ref.rocksample_features(desc, st["w"], depths, 90)).view(np.uint32) >> 16).astype(np.uint16)
    assert np.array_equal(got, want)


def test_checkpoint_roundtrip(ctx, tmp_path):
    """save/load restores the parameters, the Adam moments and step: the next
    training step from a loaded copy equals the original's bit for bit."""
    from paper_1802_06215_amd import Mlp
    from paper_1802_06215_amd.hdx import HdxError
    rng = np.random.default_rng(3)
    X = device_bf16(rng.normal(0, 1, (1024, 64)).astype(np.float32))
    t = torch.from_numpy(rng.normal(0, 1, 1024).astype(np.float32)).cuda()
    a = Mlp(ctx, seed=7)
    for _ in range(3):
        a.train_step(X, t, 1e-3)
    path = str(tmp_path / "net.ckpt")
    a.save(path)
    b = Mlp(ctx, seed=99)
    b.load(path)
    assert np.array_equal(a.params().view(np.uint32), b.params().view(np.uint32))
    a.train_step(X, t, 1e-3)
    b.train_step(X, t, 1e-3)
    torch.cuda.synchronize()
    assert np.array_equal(a.params().view(np.uint32), b.params().view(np.uint32))
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(b"not a checkpoint")
    with pytest.raises(HdxError):
        b.load(str(bad))
    a.close()
    b.close()
