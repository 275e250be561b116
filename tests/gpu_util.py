"""Helpers for the GPU parity tests: run one leaf through the C ABI and
through the oracle on the same seeded inputs, and compare.

Bar: states, ids, observations, groupings, step counts and rewards
bit-exact; floating-point values within 1e-5 of the FP64 oracle relative to
max(|value|, sum of the absolute terms that make it up)."""
import numpy as np
import torch

import oracle
from paper_1802_06215_amd import hdx as H

RTOL = 1e-5


def to_dev(st: dict) -> dict:
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in st.items()}


def ids_dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np.int64).astype(np.int32))).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def cfg_pair(policy=0, max_steps=1 << 30, max_depth=-1, const_action=0):
    return (oracle.cfg(policy, max_steps, max_depth, const_action),
            H.rollout_cfg(policy, max_steps, max_depth, const_action))


def gpu_leaf_desc(model, parent_dev, pids_dev, idx_np, depth, last_action, seed, step, hcfg,
                  per_pair=True):
    idx = H.positions(idx_np)
    out = H.LeafBuffers(model, len(idx_np), per_pair)
    leaf = H.make_leaf(model, parent_dev, pids_dev, idx, depth, last_action, out, seed, step, hcfg)
    return leaf, out, idx


def collect(model, out: H.LeafBuffers) -> dict:
    n = out.n
    res = dict(n_children=host(out.n_children), child_z=host(out.child_z).view(np.uint64),
               child_n=host(out.child_n), child_off=host(out.child_off),
               child_u0=host(out.child_u0), child_l0=host(out.child_l0), r_mean=host(out.r_mean),
               steps=host(out.steps), perm=host(out.perm)[:, :n], ids=host(out.ids)[:n].view(np.uint32))
    res["states"] = {k: host(v)[..., :n] for k, v in out.states.items()}
    if out.per_pair:
        A = out.A
        res.update(r=host(out.r)[:, :n], z=host(out.z)[:, :n].view(np.uint64), U=host(out.U)[:, :n],
                   L=host(out.L)[:, :n], child_of=host(out.child_of)[:, :n])
        sp = {k: host(v)[..., :A * n] for k, v in out.sprime.items()}
        if model.kind == H.ROCKSAMPLE:
            sp["w"] = sp["w"].reshape(A, n)
        elif model.kind in (H.MARS, H.NAV):
            sp["w"] = sp["w"].reshape(sp["w"].shape[0], A, n)
        else:
            sp["s"], sp["car"] = sp["s"].reshape(A, n), sp["car"].reshape(A, n)
            for f in ("px", "py", "goal"):
                sp[f] = sp[f].reshape(-1, A, n)
        res["sprime"] = sp
    return res


def run_gpu_leaf(ctx, model, parent_np, parent_ids, idx, depth, last_action, seed, step, hcfg,
                 per_pair=True):
    parent = to_dev(parent_np)
    pids = ids_dev(parent_ids)
    leaf, out, keep = gpu_leaf_desc(model, parent, pids, idx, depth, last_action, seed, step, hcfg,
                                    per_pair)
    ctx.expand_leaf([leaf])
    torch.cuda.synchronize()
    return collect(model, out)


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32) if a.dtype == np.float32 else a


def assert_states_equal(a: dict, b: dict):
    assert set(a) == set(b)
    for k in a:
        assert a[k].shape == b[k].shape, k
        assert np.array_equal(bits(a[k]), bits(b[k])), "state field %s differs" % k


def close(gpu, ref, scale, what):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    tol = RTOL * np.maximum(np.abs(ref), np.asarray(scale, np.float64)) + 1e-30
    bad = np.abs(gpu - ref) > tol
    assert not bad.any(), "%s: %d values off, worst %r vs %r" % (
        what, bad.sum(), gpu[bad][:3], ref[bad][:3])


def compare_leaf(desc, gpu: dict, ref: dict, n: int):
    A = desc["n_actions"]
    assert_states_equal(gpu["states"], ref["states"])
    assert np.array_equal(gpu["ids"], ref["ids"])
    assert np.array_equal(gpu["n_children"], ref["n_children"])
    # per action: (expansion steps, rollout steps), element by element
    assert np.array_equal(gpu["steps"], ref["steps"]), "per-action step counts differ"
    assert np.array_equal(gpu["perm"], ref["perm"])
    for a in range(A):
        nc = int(ref["n_children"][a])
        for f in ("child_z", "child_n", "child_off"):
            assert np.array_equal(gpu[f][a, :nc], ref[f][a, :nc]), (f, a)
    # the oracle always supplies per-scenario values (the tolerance scales)
    if "r" in gpu:
        assert np.array_equal(bits(gpu["r"]), bits(ref["r"])), "step rewards differ"
        assert np.array_equal(gpu["z"], ref["z"]), "observations differ"
        assert np.array_equal(gpu["child_of"], ref["child_of"])
        assert_states_equal(gpu["sprime"], ref["sprime"])
        close(gpu["U"], ref["U"], 0.0, "per-scenario U")
        close(gpu["L"], ref["L"], ref["Labs"], "per-scenario L")
    absr = np.abs(ref["r"].astype(np.float64)).mean(1) if n else np.zeros(A)
    close(gpu["r_mean"], ref["r_mean"], absr, "R(b,a)")
    for a in range(A):
        nc = int(ref["n_children"][a])
        for c in range(nc):
            off, cnt = ref["child_off"][a, c], ref["child_n"][a, c]
            seg = ref["perm"][a, off:off + cnt]
            close(gpu["child_u0"][a, c], ref["child_u0"][a, c], 0.0, "u0")
            close(gpu["child_l0"][a, c], ref["child_l0"][a, c], ref["Labs"][a, seg].mean(), "l0")
