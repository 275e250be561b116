"""Parity at full size, in the launch configuration bench.py times: the
autotuned, graph-replayed batch of the benchmark workloads, checked leaf by
leaf against the oracle on a sample of leaves (the oracle computes each
sampled leaf on its own)."""
import types

import numpy as np
import pytest
import torch

import oracle
from gpu_util import collect, compare_leaf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1802_06215_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("workload,sample", [("rs15", 12), ("rs7", 12), ("ped16", 6), ("ped16s", 16), ("mix64", 12)])
def test_bench_workload_sampled_leaves(ctx, workload, sample):
    import bench
    from paper_1802_06215_amd import Batch
    args = types.SimpleNamespace(workload=workload, leaves=0)
    wl = bench.build(ctx, args)
    leaves, items = wl["leaves"], wl["items"]
    n_tiles = sum(it[0]["n_actions"] for it in items)
    print("%s: %d leaves, %d tiles" % (workload, len(leaves), n_tiles), flush=True)
    b = Batch(ctx, len(leaves), n_tiles)
    b.set_leaves(leaves)
    b.autotune(1)
    b.use_graph(True)
    b.launch()
    b.launch()
    torch.cuda.synchronize()
    # per-leaf views of the slab outputs, in build() order
    views = {}
    for g, ks in enumerate(wl["groups"]):
        for j, k in enumerate(ks):
            views[k] = (g, j)
    pick = np.linspace(0, len(items) - 1, sample).astype(int)
    for k in pick:
        d, lf, seed, cfg = items[k]
        g, j = views[k]
        slab = wl["slabs"][g]
        n = len(lf["idx"])
        A = d["n_actions"]
        out = types.SimpleNamespace(n=n, A=A, per_pair=False, ids=slab["ids"][j], perm=slab["perm"][j],
                                    n_children=slab["n_children"][j], child_z=slab["child_z"][j],
                                    child_n=slab["child_n"][j], child_off=slab["child_off"][j],
                                    child_u0=slab["child_u0"][j], child_l0=slab["child_l0"][j],
                                    r_mean=slab["r_mean"][j], steps=slab["steps"][j])
        # the kernel writes perm as [A][n] contiguous inside the slab row
        flat = slab["perm"][j].reshape(-1)[:A * n].reshape(A, n)
        out.perm = flat
        cap = slab["child_z"].shape[-1]
        for f in ("child_z", "child_n", "child_off", "child_u0", "child_l0"):
            setattr(out, f, slab[f][j].reshape(-1)[:A * cap].reshape(A, cap))
        out.states = {key: v[j] for key, v in wl["state_slabs"][g].items()}
        gpu = collect(wl["models"][id(d)], out)
        ref = oracle.expand_leaf(d, oracle.cfg(*cfg), oracle.parent_states(d, lf), lf["ids"].astype(np.uint32),
                                 lf["idx"], lf["depth"], lf["last_action"], seed, 0, per_pair=True)
        compare_leaf(d, gpu, ref, n)
    b.close()
