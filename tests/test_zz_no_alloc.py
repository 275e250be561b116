"""hdx_expand_leaf_noalloc, the expansion entry point that allocates
nothing (its descriptors, tile list and queue heads in the library's fixed
per-GPU scratch array), against hdx_expand_leaf on the same leaves: every
output bit-identical, on two calls in a row, the second smaller; and the
documented capacity limits refused before anything is launched."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_util import cfg_pair, collect, gpu_leaf_desc, ids_dev, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1802_06215_amd import Context
    c = Context(0)
    yield c
    c.close()


def make_items(ctx, seed, n_mixed, n_mars, n_nav):
    """Leaves of every model kind: mixed RockSample / driving instances,
    multi-agent RockSample (11, 11) and navigation 13x13."""
    items = []
    for i, it in enumerate(W.mixed_instances(n_mixed, seed)):
        desc, K = it["model"], it["K"]
        m = ctx.upload_model(desc)
        if desc["kind"] == 0:
            lf = W.rocksample_leaf(desc, K, K - (i * 13) % (K // 2), seed + i)
            cfgs = cfg_pair(0, 1 << 30, 90)
        else:
            lf = W.pednav_leaf(desc, K, K - (i * 13) % (K // 2), seed + i)
            cfgs = cfg_pair(0, 50)
        items.append((desc, m, lf, cfgs))
    if n_mars:
        dm = W.mars_model(11, 11, 1)
        mm = ctx.upload_model(dm)
        for i in range(n_mars):
            items.append((dm, mm, W.mars_leaf(dm, 300, 200 - 37 * i, seed + 100 + i), cfg_pair(0, 1 << 30, 90)))
    if n_nav:
        dn = W.nav_model(1)
        mn = ctx.upload_model(dn)
        for i in range(n_nav):
            items.append((dn, mn, W.nav_leaf(dn, 600, 500 - 91 * i, seed + 200 + i), cfg_pair(0, 1 << 30, 90)))
    built = []
    for j, (desc, m, lf, cfgs) in enumerate(items):
        par, pids = to_dev(oracle.parent_states(desc, lf)), ids_dev(lf["ids"])
        leaf, out, idx = gpu_leaf_desc(m, par, pids, lf["idx"], lf["depth"], lf["last_action"], seed + j, 1,
                                       cfgs[1], True)
        built.append(dict(m=m, leaf=leaf, out=out, keep=(par, pids, idx)))
    return built


def poison(items):
    for it in items:
        o = it["out"]
        for t in (o.child_u0, o.child_l0, o.child_z, o.child_n, o.child_off, o.r_mean, o.perm, o.n_children,
                  o.steps, o.ids, o.r, o.z, o.U, o.L, o.child_of):
            t.fill_(-7)
        for t in list(o.states.values()) + list(o.sprime.values()):
            t.fill_(7 if t.dtype == torch.uint8 else -7)
    torch.cuda.synchronize()


def snapshot(items):
    return [collect(it["m"], it["out"]) for it in items]


def assert_identical(a, b):
    for x, y in zip(a, b):
        assert x.keys() == y.keys()
        for key in x:
            if isinstance(x[key], dict):
                for f in x[key]:
                    assert np.array_equal(x[key][f], y[key][f]), (key, f)
            elif key.startswith("child_"):
                # child slots past a leaf's child count are not written
                for a_, nc in enumerate(y["n_children"]):
                    u, v = x[key][a_, :nc], y[key][a_, :nc]
                    assert np.array_equal(u.view(np.uint32) if u.dtype == np.float32 else u,
                                          v.view(np.uint32) if v.dtype == np.float32 else v), key
            else:
                u, v = x[key], y[key]
                if u.dtype == np.float32:
                    u, v = u.view(np.uint32), v.view(np.uint32)
                assert np.array_equal(u, v), key


def run_both(ctx, items):
    leaves = [it["leaf"] for it in items]
    poison(items)
    ctx.expand_leaf(leaves)
    torch.cuda.synchronize()
    ref = snapshot(items)
    poison(items)
    ctx.expand_leaf_noalloc(leaves)
    torch.cuda.synchronize()
    return ref, snapshot(items)


def test_noalloc_equals_expand_leaf_on_two_calls(ctx):
    big = make_items(ctx, 11, 40, 3, 3)
    small = make_items(ctx, 77, 5, 1, 1)
    tiles = lambda its: sum(int(it["out"].A) for it in its)
    print("noalloc call 1: %d leaves, %d tiles" % (len(big), tiles(big)), flush=True)
    ref, got = run_both(ctx, big)
    assert_identical(got, ref)
    print("noalloc call 2: %d leaves, %d tiles" % (len(small), tiles(small)), flush=True)
    ref, got = run_both(ctx, small)
    assert_identical(got, ref)
    # and back-to-back calls on one stream without a host wait between them
    poison(small)
    ctx.expand_leaf_noalloc([it["leaf"] for it in big])
    ctx.expand_leaf_noalloc([it["leaf"] for it in small])
    torch.cuda.synchronize()
    assert_identical(snapshot(small), ref)


def test_noalloc_refuses_beyond_its_limits(ctx):
    from paper_1802_06215_amd import HdxError
    from paper_1802_06215_amd import hdx as H
    items = make_items(ctx, 5, 2, 1, 0)
    rs = [it for it in items if it["m"].kind == H.ROCKSAMPLE or it["m"].kind == H.PEDNAV][0]
    with pytest.raises(HdxError) as e:
        ctx.expand_leaf_noalloc([rs["leaf"]] * (H.NOALLOC_MAX_LEAVES + 1))
    assert e.value.code == -5
    mars = [it for it in items if it["m"].kind == H.MARS][0]
    A = int(mars["out"].A)
    with pytest.raises(HdxError) as e:
        ctx.expand_leaf_noalloc([mars["leaf"]] * (H.NOALLOC_MAX_TILES // A + 1))
    assert e.value.code == -5
    # the refused calls launched nothing: a valid call still matches
    ref, got = run_both(ctx, items)
    assert_identical(got, ref)
