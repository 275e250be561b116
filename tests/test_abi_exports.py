"""The C-ABI library loads and exports every symbol include/hdx.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def libpath():
    from paper_1802_06215_amd import build
    if not build.is_built():
        build.build()
    return build.OUT


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hdx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hdx_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for call in ("hdx_init", "hdx_upload_model", "hdx_sample_scenarios", "hdx_expand_leaf",
                 "hdx_rollout_bounds", "hdx_backup"):
        assert call in names


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_lists_every_declared_symbol():
    from paper_1802_06215_amd import EXPORTS
    assert sorted(EXPORTS) == declared_functions()


def test_version_string(libpath):
    lib = ctypes.CDLL(libpath)
    lib.hdx_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.hdx_version()


def test_tree_backup_host_side(libpath):
    # the tree and the Eq. 4 backup are host code: checked against the
    # oracle's backup on the same inputs, no GPU needed
    import numpy as np
    import oracle
    from paper_1802_06215_amd import Tree
    rng = np.random.default_rng(3)
    A, cap, n = 4, 3, 12
    t = Tree(A, 0.9, n, 50.0, -5.0)
    root = oracle.Node(None, n, 50.0, -5.0)
    nch = np.array([1, 2, 3, 2], np.int32)
    cn = np.zeros((A, cap), np.int32)
    for a in range(A):
        parts = np.sort(rng.choice(np.arange(1, n), nch[a] - 1, replace=False))
        cn[a, :nch[a]] = np.diff(np.concatenate([[0], parts, [n]]))
    u0 = rng.uniform(0, 20, (A, cap)).astype(np.float32)
    l0 = (u0 - rng.uniform(0, 10, (A, cap))).astype(np.float32)
    rm = rng.uniform(-1, 1, A).astype(np.float32)
    cz = np.arange(A * cap, dtype=np.uint64).reshape(A, cap)
    first = t.add_children(0, nch, cz, cn, u0, l0, rm, cap)
    assert first == 1
    res = dict(n_children=nch, child_n=cn, child_u0=u0.astype(np.float64),
               child_l0=l0.astype(np.float64), r_mean=rm.astype(np.float64))
    oracle.attach_children(dict(n_actions=A), root, res)
    t.backup(0)
    oracle.backup(root, 0.9)
    u, l = t.bounds(0)
    assert abs(u - root.u) < 1e-12 and abs(l - root.l) < 1e-12
    # a second level under (action 2, child 1)
    kid = first + int(nch[:2].sum()) + 1
    kn = int(cn[2, 1])
    nch2 = np.ones(A, np.int32)
    cn2 = np.zeros((A, cap), np.int32)
    cn2[:, 0] = kn
    u2 = rng.uniform(0, 20, (A, cap)).astype(np.float32)
    l2 = (u2 - 3).astype(np.float32)
    r2 = rng.uniform(-1, 1, A).astype(np.float32)
    t.add_children(kid, nch2, cz, cn2, u2, l2, r2, cap)
    okid = root.actions[2][1][1]
    oracle.attach_children(dict(n_actions=A), okid, dict(n_children=nch2, child_n=cn2,
                           child_u0=u2.astype(np.float64), child_l0=l2.astype(np.float64),
                           r_mean=r2.astype(np.float64)))
    t.backup(kid)
    oracle.backup(okid, 0.9)
    u, l = t.bounds(0)
    assert abs(u - root.u) < 1e-12 and abs(l - root.l) < 1e-12
    assert t.size() == 1 + int(nch.sum()) + A
    # child counts must add up to the node's scenario count
    with pytest.raises(Exception):
        t.add_children(first, nch2, cz, cn2 + 1, u2, l2, r2, cap)
