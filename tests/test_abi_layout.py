"""The binding's ctypes structures against the C header, field by field.

A small C program compiled with gcc here prints sizeof and the offset of
every field of the structures the binding mirrors; each must equal the
ctypes layout (a field added to one side only would shift every field
after it and corrupt the calls silently)."""
import ctypes as C
import os
import subprocess

import pytest

from paper_1802_06215_amd import hdx as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = [("hdx_model_desc", H.ModelDesc), ("hdx_belief", H.Belief), ("hdx_rollout_cfg", H.RolloutCfg),
         ("hdx_states", H.States), ("hdx_search_cfg", H.SearchCfg), ("hdx_search_result", H.SearchResult),
         ("hdx_leaf", H.Leaf)]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    d = tmp_path_factory.mktemp("abi")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "hdx.h"', "int main(void) {"]
    for cname, cls in PAIRS:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines += ["return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines))
    exe = d / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.splitlines():
        name, field, val = line.split()
        res[(name, field)] = int(val)
    return res


@pytest.mark.parametrize("cname,cls", PAIRS, ids=[p[0] for p in PAIRS])
def test_struct_layout_matches_header(c_layout, cname, cls):
    assert C.sizeof(cls) == c_layout[(cname, "size")]
    for f in cls._fields_:
        assert getattr(cls, f[0]).offset == c_layout[(cname, f[0])], f[0]
