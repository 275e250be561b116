"""The product path has no CPU fallback: without the built HIP library
the binding raises instead of computing anything, and nothing in the
package imports the oracle."""
import ast
import os

import pytest

from paper_1802_06215_amd import hdx as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1802_06215_amd")


def test_missing_library_raises(monkeypatch, tmp_path):
    monkeypatch.setattr(H, "_lib", None)
    monkeypatch.setattr(H, "LIB_PATH", str(tmp_path / "libhdx.so"))
    with pytest.raises(ImportError, match="not built"):
        H.load_library()


def test_package_does_not_import_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if not f.endswith(".py"):
                continue
            tree = ast.parse(open(os.path.join(dirpath, f)).read())
            for node in ast.walk(tree):
                names = []
                if isinstance(node, ast.Import):
                    names = [a.name for a in node.names]
                elif isinstance(node, ast.ImportFrom):
                    names = [node.module or ""]
                assert not any(n == "oracle" or n.startswith("oracle.") for n in names), (f, names)
