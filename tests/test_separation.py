"""The oracle and the HIP path share no code: no source of the library or its
binding imports or includes the oracle, the oracle reads nothing of the library,
the built library exports no oracle symbol, and bench.py loads the oracle only
inside its CPU-baseline functions.  Static checks, no GPU."""
import ast
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1802_10453_amd")
LIB = os.path.join(PKG, "libpldl.so")


def sources(top, exts):
    for d, _, files in os.walk(top):
        if "_build" in d or "__pycache__" in d:
            continue
        for f in files:
            if f.endswith(exts):
                yield os.path.join(d, f)


def code_only(path):
    """The source without comments and docstrings (what could import or include)."""
    txt = open(path, encoding="utf-8").read()
    if path.endswith(".py"):
        tree = ast.parse(txt)
        return "\n".join(ast.unparse(n) for n in ast.walk(tree) if isinstance(n, (ast.Import, ast.ImportFrom)))
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return re.sub(r"//[^\n]*", "", txt)


def test_library_and_binding_do_not_use_the_oracle():
    files = list(sources(PKG, (".py", ".hip", ".h", ".cpp"))) + list(sources(os.path.join(ROOT, "include"), (".h",)))
    assert files
    for f in files:
        code = code_only(f)
        assert not re.search(r"\boracle\b|pldl_oracle|orc_", code), f


def test_oracle_does_not_use_the_library():
    files = list(sources(os.path.join(ROOT, "oracle"), (".py", ".c", ".h")))
    assert files
    for f in files:
        code = code_only(f)
        assert not re.search(r"paper_1802_10453_amd|pldl\.h|csrc|libpldl|\bpldl\b", code), f


def test_built_library_exports_no_oracle_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libpldl.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    for name in ("orc_search", "orc_replay", "orc_reconstruct", "orc_gemm", "orc_syrdk", "orc_plduq", "orc_inv"):
        assert not hasattr(lib, name), name


def test_bench_imports_the_oracle_only_in_its_cpu_baselines():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py"), encoding="utf-8").read())
    for node in tree.body:   # module level: no oracle import
        if isinstance(node, (ast.Import, ast.ImportFrom)):
            assert "oracle" not in ast.unparse(node)
    users = set()
    for fn in (n for n in ast.walk(tree) if isinstance(n, ast.FunctionDef)):
        for node in ast.walk(fn):
            if isinstance(node, (ast.Import, ast.ImportFrom)) and "oracle" in ast.unparse(node):
                users.add(fn.name)
    assert users and all(u.startswith("cpu_baseline") for u in users), users
