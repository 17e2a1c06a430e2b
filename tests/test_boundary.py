"""C-ABI boundary checks that need no GPU: the library loads and exports every
entry point declared in include/pldl.h; argument errors are reported before any
device work (a NULL context is rejected without touching HIP)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pldl.h")
LIB = os.path.join(ROOT, "paper_1802_10453_amd", "libpldl.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pldl_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = declared()
    for f in ("pldl_create", "pldl_destroy", "pldl_last_error", "pldl_factor", "pldl_gemm", "pldl_trsm",
              "pldl_syrdk", "pldl_trss", "pldl_plduq"):
        assert f in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libpldl.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


def test_null_context_rejected_without_device():
    lib = ctypes.CDLL(LIB)
    lib.pldl_factor.restype = ctypes.c_int
    rank = ctypes.c_int64(0)
    rc = lib.pldl_factor(None, ctypes.c_uint32(65521), ctypes.c_int64(4), None, ctypes.c_int64(4), 0, None, None,
                         None, ctypes.byref(rank), None, None, None)
    assert rc == -1
    lib.pldl_last_error.restype = ctypes.c_char_p
    assert lib.pldl_last_error(None) == b"null context"
    lib.pldl_destroy.restype = ctypes.c_int
    assert lib.pldl_destroy(None) == 0
