"""ctypes binding of the plain CPU oracle (``pldl_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only users.  Nothing in the product
package imports this module.

All arrays are numpy ``uint32`` residues in [0, p) (C-contiguous, row-major);
index arrays are ``int32``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pldl_oracle.c")
_LIB = os.environ.get("ORC_LIB") or os.path.join(_HERE, "liborc.so")

_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liborc.so``."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", _LIB + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_inv.argtypes = [_u32, _u32]
        L.orc_inv.restype = _u32
        L.orc_rank.argtypes = [_u32, _i64, _i64, _u32p, _i64]
        L.orc_rank.restype = _i64
        L.orc_leading_ranks.argtypes = [_u32, _i64, _u32p, _i64, _i64p]
        L.orc_rpm_bruteforce.argtypes = [_u32, _i64, _u32p, _i64, _i32p]
        L.orc_search.argtypes = [_u32, _i64, _u32p, _i64, _i32p, _u32p, _i64, _u32p, _u32p, _i32p,
                                 ctypes.POINTER(_i64)]
        L.orc_replay.argtypes = [_u32, _i64, _u32p, _i64, _i32p, _i32p, _i64, _u32p, _i64, _u32p, _u32p]
        L.orc_reconstruct.argtypes = [_u32, _i64, _i32p, _u32p, _i64, _u32p, _u32p, _u32p, _i64]
        L.orc_char2_standard.argtypes = [_i64, _i32p, _u32p, _i64, _u32p, _u32p]
        L.orc_gemm.argtypes = [_u32, _i64, _i64, _i64, _u32p, _i64, _u32p, _i64, _u32p, _i64]
        L.orc_trsm_left.argtypes = [_u32, ctypes.c_int, _i64, _i64, _u32p, _i64, _u32p, _i64]
        L.orc_syrdk.argtypes = [_u32, _i64, _i64, _u32p, _i64, _u32p, _u32p, _u32p, _i64]
        L.orc_syrd2k.argtypes = [_u32, _i64, _i64, _u32p, _i64, _u32p, _i64, _u32p, _u32p, _u32p, _i64]
        L.orc_trss.argtypes = [_u32, _i64, _u32p, _i64, _u32p, _i64, _u32p, _i64]
        L.orc_plduq.argtypes = [_u32, _i64, _i64, _u32p, _i64, _i32p, _i32p, _u32p, _i64,
                                ctypes.POINTER(_i64)]
        L.orc_delta.argtypes = [_u32, _i64, _u32p, _i64, _u32p, _i64, _u32p]
        L.orc_det.argtypes = [_u32, _i64, _u32p, _i64, _u32p]
        L.orc_solve.argtypes = [_u32, _i64, _u32p, _i64, _u32p, _i64, _i64, _u32p, _i64, _i32p]
        for f in ("orc_leading_ranks", "orc_rpm_bruteforce", "orc_search", "orc_replay",
                  "orc_reconstruct", "orc_char2_standard", "orc_gemm", "orc_trsm_left", "orc_syrdk",
                  "orc_syrd2k", "orc_trss", "orc_plduq", "orc_delta", "orc_det", "orc_solve"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _u(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.uint32)


def _sq(A):
    A = _u(A)
    assert A.ndim == 2 and A.shape[0] == A.shape[1]
    return A


def inv(a: int, p: int) -> int:
    return int(lib().orc_inv(a, p))


def rank(A, p: int) -> int:
    A = _u(A)
    m, n = A.shape
    return int(lib().orc_rank(p, m, n, A, max(n, 1)))


def leading_ranks(A, p: int) -> np.ndarray:
    A = _sq(A)
    n = A.shape[0]
    r = np.zeros((n + 1, n + 1), dtype=np.int64)
    assert lib().orc_leading_ranks(p, n, A, max(n, 1), r) == 0
    return r


def rpm_bruteforce(A, p: int) -> np.ndarray:
    A = _sq(A)
    n = A.shape[0]
    rpm = np.zeros(n, dtype=np.int32)
    rc = lib().orc_rpm_bruteforce(p, n, A, max(n, 1), rpm)
    assert rc == 0, rc
    return rpm


def search(A, p: int) -> dict:
    """Canonical factorization (base-case pivot order).  See the C header."""
    A = _sq(A)
    n = A.shape[0]
    perm = np.zeros(n, dtype=np.int32)
    L = np.zeros((n, n), dtype=np.uint32)
    dd = np.zeros(n, dtype=np.uint32)
    de = np.zeros(n, dtype=np.uint32)
    rpm = np.zeros(n, dtype=np.int32)
    r = _i64(0)
    rc = lib().orc_search(p, n, A, max(n, 1), perm, L, max(n, 1), dd, de, rpm, ctypes.byref(r))
    assert rc == 0, rc
    return dict(perm=perm, L=L, dd=dd, de=de, rpm=rpm, rank=int(r.value))


def replay(A, p: int, perm, rpm, rank_: int):
    """Recompute (L, D) for an imposed pivot order.  Returns (rc, dict)."""
    A = _sq(A)
    n = A.shape[0]
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    rpm = np.ascontiguousarray(rpm, dtype=np.int32)
    L = np.zeros((n, n), dtype=np.uint32)
    dd = np.zeros(n, dtype=np.uint32)
    de = np.zeros(n, dtype=np.uint32)
    rc = lib().orc_replay(p, n, A, max(n, 1), perm, rpm, int(rank_), L, max(n, 1), dd, de)
    return int(rc), dict(perm=perm, L=L, dd=dd, de=de, rpm=rpm, rank=int(rank_))


def reconstruct(p: int, perm, L, dd, de) -> np.ndarray:
    L = _sq(L)
    n = L.shape[0]
    out = np.zeros((n, n), dtype=np.uint32)
    assert lib().orc_reconstruct(p, n, np.ascontiguousarray(perm, dtype=np.int32), L, max(n, 1),
                                 _u(dd), _u(de), out, max(n, 1)) == 0
    return out


def char2_standard(perm, L, dd, de):
    perm = np.array(perm, dtype=np.int32)
    L = np.array(L, dtype=np.uint32)
    dd = np.array(dd, dtype=np.uint32)
    de = np.array(de, dtype=np.uint32)
    n = L.shape[0]
    assert lib().orc_char2_standard(n, perm, L, max(n, 1), dd, de) == 0
    return perm, L, dd, de


def gemm(p: int, C, A, B) -> np.ndarray:
    """C - A B."""
    A, B, C = _u(A), _u(B), np.array(C, dtype=np.uint32)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2 and C.shape == (m, n)
    assert lib().orc_gemm(p, m, n, k, A, max(k, 1), B, max(n, 1), C, max(n, 1)) == 0
    return C


def trsm_left(p: int, T, B, lower: bool) -> np.ndarray:
    """T^{-1} B for a unit lower/upper T."""
    T, B = _u(T), np.array(B, dtype=np.uint32)
    m, n = B.shape
    assert lib().orc_trsm_left(p, 1 if lower else 0, m, n, T, max(m, 1), B, max(n, 1)) == 0
    return B


def syrdk(p: int, C, A, dd, de) -> np.ndarray:
    """Lower triangle of C - A D A^T (upper part of C returned untouched)."""
    A, C = _u(A), np.array(C, dtype=np.uint32)
    n, k = A.shape
    assert lib().orc_syrdk(p, n, k, A, max(k, 1), _u(dd), _u(de), C, max(n, 1)) == 0
    return C


def syrd2k(p: int, C, A, B, dd, de) -> np.ndarray:
    A, B, C = _u(A), _u(B), np.array(C, dtype=np.uint32)
    n, k = A.shape
    assert lib().orc_syrd2k(p, n, k, A, max(k, 1), B, max(k, 1), _u(dd), _u(de), C, max(n, 1)) == 0
    return C


def trss(p: int, U, C):
    """Upper X with X^T U + U^T X = C (Problem 1).  Returns (rc, X)."""
    U, C = _u(U), _u(C)
    n = U.shape[0]
    X = np.zeros((n, n), dtype=np.uint32)
    rc = lib().orc_trss(p, n, U, max(n, 1), C, max(n, 1), X, max(n, 1))
    return int(rc), X


def plduq(p: int, Y) -> dict:
    Y = _u(Y)
    m, n = Y.shape
    rows = np.zeros(m, dtype=np.int32)
    cols = np.zeros(n, dtype=np.int32)
    LU = np.zeros((m, n), dtype=np.uint32)
    r = _i64(0)
    assert lib().orc_plduq(p, m, n, Y, max(n, 1), rows, cols, LU, max(n, 1), ctypes.byref(r)) == 0
    return dict(rows=rows, cols=cols, LU=LU, rank=int(r.value))


def delta(p: int, U, C) -> np.ndarray:
    U, C = _u(U), _u(C)
    r = U.shape[0]
    d = np.zeros(r, dtype=np.uint32)
    assert lib().orc_delta(p, r, U, max(r, 1), C, max(r, 1), d) == 0
    return d


def det(A, p: int) -> int:
    """det(A) mod p by plain elimination (Section 1's uses: invariants of the form)."""
    A = _sq(A)
    out = np.zeros(1, dtype=np.uint32)
    assert lib().orc_det(p, A.shape[0], A, max(A.shape[0], 1), out) == 0
    return int(out[0])


def solve(A, p: int, B):
    """A X = B by Gauss-Jordan elimination (Section 1's uses: symmetric systems).
    Returns (X, cons): cons[k] = 1 when column k has a solution."""
    A = _sq(A)
    n = A.shape[0]
    B = _u(B)
    if B.ndim == 1:
        B = B.reshape(n, 1)
    nrhs = B.shape[1]
    X = np.zeros((n, nrhs), dtype=np.uint32)
    cons = np.zeros(nrhs, dtype=np.int32)
    assert lib().orc_solve(p, n, A, max(n, 1), B, max(nrhs, 1), nrhs, X, max(nrhs, 1), cons) == 0
    return X, cons


def effective_ops(n: int, r: int) -> float:
    """Classic-arithmetic operation count of the factorization (Section 6)."""
    return r ** 3 / 3.0 + n * n * r - r * r * n
