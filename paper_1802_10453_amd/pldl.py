"""Thin ctypes binding of ``libpldl.so`` (the C-ABI of ``include/pldl.h``).

Argument marshalling only: every step of the factorization runs in the HIP
library.  Tensors are torch tensors on the context's GPU; the current torch
stream is passed to every call.  If the library is missing this module raises
at import time -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpldl.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1802_10453_amd.build.build() "
                      "(hipcc for gfx950); the library has no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)
_vp, _i64, _i32, _u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32

PLDL_U32, PLDL_F64 = 0, 1
PLDL_PATH_AUTO, PLDL_PATH_F64, PLDL_PATH_I8 = 0, 1, 2
PLDL_THRESHOLD_ONLINE = -1
ERRORS = {1: "PLDL_ERANGE", 2: "PLDL_EUNSUPPORTED_P", 3: "PLDL_EHIP", 4: "PLDL_ENOMEM", 5: "PLDL_EINTERNAL",
          6: "PLDL_ETOOBIG"}
NOALLOC_SCRATCH_DOUBLES = 1 << 21
ERRORS_BY_NAME = {v: k for k, v in ERRORS.items()}


CLASS_NAMES = ("gemm", "trsm_leaf", "base_case", "plduq_leaf", "trss_leaf", "perm", "other", "host_sync", "gemm_i8")


class pldl_kstat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
                ("ops8", ctypes.c_double), ("ms", ctypes.c_double)]


class pldl_stats(ctypes.Structure):
    _fields_ = [("cls", pldl_kstat * len(CLASS_NAMES))]


class pldl_opts(ctypes.Structure):
    _fields_ = [("path", _i32), ("threshold", _i32), ("standard_form", _i32), ("check_range", _i32)]


class pldl_schedule(ctypes.Structure):
    _fields_ = [("threshold_used", _i32), ("split_rule", _i32), ("path_used", _i32), ("i8_min_log2_flops", _i32),
                ("products_f64", _i64), ("products_i8", _i64), ("launches", _i64), ("host_waits", _i64),
                ("products_winograd", _i64)]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


_lib.pldl_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int]
_lib.pldl_destroy.argtypes = [_vp]
_lib.pldl_last_error.argtypes = [_vp]
_lib.pldl_last_error.restype = ctypes.c_char_p
_lib.pldl_factor.argtypes = [_vp, _u32, _i64, _vp, _i64, _i32, _vp, _vp, _vp, ctypes.POINTER(_i64),
                             ctypes.POINTER(pldl_opts), ctypes.POINTER(pldl_schedule), _vp]
_lib.pldl_gemm.argtypes = [_vp, _u32, _i64, _i64, _i64, _vp, _i64, _i32, _vp, _i64, _i32, _vp, _i64, _i32, _vp]
_lib.pldl_trsm.argtypes = [_vp, _u32, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp]
_lib.pldl_syrdk.argtypes = [_vp, _u32, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _i64, _vp]
_lib.pldl_solve.argtypes = [_vp, _u32, _i64, _vp, _i64, _i32, _vp, _vp, _i64, _vp, _i64, _i64, _vp, _vp]
_lib.pldl_invariants.argtypes = [_vp, _u32, _i64, _vp, _i64, _i32, _vp, _i64, ctypes.POINTER(_i64), _vp]
_lib.pldl_syrdk_noalloc.argtypes = [_vp, _u32, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp, _i64, _vp]
_lib.pldl_trss.argtypes = [_vp, _u32, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp]
_lib.pldl_plduq.argtypes = [_vp, _u32, _i64, _i64, _vp, _i64, _vp, _vp, ctypes.POINTER(_i64), _vp]
_lib.pldl_profile.argtypes = [_vp, _i32, ctypes.POINTER(pldl_stats)]
_lib.pldl_set_path.argtypes = [_vp, _i32]
_lib.pldl_set_winograd.argtypes = [_vp, _i64]
_lib.pldl_char2_to_standard.argtypes = [_vp, _i64, _vp, _i64, _i32, _vp, _vp, _vp]
_lib.pldl_autotune.argtypes = [_vp, _u32, ctypes.POINTER(_i64), _i64, ctypes.c_char_p, _vp]
_lib.pldl_factor_batched.argtypes = [_vp, _u32, _i64, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp,
                                     ctypes.POINTER(pldl_opts), _vp]
for _f in ("pldl_create", "pldl_destroy", "pldl_factor", "pldl_solve", "pldl_invariants", "pldl_gemm", "pldl_trsm",
           "pldl_syrdk", "pldl_syrdk_noalloc",
           "pldl_trss",
           "pldl_plduq", "pldl_profile", "pldl_set_path", "pldl_set_winograd", "pldl_factor_batched",
           "pldl_char2_to_standard", "pldl_autotune"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTED = ("pldl_create", "pldl_destroy", "pldl_last_error", "pldl_factor", "pldl_solve", "pldl_invariants",
            "pldl_gemm", "pldl_trsm",
            "pldl_syrdk", "pldl_syrdk_noalloc", "pldl_trss", "pldl_plduq", "pldl_profile", "pldl_set_path",
            "pldl_set_winograd", "pldl_factor_batched", "pldl_char2_to_standard", "pldl_autotune")


class PldlError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ld(t):
    assert t.dim() == 2 and t.stride(1) == 1, "row-major tensor with unit column stride expected"
    return max(t.stride(0), 1)


class Context:
    """One library context on one GPU (``pldl_create`` / ``pldl_destroy``)."""

    def __init__(self, device: int = 0):
        h = _vp()
        rc = _lib.pldl_create(ctypes.byref(h), int(device))
        if rc != 0:
            raise PldlError(rc, f"pldl_create(device={device}) failed")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            _lib.pldl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise PldlError(rc, _lib.pldl_last_error(self._h).decode())

    def last_error(self) -> str:
        return _lib.pldl_last_error(self._h).decode()

    # ------------------------------------------------------------------ pldl_factor
    def set_path(self, path: int):
        """pldl_set_path: PLDL_PATH_AUTO (INT8 products in pldl_factor for p < 2^23), PLDL_PATH_F64 or
        PLDL_PATH_I8 for the products of later calls."""
        self._check(_lib.pldl_set_path(self._h, int(path)))

    def set_winograd(self, min_order: int):
        """pldl_set_winograd: dense products with m, n, k >= min_order take Winograd levels (0: off)."""
        self._check(_lib.pldl_set_winograd(self._h, int(min_order)))

    def factor(self, A: torch.Tensor, p: int, threshold: int = 0, standard_form: bool = False,
               check_range: bool = True, path: int = PLDL_PATH_AUTO):
        """Factor the symmetric A (lower triangle; int32 holding uint32 residues, or float64)
        in place.  Returns dict(perm, rpm, e, rank, schedule)."""
        n = A.shape[0]
        assert A.dim() == 2 and A.shape[1] == n and A.is_cuda
        if A.dtype == torch.int32:
            dt = PLDL_U32
        elif A.dtype == torch.float64:
            dt = PLDL_F64
        else:
            raise TypeError("A must be int32 (uint32 residues) or float64")
        e = torch.zeros(max(n, 1), dtype=A.dtype, device=A.device)
        perm = torch.zeros(max(n, 1), dtype=torch.int32, device=A.device)
        rpm = torch.zeros(max(n, 1), dtype=torch.int32, device=A.device)
        rank = _i64(0)
        o = pldl_opts(int(path), int(threshold), int(bool(standard_form)), int(bool(check_range)))
        sc = pldl_schedule()
        rc = _lib.pldl_factor(self._h, int(p), n, _ptr(A), _ld(A) if n else 1, dt, _ptr(e), _ptr(perm), _ptr(rpm),
                              ctypes.byref(rank), ctypes.byref(o), ctypes.byref(sc), _stream())
        self._check(rc)
        return dict(perm=perm[:n], rpm=rpm[:n], e=e[:n], rank=int(rank.value), schedule=sc.as_dict())

    def solve(self, p: int, F: torch.Tensor, e: torch.Tensor, perm: torch.Tensor, rank: int, B: torch.Tensor):
        """pldl_solve on pldl_factor's outputs: B (n x nrhs float64) overwritten by X.
        Returns the per-column consistency flags (int32 tensor)."""
        n = F.shape[0]
        dt = PLDL_U32 if F.dtype == torch.int32 else PLDL_F64
        assert B.dtype == torch.float64 and B.dim() == 2 and B.shape[0] == n
        cons = torch.zeros(max(B.shape[1], 1), dtype=torch.int32, device=B.device)
        self._check(_lib.pldl_solve(self._h, int(p), n, _ptr(F), _ld(F) if n else 1, dt, _ptr(e), _ptr(perm),
                                    int(rank), _ptr(B), _ld(B), B.shape[1], _ptr(cons), _stream()))
        return cons[:B.shape[1]]

    def invariants(self, p: int, F: torch.Tensor, e: torch.Tensor, rank: int) -> dict:
        """pldl_invariants: rank, det, discriminant, its quadratic character, alternating flag."""
        n = F.shape[0]
        dt = PLDL_U32 if F.dtype == torch.int32 else PLDL_F64
        out = (_i64 * 5)()
        self._check(_lib.pldl_invariants(self._h, int(p), n, _ptr(F), _ld(F) if n else 1, dt, _ptr(e), int(rank),
                                         out, _stream()))
        return dict(rank=out[0], det=out[1], disc=out[2], character=out[3], alternating=out[4])

    def char2_to_standard(self, A: torch.Tensor, e: torch.Tensor, perm: torch.Tensor):
        """pldl_char2_to_standard on pldl_factor's outputs (p = 2), in place."""
        n = A.shape[0]
        dt = PLDL_U32 if A.dtype == torch.int32 else PLDL_F64
        self._check(_lib.pldl_char2_to_standard(self._h, n, _ptr(A), _ld(A) if n else 1, dt, _ptr(e), _ptr(perm),
                                                _stream()))

    def autotune(self, p: int, n_list, table_path: str = None):
        """pldl_autotune: base-case thresholds for the orders in n_list (or, with an empty
        list, read the table at table_path)."""
        arr = (_i64 * max(len(n_list), 1))(*[int(x) for x in n_list])
        self._check(_lib.pldl_autotune(self._h, int(p), arr, len(n_list),
                                       table_path.encode() if table_path else None, _stream()))

    def batched_args(self, mats):
        """Device argument arrays of pldl_factor_batched for a list of square tensors (int32
        holding uint32 residues, or float64), all of one dtype.  Returns a dict that keeps
        every array alive; pass it to factor_batched (also inside a graph capture)."""
        dev = mats[0].device
        dt = mats[0].dtype
        assert all(m.dtype == dt and m.device == dev and m.dim() == 2 and m.shape[0] == m.shape[1] for m in mats)
        ns = [m.shape[0] for m in mats]
        e = [torch.zeros(max(k, 1), dtype=dt, device=dev) for k in ns]
        perm = [torch.zeros(max(k, 1), dtype=torch.int32, device=dev) for k in ns]
        rpm = [torch.zeros(max(k, 1), dtype=torch.int32, device=dev) for k in ns]
        ptrs = lambda ts: torch.tensor([t.data_ptr() for t in ts], dtype=torch.int64, device=dev)
        return dict(mats=mats, dtype=PLDL_U32 if dt == torch.int32 else PLDL_F64,
                    n=torch.tensor(ns, dtype=torch.int64, device=dev),
                    lda=torch.tensor([max(_ld(m), 1) for m in mats], dtype=torch.int64, device=dev),
                    A=ptrs(mats), e=e, e_p=ptrs(e), perm=perm, perm_p=ptrs(perm), rpm=rpm, rpm_p=ptrs(rpm),
                    rank=torch.zeros(len(mats), dtype=torch.int64, device=dev),
                    status=torch.zeros(len(mats), dtype=torch.int32, device=dev))

    def factor_batched(self, p: int, args: dict, check_range: bool = True):
        """pldl_factor_batched on the arrays of batched_args (asynchronous)."""
        o = pldl_opts(PLDL_PATH_AUTO, 0, 0, int(bool(check_range)))
        rc = _lib.pldl_factor_batched(self._h, int(p), len(args["mats"]), _ptr(args["n"]), _ptr(args["A"]),
                                      _ptr(args["lda"]), args["dtype"], _ptr(args["e_p"]), _ptr(args["perm_p"]),
                                      _ptr(args["rpm_p"]), _ptr(args["rank"]), _ptr(args["status"]),
                                      ctypes.byref(o), _stream())
        self._check(rc)
        return args

    def factor_raw(self, p, n, A_ptr, lda, dtype, e_ptr, perm_ptr, rpm_ptr, opts=None, rank_out=True,
                   schedule=None):
        """pldl_factor with raw device pointers and no checks on this side, returning the
        status code instead of raising (the argument-error tests use it)."""
        rank = _i64(0)
        rc = _lib.pldl_factor(self._h, p, n, A_ptr, lda, dtype, e_ptr, perm_ptr, rpm_ptr,
                              ctypes.byref(rank) if rank_out else None,
                              ctypes.byref(opts) if opts is not None else None,
                              ctypes.byref(schedule) if schedule is not None else None, _stream())
        return rc, int(rank.value)

    def profile(self, mode: int) -> dict:
        """pldl_profile: 1 = reset and start (all classes), 3 = reset and start (GEMM class only),
        0 = stop, 2 = read.  Returns per-class totals."""
        st = pldl_stats()
        self._check(_lib.pldl_profile(self._h, int(mode), ctypes.byref(st)))
        return {name: dict(launches=st.cls[i].launches, flops=st.cls[i].flops, bytes=st.cls[i].bytes,
                           ops8=st.cls[i].ops8, ms=st.cls[i].ms) for i, name in enumerate(CLASS_NAMES)}

    # ------------------------------------------------------------------ building blocks
    def gemm(self, p, C, A, B, transA=False, transB=False, lower_only=False):
        m, n = C.shape
        k = A.shape[0] if transA else A.shape[1]
        rc = _lib.pldl_gemm(self._h, p, m, n, k, _ptr(A), _ld(A), int(transA), _ptr(B), _ld(B), int(transB),
                            _ptr(C), _ld(C), int(lower_only), _stream())
        self._check(rc)
        return C

    def trsm(self, p, T, B, lower: bool):
        m, n = B.shape
        rc = _lib.pldl_trsm(self._h, p, int(lower), m, n, _ptr(T), _ld(T), _ptr(B), _ld(B), _stream())
        self._check(rc)
        return B

    def syrdk(self, p, C, A, dd, de, B=None):
        n, k = A.shape
        rc = _lib.pldl_syrdk(self._h, p, n, k, _ptr(A), _ld(A), _ptr(B), _ld(B) if B is not None else 1,
                             _ptr(dd), _ptr(de), _ptr(C), _ld(C), _stream())
        self._check(rc)
        return C

    def syrdk_noalloc(self, p, C, A, dd, de, B=None):
        """pldl_syrdk_noalloc: the same product with no device allocation (asynchronous)."""
        n, k = A.shape
        rc = _lib.pldl_syrdk_noalloc(self._h, p, n, k, _ptr(A), _ld(A), _ptr(B), _ld(B) if B is not None else 1,
                                     _ptr(dd), _ptr(de), _ptr(C), _ld(C), _stream())
        self._check(rc)
        return C

    def trss(self, p, U, C):
        n = U.shape[0]
        X = torch.zeros_like(C)
        rc = _lib.pldl_trss(self._h, p, n, _ptr(U), _ld(U), _ptr(C), _ld(C), _ptr(X), _ld(X), _stream())
        self._check(rc)
        return X

    def plduq(self, p, Y):
        m, n = Y.shape
        rows = torch.zeros(max(m, 1), dtype=torch.int32, device=Y.device)
        cols = torch.zeros(max(n, 1), dtype=torch.int32, device=Y.device)
        rank = _i64(0)
        rc = _lib.pldl_plduq(self._h, p, m, n, _ptr(Y), _ld(Y), _ptr(rows), _ptr(cols), ctypes.byref(rank),
                             _stream())
        self._check(rc)
        return dict(rows=rows[:m], cols=cols[:n], LU=Y, rank=int(rank.value))


def lib():
    return _lib
