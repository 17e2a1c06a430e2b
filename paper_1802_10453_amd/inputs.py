"""Seeded synthetic inputs shaped like the paper's experiments (Section 6).

The paper factors random symmetric matrices over Z/8388593Z of three classes:
generic rank profile, uniformly random rank profile matrix (RPM) of full rank,
and random RPM of rank n/2.  Its generator is not given; the one used here is

    A = L * R * L^T  (mod p)

with L unit lower triangular (strictly lower entries uniform in [0, p)) and R a
symmetric rook placement: f fixed points and c transpositions on a uniformly
random index set, each carrying a uniform nonzero scale.  Because L is unit
lower triangular, every leading submatrix of A has the rank of the same leading
submatrix of R, so RPM(A) = supp(R) and rank(A) = f + 2c (Theorem 1).

This module builds inputs only; it holds none of the factorization's
arithmetic.  Both the oracle side and the GPU side of every test draw their
inputs from here, and the benchmark does too.
"""
from __future__ import annotations

import hashlib

import numpy as np

C0 = dict(name="n64_p65521_r40", n=64, p=65521, f=20, c=10)
C1 = dict(name="n4096_p65521_fullrank_uniform", n=4096, p=65521)
C2 = dict(name="n16384_p8388593_r12288_randomrpm", n=16384, p=8388593, f=6144, c=3072)
C3 = dict(name="batch4096_p32749_n32to512", count=4096, p=32749, nmin=32, nmax=512)
C4 = dict(name="n8192_p2_r6000_zerodiag_half", n=8192, p=2, f=3000, c=1500)

SEED_BASE = 20180228


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def symmetric_uniform(n: int, p: int, seed: int) -> np.ndarray:
    """Full symmetric n x n uint32 matrix, lower triangle and diagonal uniform in [0, p)."""
    g = rng(seed)
    A = g.integers(0, p, size=(n, n), dtype=np.uint32)
    A = np.tril(A)
    A = A + np.tril(A, -1).T
    return np.ascontiguousarray(A, dtype=np.uint32)


def rook_placement(n: int, f: int, c: int, p: int, g: np.random.Generator, fixed_pool=None):
    """Symmetric rook placement: f fixed points, c transpositions, random scales.

    Returns ``rpm`` (int32, rpm[i] = j or -1) and ``scale`` (uint32, scale[i] =
    R[i][rpm[i]]).  ``fixed_pool`` optionally restricts where fixed points go.
    """
    rpm = np.full(n, -1, dtype=np.int32)
    scale = np.zeros(n, dtype=np.uint32)
    if fixed_pool is None:
        idx = g.permutation(n)[: f + 2 * c]
        fixed, paired = idx[:f], idx[f:]
    else:
        fixed_pool = np.asarray(fixed_pool)
        fixed = g.permutation(fixed_pool)[:f]
        rest = np.setdiff1d(np.arange(n), fixed)
        paired = g.permutation(rest)[: 2 * c]
    assert len(fixed) == f and len(paired) == 2 * c
    s = g.integers(1, p, size=f + c, dtype=np.uint32) if p > 2 else np.ones(f + c, dtype=np.uint32)
    rpm[fixed] = fixed
    scale[fixed] = s[:f]
    a, b = paired[0::2], paired[1::2]
    rpm[a] = b
    rpm[b] = a
    scale[a] = s[f:]
    scale[b] = s[f:]
    return rpm, scale


def unit_lower(n: int, p: int, g: np.random.Generator) -> np.ndarray:
    L = g.integers(0, p, size=(n, n), dtype=np.uint32)
    L = np.tril(L, -1)
    L[np.arange(n), np.arange(n)] = 1
    return L


def _lrlt(L: np.ndarray, rpm: np.ndarray, scale: np.ndarray, p: int, device=None, check: int = 64,
          seed: int = 0):
    """A = L R L^T mod p, exact.

    A = sum over the support (i, j) of R of scale * L[:, i] L[:, j]^T, i.e. X Y^T
    with X = L[:, I] * s and Y = L[:, J].  The product runs in float64 with Y cut
    into 12-bit pieces so that every partial sum is an integer below 2^53 (exact
    in any summation order); ``device`` selects numpy (None/"cpu") or a torch
    device.  ``check`` random entries are recomputed with Python integers.
    """
    n = L.shape[0]
    I = np.nonzero(rpm >= 0)[0]
    J = rpm[I]
    if len(I) == 0:
        return np.zeros((n, n), dtype=np.uint32)
    X = (L[:, I].astype(np.uint64) * scale[I].astype(np.uint64)) % p
    Y = L[:, J].astype(np.uint64)
    split = p > (1 << 17)
    if device is None or str(device) == "cpu":
        Xf = X.astype(np.float64)
        if split:
            lo = (Y & 4095).astype(np.float64)
            hi = (Y >> 12).astype(np.float64)
            A = (np.fmod(Xf @ lo.T, p) + 4096.0 * np.fmod(Xf @ hi.T, p))
        else:
            A = Xf @ Y.astype(np.float64).T
        A = np.fmod(A, p).astype(np.uint32)
    else:
        import torch
        Xf = torch.from_numpy(X.astype(np.float64)).to(device)
        if split:
            lo = torch.from_numpy((Y & 4095).astype(np.float64)).to(device)
            hi = torch.from_numpy((Y >> 12).astype(np.float64)).to(device)
            A = torch.fmod(Xf @ lo.T, p) + 4096.0 * torch.fmod(Xf @ hi.T, p)
            del lo, hi
        else:
            Yf = torch.from_numpy(Y.astype(np.float64)).to(device)
            A = Xf @ Yf.T
            del Yf
        A = torch.fmod(A, p).to(torch.int64).cpu().numpy().astype(np.uint32)
        del Xf
    if check:
        g = rng(seed ^ 0x5A5A)
        for _ in range(check):
            i, j = int(g.integers(0, n)), int(g.integers(0, n))
            v = sum(int(X[i, t]) * int(Y[j, t]) for t in range(len(I))) % p
            if v != int(A[i, j]):
                raise RuntimeError(f"input generator product not exact at ({i},{j})")
    return np.ascontiguousarray(A)


def rank_profile_matrix_input(n: int, p: int, f: int, c: int, seed: int, device=None, check: int = 64):
    """(A, rpm) with A = L R L^T, R a seeded symmetric rook placement of rank f + 2c."""
    g = rng(seed)
    rpm, scale = rook_placement(n, f, c, p, g)
    L = unit_lower(n, p, g)
    A = _lrlt(L, rpm, scale, p, device=device, check=check, seed=seed)
    return A, rpm


def char2_input(n: int, f: int, c: int, seed: int, device=None, check: int = 64):
    """Characteristic-2 input with a zero diagonal on a seeded half H of the rows.

    Fixed points of R are placed outside H; transpositions anywhere else.  Over
    F_2, A[i][i] = number of fixed points k < i with L[i][k] = 1 (mod 2), so for
    each i in H with an odd count the entry L[i][k*] at the largest fixed k* < i
    is flipped.  L stays unit lower, so RPM(A) = supp(R) still holds, and the
    rows of H need off-diagonal (often relaxed) 2x2 pivots.
    Returns (A, rpm, H).
    """
    g = rng(seed)
    H = np.sort(g.permutation(n)[: n // 2])
    inH = np.zeros(n, dtype=bool)
    inH[H] = True
    rpm, scale = rook_placement(n, f, c, 2, g, fixed_pool=np.nonzero(~inH)[0])
    L = unit_lower(n, 2, g)
    fixed = np.nonzero(rpm == np.arange(n))[0]
    isfixed = np.zeros(n, dtype=bool)
    isfixed[fixed] = True
    Lf = L[:, isfixed]                       # columns of fixed points, increasing
    cnt = np.zeros(n, dtype=np.int64)
    below = np.tril(np.ones((n, n), dtype=bool), -1)[:, isfixed]
    cnt = (Lf.astype(np.int64) * below).sum(axis=1) % 2
    for i in H:
        if cnt[i]:
            ks = fixed[fixed < i]
            L[i, ks[-1]] ^= 1
    A = _lrlt(L, rpm, scale, 2, device=device, check=check, seed=seed)
    assert not A[H, H].any()
    return A, rpm, H


def batch_params(count: int, nmin: int, nmax: int, seed: int):
    """Per-matrix (n, r, f, c, seed) of the batched workload: n ~ U{nmin..nmax},
    r ~ U{ceil(n/4)..n}, c = floor(r/4) transpositions, f = r - 2c fixed points."""
    g = rng(seed)
    out = []
    for b in range(count):
        n = int(g.integers(nmin, nmax + 1))
        r = int(g.integers((n + 3) // 4, n + 1))
        c = r // 4
        f = r - 2 * c
        h = hashlib.blake2b(f"{seed}:{b}".encode(), digest_size=8).digest()
        out.append((n, r, f, c, int.from_bytes(h, "little") & 0x7FFFFFFF))
    return out


def _batch_one(args):
    n, r, f, c, s, p = args
    return rank_profile_matrix_input(n, p, f, c, s, check=0)


def batch_input(cfg: dict, index_seed: int = 0, workers: int = 0, with_rpm: bool = False, progress=None):
    """The matrices of a batched workload (list of uint32 arrays) and their per-matrix
    (n, r, f, c, seed) (and, with_rpm, their rank profile matrices); ``workers``
    processes build them (0: serial, calling progress(done) every 256 matrices)."""
    params = batch_params(cfg["count"], cfg["nmin"], cfg["nmax"], SEED_BASE + index_seed)
    jobs = [(n, r, f, c, s, cfg["p"]) for (n, r, f, c, s) in params]
    if workers and workers > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            out = pool.map(_batch_one, jobs, chunksize=16)
    else:
        out = []
        for k, j in enumerate(jobs):
            out.append(_batch_one(j))
            if progress and (k + 1) % 256 == 0:
                progress(k + 1)
    mats = [A for A, _ in out]
    if with_rpm:
        return mats, params, [rpm for _, rpm in out]
    return mats, params


def config_input(cfg: dict, index_seed: int = 0, device=None, check: int = 64):
    """Input of one of the named single-matrix workloads; returns (A, rpm or None)."""
    seed = SEED_BASE + index_seed
    if cfg is C1:
        return symmetric_uniform(cfg["n"], cfg["p"], seed), None
    if cfg is C4:
        A, rpm, _ = char2_input(cfg["n"], cfg["f"], cfg["c"], seed, device=device, check=check)
        return A, rpm
    return rank_profile_matrix_input(cfg["n"], cfg["p"], cfg["f"], cfg["c"], seed, device=device, check=check)
