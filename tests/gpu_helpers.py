"""Shared helpers of the GPU parity tests: run the HIP path through the C-ABI
binding, pull results to the host, and compare them with the oracle."""
import numpy as np
import torch

import oracle.oracle as orc


def to_dev(A_u32: np.ndarray, dtype=torch.int32):
    if dtype == torch.int32:
        return torch.from_numpy(np.ascontiguousarray(A_u32).astype(np.int32)).cuda()
    return torch.from_numpy(np.ascontiguousarray(A_u32).astype(np.float64)).cuda()


def gpu_factor(ctx, A: np.ndarray, p: int, threshold: int = 0, dtype=torch.int32, standard_form=False):
    n = A.shape[0]
    print(f"[gpu_factor] n={n} p={p} t={threshold} dtype={dtype} std={standard_form}", flush=True)
    Ad = to_dev(A, dtype)
    out = ctx.factor(Ad, p, threshold=threshold, standard_form=standard_form)
    torch.cuda.synchronize()
    Ah = Ad.cpu().numpy()
    Ah = Ah.astype(np.int64).astype(np.uint32) if dtype == torch.int32 else Ah.astype(np.uint32)
    L = np.tril(Ah, -1).astype(np.uint32)
    L[np.arange(n), np.arange(n)] = 1
    dd = np.diag(Ah).astype(np.uint32).copy()
    e = out["e"].cpu().numpy()
    de = (e.astype(np.int64) if dtype == torch.int32 else e).astype(np.uint32)
    return dict(perm=out["perm"].cpu().numpy().astype(np.int32), rpm=out["rpm"].cpu().numpy().astype(np.int32),
                L=L, dd=dd, de=de, rank=out["rank"])


def check_against_oracle(A, p, res, exact_perm=False, ref=None):
    """r and R bit-exact against the canonical search; (L, D) bit-exact against
    the oracle's replay of the GPU's own pivot order (unique given P)."""
    ref = ref if ref is not None else orc.search(A, p)
    assert res["rank"] == ref["rank"], (res["rank"], ref["rank"])
    assert (res["rpm"] == ref["rpm"]).all(), "rank profile matrix differs"
    r = res["rank"]
    assert list(res["perm"][r:]) == sorted(res["perm"][r:]), "non-pivots not in increasing order"
    rc, rp = orc.replay(A, p, res["perm"], res["rpm"], r)
    assert rc == 0, f"oracle replay rejected the GPU pivot order: {rc}"
    assert (rp["L"] == res["L"]).all(), f"L differs at {np.argwhere(rp['L'] != res['L'])[:5]}"
    assert (rp["dd"] == res["dd"]).all(), "diag(D) differs"
    assert (rp["de"] == res["de"]).all(), "offdiag(D) differs"
    if exact_perm:
        assert (res["perm"] == ref["perm"]).all()
    return ref


def freivalds(A, p, res, trials=3, seed=0):
    """A v == P L D L^T P^T v (mod p) for random v: a property check at any size."""
    n = A.shape[0]
    g = np.random.Generator(np.random.PCG64(seed))
    perm = res["perm"].astype(np.int64)
    L = res["L"].astype(np.int64)
    dd, de = res["dd"].astype(np.int64), res["de"].astype(np.int64)
    A64 = A.astype(np.int64)
    for _ in range(trials):
        v = g.integers(0, p, size=n, dtype=np.int64)
        lhs = (A64 @ v) % p
        w = v[perm]                         # P^T v
        u = (L.T @ w) % p                   # L^T
        t = (dd * u) % p                    # D (tridiagonal)
        t = (t + np.concatenate([[0], de[:-1] * u[:-1]]) + np.concatenate([de[:-1] * u[1:], [0]])) % p
        y = (L @ t) % p                     # L
        rhs = np.zeros(n, dtype=np.int64)
        rhs[perm] = y                       # P
        assert (lhs == rhs).all(), "Freivalds reconstruction check failed"


def structure(res, p):
    """D consistent with rpm and rank (Section 2 block shapes)."""
    perm, rpm, r, dd, de, L = res["perm"], res["rpm"], res["rank"], res["dd"], res["de"], res["L"]
    n = len(perm)
    assert sorted(perm.tolist()) == list(range(n))
    q = 0
    while q < r:
        i = perm[q]
        if rpm[i] == i:
            assert dd[q] != 0 and de[q] == 0
            q += 1
        else:
            assert rpm[i] == perm[q + 1] and rpm[perm[q + 1]] == i
            assert de[q] != 0 and dd[q] == 0
            if p == 2:
                assert L[q + 1, q] == 0
            else:
                assert dd[q + 1] == 0
            q += 2
    assert (dd[r:] == 0).all() and (de[r:] == 0).all()
    assert (rpm[perm[r:]] == -1).all()


def freivalds_f2(A, res, nvec=64, seed=0):
    """Over F_2: A V == P L D L^T P^T V for nvec random 0/1 columns at once (the
    matrix products run in float64, exact: every sum is below n < 2^53).  A wrong
    factorization passes with probability at most 2^-nvec."""
    n = A.shape[0]
    g = np.random.Generator(np.random.PCG64(seed))
    V = g.integers(0, 2, size=(n, nvec)).astype(np.float64)
    perm = res["perm"].astype(np.int64)
    Lf = res["L"].astype(np.float64)
    dd, de = res["dd"].astype(np.float64), res["de"].astype(np.float64)
    lhs = np.mod(A.astype(np.float64) @ V, 2.0)
    U = np.mod(Lf.T @ V[perm], 2.0)                     # L^T P^T V
    T = dd[:, None] * U
    T[1:] += de[:-1, None] * U[:-1]
    T[:-1] += de[:-1, None] * U[1:]
    Y = np.mod(Lf @ np.mod(T, 2.0), 2.0)
    rhs = np.zeros_like(Y)
    rhs[perm] = Y
    assert (lhs == rhs).all(), "Freivalds reconstruction check over F_2 failed"
