"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle, bit-exact.

Building blocks first (GEMM/TRMM, TRSM, SYRDK/SYRD2K, TRSS, PLDUQ), then the
base case alone (canonical order: P too must match), then the full recursive
cascade at several thresholds (r, R exact; (L, D) exact through the oracle's
replay of the GPU's own pivot order).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle.oracle as orc  # noqa: E402
from paper_1802_10453_amd import inputs  # noqa: E402

from gpu_helpers import check_against_oracle, freivalds, gpu_factor, structure  # noqa: E402

PRIMES = [2, 3, 65521, 8388593, 16777213]   # the last: above 2^23, delayed-reduction chunk 128


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10453_amd import pldl
    c = pldl.Context(0)
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x).astype(np.float64)).cuda()


def host(t):
    return t.cpu().numpy().astype(np.int64).astype(np.uint32)


def rnd(g, p, *shape):
    return g.integers(0, p, size=shape).astype(np.uint32)


# ---------------------------------------------------------------- GEMM / TRMM
@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_gemm_parity(ctx, p, ta, tb):
    g = inputs.rng(p * 7 + ta * 2 + tb)
    for (m, n, k) in [(1, 1, 1), (5, 7, 3), (130, 129, 17), (257, 64, 300), (64, 200, 1100)]:
        print(f"[gemm] p={p} ta={ta} tb={tb} m={m} n={n} k={k}", flush=True)
        A = rnd(g, p, m, k)
        B = rnd(g, p, k, n)
        C = rnd(g, p, m, n)
        Ad = dev(A.T.copy() if ta else A)
        Bd = dev(B.T.copy() if tb else B)
        Cd = dev(C)
        ctx.gemm(p, Cd, Ad, Bd, transA=bool(ta), transB=bool(tb))
        assert (host(Cd) == orc.gemm(p, C, A, B)).all()


@pytest.mark.parametrize("p", [65521, 8388593, 16777213])
def test_gemm_adversarial_bounds(ctx, p):
    """All operands at the extreme centered value (p-1)/2 (and p-1), K at and past the
    delayed-reduction chunk: every partial sum sits at the 2^53 exactness limit."""
    for v in ((p - 1) // 2, (p + 1) // 2, p - 1):
        for k in (127, 128, 129, 495, 496, 497, 1000, 2049):
            m, n = 33, 65
            A = np.full((m, k), v, dtype=np.uint32)
            B = np.full((k, n), v, dtype=np.uint32)
            C = np.full((m, n), p - 1, dtype=np.uint32)
            Cd = dev(C)
            ctx.gemm(p, Cd, dev(A), dev(B))
            ref = (C.astype(object) - (A.astype(object) @ B.astype(object))) % p
            assert (host(Cd) == ref.astype(np.uint32)).all(), (v, k)


@pytest.mark.parametrize("p", [2, 65521, 8388593, 16777213])
def test_gemm_lower_only(ctx, p):
    g = inputs.rng(p + 3)
    for (n, k) in [(1, 4), (127, 33), (300, 260)]:
        A, B, C = rnd(g, p, n, k), rnd(g, p, k, n), rnd(g, p, n, n)
        Cd = dev(C)
        ctx.gemm(p, Cd, dev(A), dev(B), lower_only=True)
        out = host(Cd)
        ref = orc.gemm(p, C, A, B)
        assert (np.tril(out) == np.tril(ref)).all()
        assert (np.triu(out, 1) == np.triu(C, 1)).all()


# ---------------------------------------------------------------- TRSM
@pytest.mark.parametrize("p", PRIMES)
def test_trsm_parity(ctx, p):
    g = inputs.rng(p + 11)
    for (m, n) in [(1, 1), (3, 5), (64, 70), (65, 33), (200, 130), (517, 300)]:
        print(f"[trsm] p={p} m={m} n={n}", flush=True)
        # left, unit lower T (m x m), B m x n
        T = rnd(g, p, m, m)
        B = rnd(g, p, m, n)
        Td = dev(T)
        Bd = dev(B)
        ctx.trsm(p, Td, Bd, lower=True)
        Tl = np.tril(T, -1) + np.eye(m, dtype=np.uint32)
        assert (host(Bd) == orc.trsm_left(p, Tl, B, lower=True)).all()
        # right, unit upper T (n x n): X = B T^{-1}  <=>  T^T X^T = B^T
        T2 = rnd(g, p, n, n)
        Bd = dev(B)
        ctx.trsm(p, dev(T2), Bd, lower=False)
        Tu = np.triu(T2, 1) + np.eye(n, dtype=np.uint32)
        ref = orc.trsm_left(p, Tu.T.copy(), B.T.copy(), lower=True).T
        assert (host(Bd) == ref).all()


@pytest.mark.parametrize("p", PRIMES)
def test_trsm_stripe_orders(ctx, p):
    """Orders 65..257 (one stripe launch each, the last one split once), stripe counts
    with a ragged last stripe, both sides."""
    g = inputs.rng(p + 12)
    for (r, k) in [(65, 1), (128, 31), (192, 33), (256, 1000), (257, 95)]:
        print(f"[trsm stripe] p={p} r={r} k={k}", flush=True)
        T = rnd(g, p, r, r)
        B = rnd(g, p, r, k)
        Bd = dev(B)
        ctx.trsm(p, dev(T), Bd, lower=True)
        Tl = np.tril(T, -1) + np.eye(r, dtype=np.uint32)
        assert (host(Bd) == orc.trsm_left(p, Tl, B, lower=True)).all()
        Bt = B.T.copy()
        Bd = dev(Bt)
        ctx.trsm(p, dev(T), Bd, lower=False)
        Tu = np.triu(T, 1) + np.eye(r, dtype=np.uint32)
        ref = orc.trsm_left(p, Tu.T.copy(), Bt.T.copy(), lower=True).T
        assert (host(Bd) == ref).all()


# ---------------------------------------------------------------- SYRDK / SYRD2K
@pytest.mark.parametrize("p", PRIMES)
def test_syrdk_parity(ctx, p):
    g = inputs.rng(p + 13)
    for (n, k) in [(1, 1), (9, 6), (129, 70), (300, 257)]:
        A, B, C = rnd(g, p, n, k), rnd(g, p, n, k), rnd(g, p, n, n)
        dd = rnd(g, p, k)
        de = np.zeros(k, dtype=np.uint32)
        for q in range(0, k - 1, 5):            # some 2x2 blocks
            de[q] = 1 + q % (p - 1) if p > 2 else 1
            dd[q] = 0
            if p != 2:
                dd[q + 1] = 0
        Cd = dev(C)
        ctx.syrdk(p, Cd, dev(A), dev(dd), dev(de))
        ref = orc.syrdk(p, C, A, dd, de)
        assert (np.tril(host(Cd)) == np.tril(ref)).all()
        Cd = dev(C)
        ctx.syrdk(p, Cd, dev(A), dev(dd), dev(de), B=dev(B))
        ref2 = orc.syrd2k(p, C, A, B, dd, de)
        assert (np.tril(host(Cd)) == np.tril(ref2)).all()


# ---------------------------------------------------------------- TRSS (Algorithm 1)
@pytest.mark.parametrize("p", [3, 65521, 8388593, 2, 16777213])
def test_trss_parity(ctx, p):
    g = inputs.rng(p + 17)
    for n in (1, 2, 17, 64, 65, 130, 300):
        print(f"[trss] p={p} n={n}", flush=True)
        U = np.triu(rnd(g, p, n, n), 1) + np.eye(n, dtype=np.uint32)
        C = inputs.symmetric_uniform(n, p, int(g.integers(1 << 30)))
        if p == 2:
            C[np.arange(n), np.arange(n)] = 0
        X = ctx.trss(p, dev(U), dev(np.tril(C)))
        rc, Xr = orc.trss(p, U, C)
        assert rc == 0
        assert (host(X) == Xr).all()


def test_trss_char2_rejects_nonzero_diagonal(ctx):
    n = 5
    U = np.eye(n, dtype=np.uint32)
    C = np.zeros((n, n), dtype=np.uint32)
    C[2, 2] = 1
    from paper_1802_10453_amd.pldl import PldlError
    with pytest.raises(PldlError):
        ctx.trss(2, dev(U), dev(C))


# ---------------------------------------------------------------- PLDUQ
@pytest.mark.parametrize("p", [2, 65521, 8388593, 16777213])
def test_plduq_parity(ctx, p):
    g = inputs.rng(p + 19)
    for (m, n, k) in [(1, 1, 1), (5, 9, 3), (40, 30, 25), (33, 300, 20), (70, 600, 64), (100, 90, 100), (64, 64, 0)]:
        print(f"[plduq] p={p} m={m} n={n} k={k}", flush=True)
        X = g.integers(0, p, size=(m, k))
        Z = g.integers(0, p, size=(k, n))
        Y = ((X.astype(object) @ Z.astype(object)) % p).astype(np.uint32) if k else np.zeros((m, n), np.uint32)
        if m > 3:
            Y[1] = 0
            Y[:, min(2, n - 1)] = 0
        res = ctx.plduq(p, dev(Y))
        ref = orc.plduq(p, Y)
        r = res["rank"]
        assert r == ref["rank"]
        rows, cols = res["rows"].cpu().numpy(), res["cols"].cpu().numpy()
        # the pivot set is unique (the rank profile matrix of Y); the order may differ
        assert sorted(zip(rows[:r].tolist(), cols[:r].tolist())) == \
            sorted(zip(ref["rows"][:r].tolist(), ref["cols"][:r].tolist()))
        assert list(rows[r:]) == sorted(rows[r:]) and list(cols[r:]) == sorted(cols[r:])
        assert sorted(rows.tolist()) == list(range(m)) and sorted(cols.tolist()) == list(range(n))
        LU = host(res["LU"])
        L = np.tril(LU[:, :r], -1).astype(object)
        L[np.arange(r), np.arange(r)] = 1
        U = np.triu(LU[:r, :], 1).astype(object)
        U[np.arange(r), np.arange(r)] = 1
        D = np.diag([int(x) for x in np.diag(LU)[:r]]) if r else np.zeros((0, 0), dtype=object)
        assert all(int(x) for x in np.diag(LU)[:r])
        assert (LU[r:, r:] == 0).all()
        rec = ((L @ D) % p @ U) % p if r else np.zeros((m, n), dtype=object)
        assert (rec == Y[np.ix_(rows, cols)].astype(object)).all()


def _staircase(g, p, m, step, n):
    """Row i is zero before column step*i (a staircase): every column chunk of a
    slab holds the first nonzero of one more row, so a 64-row slab takes about
    one leaf per row, and the leaves' queued batches run out several times."""
    Y = g.integers(0, p, size=(m, n)).astype(np.uint32)
    for i in range(m):
        Y[i, : min(n, step * i)] = 0
    return Y


@pytest.mark.parametrize("p", [2, 8388593])
def test_plduq_many_leaves_per_slab(ctx, p):
    g = inputs.rng(p + 29)
    for (m, step, n) in [(64, 256, 64 * 256 + 5), (130, 300, 130 * 300), (70, 40, 3000)]:
        print(f"[plduq-staircase] p={p} m={m} step={step} n={n}", flush=True)
        Y = _staircase(g, p, m, step, n)
        if m > 3:
            Y[2] = 0   # a zero row among them
        res = ctx.plduq(p, dev(Y))
        ref = orc.plduq(p, Y)
        r = res["rank"]
        assert r == ref["rank"]
        rows, cols = res["rows"].cpu().numpy(), res["cols"].cpu().numpy()
        assert sorted(zip(rows[:r].tolist(), cols[:r].tolist())) == \
            sorted(zip(ref["rows"][:r].tolist(), ref["cols"][:r].tolist()))
        assert sorted(rows.tolist()) == list(range(m)) and sorted(cols.tolist()) == list(range(n))
        # L D U = Y[rows, cols] mod p, in int64 (r p^2 < 2^63 for these sizes)
        LU = host(res["LU"]).astype(np.int64)
        L = np.tril(LU[:, :r], -1)
        L[np.arange(r), np.arange(r)] = 1
        U = np.triu(LU[:r, :], 1)
        U[np.arange(r), np.arange(r)] = 1
        d = np.diag(LU)[:r]
        assert (d != 0).all() and (LU[r:, r:] == 0).all()
        rec = ((L * d[None, :]) % p) @ U % p
        assert (rec == Y[np.ix_(rows, cols)].astype(np.int64)).all()


# ---------------------------------------------------------------- base case alone (canonical order)
@pytest.mark.parametrize("p", PRIMES)
def test_base_case_canonical(ctx, p):
    g = inputs.rng(p + 23)
    for n in (1, 2, 3, 7, 31, 64, 100, 128):
        for kind in range(3):
            if kind == 0:
                r = int(g.integers(0, n + 1))
                c = int(g.integers(0, r // 2 + 1))
                A, _ = inputs.rank_profile_matrix_input(n, p, r - 2 * c, c, int(g.integers(1 << 30)), check=0)
            elif kind == 1:
                A = inputs.symmetric_uniform(n, p, int(g.integers(1 << 30)))
            else:
                if p == 2 and n >= 4:
                    A, _, _ = inputs.char2_input(n, n // 4, n // 8, int(g.integers(1 << 30)), check=0)
                else:
                    A = np.zeros((n, n), dtype=np.uint32)
            res = gpu_factor(ctx, A, p, threshold=128)
            check_against_oracle(A, p, res, exact_perm=True)


def test_c0_workload_base_case(ctx):
    A, rpm = inputs.config_input(inputs.C0)
    res = gpu_factor(ctx, A, inputs.C0["p"], threshold=128)
    ref = check_against_oracle(A, inputs.C0["p"], res, exact_perm=True)
    assert res["rank"] == 40 and (res["rpm"] == rpm).all()
    assert (ref["rpm"] == orc.rpm_bruteforce(A, inputs.C0["p"])).all()


# ---------------------------------------------------------------- full recursion
@pytest.mark.parametrize("t", [8, 16, 32, 64])
def test_c0_workload_recursive(ctx, t):
    A, rpm = inputs.config_input(inputs.C0)
    res = gpu_factor(ctx, A, inputs.C0["p"], threshold=t)
    check_against_oracle(A, inputs.C0["p"], res)
    assert (res["rpm"] == rpm).all()


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("t", [4, 16, 64])
def test_recursive_random(ctx, p, t):
    g = inputs.rng(p * 31 + t)
    for trial in range(6):
        n = int(g.integers(2, 200))
        kind = trial % 3
        if kind == 0:
            r = int(g.integers(0, n + 1))
            c = int(g.integers(0, r // 2 + 1))
            A, rpm = inputs.rank_profile_matrix_input(n, p, r - 2 * c, c, int(g.integers(1 << 30)), check=0)
        elif kind == 1:
            A, rpm = inputs.symmetric_uniform(n, p, int(g.integers(1 << 30))), None
        else:
            if p == 2 and n >= 8:
                A, rpm, _ = inputs.char2_input(n, n // 4, n // 8, int(g.integers(1 << 30)), check=0)
            else:
                r = n // 2
                A, rpm = inputs.rank_profile_matrix_input(n, p, r // 2, r // 4, int(g.integers(1 << 30)), check=0)
        res = gpu_factor(ctx, A, p, threshold=t)
        check_against_oracle(A, p, res)
        if rpm is not None:
            assert (res["rpm"] == rpm).all()


@pytest.mark.parametrize("p", [65521, 8388593, 2, 16777213])
def test_recursive_medium(ctx, p):
    """Several tiles of every kernel and a ragged tail (n not a tile multiple)."""
    n = 777
    r = 600 if p != 2 else 560
    c = r // 4
    if p == 2:
        A, rpm, _ = inputs.char2_input(n, 280, 140, 4242, check=0)
    else:
        A, rpm = inputs.rank_profile_matrix_input(n, p, r - 2 * c, c, 4242, check=0)
    res = gpu_factor(ctx, A, p, threshold=0)
    check_against_oracle(A, p, res)
    assert (res["rpm"] == rpm).all()


def test_float64_storage_and_determinism(ctx):
    p = 65521
    A = inputs.symmetric_uniform(300, p, 99)
    r1 = gpu_factor(ctx, A, p, threshold=32, dtype=torch.float64)
    r2 = gpu_factor(ctx, A, p, threshold=32, dtype=torch.int32)
    check_against_oracle(A, p, r1)
    for k in ("perm", "rpm", "L", "dd", "de"):
        assert (r1[k] == r2[k]).all()
    r3 = gpu_factor(ctx, A, p, threshold=32, dtype=torch.float64)
    for k in ("perm", "rpm", "L", "dd", "de"):
        assert (r1[k] == r3[k]).all()


def test_degenerate_inputs(ctx):
    p = 65521
    for n in (1, 2, 5, 130):
        Z = np.zeros((n, n), dtype=np.uint32)
        res = gpu_factor(ctx, Z, p, threshold=16)
        assert res["rank"] == 0 and (res["perm"] == np.arange(n)).all() and (res["rpm"] == -1).all()
    A = np.array([[5]], dtype=np.uint32)
    res = gpu_factor(ctx, A, p)
    assert res["rank"] == 1 and res["dd"][0] == 5
    # only the last row/column nonzero: a single 2x2 block (0, n-1) pattern at the end
    n = 70
    A = np.zeros((n, n), dtype=np.uint32)
    A[n - 1, 0] = A[0, n - 1] = 3
    res = gpu_factor(ctx, A, p, threshold=16)
    check_against_oracle(A, p, res)


def test_char2_standard_form(ctx):
    A, rpm, _ = inputs.char2_input(200, 60, 30, 77, check=0)
    res = gpu_factor(ctx, A, 2, threshold=32, standard_form=True)
    ref = orc.search(A, 2)
    assert res["rank"] == ref["rank"] and (res["rpm"] == rpm).all()
    # standard form: only antidiagonal 2x2 blocks remain, and it reconstructs A
    for q in range(199):
        if res["de"][q]:
            assert res["dd"][q] == 0 and res["dd"][q + 1] == 0
    assert (np.triu(res["L"], 1) == 0).all()
    rec = orc.reconstruct(2, res["perm"], res["L"], res["dd"], res["de"])
    assert (rec == A).all()


# ---------------------------------------------------------------- full-size properties
@pytest.mark.slow
def test_c1_workload_full_size(ctx):
    """The n = 4096 uniform workload as the bench runs it: r, R against the oracle's
    search and (L, D, e) against its replay of the GPU's P, bit-exact."""
    cfg = inputs.C1
    A, _ = inputs.config_input(cfg)
    res = gpu_factor(ctx, A, cfg["p"])
    assert res["rank"] == cfg["n"]
    structure(res, cfg["p"])
    print("[c1] oracle search and replay", flush=True)
    check_against_oracle(A, cfg["p"], res)
