"""GPU parity on the code paths that only the large workloads take, against the
CPU oracle, bit-exact: the 128 x 128 product tile (chosen for products of at
least 192 tiles), INT8-split products inside a whole factorization (products
of at least 2^27 flops), the INT32 accumulation bound of the INT8 split across
both segments of SYRD2K, and pldl_factor's argument, range and modulus errors
through the C-ABI."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle.oracle as orc  # noqa: E402
from paper_1802_10453_amd import inputs  # noqa: E402

from gpu_helpers import check_against_oracle, gpu_factor, structure  # noqa: E402


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


def profiled(ctx, fn):
    """Run fn with per-class recording on; return the class totals."""
    ctx.profile(1)
    try:
        fn()
        torch.cuda.synchronize()
        return ctx.profile(2)
    finally:
        ctx.profile(0)


# ---------------------------------------------------------------- 128 x 128 product tile
@pytest.mark.parametrize("p", [65521, 8388593])
@pytest.mark.parametrize("tb", [0, 1])
def test_gemm_big_tile_dense(ctx, p, tb):
    """m = n = 2048 (256 tiles of 128 x 128), k = 600: past the delayed-reduction
    chunk of p = 8388593 (496 products), with a ragged K tail."""
    g = inputs.rng(p + 17 * tb)
    m = n = 2048
    k = 600
    print(f"[big tile] dense p={p} tb={tb}", flush=True)
    A, B, C = rnd(g, p, m, k), rnd(g, p, k, n), rnd(g, p, m, n)
    Cd = dev(C)
    ctx.gemm(p, Cd, dev(A), dev(B.T.copy() if tb else B), transB=bool(tb))
    assert (host(Cd) == orc.gemm(p, C, A, B)).all()


@pytest.mark.parametrize("p", [8388593, 16777213])
def test_gemm_big_tile_adversarial_bounds(ctx, p):
    """Big tiles (2048 x 2048) with every operand at the extreme centered value and
    K around the delayed-reduction chunk (496 at p = 8388593, 128 at 16777213) and
    past it: the accumulators must be reduced before any partial sum passes 2^53."""
    m = n = 2048
    for v in ((p - 1) // 2, (p + 1) // 2):
        for k in (127, 129, 495, 497, 1000):
            print(f"[big tile bounds] p={p} v={v} k={k}", flush=True)
            A = np.full((m, k), v, dtype=np.uint32)
            B = np.full((k, n), v, dtype=np.uint32)
            C = np.full((m, n), p - 1, dtype=np.uint32)
            Cd = dev(C)
            ctx.gemm(p, Cd, dev(A), dev(B))
            want = (p - 1 - (k * v * v) % p) % p
            got = host(Cd)
            assert (got == want).all(), (v, k, int(got[0, 0]), want)


def test_gemm_big_tile_ragged_edges(ctx):
    """Big tiles with ragged M, N and K edges (2050 x 2000, k = 333)."""
    p = 8388593
    g = inputs.rng(99)
    m, n, k = 2050, 2000, 333
    print("[big tile] ragged", flush=True)
    A, B, C = rnd(g, p, m, k), rnd(g, p, k, n), rnd(g, p, m, n)
    Cd = dev(C)
    ctx.gemm(p, Cd, dev(A.T.copy()), dev(B), transA=True)
    assert (host(Cd) == orc.gemm(p, C, A, B)).all()


@pytest.mark.parametrize("p", [2, 8388593])
def test_gemm_big_tile_lower_only(ctx, p):
    """Lower-only output of order 2600 (231 lower tiles of 128 x 128), k = 530."""
    g = inputs.rng(p + 31)
    n, k = 2600, 530
    print(f"[big tile] lower p={p}", flush=True)
    A, B = rnd(g, p, n, k), rnd(g, p, k, n)
    C = rnd(g, p, n, n)
    Cd = dev(C)
    ctx.gemm(p, Cd, dev(A), dev(B), lower_only=True)
    got = host(Cd)
    ref = orc.gemm(p, C, A, B)
    low = np.tril(np.ones((n, n), dtype=bool))
    assert (got[low] == ref[low]).all()
    assert (got[~low] == C[~low]).all(), "upper triangle must stay untouched"


# ---------------------------------------------------------------- INT8 inside a factorization
@pytest.mark.parametrize("p,n,f,c", [(8388593, 2048, 750, 375), (65521, 2304, 1000, 400)])
def test_i8_factor_crosses_product_cut(ctx, p, n, f, c):
    """A whole factorization whose largest products reach the INT8 cut (2^27 flops):
    the schedule reports INT8 products, and r, R, (L, D) match the oracle."""
    from paper_1802_10453_amd import pldl
    A, _ = inputs.rank_profile_matrix_input(n, p, f, c, inputs.SEED_BASE + 303 + n, check=8)
    ctx.set_path(pldl.PLDL_PATH_I8)
    try:
        Ad = torch.from_numpy(A.astype(np.int32)).cuda()
        print(f"[i8 factor] n={n} p={p}", flush=True)
        out = ctx.factor(Ad, p)
        torch.cuda.synchronize()
    finally:
        ctx.set_path(pldl.PLDL_PATH_AUTO)
    sc = out["schedule"]
    assert sc["path_used"] == pldl.PLDL_PATH_I8
    assert sc["products_i8"] > 0, sc
    Ah = Ad.cpu().numpy().astype(np.int64).astype(np.uint32)
    L = np.tril(Ah, -1)
    L[np.arange(n), np.arange(n)] = 1
    res = dict(perm=out["perm"].cpu().numpy(), rpm=out["rpm"].cpu().numpy(), L=L, dd=np.diag(Ah).copy(),
               de=out["e"].cpu().numpy().astype(np.int64).astype(np.uint32), rank=out["rank"])
    assert res["rank"] == f + 2 * c
    check_against_oracle(A, p, res)


# ---------------------------------------------------------------- INT32 bound across SYRD2K segments
def test_i8_syrd2k_accumulation_bound(ctx):
    """Every residue = -32896 (balanced digits -128, -128, 0): shift class 1 gains
    2^15 per k.  SYRD2K with k = 32767 per segment (65534 in all) stays on the
    INT8 path and must be exact; k = 32768 per segment (65536, which would wrap
    INT32) must leave the INT8 path and still be exact."""
    from paper_1802_10453_amd import pldl
    p = 8388593
    a = (-32896) % p
    ctx.set_path(pldl.PLDL_PATH_I8)
    try:
        for k, want_i8 in ((32767, True), (32768, False)):
            n = 48
            print(f"[i8 bound] syrd2k k={k}", flush=True)
            A = np.full((n, k), a, dtype=np.uint32)
            dd = np.ones(k, dtype=np.uint32)
            de = np.zeros(k, dtype=np.uint32)
            C = np.tril(np.full((n, n), 12345, dtype=np.uint32))
            Cd = dev(C)
            st = profiled(ctx, lambda: ctx.syrdk(p, Cd, dev(A), dev(dd), dev(de), B=dev(A)))
            assert (st["gemm_i8"]["launches"] > 0) == want_i8, st["gemm_i8"]
            ref = (12345 - 2 * k * a * a) % p
            got = np.tril(host(Cd))
            assert (got[np.tril_indices(n)] == ref).all(), k
        # one segment at the bound: k = 65535 on INT8, exact
        k = 65535
        print(f"[i8 bound] gemm k={k}", flush=True)
        A = np.full((16, k), a, dtype=np.uint32)
        B = np.full((k, 16), a, dtype=np.uint32)
        Cd = dev(np.zeros((16, 16), dtype=np.uint32))
        st = profiled(ctx, lambda: ctx.gemm(p, Cd, dev(A), dev(B)))
        assert st["gemm_i8"]["launches"] > 0
        assert (host(Cd) == (-k * a * a) % p).all()
    finally:
        ctx.set_path(pldl.PLDL_PATH_AUTO)


# ---------------------------------------------------------------- pldl_factor's error returns
def test_factor_argument_errors(ctx):
    """Every -k return of pldl_factor (checked before any work is queued), through
    the raw C-ABI call."""
    from paper_1802_10453_amd import pldl
    p, n = 65521, 8
    A = torch.zeros((n, n), dtype=torch.int32, device="cuda")
    e = torch.zeros(n, dtype=torch.int32, device="cuda")
    perm = torch.zeros(n, dtype=torch.int32, device="cuda")
    rpm = torch.zeros(n, dtype=torch.int32, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    ok = (P(A), n, pldl.PLDL_U32, P(e), P(perm), P(rpm))

    def call(pp=p, nn=n, a=ok[0], lda=ok[1], dt=ok[2], ee=ok[3], pe=ok[4], rp=ok[5], **kw):
        return ctx.factor_raw(pp, nn, a, lda, dt, ee, pe, rp, **kw)[0]

    assert call(nn=-1) == -3
    assert call(nn=65536) == -3
    assert call(a=None) == -4
    assert call(lda=n - 1) == -5
    assert call(dt=7) == -6
    assert call(ee=None) == -7
    assert call(pe=None) == -8
    assert call(rp=None) == -9
    assert call(rank_out=False) == -10
    assert call(opts=pldl.pldl_opts(9, 0, 0, 0)) == -11
    assert call(opts=pldl.pldl_opts(0, 129, 0, 0)) == -11
    assert call(opts=pldl.pldl_opts(0, -2, 0, 0)) == -11   # (-1 is PLDL_THRESHOLD_ONLINE)
    assert call(pp=1) == pldl.ERRORS_BY_NAME["PLDL_EUNSUPPORTED_P"]
    assert call(pp=1 << 24) == pldl.ERRORS_BY_NAME["PLDL_EUNSUPPORTED_P"]
    assert "p must satisfy" in ctx.last_error()
    # n = 0 is valid and needs no arrays
    assert call(nn=0, a=None, lda=1, ee=None, pe=None, rp=None) == 0
    # the context still works after the rejected calls
    Ad, _ = inputs.rank_profile_matrix_input(40, p, 10, 5, 4040)
    res = gpu_factor(ctx, Ad, p, threshold=16)
    check_against_oracle(Ad, p, res)


def test_factor_range_error_and_schedule(ctx):
    """An entry >= p with check_range gives PLDL_ERANGE (and writes nothing); without
    it the call proceeds.  The schedule reports the threshold and split rule used."""
    from paper_1802_10453_amd import pldl
    p, n = 65521, 200
    A, _ = inputs.rank_profile_matrix_input(n, p, 60, 30, 5151)
    bad = A.copy()
    bad[150, 20] = p + 3
    Ad = torch.from_numpy(bad.astype(np.int32)).cuda()
    before = Ad.clone()
    with pytest.raises(pldl.PldlError) as ei:
        ctx.factor(Ad, p, threshold=32)
    assert ei.value.code == pldl.ERRORS_BY_NAME["PLDL_ERANGE"]
    torch.cuda.synchronize()
    assert torch.equal(Ad, before), "a rejected input must be left as it was"
    # without the range check the entry is read mod p: the same result as the reduced input
    red = bad.copy()
    red[150, 20] = 3
    out_bad = ctx.factor(Ad, p, threshold=32, check_range=False)
    Ar = torch.from_numpy(red.astype(np.int32)).cuda()
    out_red = ctx.factor(Ar, p, threshold=32)
    torch.cuda.synchronize()
    assert torch.equal(Ad, Ar) and torch.equal(out_bad["perm"], out_red["perm"])
    # a valid input: schedule fields
    ctx.set_path(pldl.PLDL_PATH_AUTO)
    Ad = torch.from_numpy(A.astype(np.int32)).cuda()
    out = ctx.factor(Ad, p, threshold=48)
    sc = out["schedule"]
    assert sc["threshold_used"] == 48 and sc["split_rule"] == 64
    # the context's default path takes INT8 products for p < 2^23, none this small
    assert sc["path_used"] == pldl.PLDL_PATH_I8 and sc["products_i8"] == 0
    assert sc["products_f64"] > 0 and sc["launches"] > sc["products_f64"] and sc["host_waits"] >= 1


# ---------------------------------------------------------------- online threshold
def _factor_host(ctx, A, p, threshold):
    n = A.shape[0]
    Ad = torch.from_numpy(A.astype(np.int32)).cuda()
    out = ctx.factor(Ad, p, threshold=threshold)
    torch.cuda.synchronize()
    Ah = Ad.cpu().numpy().astype(np.int64).astype(np.uint32)
    L = np.tril(Ah, -1)
    L[np.arange(n), np.arange(n)] = 1
    res = dict(perm=out["perm"].cpu().numpy().astype(np.int32), rpm=out["rpm"].cpu().numpy().astype(np.int32), L=L,
               dd=np.diag(Ah).copy(), de=out["e"].cpu().numpy().astype(np.int64).astype(np.uint32), rank=out["rank"])
    return res, out["schedule"]


def test_online_threshold(ctx):
    """threshold = PLDL_THRESHOLD_ONLINE: the first calls of an order class time
    each candidate once (128, 96, 64 in that order), later ones use the fastest;
    every call's result matches the oracle and equals the explicit call with the
    threshold it reports."""
    from paper_1802_10453_amd import pldl
    p, n = 65521, 900
    A, _ = inputs.rank_profile_matrix_input(n, p, 300, 150, inputs.SEED_BASE + 611, check=8)
    ref = orc.search(A, p)
    used = []
    for call in range(5):
        print(f"[online] call {call}", flush=True)
        res, sc = _factor_host(ctx, A, p, pldl.PLDL_THRESHOLD_ONLINE)
        used.append(sc["threshold_used"])
        check_against_oracle(A, p, res, ref=ref)
        exp, sc2 = _factor_host(ctx, A, p, sc["threshold_used"])
        assert sc2["threshold_used"] == sc["threshold_used"]
        assert (exp["perm"] == res["perm"]).all() and (exp["L"] == res["L"]).all()
    print("[online] thresholds used:", used, flush=True)
    assert used[:3] == [128, 96, 64], used
    assert all(t in (128, 96, 64) for t in used[3:]), used


def test_online_threshold_rejects_other_negatives(ctx):
    from paper_1802_10453_amd import pldl
    A = np.zeros((8, 8), dtype=np.uint32)
    with pytest.raises(pldl.PldlError):
        ctx.factor(torch.from_numpy(A.astype(np.int32)).cuda(), 65521, threshold=-2)
