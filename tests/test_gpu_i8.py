"""GPU parity of the INT8-split product path (signed-byte limbs, INT32 MFMA
accumulation, mod-p recombination) against the CPU oracle, bit-exact, and
against the FP64 path on whole factorizations (both are exact, so the outputs
must be identical)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle.oracle as orc  # noqa: E402
from paper_1802_10453_amd import inputs  # noqa: E402

from gpu_helpers import check_against_oracle, gpu_factor  # noqa: E402

# one, two and three limbs, each near its limb-count boundary
PRIMES = [2, 3, 251, 257, 32749, 32771, 65521, 8388593, 16777213]   # the last runs on FP64 products


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10453_amd import pldl
    c = pldl.Context(0)
    c.set_path(pldl.PLDL_PATH_I8)
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x).astype(np.float64)).cuda()


def host(t):
    return t.cpu().numpy().astype(np.int64).astype(np.uint32)


def rnd(g, p, *shape):
    return g.integers(0, p, size=shape).astype(np.uint32)


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_i8_gemm_parity(ctx, p, ta, tb):
    g = inputs.rng(p * 11 + ta * 2 + tb)
    for (m, n, k) in [(1, 1, 1), (5, 7, 3), (130, 129, 17), (257, 64, 300), (64, 200, 1100), (100, 70, 2049)]:
        print(f"[i8 gemm] p={p} ta={ta} tb={tb} m={m} n={n} k={k}", flush=True)
        A = rnd(g, p, m, k)
        B = rnd(g, p, k, n)
        C = rnd(g, p, m, n)
        Cd = dev(C)
        ctx.gemm(p, Cd, dev(A.T.copy() if ta else A), dev(B.T.copy() if tb else B), transA=bool(ta),
                 transB=bool(tb))
        assert (host(Cd) == orc.gemm(p, C, A, B)).all()


@pytest.mark.parametrize("p", [251, 257, 32749, 32771, 65521, 8388593])
def test_i8_digit_extremes(ctx, p):
    """Residues whose balanced digits sit at -128, 127 and the top-digit bound, and K
    up to the INT32 accumulation bound of one shift class."""
    h = (p - 1) // 2
    vals = sorted({v % p for v in (0, 1, 127, 128, 129, 255, 256, 32767, 32768, h, h + 1, p - 1, p - 127, p - 128,
                                   p - 129, p - 32768)})
    g = inputs.rng(p)
    for k in (64, 1000, 4100, 32768):
        m, n = 17, 33
        print(f"[i8 extremes] p={p} k={k}", flush=True)
        A = np.asarray(g.choice(vals, size=(m, k)), dtype=np.uint32)
        B = np.asarray(g.choice(vals, size=(k, n)), dtype=np.uint32)
        A[0, :] = h
        B[:, 0] = h
        A[1, :] = h + 1
        B[:, 1] = h + 1
        C = rnd(g, p, m, n)
        Cd = dev(C)
        ctx.gemm(p, Cd, dev(A), dev(B))
        # exact in int64: k (p-1)^2 < 2^61 for every case here
        ref = (C.astype(np.int64) - (A.astype(np.int64) @ B.astype(np.int64)) % p) % p
        assert (host(Cd) == ref.astype(np.uint32)).all(), k


@pytest.mark.parametrize("p", [2, 32749, 65521, 8388593])
def test_i8_lower_only_and_syrd2k(ctx, p):
    g = inputs.rng(p + 5)
    for (n, k) in [(1, 4), (127, 33), (300, 260)]:
        print(f"[i8 syrd2k] p={p} n={n} k={k}", flush=True)
        A = rnd(g, p, n, k)
        B = rnd(g, p, n, k)
        C = np.tril(rnd(g, p, n, n))
        dd = rnd(g, p, k)
        de = np.zeros(k, dtype=np.uint32)
        for q in range(0, k - 1, 5):            # some 2x2 blocks
            de[q] = 1 + q % (p - 1) if p > 2 else 1
            dd[q] = 0
            if p != 2:
                dd[q + 1] = 0
        Cd = dev(C)
        ctx.syrdk(p, Cd, dev(A), dev(dd), dev(de))
        assert (np.tril(host(Cd)) == np.tril(orc.syrdk(p, C, A, dd, de))).all()
        Cd = dev(C)
        ctx.syrdk(p, Cd, dev(A), dev(dd), dev(de), B=dev(B))
        assert (np.tril(host(Cd)) == np.tril(orc.syrd2k(p, C, A, B, dd, de))).all()


# ---------------------------------------------------------------- the 128 x 128 INT8 tile
# (products of at least 128 tiles of 128 x 128: LDS-staged limb planes, eight waves)
@pytest.mark.parametrize("p", [251, 32749, 8388593])
@pytest.mark.parametrize("tb", [0, 1])
def test_i8_big_tile_dense(ctx, p, tb):
    """m = n = 2048 (256 tiles), k = 600 (a ragged last 64-deep step): one, two and
    three limbs against the oracle."""
    g = inputs.rng(p * 3 + tb)
    m = n = 2048
    k = 600
    print(f"[i8 big tile] dense p={p} tb={tb}", flush=True)
    A, B, C = rnd(g, p, m, k), rnd(g, p, k, n), rnd(g, p, m, n)
    Cd = dev(C)
    ctx.gemm(p, Cd, dev(A), dev(B.T.copy() if tb else B), transB=bool(tb))
    assert (host(Cd) == orc.gemm(p, C, A, B)).all()


def test_i8_big_tile_ragged_edges(ctx):
    """Ragged M, N and K edges on the big tile (2100 x 2050, k = 333, A transposed)."""
    p = 8388593
    g = inputs.rng(777)
    m, n, k = 2100, 2050, 333
    print("[i8 big tile] ragged", flush=True)
    A, B, C = rnd(g, p, m, k), rnd(g, p, k, n), rnd(g, p, m, n)
    Cd = dev(C)
    ctx.gemm(p, Cd, dev(A.T.copy()), dev(B), transA=True)
    assert (host(Cd) == orc.gemm(p, C, A, B)).all()


@pytest.mark.parametrize("p", [32749, 8388593])
def test_i8_big_tile_lower_syrd2k(ctx, p):
    """SYRDK and SYRD2K of order 2900 (276 lower tiles of 128 x 128), k = 200: the
    lower-triangle tile order and both segments in one accumulator set."""
    g = inputs.rng(p + 55)
    n, k = 2900, 200
    print(f"[i8 big tile] syrd2k p={p}", flush=True)
    A, B = rnd(g, p, n, k), rnd(g, p, n, k)
    C = np.tril(rnd(g, p, n, n))
    dd = rnd(g, p, k)
    de = np.zeros(k, dtype=np.uint32)
    for q in range(0, k - 1, 7):
        de[q] = 1 + q
        dd[q] = dd[q + 1] = 0
    Cd = dev(C)
    ctx.syrdk(p, Cd, dev(A), dev(dd), dev(de))
    assert (np.tril(host(Cd)) == np.tril(orc.syrdk(p, C, A, dd, de))).all()
    Cd = dev(C)
    ctx.syrdk(p, Cd, dev(A), dev(dd), dev(de), B=dev(B))
    assert (np.tril(host(Cd)) == np.tril(orc.syrd2k(p, C, A, B, dd, de))).all()


@pytest.mark.parametrize("p,c", [(8388593, -32896), (32749, -16256)])
def test_i8_big_tile_accumulation_bound(ctx, p, c):
    """Every operand the residue with centered value c, whose two low balanced digits
    are -128 (three limbs: shift class 1 then gains 2 * 128^2 = 2^15 per k, the
    bound), with K = 65535, the longest product the INT32 classes take: the closed
    form C - K c^2 mod p on the whole 2048 x 2048 output."""
    m = n = 2048
    k = 65535
    v = c % p
    print(f"[i8 big tile] bound p={p}", flush=True)
    A = torch.full((m, k), float(v), dtype=torch.float64, device="cuda")
    B = torch.full((k, n), float(v), dtype=torch.float64, device="cuda")
    Cd = torch.full((m, n), float(p - 1), dtype=torch.float64, device="cuda")
    ctx.gemm(p, Cd, A, B)
    want = (p - 1 - (k * v * v) % p) % p
    got = host(Cd)
    assert (got == want).all(), (int(got[0, 0]), want)


@pytest.mark.parametrize("p", [3, 65521, 8388593])
def test_i8_trsm(ctx, p):
    g = inputs.rng(p + 9)
    for (m, n) in [(200, 150), (530, 77)]:
        print(f"[i8 trsm] p={p} m={m} n={n}", flush=True)
        T = rnd(g, p, m, m)
        B = rnd(g, p, m, n)
        Bd = dev(B)
        ctx.trsm(p, dev(T), Bd, lower=True)
        Tl = np.tril(T, -1) + np.eye(m, dtype=np.uint32)
        assert (host(Bd) == orc.trsm_left(p, Tl, B, lower=True)).all()


@pytest.mark.parametrize("p,n,f,c", [(8388593, 1100, 300, 200), (65521, 900, 500, 150), (32749, 1024, 0, 300)])
def test_i8_factor_parity(ctx, p, n, f, c):
    """Whole factorizations with the large products on INT8 matrix cores: r and R
    against the canonical search, (L, D) against the oracle's replay."""
    A, rpm = inputs.rank_profile_matrix_input(n, p, f, c, inputs.SEED_BASE + 77 + n, check=8)
    res = gpu_factor(ctx, A, p)
    assert res["rank"] == f + 2 * c
    check_against_oracle(A, p, res)


def test_i8_factor_char2(ctx):
    n = 1024
    A, rpm, _ = inputs.char2_input(n, 300, 150, inputs.SEED_BASE + 91, check=8)
    res = gpu_factor(ctx, A, 2)
    check_against_oracle(A, 2, res)


def test_i8_matches_f64_factor(ctx):
    """Same control flow, exact arithmetic on both paths: identical outputs."""
    from paper_1802_10453_amd import pldl
    p, n = 8388593, 1500
    A, _ = inputs.rank_profile_matrix_input(n, p, 500, 250, inputs.SEED_BASE + 123, check=8)
    res8 = gpu_factor(ctx, A, p)
    ctx.set_path(pldl.PLDL_PATH_F64)
    try:
        res64 = gpu_factor(ctx, A, p)
    finally:
        ctx.set_path(pldl.PLDL_PATH_I8)
    for key in ("perm", "rpm", "L", "dd", "de"):
        assert (res8[key] == res64[key]).all(), key
    assert res8["rank"] == res64["rank"] == 1000
