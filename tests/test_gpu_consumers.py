"""GPU parity of the uses of the factorization (Section 1: solving symmetric
systems, invariants of symmetric forms): pldl_solve and pldl_invariants on
pldl_factor's outputs, against the oracle's independent Gaussian elimination
(solutions bit-exact where unique; A X = B and the consistency flags where
not), determinants, and quadratic characters."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle.oracle as orc  # noqa: E402
from paper_1802_10453_amd import inputs  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1802_10453_amd import pldl
    c = pldl.Context(0)
    yield c
    c.close()


def factor(ctx, A, p, threshold=0, dtype=torch.int32):
    Ad = torch.from_numpy(A.astype(np.int64).astype(np.int32) if dtype == torch.int32 else A.astype(np.float64)).cuda()
    out = ctx.factor(Ad, p, threshold=threshold)
    return Ad, out


def solve(ctx, p, Ad, out, B):
    Bd = torch.from_numpy(B.astype(np.float64)).cuda()
    cons = ctx.solve(p, Ad, out["e"], out["perm"], out["rank"], Bd)
    torch.cuda.synchronize()
    return Bd.cpu().numpy().astype(np.int64).astype(np.uint32), cons.cpu().numpy()


def matmul_mod(A, X, p):
    return (A.astype(object) @ X.astype(object)) % p


@pytest.mark.parametrize("p,n", [(65521, 300), (8388593, 520), (3, 200), (2, 256)])
def test_solve_nonsingular_matches_oracle(ctx, p, n):
    g = inputs.rng(1000 + p + n)
    if p == 2:
        # full rank with a zero diagonal on half the rows: relaxed 2x2 blocks are solved too
        A, _, _ = inputs.char2_input(n, n // 2, n // 4, 2000 + n, check=0)
    else:
        for trial in range(20):
            A = inputs.symmetric_uniform(n, p, 2000 + trial + n)
            if orc.det(A, p) != 0:
                break
    assert orc.det(A, p) != 0
    B = g.integers(0, p, size=(n, 5)).astype(np.uint32)
    print(f"[solve] p={p} n={n}", flush=True)
    Ad, out = factor(ctx, A, p, threshold=32)
    assert out["rank"] == n
    X, cons = solve(ctx, p, Ad, out, B)
    Xo, co = orc.solve(A, p, B)
    assert (cons == 1).all() and (co == 1).all()
    assert (X == Xo).all()


@pytest.mark.parametrize("p", [65521, 8388593, 2])
def test_solve_singular_consistency(ctx, p):
    """Rank-deficient L R L^T inputs: columns in the range are solved (A X = B), a
    column outside it is flagged, as the oracle's rank test says."""
    g = inputs.rng(3000 + p)
    n, f, c = 200, 60, 30
    if p == 2:
        A, _, _ = inputs.char2_input(n, f, c, 3100, check=0)
    else:
        A, _ = inputs.rank_profile_matrix_input(n, p, f, c, 3100, check=0)
    y = g.integers(0, p, size=(n, 3)).astype(np.uint32)
    B = matmul_mod(A, y, p).astype(np.uint32)
    Bbad = B[:, :1].copy()
    for j in range(n):
        cand = Bbad.astype(np.int64)
        cand[j, 0] = (cand[j, 0] + 1) % p
        if orc.rank(np.concatenate([A, cand.astype(np.uint32)], axis=1), p) > f + 2 * c:
            Bbad = cand.astype(np.uint32)
            break
    Ball = np.concatenate([B, Bbad], axis=1)
    print(f"[solve singular] p={p}", flush=True)
    Ad, out = factor(ctx, A, p, threshold=32)
    X, cons = solve(ctx, p, Ad, out, Ball)
    _, co = orc.solve(A, p, Ball)
    assert cons.tolist() == co.tolist() == [1, 1, 1, 0]
    assert (matmul_mod(A, X[:, :3], p) == B).all()


def test_solve_c1_workload(ctx):
    """The n = 4096 uniform workload: four right-hand sides, against the oracle."""
    cfg = inputs.C1
    A, _ = inputs.config_input(cfg)
    p, n = cfg["p"], cfg["n"]
    g = inputs.rng(4096)
    B = g.integers(0, p, size=(n, 4)).astype(np.uint32)
    print("[solve] C1", flush=True)
    Ad, out = factor(ctx, A, p)
    X, cons = solve(ctx, p, Ad, out, B)
    print("[solve] C1 oracle", flush=True)
    Xo, co = orc.solve(A, p, B)
    assert (cons == 1).all() and (co == 1).all()
    assert (X == Xo).all()


@pytest.mark.parametrize("p", [3, 65521, 8388593])
def test_invariants_against_oracle(ctx, p):
    g = inputs.rng(5000 + p)
    for n in (1, 17, 300):
        A = inputs.symmetric_uniform(n, p, 5100 + n)
        print(f"[invariants] p={p} n={n}", flush=True)
        Ad, out = factor(ctx, A, p, threshold=32)
        inv = ctx.invariants(p, Ad, out["e"], out["rank"])
        d = orc.det(A, p)
        assert inv["rank"] == out["rank"] == orc.rank(A, p)
        assert inv["det"] == (d if out["rank"] == n else 0)
        if out["rank"] == n:
            assert inv["disc"] == d
            assert inv["character"] == (1 if pow(d, (p - 1) // 2, p) == 1 else -1)
    # a singular form: the discriminant class of its nondegenerate part equals the one the
    # oracle's own factorization gives (product of its D blocks)
    A, _ = inputs.rank_profile_matrix_input(120, p, 40, 20, 5200 + p, check=0)
    Ad, out = factor(ctx, A, p, threshold=32)
    inv = ctx.invariants(p, Ad, out["e"], out["rank"])
    ref = orc.search(A, p)
    prod, q = 1, 0
    while q < ref["rank"]:
        if ref["de"][q]:
            prod = prod * (-(int(ref["de"][q]) ** 2)) % p
            q += 2
        else:
            prod = prod * int(ref["dd"][q]) % p
            q += 1
    assert inv["rank"] == ref["rank"] == 80 and inv["det"] == 0
    assert inv["character"] == (1 if pow(prod, (p - 1) // 2, p) == 1 else -1)


def test_invariants_char2_alternating(ctx):
    """p = 2: alternating exactly when diag(A) = 0."""
    n = 160
    A, _, _ = inputs.char2_input(n, 40, 30, 6100, check=0)
    Ad, out = factor(ctx, A, 2, threshold=32)
    inv = ctx.invariants(2, Ad, out["e"], out["rank"])
    assert inv["alternating"] == int((np.diag(A) == 0).all())
    Z = A.copy()
    np.fill_diagonal(Z, 0)                      # an alternating form
    Ad, out = factor(ctx, Z, 2, threshold=32)
    inv = ctx.invariants(2, Ad, out["e"], out["rank"])
    assert inv["alternating"] == 1 and inv["rank"] == orc.rank(Z, 2)
