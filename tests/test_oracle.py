"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics.

Every check here is independent of the oracle's own elimination: brute-force
rank profiles from Theorem 1, exact reconstruction by plain integer products,
determinants by an independent elimination in Python integers, the worked
examples of the paper, exhaustive enumeration over tiny fields, and closed forms
of the input generator.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle.oracle as orc
from paper_1802_10453_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")
PRIMES = [2, 3, 5, 7, 65521, 8388593, 16777213]


# ---------------------------------------------------------------- helpers (independent)
def mm(A, B, p):
    return (np.asarray(A, dtype=object) @ np.asarray(B, dtype=object)) % p


def D_full(dd, de):
    n = len(dd)
    D = np.zeros((n, n), dtype=object)
    for q in range(n):
        D[q, q] = int(dd[q])
        if q + 1 < n:
            D[q + 1, q] = D[q, q + 1] = int(de[q])
    return D


def P_mat(perm):
    n = len(perm)
    P = np.zeros((n, n), dtype=object)
    for q, i in enumerate(perm):
        P[i, q] = 1
    return P


def reconstruct_indep(p, perm, L, dd, de):
    P = P_mat(perm)
    return mm(mm(mm(mm(P, L, p), D_full(dd, de), p), np.asarray(L, dtype=object).T, p), P.T, p)


def det_indep(A, p):
    """Determinant mod p by Gaussian elimination on Python integers."""
    M = [[int(x) % p for x in row] for row in A]
    n, det = len(M), 1
    for c in range(n):
        piv = next((r for r in range(c, n) if M[r][c]), None)
        if piv is None:
            return 0
        if piv != c:
            M[c], M[piv] = M[piv], M[c]
            det = -det
        det = det * M[c][c] % p
        inv = pow(M[c][c], p - 2, p)
        for r in range(c + 1, n):
            f = M[r][c] * inv % p
            for k in range(c, n):
                M[r][k] = (M[r][k] - f * M[c][k]) % p
    return det % p


def rpm_from_ranks_python(A, p):
    """Theorem 1 with ranks from an independent Python elimination (tiny n)."""
    n = len(A)

    def rk(a, b):
        M = [[int(A[i][j]) % p for j in range(b)] for i in range(a)]
        r = 0
        for c in range(b):
            piv = next((i for i in range(r, a) if M[i][c]), None)
            if piv is None:
                continue
            M[r], M[piv] = M[piv], M[r]
            inv = pow(M[r][c], p - 2, p)
            for i in range(r + 1, a):
                f = M[i][c] * inv % p
                for k in range(c, b):
                    M[i][k] = (M[i][k] - f * M[r][k]) % p
            r += 1
        return r

    R = np.zeros(n, dtype=np.int32) - 1
    for i in range(n):
        for j in range(n):
            e = rk(i + 1, j + 1) - rk(i, j + 1) - rk(i + 1, j) + rk(i, j)
            if e:
                R[i] = j
    return R


def check_structure(f, p):
    """L unit lower, D block structure consistent with rpm and rank."""
    L, dd, de, rpm, perm, r = f["L"], f["dd"], f["de"], f["rpm"], f["perm"], f["rank"]
    n = len(perm)
    assert sorted(perm.tolist()) == list(range(n))
    assert (np.triu(L, 1) == 0).all() and (np.diag(L) == 1).all()
    q = 0
    while q < r:
        i = perm[q]
        if rpm[i] == i:
            assert dd[q] != 0 and de[q] == 0
            q += 1
        else:
            j = perm[q + 1]
            assert rpm[i] == j and rpm[j] == i
            assert de[q] != 0 and dd[q] == 0 and de[q + 1] == 0
            if p != 2:
                assert dd[q + 1] == 0
            else:
                assert L[q + 1, q] == 0
            q += 2
    assert (dd[r:] == 0).all() and (de[max(r - 1, 0):] == 0).all() if r > 0 else (dd == 0).all()
    for q in range(r, n):
        assert rpm[perm[q]] == -1
        assert (L[q + 1:, q] == 0).all()            # non-pivot columns are identity columns
    # non-pivots keep their precedence
    assert list(perm[r:]) == sorted(perm[r:])


def full_check(A, p):
    f = orc.search(A, p)
    check_structure(f, p)
    assert (reconstruct_indep(p, f["perm"], f["L"], f["dd"], f["de"]) == np.asarray(A, dtype=object)).all()
    return f


# ---------------------------------------------------------------- field
@pytest.mark.parametrize("p", [2, 3, 5, 7, 31, 251, 32749])
def test_inverse_exhaustive(p):
    for a in range(1, p):
        assert a * orc.inv(a, p) % p == 1


def test_inverse_large_primes():
    g = inputs.rng(1)
    for p in (65521, 8388593):
        for a in list(g.integers(1, p, size=2000)) + [1, 2, p - 1, p - 2, (p - 1) // 2]:
            assert int(a) * orc.inv(int(a), p) % p == 1


# ---------------------------------------------------------------- worked examples of the paper
def _gold():
    with open(GOLD) as fh:
        return json.load(fh)


@pytest.mark.parametrize("name", ["antidiagonal_2x2", "lemma1_char2", "hand_3x3"])
def test_golden_examples(name):
    g = _gold()[name]
    p = g["p"]
    A = np.array(g["A"], dtype=np.uint32)
    f = orc.search(A, p)
    assert f["rank"] == g["rank"]
    assert f["perm"].tolist() == g["perm"]
    assert f["L"].tolist() == g["L"]
    assert f["dd"].tolist() == g["dd"]
    assert f["de"].tolist() == g["de"]
    assert f["rpm"].tolist() == g["rpm"]
    assert orc.rpm_bruteforce(A, p).tolist() == g["rpm"]
    if "standard_form" in g:
        s = g["standard_form"]
        perm, L, dd, de = orc.char2_standard(f["perm"], f["L"], f["dd"], f["de"])
        assert perm.tolist() == s["perm"] and L.tolist() == s["L"]
        assert dd.tolist() == s["dd"] and de.tolist() == s["de"]
        assert (reconstruct_indep(2, perm, L, dd, de) == A.astype(object)).all()


def test_lemma1_no_antidiagonal_solution():
    """Lemma 1: over F_2 no P, L with D antidiagonal or diagonal reproduces [[0,1],[1,1]]
    while revealing R = J; brute force over every candidate."""
    A = np.array([[0, 1], [1, 1]], dtype=object)
    found = []
    for perm in ([0, 1], [1, 0]):
        for x in range(2):
            for y in range(2):
                for z in range(2):
                    L = np.array([[1, 0], [x, 1]], dtype=object)
                    for D in (np.array([[y, 0], [0, z]], dtype=object), np.array([[0, y], [y, 0]], dtype=object)):
                        if (reconstruct_indep(2, perm, L, [D[0, 0], D[1, 1]], [D[1, 0], 0]) == A).all():
                            Psi = (D != 0).astype(object)
                            P = P_mat(perm)
                            Pi = (P @ Psi @ P.T)
                            found.append((perm, Pi.tolist()))
    assert all(Pi != [[0, 1], [1, 0]] for _, Pi in found)


# ---------------------------------------------------------------- exhaustive small fields
@pytest.mark.parametrize("p,nmax", [(2, 4), (3, 3), (5, 2)])
def test_exhaustive_small_fields(p, nmax):
    """Every symmetric matrix over F_p up to order nmax: the pivoting matrix of the
    canonical factorization equals the rank profile matrix of Theorem 1, and the
    factorization reconstructs A."""
    for n in range(1, nmax + 1):
        tri = [(i, j) for i in range(n) for j in range(i + 1)]
        for vals in itertools.product(range(p), repeat=len(tri)):
            A = np.zeros((n, n), dtype=np.uint32)
            for (i, j), v in zip(tri, vals):
                A[i, j] = A[j, i] = v
            f = full_check(A, p)
            assert f["rpm"].tolist() == rpm_from_ranks_python(A, p).tolist()
            assert f["rank"] == sum(1 for x in f["rpm"] if x >= 0)


def test_exhaustive_f2_order5_rpm():
    """All 2^15 symmetric 5x5 matrices over F_2 (search vs Theorem 1 via the
    independent leading-rank routine, plus reconstruction)."""
    n, p = 5, 2
    tri = [(i, j) for i in range(n) for j in range(i + 1)]
    g = inputs.rng(5)
    sample = set(int(x) for x in g.integers(0, 1 << 15, size=600))
    for code in range(1 << 15):
        A = np.zeros((n, n), dtype=np.uint32)
        for b, (i, j) in enumerate(tri):
            A[i, j] = A[j, i] = (code >> b) & 1
        f = orc.search(A, p)
        assert (f["rpm"] == orc.rpm_bruteforce(A, p)).all()
        if code in sample:
            check_structure(f, p)
            assert (reconstruct_indep(p, f["perm"], f["L"], f["dd"], f["de"]) == A.astype(object)).all()


# ---------------------------------------------------------------- brute force pinned itself
def test_bruteforce_rpm_matches_python_theorem1():
    g = inputs.rng(7)
    for p in (3, 7, 65521):
        for _ in range(6):
            n = int(g.integers(1, 7))
            A = inputs.symmetric_uniform(n, p, int(g.integers(1 << 30)))
            A[g.integers(0, n, size=n), :] = 0
            A = np.minimum(A, A.T)
            assert orc.rpm_bruteforce(A, p).tolist() == rpm_from_ranks_python(A, p).tolist()


@pytest.mark.parametrize("p", PRIMES)
def test_generator_closed_form_rpm(p):
    """A = L R L^T with L unit lower has RPM(A) = supp(R): brute force agrees."""
    for seed in range(4):
        n, f, c = 24, 5, 4
        A, rpm = inputs.rank_profile_matrix_input(n, p, f, c, 100 + seed)
        assert (A == A.T).all()
        assert orc.rpm_bruteforce(A, p).tolist() == rpm.tolist()
        assert orc.rank(A, p) == f + 2 * c


def test_rank_textbook():
    g = inputs.rng(11)
    for p in (2, 65521):
        for _ in range(10):
            m, n, k = (int(x) for x in g.integers(1, 12, size=3))
            X = g.integers(0, p, size=(m, k))
            Y = g.integers(0, p, size=(k, n))
            A = mm(X, Y, p).astype(np.uint32)
            r = orc.rank(A, p)
            assert r <= min(m, n, k)
            # rank equals the number of nonzero rows of R computed from leading ranks
            sq = np.zeros((max(m, n),) * 2, dtype=np.uint32)
            sq[:m, :n] = A
            assert r == int((orc.rpm_bruteforce(sq, p) >= 0).sum())


# ---------------------------------------------------------------- the factorization
@pytest.mark.parametrize("p", PRIMES)
def test_search_random_generator_inputs(p):
    g = inputs.rng(p)
    for trial in range(5):
        n = int(g.integers(2, 40))
        r = int(g.integers(0, n + 1))
        c = int(g.integers(0, r // 2 + 1))
        f = r - 2 * c
        A, rpm = inputs.rank_profile_matrix_input(n, p, f, c, int(g.integers(1 << 30)))
        fa = full_check(A, p)
        assert fa["rank"] == r
        assert fa["rpm"].tolist() == rpm.tolist()


def test_search_c0_workload():
    cfg = inputs.C0
    A, rpm = inputs.config_input(cfg)
    f = full_check(A, cfg["p"])
    assert f["rank"] == 40
    assert f["rpm"].tolist() == rpm.tolist() == orc.rpm_bruteforce(A, cfg["p"]).tolist()


@pytest.mark.parametrize("p", [3, 65521, 8388593])
def test_det_equals_det_D(p):
    g = inputs.rng(3 * p)
    for _ in range(6):
        n = int(g.integers(1, 9))
        A = inputs.symmetric_uniform(n, p, int(g.integers(1 << 30)))
        f = orc.search(A, p)
        d = det_indep(A, p)
        if f["rank"] < n:
            assert d == 0
            continue
        assert d == det_indep(D_full(f["dd"], f["de"]), p)


def test_generic_rank_profile_is_plain_ldlt():
    """All leading principal minors nonzero => P = I, D diagonal with
    D_kk = det(A_k)/det(A_{k-1}) (plain LDL^T)."""
    p = 65521
    g = inputs.rng(21)
    done = 0
    while done < 5:
        n = int(g.integers(2, 9))
        A = inputs.symmetric_uniform(n, p, int(g.integers(1 << 30)))
        minors = [1] + [det_indep(A[:k, :k], p) for k in range(1, n + 1)]
        if any(m == 0 for m in minors):
            continue
        f = orc.search(A, p)
        assert f["perm"].tolist() == list(range(n))
        assert (f["de"] == 0).all()
        for k in range(n):
            assert int(f["dd"][k]) == minors[k + 1] * pow(minors[k], p - 2, p) % p
        done += 1


def test_char2_inputs_relaxed_blocks_and_standard_form():
    for seed in range(3):
        A, rpm, H = inputs.char2_input(40, 8, 6, 50 + seed)
        assert (np.diag(A)[H] == 0).all()
        f = full_check(A, 2)
        assert f["rpm"].tolist() == rpm.tolist() == orc.rpm_bruteforce(A, 2).tolist()
        perm, L, dd, de = orc.char2_standard(f["perm"], f["L"], f["dd"], f["de"])
        assert (np.triu(L, 1) == 0).all() and (np.diag(L) == 1).all()
        for q in range(39):
            if de[q]:
                assert dd[q] == 0 and dd[q + 1] == 0      # only antidiagonal blocks remain
        assert (reconstruct_indep(2, perm, L, dd, de) == A.astype(object)).all()


def test_relaxed_blocks_occur_on_char2_workload_shape():
    A, rpm, _ = inputs.char2_input(96, 30, 15, 7)
    f = orc.search(A, 2)
    n2 = sum(1 for q in range(95) if f["de"][q])
    relaxed = sum(1 for q in range(95) if f["de"][q] and f["dd"][q + 1])
    assert n2 > 0 and relaxed > 0 and relaxed < n2 + 1


@pytest.mark.parametrize("p", [2, 65521, 8388593])
def test_replay_reproduces_search(p):
    g = inputs.rng(p + 1)
    for _ in range(4):
        n = int(g.integers(2, 30))
        r = int(g.integers(0, n + 1))
        c = int(g.integers(0, r // 2 + 1))
        A, _ = inputs.rank_profile_matrix_input(n, p, r - 2 * c, c, int(g.integers(1 << 30)))
        f = orc.search(A, p)
        rc, rp = orc.replay(A, p, f["perm"], f["rpm"], f["rank"])
        assert rc == 0
        for k in ("L", "dd", "de"):
            assert (rp[k] == f[k]).all()


def test_replay_other_valid_order():
    """A different valid pivot order (the recursive one of Section 4 for the
    hand 3x3 example with split m = 2: A's pivot 1 first, then the pair (0, 2))
    gives another factorization that reconstructs A and reveals the same R."""
    A = np.array([[0, 0, 5], [0, 3, 7], [5, 7, 11]], dtype=np.uint32)
    p = 65521
    rc, f = orc.replay(A, p, np.array([1, 0, 2]), np.array([2, 1, 0]), 3)
    assert rc == 0
    assert (reconstruct_indep(p, f["perm"], f["L"], f["dd"], f["de"]) == A.astype(object)).all()
    assert f["dd"].tolist() == [3, 0, 0] and f["de"].tolist() == [0, 5, 0]


def test_replay_rejects_invalid():
    A = np.array([[0, 0, 5], [0, 3, 7], [5, 7, 11]], dtype=np.uint32)
    p = 65521
    assert orc.replay(A, p, np.array([2, 0, 1]), np.array([2, 1, 0]), 3)[0] == -5   # leading diag 11 != 0
    assert orc.replay(A, p, np.array([0, 1, 2]), np.array([2, 1, 0]), 3)[0] == -3   # partners not adjacent
    assert orc.replay(A, p, np.array([0, 1, 2]), np.array([0, 1, 2]), 3)[0] == -4   # zero 1x1 pivot
    assert orc.replay(A, p, np.array([1, 0, 2]), np.array([-1, 1, -1]), 1)[0] == -6  # Schur not zero
    assert orc.replay(A, p, np.array([0, 0, 2]), np.array([2, 1, 0]), 3)[0] == -2


# ---------------------------------------------------------------- building blocks
def test_gemm_trsm_syrdk_definitions():
    g = inputs.rng(99)
    for p in (2, 65521, 8388593):
        m, n, k = 7, 5, 6
        A = g.integers(0, p, size=(m, k)).astype(np.uint32)
        B = g.integers(0, p, size=(k, n)).astype(np.uint32)
        C = g.integers(0, p, size=(m, n)).astype(np.uint32)
        assert (orc.gemm(p, C, A, B) == (C.astype(object) - mm(A, B, p)) % p).all()
        T = np.tril(g.integers(0, p, size=(m, m)), -1).astype(np.uint32) + np.eye(m, dtype=np.uint32)
        Bm = g.integers(0, p, size=(m, n)).astype(np.uint32)
        X = orc.trsm_left(p, T, Bm, lower=True)
        assert (mm(T, X, p) == Bm).all()
        Tu = T.T.copy()
        X = orc.trsm_left(p, Tu, Bm, lower=False)
        assert (mm(Tu, X, p) == Bm).all()
        # SYRDK / SYRD2K with a block diagonal D
        dd = g.integers(0, p, size=k).astype(np.uint32)
        de = np.zeros(k, dtype=np.uint32)
        de[1] = 3 % p or 1
        dd[1] = 0
        dd[2] = 0 if p != 2 else dd[2]
        Cs = g.integers(0, p, size=(m, m)).astype(np.uint32)
        Ak = g.integers(0, p, size=(m, k)).astype(np.uint32)
        Bk = g.integers(0, p, size=(m, k)).astype(np.uint32)
        D = D_full(dd, de)
        ref = (Cs.astype(object) - mm(mm(Ak, D, p), Ak.T, p)) % p
        out = orc.syrdk(p, Cs, Ak, dd, de)
        assert (np.tril(out) == np.tril(ref)).all() and (np.triu(out, 1) == np.triu(Cs, 1)).all()
        ref2 = (Cs.astype(object) - mm(mm(Ak, D, p), Bk.T, p) - mm(mm(Bk, D, p), Ak.T, p)) % p
        out2 = orc.syrd2k(p, Cs, Ak, Bk, dd, de)
        assert (np.tril(out2) == np.tril(ref2)).all()


@pytest.mark.parametrize("p", [3, 65521, 8388593])
def test_trss_defining_equation(p):
    g = inputs.rng(p + 5)
    for n in (1, 2, 3, 8, 17):
        U = np.triu(g.integers(0, p, size=(n, n)), 1).astype(np.uint32) + np.eye(n, dtype=np.uint32)
        C = inputs.symmetric_uniform(n, p, int(g.integers(1 << 30)))
        rc, X = orc.trss(p, U, C)
        assert rc == 0
        assert (np.tril(X, -1) == 0).all()
        lhs = (mm(X.T, U, p) + mm(U.T, X, p)) % p
        assert (lhs == C.astype(object)).all()


def test_trss_char2():
    g = inputs.rng(77)
    for n in (1, 2, 5, 12):
        U = np.triu(g.integers(0, 2, size=(n, n)), 1).astype(np.uint32) + np.eye(n, dtype=np.uint32)
        C = inputs.symmetric_uniform(n, 2, int(g.integers(1 << 30)))
        C[np.arange(n), np.arange(n)] = 0
        rc, X = orc.trss(2, U, C)
        assert rc == 0 and (np.diag(X) == 0).all()
        assert ((mm(X.T, U, 2) + mm(U.T, X, 2)) % 2 == C.astype(object)).all()
        C[0, 0] = 1
        assert orc.trss(2, U, C)[0] == -2          # no solution with a nonzero diagonal (Section 3)


@pytest.mark.parametrize("p", [2, 65521, 8388593])
def test_plduq_reveals_rpm_and_reconstructs(p):
    g = inputs.rng(p + 9)
    for _ in range(8):
        m, n = (int(x) for x in g.integers(1, 14, size=2))
        k = int(g.integers(0, min(m, n) + 1))
        X = g.integers(0, p, size=(m, k))
        Z = g.integers(0, p, size=(k, n))
        Y = mm(X, Z, p).astype(np.uint32)
        Y[g.integers(0, m)] = 0
        f = orc.plduq(p, Y)
        r, rows, cols, LU = f["rank"], f["rows"], f["cols"], f["LU"]
        assert r == orc.rank(Y, p)
        assert list(rows[:r]) == sorted(rows[:r]) and list(rows[r:]) == sorted(rows[r:])
        assert list(cols[r:]) == sorted(cols[r:])
        L = np.tril(LU[:, :r], -1).astype(object)
        L[np.arange(r), np.arange(r)] = 1
        U = np.triu(LU[:r, :], 1).astype(object)
        U[np.arange(r), np.arange(r)] = 1
        D = np.diag([int(x) for x in np.diag(LU)[:r]]) if r else np.zeros((0, 0), dtype=object)
        assert all(int(x) != 0 for x in np.diag(LU)[:r])
        assert (LU[r:, r:] == 0).all()
        rec = mm(mm(L, D, p), U, p) if r else np.zeros((m, n), dtype=object)
        assert (rec == Y[np.ix_(rows, cols)].astype(object)).all()
        # the pivot set is the rank profile matrix of Y (Theorem 1 on a square padding)
        s = max(m, n)
        sq = np.zeros((s, s), dtype=np.uint32)
        sq[:m, :n] = Y
        R = orc.rpm_bruteforce(sq, p)
        assert sorted((int(rows[t]), int(cols[t])) for t in range(r)) == \
            sorted((i, int(R[i])) for i in range(m) if R[i] >= 0)


def test_delta_zeroes_diagonal():
    g = inputs.rng(123)
    for p in (2, 65521):
        r = 9
        U = np.triu(g.integers(0, p, size=(r, r)), 1).astype(np.uint32) + np.eye(r, dtype=np.uint32)
        C = inputs.symmetric_uniform(r, p, 5)
        d = orc.delta(p, U, C)
        M = (C.astype(object) - mm(mm(U.T, np.diag([int(x) for x in d]), p), U, p)) % p
        assert all(M[i, i] == 0 for i in range(r))


def test_effective_ops_formula():
    # Section 6: r^3/3 + n^2 r - r^2 n; full rank gives n^3/3
    assert orc.effective_ops(30, 30) == pytest.approx(30 ** 3 / 3)
    assert orc.effective_ops(16384, 12288) == pytest.approx(1.4431e12, rel=1e-4)


# ---------------------------------------------------------------- reconstruction routine
def _random_factors(g, n, p, char2_relaxed=False):
    """A random (perm, L, D) with 1x1 and 2x2 blocks (relaxed ones in characteristic 2),
    built directly: no elimination involved."""
    perm = g.permutation(n).astype(np.int32)
    L = np.tril(g.integers(0, p, size=(n, n)), -1).astype(np.uint32)
    L[np.arange(n), np.arange(n)] = 1
    dd = np.zeros(n, dtype=np.uint32)
    de = np.zeros(n, dtype=np.uint32)
    q = 0
    r = int(g.integers(0, n + 1))
    while q < r:
        if q + 1 < r and g.integers(0, 2):
            de[q] = int(g.integers(1, p))
            if char2_relaxed:
                dd[q + 1] = int(g.integers(0, p))
            q += 2
        else:
            dd[q] = int(g.integers(1, p))
            q += 1
    return perm, L, dd, de


@pytest.mark.parametrize("p", [2, 3, 65521, 8388593])
def test_reconstruct_matches_independent_product(p):
    """orc_reconstruct (the checker of the standard-form tests) equals P L D L^T P^T
    computed with Python integers, for random factors with a nontrivial P (an
    inverted permutation convention gives a different matrix on these inputs)."""
    g = inputs.rng(4242 + p)
    for t in range(6):
        n = int(g.integers(1, 24))
        perm, L, dd, de = _random_factors(g, n, p, char2_relaxed=(p == 2))
        ref = reconstruct_indep(p, perm, L, dd, de)
        got = orc.reconstruct(p, perm, L, dd, de)
        assert (got.astype(object) == ref).all()
        inv = np.argsort(perm).astype(np.int32)
        if n >= 3 and not (inv == perm).all():
            bad = reconstruct_indep(p, inv, L, dd, de)
            # the check separates the two conventions whenever they give different matrices
            if not (bad == ref).all():
                assert not (got.astype(object) == bad).all()


@pytest.mark.parametrize("name", ["antidiagonal_2x2", "lemma1_char2", "hand_3x3"])
def test_reconstruct_golden(name):
    g = _gold()[name]
    A = np.array(g["A"], dtype=np.uint32)
    out = orc.reconstruct(g["p"], g["perm"], np.array(g["L"], dtype=np.uint32), g["dd"], g["de"])
    assert (out == A).all()
    if "standard_form" in g:
        s = g["standard_form"]
        out = orc.reconstruct(2, s["perm"], np.array(s["L"], dtype=np.uint32), s["dd"], s["de"])
        assert (out == A).all()


def test_reconstruct_of_search_on_generator_inputs():
    for p in (2, 65521):
        for seed in range(3):
            if p == 2:
                A, _, _ = inputs.char2_input(40, 8, 6, 90 + seed)
            else:
                A, _ = inputs.rank_profile_matrix_input(40, p, 12, 6, 90 + seed)
            f = orc.search(A, p)
            assert (orc.reconstruct(p, f["perm"], f["L"], f["dd"], f["de"]) == A).all()


# ---------------------------------------------------------------- uses of the factorization (Section 1)
@pytest.mark.parametrize("p", [2, 3, 65521, 8388593])
def test_det_against_independent_elimination(p):
    g = inputs.rng(77 + p)
    for t in range(8):
        n = int(g.integers(1, 14))
        A = g.integers(0, p, size=(n, n)).astype(np.uint32)
        if t % 3 == 2 and n > 1:
            A[n - 1] = A[0]                         # singular
        assert orc.det(A, p) == det_indep(A, p)


def test_det_of_symmetric_generator_inputs_is_det_of_D():
    """For a full-rank L R L^T, det A = det R (L unit lower): a closed form."""
    p = 65521
    for seed in range(3):
        A, rpm = inputs.rank_profile_matrix_input(24, p, 10, 7, 300 + seed)
        assert orc.det(A, p) == det_indep(A, p)


@pytest.mark.parametrize("p", [3, 65521, 8388593])
def test_solve_nonsingular_cramer(p):
    """x_i = det(A with column i replaced by b) / det(A) (Cramer), Python integers."""
    g = inputs.rng(91 + p)
    done = 0
    while done < 5:
        n = int(g.integers(1, 7))
        A = g.integers(0, p, size=(n, n)).astype(np.uint32)
        d = det_indep(A, p)
        if d == 0:
            continue
        b = g.integers(0, p, size=n).astype(np.uint32)
        X, cons = orc.solve(A, p, b)
        assert cons[0] == 1
        dinv = pow(d, p - 2, p)
        for i in range(n):
            Ai = A.copy()
            Ai[:, i] = b
            assert int(X[i, 0]) == det_indep(Ai, p) * dinv % p
        done += 1


@pytest.mark.parametrize("p", [2, 65521])
def test_solve_singular_consistency(p):
    g = inputs.rng(5 + p)
    for seed in range(4):
        A, _ = inputs.rank_profile_matrix_input(20, p, 6, 4, 400 + seed)   # rank 14
        y = g.integers(0, p, size=(20, 3)).astype(np.uint32)
        B = (A.astype(object) @ y.astype(object)) % p                       # in the range
        X, cons = orc.solve(A, p, B.astype(np.uint32))
        assert (cons == 1).all()
        assert ((A.astype(object) @ X.astype(object)) % p == B).all()
        # b + e_j leaves the range for some j (A has rank 14 < 20): the rank of [A | b] grows
        found = False
        for j in range(20):
            cand = B[:, 0].astype(np.int64)
            cand[j] = (cand[j] + 1) % p
            cand = cand.astype(np.uint32)
            if orc.rank(np.concatenate([A, cand.reshape(20, 1)], axis=1), p) > 14:
                Xb, cb = orc.solve(A, p, cand)
                assert cb[0] == 0
                found = True
                break
        assert found
