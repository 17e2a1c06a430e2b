/*
 * pldl_oracle.c -- plain CPU oracle (test infrastructure only; see the header).
 *
 * Arithmetic: residues in [0,p) held in uint32, products in uint64 reduced with
 * '%' at once.  Nothing here is tuned; the only concession to size is an OpenMP
 * loop over the rows of a trailing update, which does not change any result.
 */
#include "pldl_oracle.h"
#include <stdlib.h>
#include <string.h>

typedef uint32_t u32;
typedef uint64_t u64;

static inline u32 m_add(u32 a, u32 b, u32 p) { u64 s = (u64)a + b; return (u32)(s % p); }
static inline u32 m_sub(u32 a, u32 b, u32 p) { return (u32)(((u64)a + p - b) % p); }
static inline u32 m_mul(u32 a, u32 b, u32 p) { return (u32)(((u64)a * b) % p); }

/* Extended Euclid on signed 64-bit integers. */
u32 orc_inv(u32 a, u32 p) {
    int64_t r0 = p, r1 = a % p, s0 = 0, s1 = 1;
    while (r1 != 0) {
        int64_t q = r0 / r1, t;
        t = r0 - q * r1; r0 = r1; r1 = t;
        t = s0 - q * s1; s0 = s1; s1 = t;
    }
    /* r0 == gcd == 1 for a != 0 and p prime */
    s0 %= (int64_t)p;
    if (s0 < 0) s0 += p;
    return (u32)s0;
}

/* ------------------------------------------------------------------------ */
/* Textbook rank: forward elimination choosing, column by column, the first  */
/* row at or below the current one with a nonzero entry.                     */
int64_t orc_rank(u32 p, int64_t m, int64_t n, const u32 *A, int64_t lda) {
    u32 *W = (u32 *)malloc(sizeof(u32) * (size_t)(m * n > 0 ? m * n : 1));
    if (!W) return -1;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) W[i * n + j] = A[i * lda + j] % p;
    int64_t r = 0;
    for (int64_t c = 0; c < n && r < m; ++c) {
        int64_t piv = -1;
        for (int64_t i = r; i < m; ++i)
            if (W[i * n + c]) { piv = i; break; }
        if (piv < 0) continue;
        if (piv != r)
            for (int64_t j = 0; j < n; ++j) { u32 t = W[r * n + j]; W[r * n + j] = W[piv * n + j]; W[piv * n + j] = t; }
        u32 inv = orc_inv(W[r * n + c], p);
        for (int64_t i = r + 1; i < m; ++i) {
            u32 f = m_mul(W[i * n + c], inv, p);
            if (!f) continue;
            for (int64_t j = c; j < n; ++j) W[i * n + j] = m_sub(W[i * n + j], m_mul(f, W[r * n + j], p), p);
        }
        ++r;
    }
    free(W);
    return r;
}

/* For every row count a, rank(A[0:a, 0:b]) for all b is the number of columns
 * among the first b that are independent of the columns before them; that is
 * found by reducing each column of the a x n prefix against the reduced columns
 * kept so far (column-by-column Gaussian elimination of the prefix). */
int orc_leading_ranks(u32 p, int64_t n, const u32 *A, int64_t lda, int64_t *r) {
    int64_t N1 = n + 1;
    for (int64_t b = 0; b <= n; ++b) r[0 * N1 + b] = 0;
    u32 *basis = (u32 *)malloc(sizeof(u32) * (size_t)(n * n > 0 ? n * n : 1)); /* kept columns, length a */
    int64_t *lead = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1)); /* leading row of each kept column */
    u32 *v = (u32 *)malloc(sizeof(u32) * (size_t)(n > 0 ? n : 1));
    if (!basis || !lead || !v) { free(basis); free(lead); free(v); return -1; }
    for (int64_t a = 1; a <= n; ++a) {
        int64_t nb = 0;
        r[a * N1 + 0] = 0;
        for (int64_t b = 0; b < n; ++b) {
            for (int64_t i = 0; i < a; ++i) v[i] = A[i * lda + b] % p;
            for (int64_t t = 0; t < nb; ++t) {
                u32 *w = basis + t * n;
                u32 f = v[lead[t]];           /* kept column t has w[lead[t]] = 1 */
                if (!f) continue;
                for (int64_t i = 0; i < a; ++i) v[i] = m_sub(v[i], m_mul(f, w[i], p), p);
            }
            int64_t ld = -1;
            for (int64_t i = 0; i < a; ++i) if (v[i]) { ld = i; break; }
            if (ld >= 0) {
                u32 inv = orc_inv(v[ld], p);
                u32 *w = basis + nb * n;
                for (int64_t i = 0; i < a; ++i) w[i] = m_mul(v[i], inv, p);
                /* keep the basis reduced at its leading rows */
                for (int64_t t = 0; t < nb; ++t) {
                    u32 *o = basis + t * n;
                    u32 f = o[ld];
                    if (!f) continue;
                    for (int64_t i = 0; i < a; ++i) o[i] = m_sub(o[i], m_mul(f, w[i], p), p);
                }
                lead[nb++] = ld;
            }
            r[a * N1 + b + 1] = nb;
        }
    }
    free(basis); free(lead); free(v);
    return 0;
}

int orc_rpm_bruteforce(u32 p, int64_t n, const u32 *A, int64_t lda, int32_t *rpm) {
    int64_t N1 = n + 1;
    int64_t *r = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N1 * N1));
    if (!r) return -1;
    if (orc_leading_ranks(p, n, A, lda, r)) { free(r); return -1; }
    int rc = 0;
    for (int64_t i = 0; i < n; ++i) rpm[i] = -1;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            int64_t e = r[(i + 1) * N1 + j + 1] - r[i * N1 + j + 1] - r[(i + 1) * N1 + j] + r[i * N1 + j];
            if (e == 1) {
                if (rpm[i] != -1) rc = -2;
                rpm[i] = (int32_t)j;
            } else if (e != 0) rc = -2;
        }
    free(r);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Elimination shared by search and replay.                                  */
/* S is the full symmetric Schur complement in original coordinates; Lo holds */
/* L in original coordinates: Lo[k][c] is the multiplier of row k for the     */
/* pivot column owned by original index c.                                   */

typedef struct {
    u32 p; int64_t n;
    u32 *S;      /* n*n */
    u32 *Lo;     /* n*n */
    char *alive; /* 1 = not yet eliminated nor set aside */
    u32 *dx, *dy;/* per original index: D block data (see below) */
} elim_t;

static int elim_init(elim_t *E, u32 p, int64_t n, const u32 *A, int64_t lda) {
    E->p = p; E->n = n;
    size_t nn = (size_t)(n * n > 0 ? n * n : 1);
    E->S = (u32 *)malloc(sizeof(u32) * nn);
    E->Lo = (u32 *)calloc(nn, sizeof(u32));
    E->alive = (char *)malloc((size_t)(n > 0 ? n : 1));
    if (!E->S || !E->Lo || !E->alive) return -1;
    /* the lower triangle of A defines the symmetric matrix */
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            u32 v = A[i * lda + j] % p;
            E->S[i * n + j] = v; E->S[j * n + i] = v;
        }
    for (int64_t i = 0; i < n; ++i) { E->alive[i] = 1; E->Lo[i * n + i] = 1; }
    return 0;
}
static void elim_free(elim_t *E) { free(E->S); free(E->Lo); free(E->alive); }

/* 1x1 pivot at original index i (Section 5: x = diagonal entry, the column is
 * scaled by x^{-1}, the Schur complement loses L D L^T of that column). */
static void elim_1x1(elim_t *E, int64_t i) {
    u32 p = E->p; int64_t n = E->n; u32 *S = E->S;
    u32 x = S[i * n + i], xi = orc_inv(x, p);
    E->alive[i] = 0;
    for (int64_t k = 0; k < n; ++k)
        if (E->alive[k]) E->Lo[k * n + i] = m_mul(S[k * n + i], xi, p);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        if (!E->alive[k]) continue;
        u32 bk = E->Lo[k * n + i];
        if (!bk) continue;
        for (int64_t l = 0; l < n; ++l)
            if (E->alive[l]) S[k * n + l] = m_sub(S[k * n + l], m_mul(bk, S[l * n + i], p), p);
    }
    for (int64_t k = 0; k < n; ++k) { S[k * n + i] = 0; S[i * n + k] = 0; }
}

/* 2x2 pivot on the pair (i, j), S[i][i] = 0, x = S[i][j] != 0, y = S[j][j].
 * Section 5 (odd p: y' = y/2, D block [[0,x],[x,0]], L[j][i] = y'/x;
 * p = 2: D block [[0,x],[x,y]], L[j][i] = 0); the multipliers of a remaining
 * row k are  b_k = S[k][i]/x  (column of j)  and  a_k = (S[k][j] - w b_k)/x
 * (column of i) with w = y/2 (odd) or y (p = 2); the Schur complement then
 * loses [a b] D [a b]^T. */
static void elim_2x2(elim_t *E, int64_t i, int64_t j) {
    u32 p = E->p; int64_t n = E->n; u32 *S = E->S;
    u32 x = S[i * n + j], y = S[j * n + j], xi = orc_inv(x, p);
    u32 w, d22;
    if (p == 2) { w = y; d22 = y; E->Lo[j * n + i] = 0; }
    else {
        u32 half = (u32)(((u64)p + 1) / 2);
        w = m_mul(y, half, p); d22 = 0;
        E->Lo[j * n + i] = m_mul(w, xi, p);
    }
    E->alive[i] = 0; E->alive[j] = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (!E->alive[k]) continue;
        u32 b = m_mul(S[k * n + i], xi, p);
        u32 a = m_mul(m_sub(S[k * n + j], m_mul(w, b, p), p), xi, p);
        E->Lo[k * n + j] = b;
        E->Lo[k * n + i] = a;
    }
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        if (!E->alive[k]) continue;
        u32 ak = E->Lo[k * n + i], bk = E->Lo[k * n + j];
        for (int64_t l = 0; l < n; ++l) {
            if (!E->alive[l]) continue;
            u32 al = E->Lo[l * n + i], bl = E->Lo[l * n + j];
            /* [a_k b_k] [[0,x],[x,d22]] [a_l b_l]^T */
            u32 t = m_add(m_mul(ak, bl, p), m_mul(bk, al, p), p);
            t = m_add(m_mul(x, t, p), m_mul(d22, m_mul(bk, bl, p), p), p);
            S[k * n + l] = m_sub(S[k * n + l], t, p);
        }
    }
    for (int64_t k = 0; k < n; ++k) { S[k * n + i] = 0; S[i * n + k] = 0; S[k * n + j] = 0; S[j * n + k] = 0; }
}

/* Write L (position coordinates) and D from the order of pivots. */
static void elim_output(elim_t *E, const int32_t *perm, int64_t rank, const char *blk2,
                        const u32 *bx, const u32 *by, u32 *L, int64_t ldl, u32 *dd, u32 *de) {
    int64_t n = E->n;
    for (int64_t q = 0; q < n; ++q) {
        for (int64_t c = 0; c < n; ++c) {
            u32 v = 0;
            if (c == q) v = 1;
            else if (c < q && c < rank) v = E->Lo[(int64_t)perm[q] * n + perm[c]];
            L[q * ldl + c] = v;
        }
    }
    for (int64_t q = 0; q < n; ++q) { dd[q] = 0; de[q] = 0; }
    for (int64_t q = 0; q < rank;) {
        if (blk2[q]) {
            de[q] = bx[q];
            dd[q] = 0;
            dd[q + 1] = (E->p == 2) ? by[q] : 0;
            q += 2;
        } else {
            dd[q] = bx[q];
            q += 1;
        }
    }
}

int orc_search(u32 p, int64_t n, const u32 *A, int64_t lda, int32_t *perm, u32 *L, int64_t ldl,
               u32 *dd, u32 *de, int32_t *rpm, int64_t *rank_out) {
    elim_t E;
    if (elim_init(&E, p, n, A, lda)) { elim_free(&E); return -1; }
    int32_t *zeros = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    char *blk2 = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    u32 *bx = (u32 *)calloc((size_t)(n > 0 ? n : 1), sizeof(u32));
    u32 *by = (u32 *)calloc((size_t)(n > 0 ? n : 1), sizeof(u32));
    if (!zeros || !blk2 || !bx || !by) { free(zeros); free(blk2); free(bx); free(by); elim_free(&E); return -1; }
    int64_t r = 0, nz = 0;
    for (int64_t i = 0; i < n; ++i) rpm[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (!E.alive[i]) continue;                 /* consumed as the partner of a 2x2 block */
        int64_t j = -1;
        for (int64_t c = i; c < n; ++c)
            if (E.alive[c] && E.S[i * n + c]) { j = c; break; }
        if (j < 0) {                               /* zero row: set aside, precedence kept */
            E.alive[i] = 0;
            zeros[nz++] = (int32_t)i;
        } else if (j == i) {
            bx[r] = E.S[i * n + i];
            perm[r] = (int32_t)i; rpm[i] = (int32_t)i;
            elim_1x1(&E, i);
            r += 1;
        } else {
            bx[r] = E.S[i * n + j]; by[r] = E.S[j * n + j]; blk2[r] = 1;
            perm[r] = (int32_t)i; perm[r + 1] = (int32_t)j;
            rpm[i] = (int32_t)j; rpm[j] = (int32_t)i;
            elim_2x2(&E, i, j);
            r += 2;
        }
    }
    for (int64_t t = 0; t < nz; ++t) perm[r + t] = zeros[t];
    elim_output(&E, perm, r, blk2, bx, by, L, ldl, dd, de);
    *rank_out = r;
    free(zeros); free(blk2); free(bx); free(by); elim_free(&E);
    return 0;
}

int orc_replay(u32 p, int64_t n, const u32 *A, int64_t lda, const int32_t *perm, const int32_t *rpm,
               int64_t rank, u32 *L, int64_t ldl, u32 *dd, u32 *de) {
    if (rank < 0 || rank > n) return -2;
    char *seen = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!seen) return -1;
    for (int64_t q = 0; q < n; ++q) {
        if (perm[q] < 0 || perm[q] >= n || seen[perm[q]]) { free(seen); return -2; }
        seen[perm[q]] = 1;
    }
    free(seen);
    for (int64_t q = rank; q < n; ++q)
        if (rpm[perm[q]] != -1) return -7;
    elim_t E;
    if (elim_init(&E, p, n, A, lda)) { elim_free(&E); return -1; }
    char *blk2 = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    u32 *bx = (u32 *)calloc((size_t)(n > 0 ? n : 1), sizeof(u32));
    u32 *by = (u32 *)calloc((size_t)(n > 0 ? n : 1), sizeof(u32));
    int rc = 0;
    if (!blk2 || !bx || !by) rc = -1;
    for (int64_t q = 0; q < rank && rc == 0;) {
        int64_t i = perm[q];
        if (rpm[i] == i) {
            if (E.S[i * n + i] == 0) { rc = -4; break; }
            bx[q] = E.S[i * n + i];
            elim_1x1(&E, i);
            q += 1;
        } else {
            if (q + 1 >= rank || rpm[i] < 0 || perm[q + 1] != rpm[i] || rpm[rpm[i]] != i) { rc = -3; break; }
            int64_t j = perm[q + 1];
            if (E.S[i * n + i] != 0 || E.S[i * n + j] == 0) { rc = -5; break; }
            bx[q] = E.S[i * n + j]; by[q] = E.S[j * n + j]; blk2[q] = 1;
            elim_2x2(&E, i, j);
            q += 2;
        }
    }
    if (rc == 0) {
        for (int64_t a = rank; a < n && rc == 0; ++a)
            for (int64_t b = rank; b < n; ++b)
                if (E.S[(int64_t)perm[a] * n + perm[b]]) { rc = -6; break; }
    }
    if (rc == 0) elim_output(&E, perm, rank, blk2, bx, by, L, ldl, dd, de);
    free(blk2); free(bx); free(by); elim_free(&E);
    return rc;
}

int orc_reconstruct(u32 p, int64_t n, const int32_t *perm, const u32 *L, int64_t ldl,
                    const u32 *dd, const u32 *de, u32 *Out, int64_t ldo) {
    /* T = L D (D symmetric tridiagonal), then B = T L^T, then Out[perm[a]][perm[b]] = B[a][b] */
    size_t nn = (size_t)(n * n > 0 ? n * n : 1);
    u32 *T = (u32 *)malloc(sizeof(u32) * nn);
    if (!T) return -1;
    for (int64_t a = 0; a < n; ++a)
        for (int64_t c = 0; c < n; ++c) {
            u32 t = m_mul(L[a * ldl + c], dd[c], p);
            if (c + 1 < n) t = m_add(t, m_mul(L[a * ldl + c + 1], de[c], p), p);   /* D[c+1][c] */
            if (c > 0) t = m_add(t, m_mul(L[a * ldl + c - 1], de[c - 1], p), p);   /* D[c-1][c] */
            T[a * n + c] = t;
        }
    #pragma omp parallel for schedule(dynamic, 8)
    for (int64_t a = 0; a < n; ++a)
        for (int64_t b = 0; b < n; ++b) {
            u32 s = 0;
            for (int64_t c = 0; c < n; ++c) s = m_add(s, m_mul(T[a * n + c], L[b * ldl + c], p), p);
            Out[(int64_t)perm[a] * ldo + perm[b]] = s;
        }
    free(T);
    return 0;
}

int orc_char2_standard(int64_t n, int32_t *perm, u32 *L, int64_t ldl, u32 *dd, u32 *de) {
    const u32 p = 2;
    for (int64_t q = 0; q + 1 < n; ++q) {
        if (!de[q]) continue;
        u32 c = de[q], d = dd[q + 1];
        if (d) {
            int32_t t = perm[q]; perm[q] = perm[q + 1]; perm[q + 1] = t;
            for (int64_t c2 = 0; c2 < n; ++c2) { u32 s = L[q * ldl + c2]; L[q * ldl + c2] = L[(q + 1) * ldl + c2]; L[(q + 1) * ldl + c2] = s; }
            for (int64_t r = 0; r < n; ++r) { u32 s = L[r * ldl + q]; L[r * ldl + q] = L[r * ldl + q + 1]; L[r * ldl + q + 1] = s; }
            u32 f = m_mul(c, orc_inv(d, p), p);
            for (int64_t r = 0; r < n; ++r) L[r * ldl + q] = m_add(L[r * ldl + q], m_mul(f, L[r * ldl + q + 1], p), p);
            dd[q] = d;
            dd[q + 1] = m_mul(m_mul(c, c, p), orc_inv(d, p), p);  /* -c^2/d == c^2/d mod 2 */
            de[q] = 0;
        }
        ++q;  /* skip the second position of the block */
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
int orc_gemm(u32 p, int64_t m, int64_t n, int64_t k, const u32 *A, int64_t lda, const u32 *B, int64_t ldb,
             u32 *C, int64_t ldc) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            u32 s = C[i * ldc + j] % p;
            for (int64_t t = 0; t < k; ++t) s = m_sub(s, m_mul(A[i * lda + t], B[t * ldb + j], p), p);
            C[i * ldc + j] = s;
        }
    return 0;
}

int orc_trsm_left(u32 p, int lower, int64_t m, int64_t n, const u32 *T, int64_t ldt, u32 *B, int64_t ldb) {
    for (int64_t j = 0; j < n; ++j) {
        if (lower) {
            for (int64_t i = 0; i < m; ++i) {
                u32 s = B[i * ldb + j] % p;
                for (int64_t t = 0; t < i; ++t) s = m_sub(s, m_mul(T[i * ldt + t], B[t * ldb + j], p), p);
                B[i * ldb + j] = s;
            }
        } else {
            for (int64_t i = m - 1; i >= 0; --i) {
                u32 s = B[i * ldb + j] % p;
                for (int64_t t = i + 1; t < m; ++t) s = m_sub(s, m_mul(T[i * ldt + t], B[t * ldb + j], p), p);
                B[i * ldb + j] = s;
            }
        }
    }
    return 0;
}

/* (A D)[i][c] for a block diagonal D given by (dd, de) */
static u32 ad_entry(u32 p, int64_t k, const u32 *Ai, const u32 *dd, const u32 *de, int64_t c) {
    u32 t = m_mul(Ai[c], dd[c], p);
    if (c + 1 < k) t = m_add(t, m_mul(Ai[c + 1], de[c], p), p);
    if (c > 0) t = m_add(t, m_mul(Ai[c - 1], de[c - 1], p), p);
    return t;
}

int orc_syrdk(u32 p, int64_t n, int64_t k, const u32 *A, int64_t lda, const u32 *dd, const u32 *de,
              u32 *C, int64_t ldc) {
    #pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            u32 s = C[i * ldc + j] % p;
            for (int64_t c = 0; c < k; ++c)
                s = m_sub(s, m_mul(ad_entry(p, k, A + i * lda, dd, de, c), A[j * lda + c], p), p);
            C[i * ldc + j] = s;
        }
    return 0;
}

int orc_syrd2k(u32 p, int64_t n, int64_t k, const u32 *A, int64_t lda, const u32 *B, int64_t ldb,
               const u32 *dd, const u32 *de, u32 *C, int64_t ldc) {
    #pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            u32 s = C[i * ldc + j] % p;
            for (int64_t c = 0; c < k; ++c) {
                s = m_sub(s, m_mul(ad_entry(p, k, A + i * lda, dd, de, c), B[j * ldb + c], p), p);
                s = m_sub(s, m_mul(ad_entry(p, k, B + i * ldb, dd, de, c), A[j * lda + c], p), p);
            }
            C[i * ldc + j] = s;
        }
    return 0;
}

/* Entry (i, j), i <= j, of X^T U + U^T X with X, U upper and U unit:
 *   sum_{t<=i} X[t][i] U[t][j] + sum_{t<=i} U[t][i] X[t][j].
 * The only occurrence of X[i][j] (i < j) is the term t = i of the second sum
 * (U[i][i] = 1); for i = j, X[j][j] appears twice.  Solving the equations in
 * the order (column j ascending, row i ascending) uses only known entries. */
int orc_trss(u32 p, int64_t n, const u32 *U, int64_t ldu, const u32 *C, int64_t ldc, u32 *X, int64_t ldx) {
    if (p == 2)
        for (int64_t i = 0; i < n; ++i) if (C[i * ldc + i] % 2) return -2;
    for (int64_t i = 0; i < n; ++i) for (int64_t j = 0; j < n; ++j) X[i * ldx + j] = 0;
    u32 half = (u32)(((u64)p + 1) / 2);
    #define UU(a, b) ((a) == (b) ? 1u : ((a) < (b) ? U[(a) * ldu + (b)] % p : 0u))
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < j; ++i) {
            u32 cij = C[j * ldc + i] % p;               /* lower triangle holds C[j][i] = C[i][j] */
            u32 s = 0;
            for (int64_t t = 0; t <= i; ++t) s = m_add(s, m_mul(X[t * ldx + i], UU(t, j), p), p);
            for (int64_t t = 0; t < i; ++t) s = m_add(s, m_mul(UU(t, i), X[t * ldx + j], p), p);
            X[i * ldx + j] = m_sub(cij, s, p);
        }
        if (p == 2) { X[j * ldx + j] = 0; continue; }
        u32 s = 0;
        for (int64_t t = 0; t < j; ++t) s = m_add(s, m_mul(X[t * ldx + j], UU(t, j), p), p);
        /* C_jj = 2 s + 2 X_jj */
        X[j * ldx + j] = m_sub(m_mul(C[j * ldc + j] % p, half, p), s, p);
    }
    #undef UU
    return 0;
}

int orc_plduq(u32 p, int64_t m, int64_t n, const u32 *Y, int64_t ldy, int32_t *rows, int32_t *cols,
              u32 *LU, int64_t ldlu, int64_t *rank_out) {
    size_t mn = (size_t)(m * n > 0 ? m * n : 1);
    u32 *W = (u32 *)malloc(sizeof(u32) * mn);        /* Schur complement, original coordinates */
    u32 *Lc = (u32 *)calloc(mn, sizeof(u32));        /* Lc[i][t]: multiplier of row i for pivot t */
    int32_t *prow = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
    int32_t *pcol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
    u32 *pv = (u32 *)malloc(sizeof(u32) * (size_t)(m + 1));
    u32 *Ur = (u32 *)calloc((size_t)((m + 1) * (n > 0 ? n : 1)), sizeof(u32)); /* U rows, original column coords */
    char *ispr = (char *)calloc((size_t)(m + 1), 1), *ispc = (char *)calloc((size_t)(n + 1), 1);
    if (!W || !Lc || !prow || !pcol || !pv || !Ur || !ispr || !ispc) return -1;
    for (int64_t i = 0; i < m; ++i) for (int64_t j = 0; j < n; ++j) W[i * n + j] = Y[i * ldy + j] % p;
    int64_t r = 0;
    for (int64_t i = 0; i < m; ++i) {
        int64_t c = -1;
        for (int64_t j = 0; j < n; ++j) if (W[i * n + j]) { c = j; break; }
        if (c < 0) continue;
        u32 x = W[i * n + c], xi = orc_inv(x, p);
        prow[r] = (int32_t)i; pcol[r] = (int32_t)c; pv[r] = x; ispr[i] = 1; ispc[c] = 1;
        for (int64_t j = 0; j < n; ++j) Ur[r * n + j] = m_mul(W[i * n + j], xi, p);
        for (int64_t k = i + 1; k < m; ++k) {
            u32 f = m_mul(W[k * n + c], xi, p);
            Lc[k * n + r] = f;
            if (!f) continue;
            for (int64_t j = 0; j < n; ++j) W[k * n + j] = m_sub(W[k * n + j], m_mul(f, W[i * n + j], p), p);
        }
        ++r;
    }
    int64_t a = 0;
    for (int64_t t = 0; t < r; ++t) rows[a++] = prow[t];
    for (int64_t i = 0; i < m; ++i) if (!ispr[i]) rows[a++] = (int32_t)i;
    int64_t b = 0;
    for (int64_t t = 0; t < r; ++t) cols[b++] = pcol[t];
    for (int64_t j = 0; j < n; ++j) if (!ispc[j]) cols[b++] = (int32_t)j;
    for (int64_t aa = 0; aa < m; ++aa)
        for (int64_t bb = 0; bb < n; ++bb) {
            u32 v = 0;
            if (aa == bb && aa < r) v = pv[aa];
            else if (bb < aa && bb < r) v = Lc[(int64_t)rows[aa] * n + bb];
            else if (aa < bb && aa < r) v = Ur[aa * n + cols[bb]];
            LU[aa * ldlu + bb] = v;
        }
    *rank_out = r;
    free(W); free(Lc); free(prow); free(pcol); free(pv); free(Ur); free(ispr); free(ispc);
    return 0;
}

int orc_delta(u32 p, int64_t r, const u32 *U, int64_t ldu, const u32 *C, int64_t ldc, u32 *delta) {
    for (int64_t i = 0; i < r; ++i) {
        u32 s = C[i * ldc + i] % p;
        for (int64_t j = 0; j < i; ++j) {
            u32 u = U[j * ldu + i] % p;
            s = m_sub(s, m_mul(delta[j], m_mul(u, u, p), p), p);
        }
        delta[i] = s;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Determinant: reduce to upper triangular form with row exchanges (each one */
/* flips the sign); det = sign * product of the pivots.                      */
int orc_det(u32 p, int64_t n, const u32 *A, int64_t lda, u32 *det) {
    u32 *W = (u32 *)malloc(sizeof(u32) * (size_t)(n * n > 0 ? n * n : 1));
    if (!W) return -1;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) W[i * n + j] = A[i * lda + j] % p;
    u32 d = 1 % p;
    for (int64_t c = 0; c < n; ++c) {
        int64_t piv = -1;
        for (int64_t i = c; i < n; ++i)
            if (W[i * n + c]) { piv = i; break; }
        if (piv < 0) { d = 0; break; }
        if (piv != c) {
            for (int64_t j = 0; j < n; ++j) { u32 t = W[c * n + j]; W[c * n + j] = W[piv * n + j]; W[piv * n + j] = t; }
            d = m_sub(0, d, p);
        }
        d = m_mul(d, W[c * n + c], p);
        u32 inv = orc_inv(W[c * n + c], p);
        #pragma omp parallel for schedule(static)
        for (int64_t i = c + 1; i < n; ++i) {
            u32 f = m_mul(W[i * n + c], inv, p);
            if (!f) continue;
            for (int64_t j = c; j < n; ++j) W[i * n + j] = m_sub(W[i * n + j], m_mul(f, W[c * n + j], p), p);
        }
    }
    free(W);
    *det = d;
    return 0;
}

/* Solve A X = B: Gauss-Jordan elimination of [A | B] to reduced row echelon */
/* form (pivot columns found left to right, the first nonzero row below the   */
/* current one as pivot row), then read each column's solution off it.        */
int orc_solve(u32 p, int64_t n, const u32 *A, int64_t lda, const u32 *B, int64_t ldb, int64_t nrhs, u32 *X,
              int64_t ldx, int32_t *cons) {
    const int64_t w = n + nrhs;
    u32 *W = (u32 *)malloc(sizeof(u32) * (size_t)(n * w > 0 ? n * w : 1));
    int64_t *pc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!W || !pc) { free(W); free(pc); return -1; }
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) W[i * w + j] = A[i * lda + j] % p;
        for (int64_t k = 0; k < nrhs; ++k) W[i * w + n + k] = B[i * ldb + k] % p;
    }
    int64_t r = 0;
    for (int64_t c = 0; c < n && r < n; ++c) {
        int64_t piv = -1;
        for (int64_t i = r; i < n; ++i)
            if (W[i * w + c]) { piv = i; break; }
        if (piv < 0) continue;
        if (piv != r)
            for (int64_t j = 0; j < w; ++j) { u32 t = W[r * w + j]; W[r * w + j] = W[piv * w + j]; W[piv * w + j] = t; }
        u32 inv = orc_inv(W[r * w + c], p);
        for (int64_t j = c; j < w; ++j) W[r * w + j] = m_mul(W[r * w + j], inv, p);
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            if (i == r) continue;
            u32 f = W[i * w + c];
            if (!f) continue;
            for (int64_t j = c; j < w; ++j) W[i * w + j] = m_sub(W[i * w + j], m_mul(f, W[r * w + j], p), p);
        }
        pc[r] = c;
        ++r;
    }
    for (int64_t k = 0; k < nrhs; ++k) {
        int32_t ok = 1;
        for (int64_t i = r; i < n; ++i)
            if (W[i * w + n + k]) { ok = 0; break; }
        cons[k] = ok;
        for (int64_t j = 0; j < n; ++j) X[j * ldx + k] = 0;
        if (ok)
            for (int64_t i = 0; i < r; ++i) X[pc[i] * ldx + k] = W[i * w + n + k];
    }
    free(W); free(pc);
    return 0;
}
