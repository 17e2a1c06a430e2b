/* Host memory-safety check of the C oracle: every oracle routine runs on seeded
 * random inputs (five primes, characteristic 2 included, orders 0..40, dense,
 * sparse and zero-diagonal symmetric matrices) in a program built with
 * AddressSanitizer and UndefinedBehaviorSanitizer.  The factorization is also
 * checked against itself: the replay of its own pivot order succeeds, P L D L^T P^T
 * gives A back, and on small orders the rank profile matrix equals the one of
 * Theorem 1 by brute force.  Exit 0 and "ok" when nothing was reported. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "pldl_oracle.h"

static uint64_t s = 88172645463325252ull;
static uint32_t rnd(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return (uint32_t)s; }
static uint32_t* mat(int64_t r, int64_t c, uint32_t p) {
    uint32_t* a = malloc((size_t)(r * c + 1) * 4);
    for (int64_t i = 0; i < r * c; ++i) a[i] = rnd() % p;
    return a;
}

static int factorizations(void) {
    const uint32_t ps[] = {2, 3, 65521, 8388593, 16777213};
    int bad = 0;
    for (int pi = 0; pi < 5; ++pi) for (int n = 0; n <= 40; n += 7) for (int mode = 0; mode < 3; ++mode) {
        uint32_t p = ps[pi];
        uint32_t *A = calloc((size_t)n * n + 1, 4), *L = calloc((size_t)n * n + 1, 4), *O = calloc((size_t)n * n + 1, 4);
        uint32_t *dd = calloc(n + 1, 4), *de = calloc(n + 1, 4), *L2 = calloc((size_t)n * n + 1, 4), *dd2 = calloc(n + 1, 4), *de2 = calloc(n + 1, 4);
        int32_t *perm = calloc(n + 1, 4), *rpm = calloc(n + 1, 4), *rb = calloc(n + 1, 4);
        for (int i = 0; i < n; ++i) for (int j = 0; j <= i; ++j) {
            uint32_t v = rnd() % p;
            if (mode == 1 && (i % 3 == 0 || j % 2 == 0)) v = 0;
            if (mode == 2 && i == j) v = 0;
            A[i * n + j] = A[j * n + i] = v;
        }
        int64_t r = -1;
        orc_search(p, n, A, n ? n : 1, perm, L, n ? n : 1, dd, de, rpm, &r);
        if (orc_replay(p, n, A, n ? n : 1, perm, rpm, r, L2, n ? n : 1, dd2, de2) != 0) bad++;
        orc_reconstruct(p, n, perm, L, n ? n : 1, dd, de, O, n ? n : 1);
        if (n && memcmp(O, A, (size_t)n * n * 4)) bad++;
        if (n <= 21) { orc_rpm_bruteforce(p, n, A, n ? n : 1, rb); if (n && memcmp(rb, rpm, n * 4)) bad++; }
        if (p == 2) orc_char2_standard(n, perm, L, n ? n : 1, dd, de);
        free(A); free(L); free(O); free(dd); free(de); free(L2); free(dd2); free(de2); free(perm); free(rpm); free(rb);
    }
    return bad;
}

static void building_blocks(void) {
    const uint32_t ps[] = {2, 3, 65521, 8388593, 16777213};
    for (int pi = 0; pi < 5; ++pi) for (int m = 1; m <= 33; m += 8) for (int n = 1; n <= 29; n += 7) for (int k = 1; k <= 19; k += 6) {
        uint32_t p = ps[pi];
        uint32_t *A = mat(m, k, p), *B = mat(k, n, p), *C = mat(m, n, p);
        orc_gemm(p, m, n, k, A, k, B, n, C, n);
        uint32_t *T = mat(m, m, p), *X = mat(m, n, p);
        orc_trsm_left(p, 1, m, n, T, m, X, n); orc_trsm_left(p, 0, m, n, T, m, X, n);
        uint32_t *G = mat(m, k, p), *H = mat(m, k, p), *dd = mat(k, 1, p), *de = mat(k, 1, p), *S = mat(m, m, p);
        /* 2x2 blocks may start at even positions only: no two overlap */
        for (int q = 0; q < k; q += 2) de[q + 1 < k ? q + 1 : q] = 0;
        de[k - 1] = 0;
        orc_syrdk(p, m, k, G, k, dd, de, S, m); orc_syrd2k(p, m, k, G, k, H, k, dd, de, S, m);
        uint32_t *U = mat(m, m, p), *Cs = mat(m, m, p), *Xs = mat(m, m, p), *dl = mat(m, 1, p);
        for (int i = 0; i < m; ++i) { for (int j = 0; j < i; ++j) Cs[j * m + i] = Cs[i * m + j]; if (p == 2) Cs[i * m + i] = 0; }
        orc_trss(p, m, U, m, Cs, m, Xs, m);
        orc_delta(p, m, U, m, Cs, m, dl);
        int32_t *rows = malloc((m + 1) * 4), *cols = malloc((n + 1) * 4), *cons = malloc((n + 1) * 4);
        uint32_t* LU = mat(m, n, p); int64_t r;
        orc_plduq(p, m, n, C, n, rows, cols, LU, n, &r);
        uint32_t det; uint32_t* Q = mat(m, m, p); uint32_t* R = mat(m, n, p); uint32_t* Y = mat(m, n, p);
        orc_det(p, m, Q, m, &det); orc_solve(p, m, Q, m, R, n, n, Y, n, cons);
        orc_rank(p, m, n, C, n);
        free(A); free(B); free(C); free(T); free(X); free(G); free(H); free(dd); free(de); free(S); free(U); free(Cs); free(Xs);
        free(dl); free(rows); free(cols); free(cons); free(LU); free(Q); free(R); free(Y);
    }
    }

int main(void) {
    const int bad = factorizations();
    building_blocks();
    printf(bad ? "mismatches: %d\n" : "ok\n", bad);
    return bad != 0;
}
