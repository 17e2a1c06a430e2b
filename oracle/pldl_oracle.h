/*
 * pldl_oracle.h -- plain CPU oracle for the symmetric PLDL^TP^T factorization
 * over a prime field F_p that reveals the rank profile matrix
 * (Dumas & Pernet, "Symmetric indefinite triangular factorization revealing
 * the rank profile matrix").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the checker: only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  The GPU
 * library shares no code, header, table or helper with it.
 *
 * Every routine is a direct, slow, scalar transcription of a definition:
 *   - arithmetic is exact: residues are uint32 in [0, p), every product is
 *     formed in uint64 and reduced with '%' immediately;
 *   - p must be prime and below 2^31 (the caller checks primality);
 *   - matrices are row-major with an explicit leading dimension;
 *   - no blocking, no fusion, no reordering beyond what the definition states.
 *
 * Return codes: 0 = success, negative = the definition cannot be met on this
 * input (documented per routine), -1 = allocation failure.
 */
#ifndef PLDL_ORACLE_H
#define PLDL_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* ---- field ------------------------------------------------------------- */
uint32_t orc_inv(uint32_t a, uint32_t p);  /* a^{-1} mod p, a != 0 */

/* ---- reference linear algebra (definitions) ---------------------------- */

/* Rank of the m x n matrix A by textbook Gaussian elimination. */
int64_t orc_rank(uint32_t p, int64_t m, int64_t n, const uint32_t *A, int64_t lda);

/* r[a*(n+1)+b] = rank of the leading a x b submatrix of the n x n matrix A,
 * 0 <= a,b <= n (the quantities of Theorem 1 of the paper, Section 2.1). */
int orc_leading_ranks(uint32_t p, int64_t n, const uint32_t *A, int64_t lda, int64_t *r);

/* Rank profile matrix by Theorem 1: R[i][j] = r(i+1,j+1) - r(i,j+1) - r(i+1,j) + r(i,j).
 * Output as a rook placement: rpm[i] = j if R[i][j] = 1, else -1.
 * Returns -2 if the result is not a rook placement (cannot happen for a field). */
int orc_rpm_bruteforce(uint32_t p, int64_t n, const uint32_t *A, int64_t lda, int32_t *rpm);

/* ---- the factorization -------------------------------------------------- */
/*
 * Output convention shared by orc_search / orc_replay / orc_reconstruct:
 *   perm[q]  original index placed at position q (A = P L D L^T P^T with
 *            P = [e_perm[0] ... e_perm[n-1]]); pivots first, non-pivots last.
 *   L        n x n unit lower triangular in position coordinates (the unit
 *            diagonal is written as 1); non-pivot columns are identity columns.
 *   dd[q]    D[q][q];   de[q] = D[q+1][q] (nonzero only at a 2x2 block), de
 *            has n entries, de[n-1] = 0.
 *   rpm[i]   R[i][j] = 1  <=>  rpm[i] = j; -1 for a zero row of R.
 * In odd characteristic a 2x2 block of D is [[0,x],[x,0]] and the matching
 * entry of L is L[q+1][q] = y/(2x); in characteristic 2 the block is the
 * relaxed [[0,x],[x,y]] and L[q+1][q] = 0 (Sections 2.2, 4.3, 5).
 */

/* Canonical factorization: right-looking elimination with the pivot search of
 * the base case (Section 5): the current row is the first unprocessed one; the
 * pivot is the first nonzero of its Schur-complement row; a diagonal pivot gives
 * a 1x1 block, an off-diagonal one a 2x2 block, an all-zero row is set aside
 * keeping its precedence.  Returns 0. */
int orc_search(uint32_t p, int64_t n, const uint32_t *A, int64_t lda,
               int32_t *perm, uint32_t *L, int64_t ldl, uint32_t *dd, uint32_t *de,
               int32_t *rpm, int64_t *rank);

/* Same elimination, but the pivot order and block structure are imposed:
 * positions 0..rank-1 of perm hold the pivots; a position q with rpm[perm[q]] ==
 * perm[q] is a 1x1 block, otherwise perm[q+1] must be its partner rpm[perm[q]]
 * and (perm[q], perm[q+1]) is a 2x2 block.  Computes the unique (L, D).
 * Returns 0, or a negative code telling which requirement failed:
 *   -2 perm is not a permutation / rank out of range
 *   -3 a 2x2 block is not formed by consecutive partners
 *   -4 a 1x1 pivot is zero
 *   -5 a 2x2 block has a nonzero leading diagonal entry or zero off-diagonal
 *   -6 the trailing Schur complement is not zero
 *   -7 rpm of a non-pivot is not -1                                        */
int orc_replay(uint32_t p, int64_t n, const uint32_t *A, int64_t lda,
               const int32_t *perm, const int32_t *rpm, int64_t rank,
               uint32_t *L, int64_t ldl, uint32_t *dd, uint32_t *de);

/* Out = P L D L^T P^T (n x n, full).  */
int orc_reconstruct(uint32_t p, int64_t n, const int32_t *perm, const uint32_t *L, int64_t ldl,
                    const uint32_t *dd, const uint32_t *de, uint32_t *Out, int64_t ldo);

/* Characteristic 2 only: turn every relaxed block [[0,c],[c,d]] (d != 0) into
 * the standard form of Section 2.3: swap the two positions in perm, conjugate
 * L by the swap, add (c/d) x column q+1 to column q, and set the block to
 * diag(d, c^2/d).  In place.  Returns 0. */
int orc_char2_standard(int64_t n, int32_t *perm, uint32_t *L, int64_t ldl,
                       uint32_t *dd, uint32_t *de);

/* ---- building blocks (Section 3), by their definitions ------------------ */

/* C <- C - A*B ; A m x k, B k x n, C m x n. */
int orc_gemm(uint32_t p, int64_t m, int64_t n, int64_t k, const uint32_t *A, int64_t lda,
             const uint32_t *B, int64_t ldb, uint32_t *C, int64_t ldc);

/* B <- T^{-1} B with T unit lower (lower=1) or unit upper (lower=0) triangular
 * of order m (diagonal of T not read), B m x n.  Substitution. */
int orc_trsm_left(uint32_t p, int lower, int64_t m, int64_t n, const uint32_t *T, int64_t ldt,
                  uint32_t *B, int64_t ldb);

/* Lower triangle (j <= i) of C <- C - A D A^T, A n x k, D block diagonal given
 * by (dd, de) of order k (de[q] = D[q+1][q] = D[q][q+1]). Upper part untouched. */
int orc_syrdk(uint32_t p, int64_t n, int64_t k, const uint32_t *A, int64_t lda,
              const uint32_t *dd, const uint32_t *de, uint32_t *C, int64_t ldc);

/* Lower triangle of C <- C - A D B^T - B D A^T. */
int orc_syrd2k(uint32_t p, int64_t n, int64_t k, const uint32_t *A, int64_t lda,
               const uint32_t *B, int64_t ldb, const uint32_t *dd, const uint32_t *de,
               uint32_t *C, int64_t ldc);

/* Problem 1 (TRSS): given U unit upper (n x n, diagonal not read) and C
 * symmetric (lower triangle read), write into X (n x n, upper triangle, strict
 * lower set to 0) the upper triangular X with X^T U + U^T X = C.  In odd
 * characteristic X is unique.  In characteristic 2 the diagonal of C must be 0
 * (else -2 is returned) and the diagonal of X is set to 0, which makes X unique.
 * Solved entry by entry from the defining equation. */
int orc_trss(uint32_t p, int64_t n, const uint32_t *U, int64_t ldu,
             const uint32_t *C, int64_t ldc, uint32_t *X, int64_t ldx);

/* Rank-profile-revealing PLDUQ of the m x n matrix Y by row-by-row elimination
 * in lexicographic order (row i's pivot is the first nonzero of its reduced
 * row; an all-zero row is skipped keeping its precedence).
 *   rows[0..m): pivot rows in increasing order, then non-pivot rows increasing
 *   cols[0..n): pivot columns in pivot order, then non-pivot columns increasing
 *   LU (m x n, in (rows, cols) coordinates): strictly lower part of the leading
 *     rank columns = L (and M), diagonal = D, strictly upper part of the leading
 *     rank rows = U (and V); the trailing (m-rank) x (n-rank) block is zero.
 * So that Y[rows[a]][cols[b]] = sum_t L[a][t] D[t] U[t][b].  Returns 0. */
int orc_plduq(uint32_t p, int64_t m, int64_t n, const uint32_t *Y, int64_t ldy,
              int32_t *rows, int32_t *cols, uint32_t *LU, int64_t ldlu, int64_t *rank);

/* Characteristic-2 diagonal of Section 4.1.2: Delta_ii = C_ii - sum_{j<i}
 * Delta_jj U_ji^2 for a unit upper U of order r (general p accepted). */
int orc_delta(uint32_t p, int64_t r, const uint32_t *U, int64_t ldu,
              const uint32_t *C, int64_t ldc, uint32_t *delta);

/* Uses of the factorization named in Section 1 (solving symmetric systems,
 * invariants of symmetric forms), computed here without it, by plain Gaussian
 * elimination with row exchanges on the matrix itself.
 * orc_det: det(A) mod p of the n x n A.
 * orc_solve: for each of the nrhs columns of B (n x nrhs), cons[k] = 1 when
 * A x = B[:, k] has a solution (then X[:, k] is the one whose free variables
 * of the reduced row echelon form of A are 0), else cons[k] = 0 and X[:, k]
 * = 0.  Returns 0. */
int orc_det(uint32_t p, int64_t n, const uint32_t *A, int64_t lda, uint32_t *det);
int orc_solve(uint32_t p, int64_t n, const uint32_t *A, int64_t lda, const uint32_t *B, int64_t ldb,
              int64_t nrhs, uint32_t *X, int64_t ldx, int32_t *cons);

#ifdef __cplusplus
}
#endif
#endif
