/*
 * pldl.h -- C-ABI of the MI355X (gfx950) library computing the symmetric
 * indefinite factorization  A = P L D L^T P^T  over a prime field F_p that
 * reveals the rank profile matrix (Dumas & Pernet, "Symmetric indefinite
 * triangular factorization revealing the rank profile matrix").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All matrix arguments are DEVICE pointers (memory of the context's GPU),
 *    row-major with an explicit leading dimension (elements, >= row length).
 *  - Residues are canonical, in [0, p).  The building-block calls take and
 *    return FP64 residues (integers held exactly in doubles).
 *  - p must be prime with 2 <= p < 2^24 (primality is the caller's duty;
 *    p >= 2^24 or p < 2 gives PLDL_EUNSUPPORTED_P).  The INT8 product path
 *    covers p < 2^23; for larger p its products run on FP64.
 *  - `stream` is a hipStream_t (NULL = default stream).  Every call is ordered
 *    on that stream; calls that must return a rank to the host synchronise it.
 *  - The caller owns every array; the library never frees or reallocates
 *    caller memory.  The context owns its workspace (grown on demand, freed by
 *    pldl_destroy).  A context is not thread-safe: one per host thread.
 *  - Return value: 0 on success; -k when argument k (1-based) is invalid;
 *    a positive PLDL_E* code for runtime failures (text: pldl_last_error).
 *    Arguments are checked before any work is queued.
 */
#ifndef PLDL_H
#define PLDL_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define PLDL_OK 0
#define PLDL_ERANGE 1          /* an input entry is >= p                         */
#define PLDL_EUNSUPPORTED_P 2  /* p outside [2, 2^24)                            */
#define PLDL_EHIP 3            /* HIP runtime error (text in pldl_last_error)    */
#define PLDL_ENOMEM 4          /* workspace allocation failed                    */
#define PLDL_EINTERNAL 5       /* internal consistency check failed              */
#define PLDL_ETOOBIG 6         /* larger than the fixed scratch of an allocation-free call */

#define PLDL_U32 0             /* uint32 residues */
#define PLDL_F64 1             /* FP64 residues   */

#define PLDL_THRESHOLD_ONLINE (-1)  /* pldl_opts.threshold: chosen online by the context */

#define PLDL_PATH_AUTO 0       /* the context's path (pldl_set_path; by prime at creation) */
#define PLDL_PATH_F64 1        /* products on FP64 MFMA with delayed reduction         */
#define PLDL_PATH_I8 2         /* products on INT8 MFMA: residues split into 1-3 signed
                                  bytes, INT32 accumulation, mod-p recombination         */

typedef struct pldl_ctx pldl_ctx;

/* What a pldl_factor call did, for reproducing it (filled when sched_out is
 * not NULL).  The factorization is a function of (A, p, threshold_used,
 * split_rule); path_used and the product counts change no result (both
 * product paths are exact). */
typedef struct {
    int32_t threshold_used;   /* base-case order t of the cascade (Section 5)           */
    int32_t split_rule;       /* granule g of the recursive split: a range of order N
                                 >= 2g splits at m = floor(N/2) rounded down to a
                                 multiple of g (g = 64); smaller ones at floor(N/2)   */
    int32_t path_used;        /* PLDL_PATH_F64 or PLDL_PATH_I8                          */
    int32_t i8_min_log2_flops;/* INT8 path: products of fewer flops stay on FP64 (2^k) */
    int64_t products_f64;     /* products run on the FP64 matrix cores                  */
    int64_t products_i8;      /* products run on the INT8 matrix cores                  */
    int64_t launches;         /* kernel launches and stream memory operations queued    */
    int64_t host_waits;       /* host synchronisations of the stream inside the call    */
    int64_t products_winograd;/* products split by a Winograd level (pldl_set_winograd) */
} pldl_schedule;

typedef struct {
    int32_t path;          /* PLDL_PATH_*                                              */
    int32_t threshold;     /* base-case order t of the cascade (Section 5), 1..128;
                              0 = the context's autotuned value (pldl_autotune), else 128;
                              PLDL_THRESHOLD_ONLINE = chosen by the context from the wall
                              times of its earlier calls of the same p and order class
                              (each of 128, 96, 64 timed once, then the fastest, with
                              every 16th call re-timing the oldest measurement; the
                              end of Section 6 suggests such introspective tuning).
                              sched_out reports the value used, which with A and p
                              fixes the result.                                       */
    int32_t standard_form; /* p == 2 only: turn relaxed 2x2 blocks into the standard
                              form of Section 2.3 (after the rank profile is taken)     */
    int32_t check_range;   /* nonzero: reject inputs with an entry >= p (PLDL_ERANGE);
                              zero: such entries are read mod p (a negative or
                              fractional FP64 entry as 0)                              */
} pldl_opts;

/* Create a context bound to HIP device `device`.  *ctx receives the handle. */
int pldl_create(pldl_ctx **ctx, int device);
/* Release the context and its workspace.  NULL is accepted. */
int pldl_destroy(pldl_ctx *ctx);
/* Text of the last error recorded on this context ("" if none). */
const char *pldl_last_error(const pldl_ctx *ctx);

/*
 * pldl_factor -- Algorithm 2 of the paper (recursive symmetric elimination,
 * Section 4) cascaded with the Crout-style base case of Section 5 below order
 * `threshold`, with Algorithm 3 (zero leading block) and Algorithm 1 (TRSS) as
 * sub-steps.  Computes P, L, D with A = P L D L^T P^T, the rank r, and the rank
 * profile matrix R = P Psi P^T (Section 2.1, pivoting matrix).
 *
 *  p      prime modulus.
 *  n      order of A (n >= 0).
 *  A      device, n x n, leading dimension lda >= max(1, n), dtype `dtype`.
 *         In: the lower triangle (j <= i) of the symmetric A; the strict upper
 *         triangle is neither read nor written.
 *         Out: strict lower triangle = L (unit diagonal implied), including the
 *         entry L[q+1][q] of a 2x2 block; diagonal = diag(D) (x for a 1x1 block,
 *         0 and 0 for an odd-characteristic 2x2 block, 0 and d for a relaxed
 *         characteristic-2 block [[0,c],[c,d]]).
 *  e      device, n entries (dtype `dtype`): e[q] = D[q+1][q] for a 2x2 block
 *         starting at position q, else 0.
 *  perm   device int32[n]: perm[q] = original index at position q, i.e.
 *         P = [e_perm[0] ... e_perm[n-1]]; the rank pivots come first, the n - r
 *         non-pivots last in increasing original order.
 *  rpm    device int32[n]: rpm[i] = j if R[i][j] = 1, else -1 (R is a symmetric
 *         rook placement with r ones).
 *  rank   host int64*: receives r (the call synchronises `stream`).
 *  opts   may be NULL (defaults).
 *  sched_out  host, may be NULL: receives the schedule the call used
 *         (threshold, split rule, product path and counts, launches, waits).
 * Errors: -1 ctx NULL; -3 n outside [0, 65535]; -4 A NULL; -5 lda < max(1, n);
 * -6 unknown dtype; -7 e NULL; -8 perm NULL; -9 rpm NULL; -10 rank NULL;
 * -11 opts invalid (path, or threshold neither PLDL_THRESHOLD_ONLINE nor in
 * [0, 128]); PLDL_EUNSUPPORTED_P
 * for p outside [2, 2^24); PLDL_ERANGE when opts->check_range is set and an
 * input entry is >= p (nothing else is written); PLDL_ENOMEM, PLDL_EHIP.
 * With standard_form set and p == 2, perm/L/diag/e are returned in the standard
 * form of Section 2.3 while rpm still holds R.
 */
int pldl_factor(pldl_ctx *ctx, uint32_t p, int64_t n, void *A, int64_t lda, int32_t dtype,
                void *e, int32_t *perm, int32_t *rpm, int64_t *rank, const pldl_opts *opts,
                pldl_schedule *sched_out, void *stream);

/*
 * pldl_factor_batched -- `batch` independent factorizations (each as
 * pldl_factor, order n_b <= 512) in one persistent launch: workgroups take
 * matrices from a device counter, largest order first (a counting sort on the
 * device), so uneven orders and ranks balance and the last matrices started
 * are the small ones.  Each matrix is factored by the base-case elimination of
 * Section 5 (rows in increasing order, lexicographically first nonzero of the
 * Schur-complement row as pivot, 1x1 / 2x2 blocks, relaxed 2x2 blocks in
 * characteristic 2, zero rows set aside): perm is that elimination's
 * canonical order, and rpm is the rank profile matrix (Theorem 1).
 *
 *  n, lda, rank   device int64[batch]: order, leading dimension, rank out.
 *  A, e           device arrays of batch device pointers (dtype `dtype`): the
 *                 matrices (lower triangle in, L / diag(D) out, as pldl_factor)
 *                 and their e vectors (n_b entries each).
 *  perm, rpm      device arrays of batch device pointers to int32[n_b].
 *  status         device int32[batch]: 0, PLDL_ERANGE (an entry >= p, when
 *                 opts->check_range), or -3 (n_b outside [0, 512], lda_b < n_b
 *                 or a NULL pointer); outputs of a failed matrix are undefined.
 *  opts           may be NULL; threshold and path are ignored; standard_form
 *                 must be 0 (-13).
 * The call is asynchronous (no host synchronisation: read rank and status
 * after synchronising `stream`) and launches three kernels, so it can be
 * captured in a HIP graph.  The first call on a context allocates its
 * workspace (four workgroup slots per compute unit, 1 MiB each) and the
 * inverse table of p and the order array (int32, 65536 entries, grown by a
 * larger batch than every earlier one): make such calls outside a capture.  Per-matrix pointers are
 * trusted (the host cannot check device arrays without synchronising).
 */
int pldl_factor_batched(pldl_ctx *ctx, uint32_t p, int64_t batch, const int64_t *n, void *const *A,
                        const int64_t *lda, int32_t dtype, void *const *e, int32_t *const *perm,
                        int32_t *const *rpm, int64_t *rank, int32_t *status, const pldl_opts *opts,
                        void *stream);

/*
 * pldl_char2_to_standard -- the transform of Section 2.3 applied to a
 * characteristic-2 factorization returned by pldl_factor (p = 2, standard_form
 * 0): every relaxed 2x2 block [[0,c],[c,d]] with d != 0 is turned into the
 * 1x1 blocks (d) and (c^2/d) by P~ = P P_J, L~ = (P_J^T L P_J) L_J.
 * A (lda), e, perm: pldl_factor's outputs, updated in place (same layout);
 * rpm is not changed by the transform (take it from pldl_factor).  Entries
 * outside {0, 1} give PLDL_ERANGE.  Synchronises `stream`.
 */
int pldl_char2_to_standard(pldl_ctx *ctx, int64_t n, void *A, int64_t lda, int32_t dtype, void *e,
                           int32_t *perm, void *stream);

/*
 * pldl_autotune -- picks the base-case threshold of the cascade (Section 5)
 * for each order in n_list[0 .. count) (host array, 1 <= n <= 16384) over F_p:
 * builds two synthetic matrices of that order on the device (uniform
 * symmetric, i.e. a generic rank profile; and L R L^T with a random rank
 * profile of rank about n/2), times pldl_factor at thresholds 32, 48, 64, 96
 * and 128 (best of two runs each) and keeps the threshold with the smallest
 * total.  Later pldl_factor calls on this context with opts->threshold = 0
 * use the entry of the same p (else of any p) nearest to their n on a log
 * scale.  table_path (may be NULL): the table is written there as text lines
 * "p n threshold ms_uniform ms_rank_profile".  With count = 0, the table at
 * table_path is read instead.  Allocates five n x n FP64 buffers per order
 * while it runs; synchronises `stream`.
 */
int pldl_autotune(pldl_ctx *ctx, uint32_t p, const int64_t *n_list, int64_t count, const char *table_path,
                  void *stream);

/* ---------------- uses of a factorization (Section 1) ---------------- */

/*
 * pldl_solve -- X with A X = B for the symmetric A whose factorization
 * pldl_factor returned (the introduction names solving symmetric systems as
 * the first use of the factorization): A = P L D L^T P^T gives
 * X = P L^{-T} D^+ L^{-1} P^T B, with D^+ inverting D's 1x1 blocks and its 2x2
 * blocks [[0,c],[c,d]] on the r pivot positions.  For a singular A a column b
 * has a solution when L^{-1} P^T b vanishes on the n - r non-pivot positions;
 * the solution returned is the one with L^T P^T x zero there.
 *  F (lda, dtype), e, perm, rank: pldl_factor's outputs, unchanged (not in the
 *            characteristic-2 standard form: the relaxed blocks are expected).
 *  B         device, n x nrhs FP64 residues, leading dimension ldb >= nrhs; in:
 *            the right-hand sides, out: the solutions (a column without a
 *            solution is left undefined).
 *  consistent device int32[nrhs] (may be NULL): 1 if the column has a solution, else 0.
 * Errors: -1 ctx; -3 n; -4 F; -5 lda; -6 dtype; -7 e; -8 perm; -9 rank outside
 * [0, n]; -10 B; -11 ldb; -12 nrhs < 0; PLDL_ERANGE for an entry of F >= p.
 * Synchronises `stream`.
 */
int pldl_solve(pldl_ctx *ctx, uint32_t p, int64_t n, const void *F, int64_t lda, int32_t dtype,
               const void *e, const int32_t *perm, int64_t rank, double *B, int64_t ldb, int64_t nrhs,
               int32_t *consistent, void *stream);

/*
 * pldl_invariants -- invariants of the symmetric bilinear form x^T A y read
 * off its factorization (the introduction's second use: invariants of
 * symmetric forms, such as the signature).  Over F_p the form is classified by
 * its rank and, for odd p, by the discriminant of its nondegenerate part
 * modulo squares (two nondegenerate forms of the same rank are equivalent iff
 * these agree); in characteristic 2 by its rank and whether it is alternating.
 *  out (host int64[5]): [0] rank r; [1] det(A) mod p (0 when r < n);
 *   [2] the product of the determinants of D's blocks (1x1: x; 2x2: -c^2), a
 *       discriminant of the nondegenerate part; [3] its quadratic character,
 *       1 (a square) or -1 (p odd; 1 for p = 2); [4] p = 2: 1 if the form is
 *       alternating (diag(D) = 0, i.e. diag(A) = 0), else 0 (odd p: 0).
 * Errors: -1 ctx; -3 n; -4 F; -5 lda; -6 dtype; -7 e; -8 rank; -9 out.
 * Synchronises `stream`.
 */
int pldl_invariants(pldl_ctx *ctx, uint32_t p, int64_t n, const void *F, int64_t lda, int32_t dtype,
                    const void *e, int64_t rank, int64_t *out, void *stream);

/* ---------------- building blocks (Section 3), FP64 residues ---------------- */

/*
 * GEMM (Section 3): C <- C - op(A) op(B) mod p, C m x n, op(A) m x k, op(B) k x n;
 * op(X) = X (trans = 0) or X^T (trans = 1).  With lower_only = 1 (m == n) only
 * the entries j <= i of C are updated: this is SYRDK / SYRD2K's output mode.
 */
int pldl_gemm(pldl_ctx *ctx, uint32_t p, int64_t m, int64_t n, int64_t k,
              const double *A, int64_t lda, int32_t transA,
              const double *B, int64_t ldb, int32_t transB,
              double *C, int64_t ldc, int32_t lower_only, void *stream);

/*
 * TRSM (Section 3) with a unit triangular T of order m (its diagonal and other
 * triangle are not read), B m x n in place:
 *   lower = 1: B <- T^{-1} B with T unit lower;   lower = 0: T unit upper.
 */
int pldl_trsm(pldl_ctx *ctx, uint32_t p, int32_t lower, int64_t m, int64_t n,
              const double *T, int64_t ldt, double *B, int64_t ldb, void *stream);

/*
 * SYRDK (Section 3): lower triangle of C <- C - A D A^T, A n x k, D block
 * diagonal of order k with diagonal dd[k] and off-diagonal de[k]
 * (de[q] = D[q+1][q] = D[q][q+1]).  SYRD2K: C <- C - A D B^T - B D A^T.
 * B may be NULL for SYRDK.
 */
int pldl_syrdk(pldl_ctx *ctx, uint32_t p, int64_t n, int64_t k, const double *A, int64_t lda,
               const double *B, int64_t ldb, const double *dd, const double *de,
               double *C, int64_t ldc, void *stream);

/*
 * TRSS (Problem 1, Algorithm 1): given U unit upper (n x n, diagonal and strict
 * lower part not read) and symmetric C (lower triangle read), overwrite the
 * upper triangle of X (n x n, strict lower part set to 0) with the upper
 * triangular solution of X^T U + U^T X = C.  For p = 2 the diagonal of C must be
 * zero (else -6 ... see return codes) and the diagonal of X is set to 0.
 */
int pldl_trss(pldl_ctx *ctx, uint32_t p, int64_t n, const double *U, int64_t ldu,
              const double *C, int64_t ldc, double *X, int64_t ldx, void *stream);

/*
 * PLDUQ revealing the rank profile matrix of the m x n matrix Y (the
 * elimination Algorithm 3 starts with; Sections 4.2 and 5 for its pivoting):
 * Y = P [L1; M1] D1 [U1 V1] Q.  On return:
 *   rows[0..m): original row indices, the rank pivot rows first (pivot order),
 *               then the non-pivot rows in increasing order;
 *   cols[0..n): pivot columns in pivot order, then non-pivot columns increasing;
 *   Y (in place, in (rows, cols) coordinates): strict lower part of the leading
 *     r columns = L1/M1, diagonal = D1, strict upper part of the leading r rows =
 *     U1/V1, trailing block zero.  The pivot set {(rows[t], cols[t])} is the rank
 *     profile matrix of Y; the pivot order is the one of the recursive search.
 *   rank: host int64*.
 */
int pldl_plduq(pldl_ctx *ctx, uint32_t p, int64_t m, int64_t n, double *Y, int64_t ldy,
               int32_t *rows, int32_t *cols, int64_t *rank, void *stream);

/*
 * pldl_syrdk_noalloc -- pldl_syrdk (same arguments, same result) for callers
 * that cannot allocate device memory: code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc.  The call allocates nothing: A D (and
 * B D) are staged in a fixed device array of PLDL_NOALLOC_SCRATCH_DOUBLES
 * doubles per GPU (16 MiB, held from the context's creation to the end of the
 * process), and the products run on the FP64 matrix cores whatever the
 * context's path.  Limit: n * k (2 n k with B) <= PLDL_NOALLOC_SCRATCH_DOUBLES,
 * else PLDL_ETOOBIG.  Asynchronous: nothing is waited for (read C after
 * synchronising `stream`).  Calls that overlap on one GPU share the array and
 * race: serialise them.
 */
#define PLDL_NOALLOC_SCRATCH_DOUBLES (1 << 21)
int pldl_syrdk_noalloc(pldl_ctx *ctx, uint32_t p, int64_t n, int64_t k, const double *A, int64_t lda,
                       const double *B, int64_t ldb, const double *dd, const double *de,
                       double *C, int64_t ldc, void *stream);

/*
 * Matrix cores used by the products (GEMM, TRMM, SYRDK, SYRD2K of Section 3)
 * of every later call on this context whose options say PLDL_PATH_AUTO, and of
 * the building-block calls above.  path: PLDL_PATH_AUTO (the default at
 * creation: pldl_factor takes the INT8 path when p < 2^23, where three
 * balanced limbs cover the residues, and FP64 otherwise; the building-block
 * calls take FP64), PLDL_PATH_F64 or PLDL_PATH_I8.  The INT8 path writes each operand as L signed-byte digit
 * planes (L = 1 for p < 2^8, 2 for p < 2^15, else 3) into a context buffer
 * grown on demand, and runs the L^2 byte products on v_mfma_i32_16x16x64_i8;
 * results are identical to the FP64 path (both are exact).  Inside
 * pldl_factor, products below 2^27 flops, and products whose two segments
 * together exceed the INT32 bound (K0 + K1 > 65535), stay on FP64.  Returns
 * -2 for another value.
 */
int pldl_set_path(pldl_ctx *ctx, int32_t path);

/*
 * Sub-cubic products (the paper's introduction: fast matrix multiplication is
 * exact over F_p, so the factorization inherits its exponent).  Every later
 * dense product of this context (a GEMM of the recursion, of PLDUQ or of
 * pldl_gemm; not the triangular-output SYRDK / SYRD2K nor the TRMM) whose m,
 * n and k are all >= min_order takes one level of Winograd's variant of
 * Strassen's algorithm: seven products of half size and fifteen additions,
 * all mod p, on the leading part whose halves are multiples of 64; the rest
 * of the product is plain.  The half-size products take another level while
 * they are still large enough.  Temporaries come from a context buffer grown
 * on demand (about 4/3 of (m k + k n + 2 m n) / 2 doubles).  Results are
 * identical (exact arithmetic).  min_order: 0 (off, the default) or
 * 256 .. 65535; returns -2 for another value.
 */
int pldl_set_winograd(pldl_ctx *ctx, int64_t min_order);

/* ---------------- measurement ---------------- */

/* Per-kernel-class totals collected with HIP events recorded around every
 * launch the library makes on the caller's stream while profiling is on. */
#define PLDL_NCLASS 9
#define PLDL_CLASS_GEMM 0        /* mod-p FP64 MFMA products (GEMM/TRMM/SYRDK/SYRD2K) */
#define PLDL_CLASS_TRSM_LEAF 1   /* triangular-solve leaves                         */
#define PLDL_CLASS_BASE_CASE 2   /* base case of Section 5                          */
#define PLDL_CLASS_PLDUQ_LEAF 3  /* PLDUQ tile leaves                               */
#define PLDL_CLASS_TRSS_LEAF 4   /* TRSS leaves                                     */
#define PLDL_CLASS_PERM 5        /* symmetric permutations / assembly moves          */
#define PLDL_CLASS_OTHER 6       /* scaling, bookkeeping, input/output kernels      */
#define PLDL_CLASS_HOST_SYNC 7   /* host waits for a rank (launches = count, ms = wall) */
#define PLDL_CLASS_GEMM_I8 8     /* mod-p INT8-split MFMA products (limb split: OTHER) */
typedef struct {
    int64_t launches;  /* number of launches (or synchronisations)               */
    double flops;      /* algorithmic mod-p flops (2 per multiply-add), classes 0, 8 */
    double bytes;      /* algorithmic HBM bytes (read + write): class 5; classes
                          0 and 8 count each operand read once and C read and
                          written (8 B per FP64 residue, L B per INT8 limb set) */
    double ops8;       /* class 8: INT8 MFMA operations (L^2 byte products per
                          mod-p product, 2 per multiply-add)                        */
    double ms;         /* summed GPU duration of the launches (event-timed)        */
} pldl_kstat;
typedef struct {
    pldl_kstat cls[PLDL_NCLASS];
} pldl_stats;

/*
 * Profiling control.  mode 1: reset the totals and start recording every
 * class with two HIP events around each launch (a few microseconds of queue
 * time each); mode 3: reset and record the two product classes only, timed
 * inside the kernels (first workgroup start to last workgroup end on the
 * device wall clock; no events, no extra launches: the light mode a timed run
 * uses); mode 0: stop recording; mode 2: leave the state unchanged.  In every
 * mode `out` (host, may be NULL) receives the totals gathered so far.
 * Recording never changes results.
 */
int pldl_profile(pldl_ctx *ctx, int32_t mode, pldl_stats *out);

#ifdef __cplusplus
}
#endif
#endif
