// kernels.h -- declarations of the kernels in kernels.hip (see there for semantics).
#pragma once
#include "common.h"

namespace pldl {

// Leaf and bookkeeping constants shared by the kernels and the driver (the
// product kernels do not depend on them).
// "No nonzero seen" value of the first-nonzero slots (a column index above any n).
constexpr int32_t NZ_NONE = 0x7F7F7F7F;
// Threads of the base-case leaf (128 x 128 block, 4 rows x 4096/BC_THREADS columns each).
constexpr int BC_THREADS = 1024;
// PLDUQ slab in one launch (plduq.hip): chunk of PS_CHUNK columns per
// workgroup of PS_THREADS threads (lane = slab row, each wave PS_CPW columns),
// at most PS_MAXCH chunks; a wait gives up after PS_SPIN polls.
constexpr int PS_CPW = 16, PS_THREADS = 1024, PS_CHUNK = PS_CPW * (PS_THREADS / 64), PS_MAXCH = 256;
constexpr int PS_SPIN = 1 << 20;
// Device words one slab launch shares between its workgroups.  Once chunk b has
// published its pivot records (slab row, column (T row), scaled pivot value and
// scaled pivot column: 64 entries, 0 for rows it does not eliminate) it sets
// flag[b] = gen << 32 | base << 8 | cnt, with gen the launch's generation, base
// the slab pivots of the chunks before it and cnt its own: one read gives a
// waiting chunk everything it needs to fetch the records.  abort_gen equals the
// generation of an aborted launch.
constexpr int PS_FLAG_STRIDE = 16;   // flags 128 bytes apart: one cache line each
struct PsShared {
    uint64_t flag[PS_MAXCH * PS_FLAG_STRIDE];
    int32_t abort_gen;
    int32_t prow[64];
    int32_t pcol[64];
    double px[64];
    double pf[64 * 64];
};
struct PsArgs {
    double* T;
    int64_t ld;
    int64_t a0;           // first slab row (T column)
    int m;                // slab rows, 1 .. 64
    int nch;              // chunks: ceil((c1 - c0) / PS_CHUNK) <= PS_MAXCH
    int64_t c0, c1;       // slab columns (T rows)
    Field F;
    const uint32_t* itab;
    int32_t* pR;          // original index of each slab row position (T column), updated
    int32_t* pC;          // original index of each column position (T row), updated
    PsShared* sh;
    int32_t gen;          // this launch's generation (> every earlier one on sh)
    int32_t* hout;        // mapped host words: [0] = slab rank, [1] = 1 if the launch aborted
    int32_t* hflag;       // mapped host word raised to hgen once hout[0] is written
    int32_t hgen;
    int32_t* srcC;        // out: column position c0 + q holds the column that was at c0 + srcC[q]
    int32_t* srcR;        // out: slab row a0 + q holds the row that was at a0 + srcR[q]
    int32_t* rdev;        // out: device word, the slab rank (read by launches queued behind the slab)
};
__global__ void k_plduq_slab(PsArgs g);

__global__ void k_bc_leaf(double* W, int64_t ld, int64_t lo, int s, Field F, const uint32_t* itab, double* dd,
                          double* de, int32_t* sig_out, int32_t* rank_out, int32_t* hsig, int32_t* hflag, int32_t hgen);
constexpr int TS_THREADS = 256, TS_COLS = 2;   // small TRSM: workgroup size, right-hand sides per wave
__global__ void k_trsm_small(double* B, int64_t ldb, int64_t nrhs, int r, MatV T, int right, Field F);
__global__ void k_ew3(MatV D, MatV X, MatV Y, MatV Z, int64_t rows, int64_t cols, int sx, int sy, int sz, Field F);
constexpr int TSR = 16, TS_MAXR = 256;   // stripe TRSM: rows per workgroup, largest order
__global__ void k_trsm_stripe(MatV B, int64_t m, int r, MatV T, const double* N, int n_trans, Field F);
__global__ void k_inv_scatter(const int32_t* snap, int64_t len, int32_t* inv);
__global__ void k_src_gather(const int32_t* cur, int64_t len, const int32_t* inv, int32_t* src);
__global__ void k_rot_src(int64_t len, int64_t rot1, int32_t* src);
__global__ void k_compose(int32_t* srcc, const int32_t* topc, const int32_t* botc, int64_t len, int32_t* srcr,
                          const int32_t* topr, const int32_t* botr, int64_t h, int64_t m, int64_t r1, int64_t r2);
__global__ void k_reorder_src_1wg(const int32_t* snap, const int32_t* cur, int64_t len, int32_t* inv, int32_t* src);
__global__ void k_idx_reorder_1wg(int32_t* idx, int64_t a, int64_t len, const int32_t* src);
__global__ void k_tcolperm(double* T, int64_t ld, int64_t j0, int64_t len, const int32_t* src, int64_t i0,
                           int64_t ni, double* tmp, int phase, const int32_t* skip_zero);
__global__ void k_trowperm(double* T, int64_t ld, int64_t j0, int64_t nj, int64_t i0, int64_t len,
                           const int32_t* src, double* tmp, int phase);
__global__ void k_inv_table(uint32_t* tab, Field F);
__global__ void k_transpose(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t rows, int64_t cols);
__global__ void k_idx_gather(const int32_t* idx, int64_t a, int64_t len, const int32_t* sig, int32_t* tmp);
__global__ void k_idx_copy(int32_t* idx, int64_t a, int64_t len, const int32_t* tmp);
__global__ void k_zlp_sigma_total(int32_t* sig, int64_t mz, int64_t nc, int64_t rY, const int32_t* pR,
                                  const int32_t* pC);
__global__ void k_trinv_blocks(MatV T, int64_t r, int lower, double* N, Field F);
__global__ void k_trss_leaf(double* W, int64_t ld, int64_t s0, int64_t u0, int r, Field F);
struct PermGeom { int64_t n, lo, hi, s, c0, nb0, nb1, B0, B1, B2, B3; int parts, skip_ident; };
__global__ void k_perm_sym(double* W, int64_t ld, PermGeom g, const int32_t* sig, double* tmp,
                           int32_t* orig, int32_t* tmpo, int dir);
__global__ void k_scale_pack(double* X, int64_t ld, int64_t rows, int64_t cols, const double* P, int64_t ldp,
                             int by_row, const uint32_t* itab, Field F);
__global__ void k_sigma_merge(const int32_t* orig, int64_t a, int64_t n1, int64_t n2, int32_t* sig);
__global__ void k_block_dinv(const double* dd, const double* de, int64_t lo, int64_t r, Field F, double* xinv,
                             double* yy, int8_t* kind);
__global__ void k_scal_dinv(double* X, int64_t ldx, int64_t rows, int64_t r, const double* xinv, const double* yy,
                            const int8_t* kind, double* T, int64_t ldt, Field F);
__global__ void k_pack_dinv(const double* W, int64_t ld, int64_t c0, int64_t a0, int64_t r, Field F, double* dinv);
__global__ void k_mul_cols(const double* X, int64_t ldx, int64_t rows, int64_t cols, const double* dinv, int lower,
                           double* out, int64_t ldo, Field F);
__global__ void k_copy2d(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t rows, int64_t cols);
__global__ void k_zlp_assemble(const double* W, int64_t ld, int64_t lo, int64_t mz, int64_t hi, int64_t rY,
                               const double* G1, int64_t ldg1, const double* G2, int64_t ldg2, double* tmp);
__global__ void k_zlp_orig_d(int32_t* orig, int32_t* tmpo, int64_t lo, int64_t mz, int64_t hi, int64_t rY,
                             const double* W, int64_t ld, const double* delta, double* dd, double* de, int phase);
__global__ void k_save_pack_diag(const double* W, int64_t ld, int64_t s0, int64_t lo, int64_t rY, double* out);
__global__ void k_delta(const double* W, int64_t ld, int64_t s0, int64_t u0, int64_t r, Field F, double* delta);
__global__ void k_u1t_delta(const double* W, int64_t ld, int64_t s0, int64_t u0, int64_t r, const double* delta,
                            double* UT, double* UTD, Field F);
__global__ void k_dadd(double* W, int64_t ld, int64_t s0, int64_t u0, int64_t r, const double* delta, Field F);
__global__ void k_mul_delta(const double* V, int64_t ldv, int64_t rows, int64_t r, const double* delta, double* out,
                            Field F);
template <typename T>
__global__ void k_load_input(const T* A, int64_t lda, double* W, int64_t ld, int64_t n, Field F, int32_t* err);
template <typename T>
__global__ void k_store_output(T* A, int64_t lda, const double* W, int64_t ld, int64_t n, const double* dd,
                               const double* de, T* e, const int32_t* orig, int32_t* perm, const int32_t* colblk,
                               const int32_t* dinv);
__global__ void k_seg_perm(double* W, int64_t ld, int64_t lo, int64_t s, int64_t hi, int64_t n, const int32_t* sig,
                             int rpw, int skip_ident);
__global__ void k_dead_snapshot(const int32_t* orig, int64_t d0, int64_t d1, int64_t n, int32_t blk, int32_t* colblk,
                                int32_t* inv);
__global__ void k_dead_gather(const double* W, int64_t ld, int64_t n, const int32_t* orig, const int32_t* colblk,
                              const int32_t* dinv, double* tmp);
// LDS a k_seg_perm workgroup may stage (doubles); rows it takes target
// SEG_PERM_ROWS_LDS doubles; elements per thread of k_perm_sym
constexpr int64_t SEG_PERM_LDS = 8192, SEG_PERM_ROWS_LDS = 4096;
constexpr int PERM_EPT = 4;
__global__ void k_rpm(const int32_t* orig, const double* de, int64_t n, int64_t r, int32_t* rpm);
__global__ void k_char2_std(double* W, int64_t ld, int64_t n, double* dd, double* de, int32_t* orig, double* tmp,
                            int phase);

__global__ void k_iota(int32_t* a, int64_t n);
__global__ void k_iota2(int32_t* a, int64_t na, int32_t* b, int64_t nb);
__global__ void k_zlp_sigma(int32_t* sig, int64_t mz, int64_t nc, int64_t rY);
__global__ void k_apply_d(const double* A, int64_t lda, int64_t n, int64_t k, const double* dd, const double* de,
                          double* out, Field F);
__global__ void k_trss_pack(const double* U, int64_t ldu, const double* C, int64_t ldc, double* W, int64_t ldw,
                            int64_t n, int32_t* info, int check_char2);
__global__ void k_trss_unpack(const double* W, int64_t ldw, int64_t n, double* X, int64_t ldx);


template <typename T>
__global__ void k_load_factors(const double* W, int64_t ld, int64_t n, const T* e, const int32_t* perm, double* dd,
                               double* de, int32_t* orig);
// consumers.hip: solving with and reading invariants off a finished factorization
__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v);
__global__ void k_solve_gather(const double* B, int64_t ldb, const int32_t* perm, int64_t n, int64_t nrhs, double* Y);
__global__ void k_solve_dblock(const double* Y, int64_t n, int64_t nrhs, int64_t r, const void* Fd, int64_t lda,
                               int32_t dtype, const void* e, const uint32_t* itab, Field F, int32_t* cons, double* U);
__global__ void k_solve_revlt(const void* Fd, int64_t lda, int32_t dtype, int64_t n, double* Mt, int64_t ldm);
__global__ void k_solve_scatter(const double* Wt, int64_t n, int64_t nrhs, const int32_t* perm, double* B,
                                int64_t ldb);
__global__ void k_invariants(const void* Fd, int64_t lda, int32_t dtype, const void* e, int64_t n, int64_t r, Field F,
                             int64_t* out);
__global__ void k_fill_uniform_sym(double* A, int64_t n, uint32_t p, uint64_t seed);
__global__ void k_fill_unit_lower(double* L, int64_t n, uint32_t p, uint64_t seed);
__global__ void k_fill_neg_rlt(double* B, const double* L, int64_t n, const int32_t* rpm, const double* scale, Field F);

}  // namespace pldl
