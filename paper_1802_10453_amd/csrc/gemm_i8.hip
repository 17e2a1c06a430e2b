// gemm_i8.hip -- mod-p matrix product on the INT8 matrix cores of gfx950.
//
// The same operation as gemm.hip (C <- C - sum_seg A_seg B_seg mod p, with the
// lower-triangle and triangular-B variants of Section 3's SYRDK, SYRD2K and
// TRMM), with the residues split into signed bytes:
//
//   a = sum_{t < L} 256^t a_t,  a_t in [-128, 127]   (balanced digits of the
//   centered residue |a| <= (p-1)/2; L = 1 for p < 2^8, 2 for p < 2^15, 3 for
//   p < 2^23, the top digit then has |a_{L-1}| <= 64),
//
// so that A B = sum_s 256^s C_s with C_s = sum_{t+u=s} A_t B_u.  Every C_s is
// accumulated exactly in INT32 by v_mfma_i32_16x16x64_i8 and recombined once,
// in the epilogue: sum_s w_s (C_s mod p) with w_s = 256^s mod p, reduced in
// FP64.  Bound: a digit pair contributes at most 2^14 per k (2^13 when one
// digit is a top digit, |top| <= 64), so a shift class gains at most 2^15 per
// k for every L (L = 3, s = 1: two pairs of full digits; s = 2: one pair of
// full digits and two with a top digit).  Both segments of SYRD2K accumulate
// into the same registers, hence the condition K0 + K1 <= 65535
// (65535 * 2^15 < 2^31); a longer product falls back to FP64.
//
// Operands are first split into K-contiguous limb planes (one pass, 8 bytes
// read and L bytes written per element, every operand of a product in one
// launch; K padded to a multiple of 64 with zeros): plane t of A is m x Kp,
// plane t of B holds B^T (n x Kp).  A wave's
// MFMA fragment is then 16 contiguous bytes per lane: lane l takes row l%16
// (of A) or column l%16 (of B^T) and the k-group l/16 of each 64-wide K step,
// the same k map on both sides as the instruction requires.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace pldl {

namespace {
typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int SPLIT_T = 64;   // split tile: 64 rows x 64 k

// Balanced base-256 digits of the centered residue of the canonical v.
template <int L>
__device__ __forceinline__ void split_digits(double v, const Field& F, int8_t* d) {
    int a = (int)fcen(v, F);
#pragma unroll
    for (int t = 0; t < L; ++t) {
        int lo = ((a + 128) & 255) - 128;
        d[t] = (int8_t)lo;
        a = (a - lo) >> 8;
    }
}

// X (rows x K view, element (i, k) at X.p[i*X.rs + k*X.cs]) -> L planes of
// rows x Kp int8.  upper_mask: X(i, k) is taken as 0 for k > i (the TRMM
// triangle of B, seen transposed).  A 64 x 64 tile goes through LDS so that the
// global reads follow whichever stride is 1.
// All the operands of one product are split in one launch: blocks
// [blk0[q], blk0[q+1]) take operand q, 64 x 64 tiles in row-major order of its
// (rows / 64) x (Kp / 64) tile grid.
struct SplitArgs {
    MatV X[4];
    int64_t rows[4], K[4], Kp[4];
    int upper[4];
    int8_t* planes[4];
    int64_t blk0[5];
    int nx;
};

template <int L>
__global__ __launch_bounds__(256) void k_split_i8(SplitArgs sa, Field F) {
    __shared__ double tile[SPLIT_T][SPLIT_T + 1];
    const int tid = threadIdx.x;
    const int64_t blk = blockIdx.x;
    int op = 0;
    while (op + 1 < sa.nx && blk >= sa.blk0[op + 1]) ++op;
    const MatV X = sa.X[op];
    const int64_t rows = sa.rows[op], K = sa.K[op], Kp = sa.Kp[op];
    const int upper_mask = sa.upper[op];
    int8_t* planes = sa.planes[op];
    const int64_t local = blk - sa.blk0[op], kt = Kp / SPLIT_T;
    const int64_t r0 = (local / kt) * SPLIT_T, k0 = (local % kt) * SPLIT_T;
    const bool kfast = X.cs == 1;
#pragma unroll
    for (int e = 0; e < SPLIT_T * SPLIT_T / 256; ++e) {
        const int q = tid + 256 * e;
        const int a = q / SPLIT_T, b = q % SPLIT_T;     // b runs along the unit stride
        const int i = kfast ? a : b, k = kfast ? b : a;
        const int64_t gi = r0 + i, gk = k0 + k;
        double v = 0.0;
        if (gi < rows && gk < K && !(upper_mask && gk > gi)) v = X.p[gi * X.rs + gk * X.cs];
        tile[i][k] = v;
    }
    __syncthreads();
    // thread: row tid/4, 16 consecutive k starting at 16*(tid%4)
    const int i = tid >> 2, kb = (tid & 3) * 16;
    const int64_t gi = r0 + i;
    if (gi >= rows) return;
    int8_t d[16][L];
#pragma unroll
    for (int c = 0; c < 16; ++c) split_digits<L>(tile[i][kb + c], F, d[c]);
    const int64_t plane = rows * Kp;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        v4i w;
        int* wp = (int*)&w;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            wp[q] = (int)(uint8_t)d[4 * q][t] | ((int)(uint8_t)d[4 * q + 1][t] << 8) |
                    ((int)(uint8_t)d[4 * q + 2][t] << 16) | ((int)(uint8_t)d[4 * q + 3][t] << 24);
        *(v4i*)(planes + t * plane + gi * Kp + k0 + kb) = w;
    }
}

struct I8Args {
    int64_t m, n;
    double* C;
    int64_t ldc;
    const int8_t* A[2];   // L planes of m x Kp each
    const int8_t* B[2];   // L planes of n x Kp each (B transposed)
    int64_t Kp[2];
    Field F;
    double w[5];          // 256^s mod p
    int tiles_n;
    Stamp stamp;
};

// Workgroup tile 64 x 64, four waves in a 2 x 2 grid, wave tile 32 x 32 (2 x 2
// MFMA blocks).  Fragments stream from the planes (L1/L2 serve the reuse
// between the two waves that share rows or columns); the next K step's
// fragments are loaded before the current step's MFMAs are issued.
template <int L, bool LOWER_C>
__global__ __launch_bounds__(256) void k_gemm_i8(I8Args g) {
    constexpr int NS = 2 * L - 1;
    stamp_begin(g.stamp);
    const int bid = blockIdx.x;
    int ti, tj;
    if (LOWER_C) {
        ti = (int)((sqrt(8.0 * (double)bid + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= bid) ++ti;
        while (ti * (ti + 1) / 2 > bid) --ti;
        tj = bid - ti * (ti + 1) / 2;
    } else {
        ti = bid / g.tiles_n;
        tj = bid - ti * g.tiles_n;
    }
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int r16 = lane & 15, kg = lane >> 4;
    const int64_t i0 = (int64_t)ti * 64 + wm * 32, j0 = (int64_t)tj * 64 + wn * 32;

    v4i acc[2][2][NS];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int s = 0; s < NS; ++s) acc[a][b][s] = v4i{0, 0, 0, 0};

#pragma unroll 1
    for (int seg = 0; seg < 2; ++seg) {
        const int64_t Kp = g.Kp[seg];
        if (Kp <= 0) continue;
        const int8_t* Ap = g.A[seg];
        const int8_t* Bp = g.B[seg];
        const int64_t pa = g.m * Kp, pb = g.n * Kp;
        // fragment base addresses (rows/columns past the edge are clamped: their
        // products land in outputs that are never stored)
        const int8_t* fa[2];
        const int8_t* fb[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const int64_t row = min(i0 + x * 16 + r16, g.m - 1), col = min(j0 + x * 16 + r16, g.n - 1);
            fa[x] = Ap + row * Kp + kg * 16;
            fb[x] = Bp + col * Kp + kg * 16;
        }
        v4i ca[2][L], cb[2][L], na[2][L], nb[2][L];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int t = 0; t < L; ++t) {
                ca[x][t] = *(const v4i*)(fa[x] + t * pa);
                cb[x][t] = *(const v4i*)(fb[x] + t * pb);
            }
#pragma unroll 1
        for (int64_t k0 = 0; k0 < Kp; k0 += 64) {
            const bool more = k0 + 64 < Kp;
            if (more) {
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int t = 0; t < L; ++t) {
                        na[x][t] = *(const v4i*)(fa[x] + t * pa + k0 + 64);
                        nb[x][t] = *(const v4i*)(fb[x] + t * pb + k0 + 64);
                    }
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
#pragma unroll
                    for (int t = 0; t < L; ++t)
#pragma unroll
                        for (int u = 0; u < L; ++u)
                            acc[x][y][t + u] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ca[x][t], cb[y][u], acc[x][y][t + u],
                                                                                    0, 0, 0);
            if (more) {
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int t = 0; t < L; ++t) { ca[x][t] = na[x][t]; cb[x][t] = nb[x][t]; }
            }
        }
    }
    // epilogue: lane l, register r of a block holds D[4*(l/16) + r][l%16]
    const Field F = g.F;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = i0 + x * 16 + 4 * kg + r, col = j0 + y * 16 + r16;
                if (row < g.m && col < g.n && (!LOWER_C || col <= row)) {
                    double v = 0.0;
#pragma unroll
                    for (int s = 0; s < NS; ++s) v = fma(fred((double)acc[x][y][s][r], F), g.w[s], v);
                    double* c = g.C + row * g.ldc + col;
                    *c = fred(*c - fred(v, F), F);
                }
            }
    stamp_end(g.stamp);
}

// Large products: workgroup tile 128 x 128, eight waves in a 2 x 4 grid, wave
// tile 64 x 32 (4 x 2 MFMA blocks).  Each 64-deep K step of every limb plane
// goes through LDS (double-buffered, one barrier per step; the next step's
// global reads are in flight during the current step's products), so an A
// fragment serves two B blocks and a B fragment four A blocks, all from LDS.
// LDS rows are 80 bytes (64 of data): the 16-byte fragment reads of 16
// consecutive rows then fall on distinct banks.
constexpr int I8B_TILE = 128, I8B_ROW = 80, I8B_THREADS = 512;

template <int L, bool LOWER_C>
__global__ __launch_bounds__(I8B_THREADS) void k_gemm_i8_big(I8Args g) {
    constexpr int NS = 2 * L - 1, T = I8B_TILE, RB = I8B_ROW;
    constexpr int PLANE = T * RB;                 // bytes of one limb plane of one operand tile
    __shared__ __attribute__((aligned(16))) int8_t lds[2 * 2 * L * PLANE];   // [buffer][A, B][limb][T][RB]
    stamp_begin(g.stamp);
    const int bid = blockIdx.x;
    int ti, tj;
    if (LOWER_C) {
        ti = (int)((sqrt(8.0 * (double)bid + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= bid) ++ti;
        while (ti * (ti + 1) / 2 > bid) --ti;
        tj = bid - ti * (ti + 1) / 2;
    } else {
        ti = bid / g.tiles_n;
        tj = bid - ti * g.tiles_n;
    }
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 2, wn = wave & 3;      // wave tile rows wm*64 .., columns wn*32 ..
    const int r16 = lane & 15, kg = lane >> 4;
    const int64_t ti0 = (int64_t)ti * T, tj0 = (int64_t)tj * T;
    // this thread's share of a stage: row (or column) tid/4 of the tile, 16 bytes at k (tid%4)*16
    const int lrow = tid >> 2, lk = (tid & 3) * 16;

    v4i acc[4][2][NS];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < NS; ++q) acc[x][y][q] = v4i{0, 0, 0, 0};

#pragma unroll 1
    for (int seg = 0; seg < 2; ++seg) {
        const int64_t Kp = g.Kp[seg];
        if (Kp <= 0) continue;
        const int64_t pa = g.m * Kp, pb = g.n * Kp;
        // rows / columns past the edge are clamped: their products land in outputs never stored
        const int8_t* ga = g.A[seg] + min(ti0 + lrow, g.m - 1) * Kp + lk;
        const int8_t* gb = g.B[seg] + min(tj0 + lrow, g.n - 1) * Kp + lk;
        v4i ra[L], rb[L];
        auto gload = [&](int64_t k0) {
#pragma unroll
            for (int t = 0; t < L; ++t) {
                ra[t] = *(const v4i*)(ga + t * pa + k0);
                rb[t] = *(const v4i*)(gb + t * pb + k0);
            }
        };
        auto lstore = [&](int buf) {
            int8_t* base = lds + buf * 2 * L * PLANE;
#pragma unroll
            for (int t = 0; t < L; ++t) {
                *(v4i*)(base + t * PLANE + lrow * RB + lk) = ra[t];
                *(v4i*)(base + (L + t) * PLANE + lrow * RB + lk) = rb[t];
            }
        };
        __syncthreads();   // LDS of a previous segment fully read
        gload(0);
        lstore(0);
        const int64_t nst = Kp / 64;
        if (nst > 1) gload(64);
        __syncthreads();
        int cur = 0;
#pragma unroll 1
        for (int64_t st = 0; st < nst; ++st) {
            const int8_t* A_l = lds + cur * 2 * L * PLANE;
            const int8_t* B_l = A_l + L * PLANE;
            v4i fb[2][L];
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int u = 0; u < L; ++u)
                    fb[y][u] = *(const v4i*)(B_l + u * PLANE + (wn * 32 + y * 16 + r16) * RB + kg * 16);
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                v4i fa[L];
#pragma unroll
                for (int t = 0; t < L; ++t)
                    fa[t] = *(const v4i*)(A_l + t * PLANE + (wm * 64 + x * 16 + r16) * RB + kg * 16);
#pragma unroll
                for (int y = 0; y < 2; ++y)
#pragma unroll
                    for (int t = 0; t < L; ++t)
#pragma unroll
                        for (int u = 0; u < L; ++u)
                            acc[x][y][t + u] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[t], fb[y][u], acc[x][y][t + u],
                                                                                    0, 0, 0);
            }
            if (st + 1 < nst) {
                lstore(cur ^ 1);
                if (st + 2 < nst) gload((st + 2) * 64);
            }
            __syncthreads();
            cur ^= 1;
        }
    }
    // epilogue: lane l, register r of a block holds D[4*(l/16) + r][l%16]
    const Field F = g.F;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = ti0 + wm * 64 + x * 16 + 4 * kg + r, col = tj0 + wn * 32 + y * 16 + r16;
                if (row < g.m && col < g.n && (!LOWER_C || col <= row)) {
                    double v = 0.0;
#pragma unroll
                    for (int q = 0; q < NS; ++q) v = fma(fred((double)acc[x][y][q][r], F), g.w[q], v);
                    double* c = g.C + row * g.ldc + col;
                    *c = fred(*c - fred(v, F), F);
                }
            }
    stamp_end(g.stamp);
}

template <int L>
void split_launch(hipStream_t s, const Field& F, const SplitArgs& sa) {
    hipLaunchKernelGGL(k_split_i8<L>, dim3((unsigned)sa.blk0[sa.nx]), dim3(256), 0, s, sa, F);
}

// The 128 x 128 tile from 128 such tiles (half the compute units; measured a little faster
// than the 64 x 64 tile there), else 64 x 64.
template <int L>
void gemm_launch(hipStream_t s, I8Args g, bool lower_c) {
    const int64_t tmb = (g.m + I8B_TILE - 1) / I8B_TILE, tnb = (g.n + I8B_TILE - 1) / I8B_TILE;
    const int64_t big = lower_c ? tmb * (tmb + 1) / 2 : tmb * tnb;
    if (big >= 128) {
        g.tiles_n = (int)tnb;
        if (lower_c) hipLaunchKernelGGL((k_gemm_i8_big<L, true>), dim3((unsigned)big), dim3(I8B_THREADS), 0, s, g);
        else hipLaunchKernelGGL((k_gemm_i8_big<L, false>), dim3((unsigned)big), dim3(I8B_THREADS), 0, s, g);
        return;
    }
    const int tm = (int)((g.m + 63) / 64);
    const int blocks = lower_c ? tm * (tm + 1) / 2 : tm * g.tiles_n;
    if (lower_c) hipLaunchKernelGGL((k_gemm_i8<L, true>), dim3(blocks), dim3(256), 0, s, g);
    else hipLaunchKernelGGL((k_gemm_i8<L, false>), dim3(blocks), dim3(256), 0, s, g);
}
}  // namespace

int i8_limbs(uint32_t p) { return p < 256u ? 1 : (p < 32768u ? 2 : 3); }

size_t i8_workspace_bytes(uint32_t p, int64_t m, int64_t n, const GemmSeg* segs, int nseg) {
    const int L = i8_limbs(p);
    size_t b = 0;
    for (int i = 0; i < nseg; ++i) {
        if (segs[i].k <= 0) continue;
        const int64_t Kp = (segs[i].k + 63) / 64 * 64;
        b += (size_t)L * (size_t)(m + n) * (size_t)Kp + 256;
    }
    return b;
}

bool i8_prepare(hipStream_t s, const Field& F, int64_t m, int64_t n, const GemmSeg* segs, int nseg, bool b_upper,
                int8_t* ws, size_t ws_bytes, I8Product* out) {
    const uint32_t p = (uint32_t)F.ip;
    if (p >= (1u << 23)) return false;   // 3 balanced digits cover |a| < 2^22 only: such products run on FP64
    const int L = i8_limbs(p);
    if (i8_workspace_bytes(p, m, n, segs, nseg) > ws_bytes) return false;
    int64_t ktot = 0;   // both segments share the INT32 accumulators
    for (int i = 0; i < nseg && i < 2; ++i) ktot += std::max<int64_t>(segs[i].k, 0);
    if (ktot > I8_MAX_KTOT) return false;
    *out = I8Product{};
    out->m = m; out->n = n; out->L = L;
    int8_t* cur = ws;
    SplitArgs sa{};
    auto add = [&](MatV X, int64_t rows, int64_t K, int64_t Kp, bool upper, int8_t* planes) {
        const int q = sa.nx++;
        sa.X[q] = X; sa.rows[q] = rows; sa.K[q] = K; sa.Kp[q] = Kp; sa.upper[q] = upper ? 1 : 0;
        sa.planes[q] = planes;
        sa.blk0[q + 1] = sa.blk0[q] + (rows + SPLIT_T - 1) / SPLIT_T * (Kp / SPLIT_T);
    };
    for (int i = 0; i < 2; ++i) {
        if (i >= nseg || segs[i].k <= 0) continue;
        const int64_t K = segs[i].k, Kp = (K + 63) / 64 * 64;
        int8_t* ap = cur;
        int8_t* bp = ap + (size_t)L * m * Kp;
        cur = bp + (size_t)L * n * Kp;
        cur += (256 - ((uintptr_t)cur & 255)) & 255;
        // B^T (n x K): element (j, k) = B(k, j)
        const MatV bt{segs[i].B.p, segs[i].B.cs, segs[i].B.rs};
        add(segs[i].A, m, K, Kp, false, ap);
        add(bt, n, K, Kp, b_upper && i == 0, bp);
        out->A[i] = ap; out->B[i] = bp; out->Kp[i] = Kp;
    }
    if (sa.nx > 0) {
        if (sa.blk0[sa.nx] >= ((int64_t)1 << 31)) return false;
        if (L == 1) split_launch<1>(s, F, sa);
        if (L == 2) split_launch<2>(s, F, sa);
        if (L == 3) split_launch<3>(s, F, sa);
    }
    return true;
}

void i8_run(hipStream_t s, const Field& F, const I8Product& pr, double* C, int64_t ldc, bool lower_c, Stamp stamp) {
    if (pr.m <= 0 || pr.n <= 0 || (pr.Kp[0] <= 0 && pr.Kp[1] <= 0)) return;
    const uint32_t p = (uint32_t)F.ip;
    I8Args g{};
    g.m = pr.m; g.n = pr.n; g.C = C; g.ldc = ldc; g.F = F;
    g.tiles_n = (int)((pr.n + 63) / 64);
    g.stamp = stamp;
    double w = 1.0;
    for (int sidx = 0; sidx < 5; ++sidx) { g.w[sidx] = w; w = std::fmod(w * 256.0, (double)p); }
    for (int i = 0; i < 2; ++i) { g.A[i] = pr.A[i]; g.B[i] = pr.B[i]; g.Kp[i] = pr.Kp[i]; }
    if (pr.L == 1) gemm_launch<1>(s, g, lower_c);
    if (pr.L == 2) gemm_launch<2>(s, g, lower_c);
    if (pr.L == 3) gemm_launch<3>(s, g, lower_c);
}

}  // namespace pldl
