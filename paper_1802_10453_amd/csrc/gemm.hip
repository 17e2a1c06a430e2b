// gemm.hip -- mod-p matrix product on the FP64 matrix cores of gfx950.
//
// C <- C - sum_seg A_seg * B_seg (mod p): the GEMM, TRMM (3-operand), SYRDK and
// SYRD2K building blocks of Section 3 all reduce to this kernel: SYRDK and
// SYRD2K write the lower triangle only (lower_c) and SYRD2K's two products are
// two segments of one K loop; TRMM masks the triangle of its B operand.
//
// Exactness: operands are loaded as centered residues (|v| <= (p-1)/2), the
// v_mfma_f64_16x16x4f64 products and sums are integers below 2^53 and hence
// exact in any order; the accumulators are reduced mod p every F.kred products
// (delayed reduction), and once more in the epilogue.
#include "common.h"

namespace pldl {

namespace {
constexpr int BM = 128, BN = 128, BK = 16, NT = 256, PAD = 4;
typedef double d4 __attribute__((ext_vector_type(4)));

struct GemmKArgs {
    int64_t m, n;
    double* C;
    int64_t ldc;
    MatV A[2], B[2];
    int64_t K[2];
    Field F;
    int tiles_n;
    int32_t* nzrow;   // optional: atomicMin(nzrow, nzoff + first row of C with a nonzero result)
    int32_t nzoff;
};

template <bool A_ROW, bool B_ROW, bool LOWER_C, bool B_UPPER>
__global__ __launch_bounds__(NT) void k_gemm(GemmKArgs g) {
    __shared__ double As[BK][BM + PAD];
    __shared__ double Bs[BK][BN + PAD];
    const Field F = g.F;
    int bid = blockIdx.x;
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
    const int64_t i0 = (int64_t)ti * BM, j0 = (int64_t)tj * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;

    d4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

    int since = 0;
    double ra[8], rb[8];
#pragma unroll 1
    for (int seg = 0; seg < 2; ++seg) {
        const int64_t K = g.K[seg];
        if (K <= 0) continue;
        const MatV A = g.A[seg], B = g.B[seg];
        const bool mask_b = B_UPPER && seg == 0;
        auto load = [&](int64_t kt) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                int idx = tid + e * NT;
                int r, c;
                if (A_ROW) { r = idx / BK; c = idx % BK; } else { r = idx % BM; c = idx / BM; }
                int64_t gi = i0 + r, gk = kt + c;
                double v = 0.0;
                if (gi < g.m && gk < K) v = fcen(A.p[gi * A.rs + gk * A.cs], F);
                ra[e] = v;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                int idx = tid + e * NT;
                int c, r;
                if (B_ROW) { c = idx / BN; r = idx % BN; } else { c = idx % BK; r = idx / BK; }
                int64_t gk = kt + c, gj = j0 + r;
                double v = 0.0;
                if (gk < K && gj < g.n && !(mask_b && gk > gj)) v = fcen(B.p[gk * B.rs + gj * B.cs], F);
                rb[e] = v;
            }
        };
        load(0);
#pragma unroll 1
        for (int64_t kt = 0; kt < K; kt += BK) {
            __syncthreads();
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                int idx = tid + e * NT;
                int r, c;
                if (A_ROW) { r = idx / BK; c = idx % BK; } else { r = idx % BM; c = idx / BM; }
                As[c][r] = ra[e];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                int idx = tid + e * NT;
                int c, r;
                if (B_ROW) { c = idx / BN; r = idx % BN; } else { c = idx % BK; r = idx / BK; }
                Bs[c][r] = rb[e];
            }
            __syncthreads();
            if (kt + BK < K) load(kt + BK);
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                double a[4], b[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    a[t] = As[kk + lk][wm * 64 + t * 16 + lr];
                    b[t] = Bs[kk + lk][wn * 64 + t * 16 + lr];
                }
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
            }
            since += BK;
            if (since >= F.kred) {
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y)
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[x][y][r] = fred(acc[x][y][r], F);
                since = 0;
            }
        }
    }
    // epilogue: output element (row, col) of MFMA block (x, y), register r
    int first_nz = 1 << 30;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // v_mfma_f64_16x16x4f64 result layout: lane l, register r holds D[l/16 + 4r][l%16]
                int64_t row = i0 + wm * 64 + x * 16 + lk + 4 * r;
                int64_t col = j0 + wn * 64 + y * 16 + lr;
                if (row < g.m && col < g.n && (!LOWER_C || col <= row)) {
                    double* c = g.C + row * g.ldc + col;
                    double v = fred(*c - fred(acc[x][y][r], F), F);
                    *c = v;
                    if (v != 0.0 && row < first_nz) first_nz = (int)row;
                }
            }
    if (g.nzrow) {
        // block minimum, then one atomic per block
        for (int off = 32; off > 0; off >>= 1) first_nz = min(first_nz, __shfl_xor(first_nz, off));
        __syncthreads();
        int* red = (int*)&As[0][0];
        if (lane == 0) red[wave] = first_nz;
        __syncthreads();
        if (tid == 0) {
            int v = min(min(red[0], red[1]), min(red[2], red[3]));
            if (v < (1 << 30)) atomicMin(g.nzrow, g.nzoff + v);
        }
    }
}

template <bool AR, bool BR>
void dispatch(hipStream_t s, const GemmKArgs& g, int blocks, bool lower_c, bool b_upper) {
    if (lower_c) {
        if (b_upper) hipLaunchKernelGGL((k_gemm<AR, BR, true, true>), dim3(blocks), dim3(NT), 0, s, g);
        else hipLaunchKernelGGL((k_gemm<AR, BR, true, false>), dim3(blocks), dim3(NT), 0, s, g);
    } else {
        if (b_upper) hipLaunchKernelGGL((k_gemm<AR, BR, false, true>), dim3(blocks), dim3(NT), 0, s, g);
        else hipLaunchKernelGGL((k_gemm<AR, BR, false, false>), dim3(blocks), dim3(NT), 0, s, g);
    }
}
}  // namespace

void launch_gemm(hipStream_t s, const Field& F, int64_t m, int64_t n, double* C, int64_t ldc,
                 const GemmSeg* segs, int nseg, bool lower_c, bool b_upper, int32_t* nzrow, int32_t nzoff) {
    if (m <= 0 || n <= 0) return;
    GemmKArgs g{};
    g.m = m; g.n = n; g.C = C; g.ldc = ldc; g.F = F;
    g.nzrow = nzrow; g.nzoff = nzoff;
    bool any = false;
    for (int i = 0; i < 2; ++i) {
        if (i < nseg && segs[i].k > 0) {
            g.A[i] = segs[i].A; g.B[i] = segs[i].B; g.K[i] = segs[i].k;
            any = true;
        } else {
            g.A[i] = MatV{nullptr, 0, 1}; g.B[i] = MatV{nullptr, 0, 1}; g.K[i] = 0;
        }
    }
    if (!any) return;
    // both segments share operand layouts (checked by the caller)
    int first = g.K[0] > 0 ? 0 : 1;
    bool ar = g.A[first].cs == 1, br = g.B[first].cs == 1;
    int tm = (int)((m + BM - 1) / BM), tn = (int)((n + BN - 1) / BN);
    g.tiles_n = tn;
    int blocks = lower_c ? tm * (tm + 1) / 2 : tm * tn;
    if (ar && br) dispatch<true, true>(s, g, blocks, lower_c, b_upper);
    else if (ar && !br) dispatch<true, false>(s, g, blocks, lower_c, b_upper);
    else if (!ar && br) dispatch<false, true>(s, g, blocks, lower_c, b_upper);
    else dispatch<false, false>(s, g, blocks, lower_c, b_upper);
}

}  // namespace pldl
