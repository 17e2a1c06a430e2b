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
//
// Structure: workgroup tile BM x BN (128x128 with 16 waves in a 2x8 grid, or
// 64x64 with 16 waves in a 4x4 grid when the big tiles would leave CUs idle), K
// tiles of 32 (big) or 16 (small) staged through double-buffered LDS (one
// barrier per K tile), later K tiles' global loads in flight while the current
// one feeds the matrix cores.
#include <type_traits>

#include "common.h"

namespace pldl {

namespace {
constexpr int PAD = 2;   // LDS row padding (doubles): breaks the bank conflicts of the transposed tile stores
// K depth of an LDS tile: 32 on both tiles (twice the matrix-core work per
// barrier of 16: 3-4% faster on the largest products, and fewer barriers on the
// short K loops of the small ones)
template <int BM> constexpr int gemm_bk() { return 32; }
// waves of a workgroup (up to BN/16 along n, the rest along m): more waves than
// SIMDs let one wave's loads and barrier waits overlap another's matrix-core work
constexpr int BIG_WAVES = 16, SMALL_WAVES = 16;
template <int BM> constexpr int gemm_threads() { return 64 * (BM == 128 ? BIG_WAVES : SMALL_WAVES); }
typedef double d4 __attribute__((ext_vector_type(4)));

struct GemmKArgs {
    int64_t m, n;
    double* C;
    int64_t ldc;
    MatV A[2], B[2];
    int64_t K[2];
    Field F;
    int tiles_n;
    Stamp stamp;
};

template <int BM, int BN, bool A_ROW, bool B_ROW, bool LOWER_C, bool B_UPPER>
__global__ __launch_bounds__(gemm_threads<BM>()) void k_gemm(GemmKArgs g) {
    constexpr int NT = gemm_threads<BM>(), NW = NT / 64, BK = gemm_bk<BM>();
    constexpr int WGN = NW / 2 < BN / 16 ? NW / 2 : BN / 16, WGM = NW / WGN;   // wave grid
    constexpr int WM = BM / WGM, WN = BN / WGN;  // wave tile
    static_assert(WM % 16 == 0 && WN % 16 == 0 && WGM * WGN == NW, "wave grid");
    constexpr int FM = WM / 16, FN = WN / 16;    // 16x16 MFMA blocks per wave
    constexpr int AE = BM * BK / NT, BE = BN * BK / NT;
    __shared__ double As[2][BK][BM + PAD];
    __shared__ double Bs[2][BK][BN + PAD];
    const Field F = g.F;
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
    const int64_t i0 = (int64_t)ti * BM, j0 = (int64_t)tj * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const int lr = lane & 15, lk = lane >> 4;

    // per-thread load coordinates inside a tile (element e adds a fixed step)
    //   A row-major:  row tid/BK + (NT/BK)e, col tid%BK   A col-major: row tid%BM, col tid/BM + (NT/BM)e
    //   B row-major:  k tid/BN + (NT/BN)e, col tid%BN     B col-major: k tid%BK, col tid/BK + (NT/BK)e
    const int a_r0 = A_ROW ? tid / BK : tid % BM, a_c0 = A_ROW ? tid % BK : tid / BM;
    const int a_dr = A_ROW ? NT / BK : 0, a_dc = A_ROW ? 0 : NT / BM;
    const int b_k0 = B_ROW ? tid / BN : tid % BK, b_c0 = B_ROW ? tid % BN : tid / BK;
    const int b_dk = B_ROW ? NT / BN : 0, b_dc = B_ROW ? 0 : NT / BK;

    d4 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    // The small tile reads its C entries now (clamped in bounds, used only where
    // the epilogue stores), so that their latency overlaps the K loop instead of
    // adding to it: a small product has few K tiles.  C is written only in the
    // epilogue, so an in-place product (C the A operand) reads the same values.
    constexpr bool PRE_C = BM == 64;
    double cpre[PRE_C ? FM : 1][PRE_C ? FN : 1][4];
    if (PRE_C) {
#pragma unroll
        for (int x = 0; x < FM; ++x)
#pragma unroll
            for (int y = 0; y < FN; ++y)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = min(i0 + wm * WM + x * 16 + lk + 4 * r, g.m - 1);
                    const int64_t col = min(j0 + wn * WN + y * 16 + lr, g.n - 1);
                    cpre[x][y][r] = g.C[row * g.ldc + col];
                }
    }

    // Global loads run PD K tiles ahead of the matrix cores through PD register
    // sets (two for the small tile, whose K tiles carry little work to hide a
    // memory latency behind; one for the big tile, bounded by registers); LDS is
    // double-buffered with one barrier per K tile.
    constexpr int PD = BM == 64 ? 2 : 1;
    int since = 0;
    double ra[PD][AE], rb[PD][BE];
    uint32_t va[PD], vb[PD];
#pragma unroll 1
    for (int seg = 0; seg < 2; ++seg) {
        const int64_t K = g.K[seg];
        if (K <= 0) continue;
        const MatV A = g.A[seg], B = g.B[seg];
        const bool mask_b = B_UPPER && seg == 0;
        // Loads are unconditional (out-of-range coordinates are clamped to the last
        // valid row/column) so that all of them are in flight together; the
        // validity masks are applied when the values are written to LDS.
        const int64_t mlast = g.m - 1, nlast = g.n - 1, klast = K - 1;
        auto load = [&](auto slot_c, int64_t kt) {
            constexpr int sl = decltype(slot_c)::value;
            va[sl] = 0; vb[sl] = 0;
#pragma unroll
            for (int e = 0; e < AE; ++e) {
                const int64_t gi = i0 + a_r0 + a_dr * e, gk = kt + a_c0 + a_dc * e;
                const bool ok = gi <= mlast && gk <= klast;
                va[sl] |= (ok ? 1u : 0u) << e;
                ra[sl][e] = A.p[min(gi, mlast) * A.rs + min(gk, klast) * A.cs];
            }
#pragma unroll
            for (int e = 0; e < BE; ++e) {
                const int64_t gk = kt + b_k0 + b_dk * e, gj = j0 + b_c0 + b_dc * e;
                const bool ok = gk <= klast && gj <= nlast && !(mask_b && gk > gj);
                vb[sl] |= (ok ? 1u : 0u) << e;
                rb[sl][e] = B.p[min(gk, klast) * B.rs + min(gj, nlast) * B.cs];
            }
        };
        auto store = [&](auto slot_c, int buf) {
            constexpr int sl = decltype(slot_c)::value;
#pragma unroll
            for (int e = 0; e < AE; ++e)
                As[buf][a_c0 + a_dc * e][a_r0 + a_dr * e] = ((va[sl] >> e) & 1u) ? fcen(ra[sl][e], F) : 0.0;
#pragma unroll
            for (int e = 0; e < BE; ++e)
                Bs[buf][b_k0 + b_dk * e][b_c0 + b_dc * e] = ((vb[sl] >> e) & 1u) ? fcen(rb[sl][e], F) : 0.0;
        };
        using S0 = std::integral_constant<int, 0>;
        using S1 = std::integral_constant<int, (PD > 1 ? 1 : 0)>;
        const int64_t nt = (K + BK - 1) / BK;
        __syncthreads();   // LDS of a previous segment fully consumed
        // tile 0 to LDS; tile tau waits in register set tau % PD
        load(S0{}, 0);
        store(S0{}, 0);
        if (nt > 1) load(S1{}, BK);
        if (PD > 1 && nt > 2) load(S0{}, 2 * BK);
        __syncthreads();
        int cur = 0;
        // one K tile: feed the matrix cores from LDS, move tile t+1 from its register
        // set to the other buffer, refill that set with tile t+1+PD
        // (the LDS reads of the next k step are issued before this step's products)
        auto body = [&](int64_t t, auto slot_c) {
            double a[2][FM], b[2][FN];
#pragma unroll
            for (int q = 0; q < FM; ++q) a[0][q] = As[cur][lk][wm * WM + q * 16 + lr];
#pragma unroll
            for (int q = 0; q < FN; ++q) b[0][q] = Bs[cur][lk][wn * WN + q * 16 + lr];
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                const int c = (kk / 4) & 1;
                if (kk + 4 < BK) {
#pragma unroll
                    for (int q = 0; q < FM; ++q) a[c ^ 1][q] = As[cur][kk + 4 + lk][wm * WM + q * 16 + lr];
#pragma unroll
                    for (int q = 0; q < FN; ++q) b[c ^ 1][q] = Bs[cur][kk + 4 + lk][wn * WN + q * 16 + lr];
                }
                __builtin_amdgcn_sched_barrier(0);   // keep those reads ahead of the products
#pragma unroll
                for (int x = 0; x < FM; ++x)
#pragma unroll
                    for (int y = 0; y < FN; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][x], b[c][y], acc[x][y], 0, 0, 0);
            }
            if (t + 1 < nt) {
                store(slot_c, cur ^ 1);
                if (t + 1 + PD < nt) load(slot_c, (t + 1 + PD) * BK);
            }
            __syncthreads();
            cur ^= 1;
            since += BK;
            if (since + BK > F.kred) {   // the next tile would pass the exactness bound
#pragma unroll
                for (int x = 0; x < FM; ++x)
#pragma unroll
                    for (int y = 0; y < FN; ++y)
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[x][y][r] = fred(acc[x][y][r], F);
                since = 0;
            }
        };
#pragma unroll 1
        for (int64_t t = 0; t < nt; t += PD) {
            body(t, S1{});                        // tile t+1 sits in set (t+1) % PD
            if (PD > 1 && t + 1 < nt) body(t + 1, S0{});
        }
    }
    // epilogue: v_mfma_f64_16x16x4f64 result layout: lane l, register r holds D[l/16 + 4r][l%16]
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
        for (int y = 0; y < FN; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = i0 + wm * WM + x * 16 + lk + 4 * r;
                const int64_t col = j0 + wn * WN + y * 16 + lr;
                if (row < g.m && col < g.n && (!LOWER_C || col <= row)) {
                    double* c = g.C + row * g.ldc + col;
                    const double cv = PRE_C ? cpre[PRE_C ? x : 0][PRE_C ? y : 0][r] : *c;
                    double v = fred(cv - fred(acc[x][y][r], F), F);
                    *c = v;
                }
            }
    stamp_end(g.stamp);
}

template <int BM, int BN, bool AR, bool BR>
void dispatch(hipStream_t s, const GemmKArgs& g, int blocks, bool lower_c, bool b_upper) {
    if (lower_c) {
        if (b_upper) hipLaunchKernelGGL((k_gemm<BM, BN, AR, BR, true, true>), dim3(blocks), dim3(gemm_threads<BM>()), 0, s, g);
        else hipLaunchKernelGGL((k_gemm<BM, BN, AR, BR, true, false>), dim3(blocks), dim3(gemm_threads<BM>()), 0, s, g);
    } else {
        if (b_upper) hipLaunchKernelGGL((k_gemm<BM, BN, AR, BR, false, true>), dim3(blocks), dim3(gemm_threads<BM>()), 0, s, g);
        else hipLaunchKernelGGL((k_gemm<BM, BN, AR, BR, false, false>), dim3(blocks), dim3(gemm_threads<BM>()), 0, s, g);
    }
}

template <int BM, int BN>
void dispatch_layout(hipStream_t s, GemmKArgs& g, bool ar, bool br, bool lower_c, bool b_upper) {
    const int tm = (int)((g.m + BM - 1) / BM), tn = (int)((g.n + BN - 1) / BN);
    g.tiles_n = tn;
    const int blocks = lower_c ? tm * (tm + 1) / 2 : tm * tn;
    if (ar && br) dispatch<BM, BN, true, true>(s, g, blocks, lower_c, b_upper);
    else if (ar && !br) dispatch<BM, BN, true, false>(s, g, blocks, lower_c, b_upper);
    else if (!ar && br) dispatch<BM, BN, false, true>(s, g, blocks, lower_c, b_upper);
    else dispatch<BM, BN, false, false>(s, g, blocks, lower_c, b_upper);
}
}  // namespace

void launch_gemm(hipStream_t s, const Field& F, int64_t m, int64_t n, double* C, int64_t ldc,
                 const GemmSeg* segs, int nseg, bool lower_c, bool b_upper, Stamp stamp) {
    if (m <= 0 || n <= 0) return;
    GemmKArgs g{};
    g.m = m; g.n = n; g.C = C; g.ldc = ldc; g.F = F;
    g.stamp = stamp;
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
    const int first = g.K[0] > 0 ? 0 : 1;
    const bool ar = g.A[first].cs == 1, br = g.B[first].cs == 1;
    // big tiles unless they would leave most of the 256 CUs idle
    const int64_t t128 = ((m + 127) / 128) * ((n + 127) / 128) / (lower_c ? 2 : 1);
    if (t128 >= 192) dispatch_layout<128, 128>(s, g, ar, br, lower_c, b_upper);
    else dispatch_layout<64, 64>(s, g, ar, br, lower_c, b_upper);
}

}  // namespace pldl
