// batched.hip -- many small factorizations in one persistent launch.
//
// Each workgroup takes matrix indices from a device counter until the batch is
// exhausted and factors its matrix (n <= NB_MAX) with the base-case
// elimination of Section 5: rows are visited in increasing order, the pivot of
// row i is the first nonzero of its Schur-complement row among the rows still
// alive (a diagonal pivot is a 1x1 block, an off-diagonal one j a 2x2 block
// (i, j), relaxed in characteristic 2), an all-zero row is set aside keeping
// its precedence.  The result is the canonical order of that elimination; it
// reveals the rank profile matrix (Theorem 1) like the recursive cascade.
//
// The Schur complement lives in a private slot as exact residues in FP32
// (|value| < p < 2^24), lower triangle stored by columns: entry (k, l), k >= l,
// at S[l * n + k], so the column a pivot step reads is contiguous.  Updates are
// lazy: a 1x1 pivot contributes one rank-1 term u v^T, a 2x2 pivot two; up to
// KMAX terms wait in LDS.  Only the column factor v of a term is stored (by
// row); its row factor u is recovered mod p from the row's stored factors and
// two scalars of the pivot step, which halves the LDS a term takes.  A pivot
// step reads its column from the slot and subtracts the waiting terms for that
// column only; when the window is full, one pass over the alive triangle
// applies all of them (FP64 accumulation of at most KMAX products below
// (p-1)^2/4 each onto a reduced value: far below 2^53) and stores the reduced
// result.  The multiplier of alive row k for pivot column c goes to the
// position of (k, c) as soon as c is eliminated; a row set aside leaves zeros
// in its column.  A step is a chain of short latencies (a column read, two
// barriers, a ballot), so the design keeps LDS per workgroup small enough for
// WG_PER_CU matrices in flight on each CU.  Everything happens on the device
// (no host synchronisation), so the call can be captured in a graph.
#include "../../include/pldl.h"
#include "common.h"

namespace pldl {

namespace {

constexpr int NB_MAX = 512;       // largest order of a batched matrix
constexpr int NTH = 512;          // threads per workgroup
constexpr int NWAVE = NTH / 64;   // waves per workgroup
constexpr int WG_PER_CU = 4;      // workgroups resident per CU (LDS and register budget)
constexpr int KMAX = 12;          // rank-1 terms applied per pass over the triangle
constexpr int CG = 8;             // columns whose loads are in flight together in a pass
static_assert(NB_MAX <= NTH, "one thread per row of a batched matrix");

struct BatchArgs {
    int64_t batch;
    const int64_t* n;
    void* const* A;
    const int64_t* lda;
    int32_t dtype;
    void* const* e;
    int32_t* const* perm;
    int32_t* const* rpm;
    int64_t* rank;
    int32_t* status;
    float* ws;           // one NB_MAX^2 slot per workgroup
    int32_t* queue;      // next position in `order`
    const int32_t* order; // matrix indices, largest order first
    Field F;
    int check_range;
};

__device__ __forceinline__ double ld_in(const void* A, int32_t dtype, int64_t off) {
    return dtype == PLDL_U32 ? (double)((const uint32_t*)A)[off] : ((const double*)A)[off];
}
__device__ __forceinline__ void st_out(void* A, int32_t dtype, int64_t off, double v) {
    if (dtype == PLDL_U32) ((uint32_t*)A)[off] = (uint32_t)v;
    else ((double*)A)[off] = v;
}

// Inverse of a pivot: table read through the scalar path (the index is uniform,
// the table read-only), else the extended Euclidean algorithm.
__device__ __forceinline__ double inverse(double x, const Field& F, const uint32_t* __restrict__ itab) {
    if (itab) return (double)itab[__builtin_amdgcn_readfirstlane((int)x)];
    return finv(x, F);
}

struct BatchShared {
    float v[NB_MAX][KMAX];     // column factor of each waiting term, by row
    float ta[KMAX], tb[KMAX];  // row factor of term t at row k: ta[t] v[k][t] + tb[t] v[k][tp[t]]
    int tp[KMAX];
    float colI[NB_MAX], colJ[NB_MAX];
    float bx[NB_MAX], by[NB_MAX];
    int16_t order[NB_MAX], zeros[NB_MAX], sig[NB_MAX];
    uint8_t alv[NB_MAX], bt[NB_MAX];
    int64_t m;
};

// Row factor of waiting term t at a row whose stored column factors are vk.  A
// 1x1 pivot x (term b c^T, b = c / x) stores c, so b = x^-1 c.  A 2x2 pair
// (terms (e + f) b^T and c a^T, with a = e / x, b = c / x, f = d22 b) stores b
// (term t) and a (term t + 1), so e + f = d22 b + x a and c = x b.  Both forms
// are ta[t] vk[t] + tb[t] vk[tp[t]], mod p, centered; each product is below
// p^2 / 2.
__device__ __forceinline__ double urow(const float* vk, const BatchShared& sh, int t, const Field& F) {
    return fredc(fma((double)sh.ta[t], (double)vk[t], (double)sh.tb[t] * (double)vk[sh.tp[t]]), F);
}

// Applies the npend waiting terms to every alive entry (k, l), k >= l >= i0 (all
// alive indices are >= i0).  Work items are 64x64 tiles of the lower triangle,
// dealt round-robin to the waves; a lane owns one row k of its tile and walks
// the alive columns of the tile CG at a time, all CG loads issued before use.
__device__ void flush_terms(const BatchShared& sh, float* S, int n, int i0, int npend, const Field& F, int wave,
                            int lane) {
    const int c0 = i0 >> 6, nch = (n + 63) >> 6;
    int tile = 0;
    for (int c = c0; c < nch; ++c)
        for (int b = c0; b <= c; ++b, ++tile) {
            if (tile % NWAVE != wave) continue;
            // keeps the per-term scalars from being hoisted out of the tile loop into
            // registers (they are cheap LDS broadcasts)
            __asm__ __volatile__("" ::: "memory");
            const int k = 64 * c + lane;
            const bool kal = k < n && sh.alv[k];
            const int kc = k < n ? k : n - 1;   // in-bounds row for lanes past the end
            float uk[KMAX];
#pragma unroll
            for (int t = 0; t < KMAX; ++t) uk[t] = (kal && t < npend) ? (float)urow(sh.v[kc], sh, t, F) : 0.0f;
            const int lb = 64 * b + lane;
            uint64_t live = __ballot(lb < n && sh.alv[lb]);
            while (live) {
                int ls[CG];
                float sv[CG];
#pragma unroll
                for (int q = 0; q < CG; ++q) {
                    ls[q] = live ? 64 * b + __ffsll((long long)live) - 1 : -1;
                    live &= live - 1;
                }
                // every load unconditional and in bounds (l, kc < n), so all CG are in flight
                // together; values of lanes or columns that take no update are not used
#pragma unroll
                for (int q = 0; q < CG; ++q) sv[q] = S[(ls[q] >= 0 ? ls[q] : ls[0]) * n + kc];
#pragma unroll
                for (int q = 0; q < CG; ++q) {
                    const int l = ls[q];
                    if (l >= 0 && kal && l <= k) {
                        const float* vl = sh.v[l];
                        double acc = (double)sv[q];
#pragma unroll
                        for (int t = 0; t < KMAX; ++t) acc = fma(-(double)uk[t], (double)vl[t], acc);
                        S[l * n + k] = (float)fredc(acc, F);
                    }
                }
            }
        }
}

__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(8))) void k_factor_batched(
    BatchArgs g, const uint32_t* __restrict__ itab) {
    __shared__ BatchShared sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const Field F = g.F;
    float* S = g.ws + (int64_t)blockIdx.x * NB_MAX * NB_MAX;
    // the term buffer only ever holds finite residues: a zero row factor then
    // cancels whatever a column factor slot holds
    for (int q = tid; q < KMAX * NB_MAX; q += NTH) (&sh.v[0][0])[q] = 0.0f;

    for (;;) {
        if (tid == 0) {
            const int64_t q = atomicAdd(g.queue, 1);
            sh.m = q < g.batch ? (int64_t)g.order[q] : g.batch;
        }
        __syncthreads();
        const int64_t mi = sh.m;
        __syncthreads();
        if (mi >= g.batch) return;
        const int n = (int)g.n[mi];
        const int64_t lda = g.lda[mi];
        void* A = g.A[mi];
        if (g.n[mi] < 0 || g.n[mi] > NB_MAX || lda < (int64_t)(n > 1 ? n : 1) ||
            (n > 0 && (!A || !g.e[mi] || !g.perm[mi] || !g.rpm[mi]))) {
            if (tid == 0) { g.status[mi] = -3; g.rank[mi] = 0; }
            continue;
        }
        if (n == 0) {
            if (tid == 0) { g.status[mi] = 0; g.rank[mi] = 0; }
            continue;
        }
        // ---- load the lower triangle (centered) column by column, check the range
        int bad = 0;
        for (int l = wave; l < n; l += NWAVE)
            for (int k = l + lane; k < n; k += 64) {
                const double v = ld_in(A, g.dtype, (int64_t)k * lda + l);
                bad |= (v >= F.p || v < 0.0);
                S[l * n + k] = (float)fcen(v, F);
            }
        for (int k = tid; k < n; k += NTH) sh.alv[k] = 1;
        bad = __syncthreads_or(bad);
        if (bad && g.check_range) {
            if (tid == 0) { g.status[mi] = PLDL_ERANGE; g.rank[mi] = 0; }
            continue;
        }
        // ---- elimination; thread k owns row k
        int r = 0, nz = 0, np = 0;
        const int k = tid;
        const int kc = k < n ? k : n - 1;   // in-bounds row for the unconditional column loads
        float pre = 0.0f;                   // slot column pre_i at row kc, loaded one step ahead
        int pre_i = -1;
        for (int i = 0; i < n; ++i) {
            if (!sh.alv[i]) continue;
            if (np + 2 > KMAX) {
                flush_terms(sh, S, n, i, np, F, wave, lane);
                np = 0;
                pre_i = -1;
                __syncthreads();
            }
            // Column i of the slot changes only in a pass over the triangle (pivot steps
            // write multipliers to eliminated positions only), so the copy loaded during
            // the previous step is current unless a pass ran since.  The next column is
            // loaded now, ahead of its step.
            const float raw = pre_i == i ? pre : S[i * n + kc];
            if (i + 1 < n) {
                pre = S[(i + 1) * n + kc];
                pre_i = i + 1;
            }
            // column i of the Schur complement (alive rows, all >= i), waiting terms applied
            if (k < n) {
                double c = 0.0;
                if (k >= i && sh.alv[k]) {
                    double a = (double)raw;
                    for (int t = 0; t < np; ++t) a = fma(-urow(sh.v[k], sh, t, F), (double)sh.v[i][t], a);
                    c = fredc(a, F);
                }
                sh.colI[k] = (float)c;
            }
            __syncthreads();
            int j = -1;
            for (int q = i >> 6; q * 64 < n && j < 0; ++q) {
                const int kk = q * 64 + lane;
                const unsigned long long bal = __ballot(kk < n && sh.colI[kk] != 0.0f);
                if (bal) j = q * 64 + __ffsll((long long)bal) - 1;
            }
            if (j < 0) {   // zero row: set aside, precedence kept, its column left zero
                if (k < n && k > i && sh.alv[k]) S[i * n + k] = 0.0f;
                if (tid == 0) { sh.zeros[nz] = (int16_t)i; sh.alv[i] = 0; }
                ++nz;
                __syncthreads();
                continue;
            }
            if (j == i) {  // 1x1 pivot x: term b c^T with b = c / x; L(k, i) = b_k
                const double x = fcan((double)sh.colI[i], F);
                const double xi = inverse(x, F, itab);
                if (k < n) {
                    float v = 0.0f;
                    if (k > i && sh.alv[k]) {
                        const double ck = (double)sh.colI[k];
                        S[i * n + k] = (float)fcan(fredc(ck * xi, F), F);
                        v = (float)ck;
                    }
                    sh.v[k][np] = v;
                }
                if (tid == 0) {
                    sh.bx[r] = (float)x; sh.bt[r] = 1; sh.order[r] = (int16_t)i; sh.alv[i] = 0;
                    sh.ta[np] = (float)xi; sh.tb[np] = 0.0f; sh.tp[np] = np;
                }
                np += 1;
                r += 1;
            } else {       // 2x2 pivot on (i, j), j > i
                if (k < n) {
                    double c = 0.0;
                    if (k >= i && sh.alv[k]) {
                        const int hi = k > j ? k : j, lo = k > j ? j : k;
                        double a = (double)S[lo * n + hi];
                        for (int t = 0; t < np; ++t) a = fma(-urow(sh.v[hi], sh, t, F), (double)sh.v[lo][t], a);
                        c = fredc(a, F);
                    }
                    sh.colJ[k] = (float)c;
                }
                __syncthreads();
                const double x = fcan((double)sh.colI[j], F), y = fcan((double)sh.colJ[j], F);
                const double xi = inverse(x, F, itab);
                double w, d22, lji;
                if (F.ip == 2) { w = y; d22 = y; lji = 0.0; }
                else { w = fmulm(y, F.inv2, F); d22 = 0.0; lji = fmulm(w, xi, F); }
                // per row: b_k = c_k / x, e_k = d_k - w b_k, a_k = e_k / x; terms
                // (e + f) b^T and c a^T with f = d22 b; L(k, i) = a_k, L(k, j) = b_k
                if (k < n) {
                    float vb = 0.0f, va = 0.0f;
                    if (k > i && k != j && sh.alv[k]) {
                        const double ck = (double)sh.colI[k], dk = (double)sh.colJ[k];
                        const double bk = fredc(ck * xi, F);
                        const double ek = fredc(dk - fredc(w * bk, F), F);
                        const double ak = fredc(ek * xi, F);
                        S[i * n + k] = (float)fcan(ak, F);
                        if (k > j) S[j * n + k] = (float)fcan(bk, F);
                        else S[k * n + j] = (float)fcan(bk, F);
                        vb = (float)bk;
                        va = (float)ak;
                    }
                    sh.v[k][np] = vb;
                    sh.v[k][np + 1] = va;
                }
                if (tid == 0) {
                    sh.bx[r] = (float)x; sh.by[r] = (F.ip == 2) ? (float)y : 0.0f; sh.bt[r] = 2; sh.bt[r + 1] = 0;
                    sh.order[r] = (int16_t)i; sh.order[r + 1] = (int16_t)j;
                    sh.ta[np] = (float)d22; sh.tb[np] = (float)x; sh.tp[np] = np + 1;
                    sh.ta[np + 1] = 0.0f; sh.tb[np + 1] = (float)x; sh.tp[np + 1] = np;
                    S[i * n + j] = (float)lji;
                    sh.alv[i] = 0; sh.alv[j] = 0;
                }
                np += 2;
                r += 2;
            }
            __syncthreads();
        }
        // ---- output in place: order = pivots then zero rows
        for (int q = tid; q < n; q += NTH) sh.sig[q] = q < r ? sh.order[q] : sh.zeros[q - r];
        __syncthreads();
        for (int q = wave; q < n; q += NWAVE)
            for (int c = lane; c < q; c += 64) {
                double v = 0.0;
                if (c < r) {
                    const int a = sh.sig[q], bb = sh.sig[c];
                    v = fred(a > bb ? (double)S[bb * n + a] : (double)S[a * n + bb], F);
                }
                st_out(A, g.dtype, (int64_t)q * lda + c, v);
            }
        if (tid == 0) {
            int q = 0;
            for (int t = 0; t < r;) {
                if (sh.bt[t] == 1) {
                    sh.colJ[q] = sh.bx[t]; sh.colI[q] = 0.0f;
                    q += 1; t += 1;
                } else {
                    sh.colJ[q] = 0.0f; sh.colI[q] = sh.bx[t];
                    sh.colJ[q + 1] = sh.by[t]; sh.colI[q + 1] = 0.0f;
                    q += 2; t += 2;
                }
            }
            for (; q < n; ++q) { sh.colJ[q] = 0.0f; sh.colI[q] = 0.0f; }
            g.rank[mi] = r;
            g.status[mi] = 0;
        }
        __syncthreads();
        for (int q = tid; q < n; q += NTH) {
            st_out(A, g.dtype, (int64_t)q * lda + q, (double)sh.colJ[q]);
            st_out(g.e[mi], g.dtype, q, (double)sh.colI[q]);
            g.perm[mi][q] = sh.sig[q];
            g.rpm[mi][q] = -1;
        }
        __syncthreads();
        for (int t = tid; t < r; t += NTH) {
            if (sh.bt[t] == 1) g.rpm[mi][sh.order[t]] = sh.order[t];
            else if (sh.bt[t] == 2) { g.rpm[mi][sh.order[t]] = sh.order[t + 1]; g.rpm[mi][sh.order[t + 1]] = sh.order[t]; }
        }
        __syncthreads();
    }
}

__global__ void k_zero_counter(int32_t* q) { *q = 0; }

// The order the workgroups take the matrices in: largest n first (a counting
// sort on n by one workgroup; invalid orders last).  Started largest-first, the
// persistent workgroups finish together: taken in index order, a batch of
// mixed orders leaves a tail of large matrices started last.
__global__ __launch_bounds__(1024) void k_batch_order(const int64_t* n, int64_t batch, int32_t* order) {
    constexpr int NBK = NB_MAX + 2;   // bucket NB_MAX - n for 0 <= n <= NB_MAX, NB_MAX + 1 for the rest
    __shared__ int cnt[NBK];
    const int tid = threadIdx.x;
    auto key = [&](int64_t i) -> int {
        const int64_t v = n[i];
        return (v >= 0 && v <= NB_MAX) ? NB_MAX - (int)v : NB_MAX + 1;
    };
    for (int b = tid; b < NBK; b += 1024) cnt[b] = 0;
    __syncthreads();
    for (int64_t i = tid; i < batch; i += 1024) atomicAdd(&cnt[key(i)], 1);
    __syncthreads();
    if (tid == 0) {   // exclusive prefix sums: the first position of each bucket
        int run = 0;
        for (int b = 0; b < NBK; ++b) {
            const int c = cnt[b];
            cnt[b] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int64_t i = tid; i < batch; i += 1024) order[atomicAdd(&cnt[key(i)], 1)] = (int32_t)i;
}

}  // namespace

int batched_nb_max() { return NB_MAX; }

int batched_wg_per_cu() { return WG_PER_CU; }

size_t batched_slot_bytes() { return (size_t)NB_MAX * NB_MAX * sizeof(float); }

void launch_factor_batched(hipStream_t s, const Field& F, const uint32_t* itab, int64_t batch, const int64_t* n,
                           void* const* A, const int64_t* lda, int32_t dtype, void* const* e, int32_t* const* perm,
                           int32_t* const* rpm, int64_t* rank, int32_t* status, int check_range, void* ws,
                           int slots, int32_t* queue, int32_t* order) {
    BatchArgs g{};
    g.batch = batch; g.n = n; g.A = A; g.lda = lda; g.dtype = dtype; g.e = e; g.perm = perm; g.rpm = rpm;
    g.rank = rank; g.status = status; g.ws = (float*)ws; g.queue = queue; g.order = order; g.F = F;
    g.check_range = check_range;
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, s, queue);
    hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, s, n, batch, order);
    hipLaunchKernelGGL(k_factor_batched, dim3((unsigned)slots), dim3(NTH), 0, s, g, itab);
}

}  // namespace pldl
