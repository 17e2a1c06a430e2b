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
// The Schur complement lives in a private FP64 slot (lower triangle, row-major,
// leading dimension n), updated right-looking with delayed reduction: an
// update adds at most 3 (p-1)^2/4 to an entry, and the alive part is reduced
// in place before F.kred such terms can accumulate.  The multiplier of alive
// row k for pivot column c is stored at the lower-triangle position of (k, c):
// when c is eliminated, entry (c, k) of a row k < c is no longer needed.
// Everything happens on the device (no host synchronisation), so the call can
// be captured in a graph.
#include "../../include/pldl.h"
#include "common.h"

namespace pldl {

namespace {

constexpr int NB_MAX = 512;   // largest order of a batched matrix

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
    double* ws;          // one NB_MAX^2 slot per workgroup
    int32_t* queue;      // next matrix index
    Field F;
    const uint32_t* itab;
    int check_range;
};

__device__ __forceinline__ double ld_in(const void* A, int32_t dtype, int64_t off) {
    return dtype == PLDL_U32 ? (double)((const uint32_t*)A)[off] : ((const double*)A)[off];
}
__device__ __forceinline__ void st_out(void* A, int32_t dtype, int64_t off, double v) {
    if (dtype == PLDL_U32) ((uint32_t*)A)[off] = (uint32_t)v;
    else ((double*)A)[off] = v;
}

__global__ __launch_bounds__(1024) void k_factor_batched(BatchArgs g) {
    __shared__ double colI[2][NB_MAX], colJ[NB_MAX];
    __shared__ double va[NB_MAX], vb[NB_MAX], ve[NB_MAX], vf[NB_MAX];
    __shared__ uint8_t alv[NB_MAX];
    __shared__ int order[NB_MAX], zeros[NB_MAX], sig[NB_MAX];
    __shared__ double bx[NB_MAX], by[NB_MAX];
    __shared__ uint8_t bt[NB_MAX];
    __shared__ int64_t s_m;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const Field F = g.F;
    double* S = g.ws + (int64_t)blockIdx.x * NB_MAX * NB_MAX;

    for (;;) {
        if (tid == 0) s_m = atomicAdd(g.queue, 1);
        __syncthreads();
        const int64_t mi = s_m;
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
        // ---- load the lower triangle (centered), check the range
        int bad = 0;
        for (int k = wave; k < n; k += 16)
            for (int l = lane; l <= k; l += 64) {
                const double v = ld_in(A, g.dtype, (int64_t)k * lda + l);
                bad |= (v >= F.p || v < 0.0);
                S[k * n + l] = fcen(v, F);
            }
        for (int k = tid; k < n; k += 1024) alv[k] = 1;
        bad = __syncthreads_or(bad);
        if (bad && g.check_range) {
            if (tid == 0) { g.status[mi] = PLDL_ERANGE; g.rank[mi] = 0; }
            continue;
        }
        // ---- elimination
        int r = 0, nz = 0, grow = 0, step = 0;
        for (int i = 0; i < n; ++i) {
            if (!alv[i]) continue;
            const int b = step & 1;
            ++step;
            // column i of the Schur complement (= row i), reduced; alive rows only (all >= i)
            for (int k = tid; k < n; k += 1024) colI[b][k] = alv[k] ? fredc(S[k * n + i], F) : 0.0;
            __syncthreads();
            int j = -1;
            for (int q = i >> 6; q * 64 < n && j < 0; ++q) {
                const int kk = q * 64 + lane;
                const unsigned long long bal = __ballot(kk < n && colI[b][kk] != 0.0);
                if (bal) j = q * 64 + __ffsll((long long)bal) - 1;
            }
            if (j < 0) {   // zero row: set aside, precedence kept
                if (tid == 0) { zeros[nz] = i; alv[i] = 0; }
                ++nz;
                __syncthreads();
                continue;
            }
            if (j == i) {  // 1x1 pivot x: S -= c c^T / x, L(k, i) = c_k / x
                const double x = fcan(colI[b][i], F);
                const double xi = g.itab ? (double)g.itab[(int)x] : finv(x, F);
                if (tid == 0) { bx[r] = x; bt[r] = 1; order[r] = i; }
                for (int k = wave; k < n; k += 16) {
                    if (k == i || !alv[k]) continue;
                    const double bk = fredc(colI[b][k] * xi, F);
                    for (int l = lane; l <= k; l += 64)
                        if (l != i && alv[l]) S[k * n + l] = fma(-bk, colI[b][l], S[k * n + l]);
                    if (lane == 0) S[k * n + i] = fcan(bk, F);
                }
                if (tid == 0) alv[i] = 0;
                grow += 1;
                r += 1;
            } else {       // 2x2 pivot on (i, j), j > i
                for (int k = tid; k < n; k += 1024) {
                    const int hi = k > j ? k : j, lo = k > j ? j : k;
                    colJ[k] = alv[k] ? fredc(S[hi * n + lo], F) : 0.0;
                }
                __syncthreads();
                const double x = fcan(colI[b][j], F), y = fcan(colJ[j], F);
                const double xi = g.itab ? (double)g.itab[(int)x] : finv(x, F);
                double w, d22, lji;
                if (F.ip == 2) { w = y; d22 = y; lji = 0.0; }
                else { w = fmulm(y, F.inv2, F); d22 = 0.0; lji = fmulm(w, xi, F); }
                if (tid == 0) {
                    bx[r] = x; by[r] = (F.ip == 2) ? y : 0.0; bt[r] = 2; bt[r + 1] = 0;
                    order[r] = i; order[r + 1] = j;
                }
                // per-row coefficients: b_k = c_k / x, e_k = d_k - w b_k, a_k = e_k / x, f_k = d22 b_k
                for (int k = tid; k < n; k += 1024) {
                    const bool al = alv[k] && k != i && k != j;
                    const double ci = al ? colI[b][k] : 0.0, cj = al ? colJ[k] : 0.0;
                    const double bk = fredc(ci * xi, F);
                    const double ek = fredc(cj - fredc(w * bk, F), F);
                    vb[k] = bk;
                    ve[k] = ek;
                    va[k] = fredc(ek * xi, F);
                    vf[k] = fredc(d22 * bk, F);
                }
                __syncthreads();
                // S[k][l] -= e_k b_l + c_k a_l + f_k b_l; L(k, i) = a_k, L(k, j) = b_k
                for (int k = wave; k < n; k += 16) {
                    if (k == i || k == j || !alv[k]) continue;
                    const double ek = ve[k], ck = colI[b][k], fk = vf[k];
                    for (int l = lane; l <= k; l += 64) {
                        if (l == i || l == j || !alv[l]) continue;
                        double t = S[k * n + l];
                        t = fma(-ek, vb[l], t);
                        t = fma(-ck, va[l], t);
                        t = fma(-fk, vb[l], t);
                        S[k * n + l] = t;
                    }
                    if (lane == 0) {
                        S[k * n + i] = fcan(va[k], F);
                        if (k > j) S[k * n + j] = fcan(vb[k], F);
                        else S[j * n + k] = fcan(vb[k], F);
                    }
                }
                if (tid == 0) { S[j * n + i] = lji; alv[i] = 0; alv[j] = 0; }
                grow += 3;
                r += 2;
            }
            __syncthreads();
            if (2 * (grow + 3) > F.kred) {   // reduce the alive part well before the exactness bound
                for (int k = wave; k < n; k += 16) {
                    if (!alv[k]) continue;
                    for (int l = lane; l <= k; l += 64)
                        if (alv[l]) S[k * n + l] = fredc(S[k * n + l], F);
                }
                grow = 0;
                __syncthreads();
            }
        }
        // ---- output in place: order = pivots then zero rows
        for (int q = tid; q < n; q += 1024) sig[q] = q < r ? order[q] : zeros[q - r];
        __syncthreads();
        for (int q = wave; q < n; q += 16)
            for (int c = lane; c < q; c += 64) {
                double v = 0.0;
                if (c < r) {
                    const int a = sig[q], bb = sig[c];
                    v = fred(a > bb ? S[a * n + bb] : S[bb * n + a], F);
                }
                st_out(A, g.dtype, (int64_t)q * lda + c, v);
            }
        if (tid == 0) {
            int q = 0;
            for (int t = 0; t < r;) {
                if (bt[t] == 1) {
                    colJ[q] = bx[t]; va[q] = 0.0;
                    q += 1; t += 1;
                } else {
                    colJ[q] = 0.0; va[q] = bx[t];
                    colJ[q + 1] = by[t]; va[q + 1] = 0.0;
                    q += 2; t += 2;
                }
            }
            for (; q < n; ++q) { colJ[q] = 0.0; va[q] = 0.0; }
            g.rank[mi] = r;
            g.status[mi] = 0;
        }
        __syncthreads();
        for (int q = tid; q < n; q += 1024) {
            st_out(A, g.dtype, (int64_t)q * lda + q, colJ[q]);
            st_out(g.e[mi], g.dtype, q, va[q]);
            g.perm[mi][q] = sig[q];
            g.rpm[mi][q] = -1;
        }
        __syncthreads();
        for (int t = tid; t < r; t += 1024) {
            if (bt[t] == 1) g.rpm[mi][order[t]] = order[t];
            else if (bt[t] == 2) { g.rpm[mi][order[t]] = order[t + 1]; g.rpm[mi][order[t + 1]] = order[t]; }
        }
        __syncthreads();
    }
}

__global__ void k_zero_counter(int32_t* q) { *q = 0; }

}  // namespace

int batched_nb_max() { return NB_MAX; }

size_t batched_slot_bytes() { return (size_t)NB_MAX * NB_MAX * sizeof(double); }

void launch_factor_batched(hipStream_t s, const Field& F, const uint32_t* itab, int64_t batch, const int64_t* n,
                           void* const* A, const int64_t* lda, int32_t dtype, void* const* e, int32_t* const* perm,
                           int32_t* const* rpm, int64_t* rank, int32_t* status, int check_range, double* ws,
                           int slots, int32_t* queue) {
    BatchArgs g{};
    g.batch = batch; g.n = n; g.A = A; g.lda = lda; g.dtype = dtype; g.e = e; g.perm = perm; g.rpm = rpm;
    g.rank = rank; g.status = status; g.ws = ws; g.queue = queue; g.F = F; g.itab = itab;
    g.check_range = check_range;
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, s, queue);
    hipLaunchKernelGGL(k_factor_batched, dim3((unsigned)slots), dim3(1024), 0, s, g);
}

}  // namespace pldl
