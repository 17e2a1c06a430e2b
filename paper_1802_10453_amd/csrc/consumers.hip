// consumers.hip -- uses of a finished factorization A = P L D L^T P^T
// (Section 1: the triangular factorization as the kernel of solving symmetric
// systems and of computing invariants of symmetric bilinear forms).
//
// The factorization is read as pldl_factor leaves it: L in the strict lower
// triangle and diag(D) on the diagonal of F (uint32 or FP64 residues), e the
// sub-diagonal of D's 2x2 blocks, perm the positions.  Every 2x2 block of D
// has the form [[0, c], [c, d]] (d = 0 in odd characteristic, the relaxed
// block of characteristic 2 otherwise); the n - r non-pivot positions carry D = 0.
#include "kernels.h"

namespace pldl {

namespace {
template <typename T>
__device__ __forceinline__ double rd(const void* p, int64_t i) {
    return (double)static_cast<const T*>(p)[i];
}
__device__ __forceinline__ double rdf(const void* F, int32_t dtype, int64_t i) {
    return dtype == 0 ? rd<uint32_t>(F, i) : rd<double>(F, i);
}
__device__ __forceinline__ double inv_of(double x, const uint32_t* itab, const Field& F) {
    return itab ? (double)itab[(int)x] : finv(x, F);
}
}  // namespace

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = v;
}

// Y[q][k] = B[perm[q]][k] (P^T B), rows q < n, columns k < nrhs.
__global__ void k_solve_gather(const double* B, int64_t ldb, const int32_t* perm, int64_t n, int64_t nrhs, double* Y) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x, q = blockIdx.y;
    if (k >= nrhs || q >= n) return;
    Y[q * nrhs + k] = B[(int64_t)perm[q] * ldb + k];
}

// u = D^+ y on the block-diagonal D (pivot positions q < r), in place; the
// positions q >= r must hold 0 (b in the range of A), else column k is
// inconsistent (cons[k] = 0); they are set to 0 (the solution's free part).
// The reversed copy U[n-1-q][k] = u[q][k] is written for the L^T solve.
__global__ void k_solve_dblock(const double* Y, int64_t n, int64_t nrhs, int64_t r, const void* Fd, int64_t lda,
                               int32_t dtype, const void* e, const uint32_t* itab, Field F, int32_t* cons, double* U) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x, q = blockIdx.y;
    if (k >= nrhs || q >= n) return;
    double u;
    if (q >= r) {
        if (Y[q * nrhs + k] != 0.0 && cons) cons[k] = 0;
        u = 0.0;
    } else {
        const double eq = rdf(e, dtype, q);
        const double ep = q > 0 ? rdf(e, dtype, q - 1) : 0.0;
        if (eq != 0.0 && q + 1 < r) {   // first position of a 2x2 block [[0, c], [c, d]]: u0 = (y1 - d u1) / c
            const double ci = inv_of(eq, itab, F);
            const double d = rdf(Fd, dtype, (q + 1) * lda + q + 1);
            const double u1 = fmulm(Y[q * nrhs + k], ci, F);
            u = fmulm(fcan(fred(Y[(q + 1) * nrhs + k] - fmulm(d, u1, F), F), F), ci, F);
        } else if (ep != 0.0 && q - 1 < r) {   // second position: u1 = y0 / c
            u = fmulm(Y[(q - 1) * nrhs + k], inv_of(ep, itab, F), F);
        } else {                  // 1x1 block (x): u = y / x
            u = fmulm(Y[q * nrhs + k], inv_of(rdf(Fd, dtype, q * lda + q), itab, F), F);
        }
    }
    U[(n - 1 - q) * nrhs + k] = u;
}

// M^T with M = J L J (J the reversal): M^T[a][b] = L[n-1-b][n-1-a], unit lower
// (only its strict lower part is written and read), so that L^T w = u becomes
// M^T (J w) = J u, a forward solve.
__global__ void k_solve_revlt(const void* Fd, int64_t lda, int32_t dtype, int64_t n, double* Mt, int64_t ldm) {
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x, a = blockIdx.y;
    if (a >= n || b >= a) return;
    Mt[a * ldm + b] = rdf(Fd, dtype, (n - 1 - b) * lda + (n - 1 - a));
}

// X = P J w~: B[perm[q]][k] = W~[n-1-q][k].
__global__ void k_solve_scatter(const double* Wt, int64_t n, int64_t nrhs, const int32_t* perm, double* B,
                                int64_t ldb) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x, q = blockIdx.y;
    if (k >= nrhs || q >= n) return;
    B[(int64_t)perm[q] * ldb + k] = Wt[(n - 1 - q) * nrhs + k];
}

// Invariants of the form (one workgroup of 1024 threads): the product of the
// determinants of D's blocks over the r pivot positions (1x1: x; 2x2
// [[0,c],[c,d]]: -c^2), its quadratic character by Euler's criterion, and for
// p = 2 whether the diagonal of D vanishes (the form is alternating).
// out: [0] det(A) (0 when r < n), [1] the product, [2] character (1 / -1; p = 2: 1),
// [3] p = 2: 1 if alternating else 0 (odd p: 0).
__global__ __launch_bounds__(1024) void k_invariants(const void* Fd, int64_t lda, int32_t dtype, const void* e,
                                                     int64_t n, int64_t r, Field F, int64_t* out) {
    __shared__ double part[1024];
    __shared__ int anyd[1024];
    const int tid = threadIdx.x;
    double acc = 1.0;
    int nzd = 0;
    for (int64_t q = tid; q < n; q += 1024) {
        const double d = rdf(Fd, dtype, q * lda + q);
        nzd |= d != 0.0;
        if (q >= r) continue;
        const double eq = rdf(e, dtype, q);
        const double ep = q > 0 ? rdf(e, dtype, q - 1) : 0.0;
        double f;
        if (eq != 0.0 && q + 1 < r) f = fcan(-fmulm(eq, eq, F), F);   // the 2x2 block at q: -c^2 (d times the leading 0)
        else if (ep != 0.0) f = 1.0;                      // its second position
        else f = d;
        acc = fmulm(acc, f, F);
    }
    part[tid] = acc;
    anyd[tid] = nzd;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) {
            part[tid] = fmulm(part[tid], part[tid + w], F);
            anyd[tid] |= anyd[tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double prod = part[0];
        out[0] = r == n ? (int64_t)prod : 0;
        out[1] = (int64_t)prod;
        if (F.ip == 2) {
            out[2] = 1;
            out[3] = anyd[0] ? 0 : 1;
        } else {
            // Euler's criterion: prod^((p-1)/2) = 1 for a square, p - 1 otherwise
            double res = 1.0, base = prod;
            for (int64_t ex = (F.ip - 1) / 2; ex > 0; ex >>= 1) {
                if (ex & 1) res = fmulm(res, base, F);
                base = fmulm(base, base, F);
            }
            out[2] = prod == 0.0 ? 0 : (res == 1.0 ? 1 : -1);
            out[3] = 0;
        }
    }
}

}  // namespace pldl
