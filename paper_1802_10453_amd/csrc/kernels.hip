// kernels.hip -- base-case, triangular-solve, permutation and bookkeeping kernels.
//
// Storage shared with the driver: W is the n x n working matrix (row-major,
// leading dimension ld); only its lower triangle (j <= i) is meaningful.  Every
// recursive step works on a contiguous position range; a permutation of a range
// is applied symmetrically (rows of the L part to the left, the lower block,
// columns of the rows below).  dd/de hold D in position coordinates.
#include "common.h"
#include "kernels.h"

namespace pldl {

// ===========================================================================
// Base case (Section 5, Algorithm 4): rank-profile-revealing elimination of a
// symmetric block of order s <= 128 held in registers (one workgroup, 1024
// threads, each owning a 4x4 tile of the full symmetric matrix).
//
// Pivot search as in Section 5: the current row i is the first unprocessed
// one; its pivot is the first nonzero of its Schur-complement row (found with
// one wave ballot); a diagonal pivot makes a 1x1 block, an off-diagonal pivot
// j a 2x2 block (i, j); an all-zero row is set aside keeping its precedence.
// The paper's Crout schedule delays updates to save reductions on a CPU; here
// the block is register resident and the update is right-looking with delayed
// reduction instead (one FMA per owned entry per pivot; entries grow by at most
// 3 (p-1)^2/4 per step and are reduced only when their column becomes a pivot
// column), which computes the same unique (P, L, D).
// ===========================================================================
__global__ __launch_bounds__(1024) void k_bc_leaf(double* W, int64_t ld, int64_t lo, int s, Field F,
                                                  double* dd, double* de, int32_t* sig_out,
                                                  int32_t* rank_out) {
    __shared__ double colI[128], colJ[128];
    __shared__ double vb[128], vc[128], va[128], ve[128], vf[128];
    __shared__ int alive[128], order[128], zeros[128], sig[128];
    __shared__ double bx[128], by[128];
    __shared__ int bt[128];
    __shared__ int sh_j;
    __shared__ double sh_xi, sh_w, sh_d22, sh_lji;
    __shared__ uint32_t Mo[128][129];

    const int tid = threadIdx.x, ty = tid >> 5, tx = tid & 31;
    const int r0 = ty * 4, c0 = tx * 4;
    double m[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            int i = r0 + a, j = c0 + b;
            double v = 0.0;
            if (i < s && j < s) v = (i >= j) ? W[(lo + i) * ld + lo + j] : W[(lo + j) * ld + lo + i];
            m[a][b] = v;
        }
    if (tid < 128) { alive[tid] = tid < s ? 1 : 0; bt[tid] = 0; bx[tid] = 0.0; by[tid] = 0.0; }
    __syncthreads();

    int r = 0, nz = 0;
    for (int i = 0; i < s; ++i) {
        if (!alive[i]) continue;
        // owners of column i publish the reduced column (0 on eliminated rows)
        if (tx == (i >> 2)) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                int k = r0 + a;
                double v = 0.0;
#pragma unroll
                for (int b = 0; b < 4; ++b) v = (b == (i & 3)) ? m[a][b] : v;
                colI[k] = (k < s && alive[k]) ? fred(v, F) : 0.0;
            }
        }
        __syncthreads();
        if (tid < 64) {
            int j = -1;
            for (int base = i; base < s; base += 64) {
                int c = base + tid;
                bool pr = (c < s) && colI[c] != 0.0;
                unsigned long long bal = __ballot(pr);
                if (bal) { j = base + __ffsll((long long)bal) - 1; break; }
            }
            if (tid == 0) sh_j = j;
        }
        __syncthreads();
        const int j = sh_j;
        if (j < 0) {  // zero row
            if (tid == 0) { alive[i] = 0; zeros[nz] = i; }
            ++nz;
            __syncthreads();
            continue;
        }
        if (j == i) {  // 1x1 pivot
            if (tid == 0) {
                double x = colI[i];
                sh_xi = finv(x, F);
                bx[r] = x; bt[r] = 1; order[r] = i; alive[i] = 0;
            }
            __syncthreads();
            if (tid < 128) {
                double c = (tid < s && alive[tid]) ? colI[tid] : 0.0;
                vb[tid] = fcen(fmulm(c, sh_xi, F), F);
                vc[tid] = fcen(c, F);
            }
            __syncthreads();
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) m[a][b] = fma(-vb[r0 + a], vc[c0 + b], m[a][b]);
            if (tx == (i >> 2)) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (b == (i & 3)) m[a][b] = fcan(vb[r0 + a], F);
            }
            r += 1;
            __syncthreads();
        } else {  // 2x2 pivot on (i, j)
            if (tx == (j >> 2)) {
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    int k = r0 + a;
                    double v = 0.0;
#pragma unroll
                for (int b = 0; b < 4; ++b) v = (b == (j & 3)) ? m[a][b] : v;
                colJ[k] = (k < s && alive[k]) ? fred(v, F) : 0.0;
                }
            }
            __syncthreads();
            if (tid == 0) {
                double x = colI[j], y = colJ[j];
                double xi = finv(x, F);
                double w, d22, lji;
                if (F.ip == 2) { w = y; d22 = y; lji = 0.0; }
                else { w = fmulm(y, F.inv2, F); d22 = 0.0; lji = fmulm(w, xi, F); }
                sh_xi = xi; sh_w = w; sh_d22 = d22; sh_lji = lji;
                bx[r] = x; by[r] = (F.ip == 2) ? y : 0.0; bt[r] = 2;
                order[r] = i; order[r + 1] = j; alive[i] = 0; alive[j] = 0;
            }
            __syncthreads();
            if (tid < 128) {
                bool al = tid < s && alive[tid];
                double ci = al ? colI[tid] : 0.0, cj = al ? colJ[tid] : 0.0;
                double b = fmulm(ci, sh_xi, F);                 // S[k][i] / x
                double e = fcan(cj - fmulm(sh_w, b, F), F);      // x a_k = S[k][j] - w b_k
                double av = fmulm(e, sh_xi, F);                  // a_k
                vb[tid] = fcen(b, F); va[tid] = fcen(av, F); vc[tid] = fcen(ci, F);
                ve[tid] = fcen(e, F); vf[tid] = fcen(fmulm(sh_d22, b, F), F);
            }
            __syncthreads();
            // S[k][l] -= x (a_k b_l + b_k a_l) + d22 b_k b_l = e_k b_l + c_k a_l + f_k b_l
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    double t = m[a][b];
                    t = fma(-ve[r0 + a], vb[c0 + b], t);
                    t = fma(-vc[r0 + a], va[c0 + b], t);
                    t = fma(-vf[r0 + a], vb[c0 + b], t);
                    m[a][b] = t;
                }
            if (tx == (i >> 2)) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (b == (i & 3)) m[a][b] = fcan(va[r0 + a], F);
            }
            if (tx == (j >> 2)) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (b == (j & 3)) m[a][b] = fcan(vb[r0 + a], F);
            }
            if (tx == (i >> 2) && ty == (j >> 2)) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (a == (j & 3) && b == (i & 3)) m[a][b] = sh_lji;
            }
            r += 2;
            __syncthreads();
        }
    }
    // ---- write out: order = pivots then zero rows (their precedence kept)
    if (tid < s) sig[tid] = tid < r ? order[tid] : zeros[tid - r];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            int i = r0 + a, j = c0 + b;
            if (i < 128 && j < 128) Mo[i][j] = (uint32_t)fred(m[a][b], F);
        }
    __syncthreads();
    for (int e = tid; e < s * s; e += 1024) {
        int q = e / s, c = e - q * s;
        if (c >= q) continue;   // strict lower part: L (the diagonal holds D, written below)
        W[(lo + q) * ld + lo + c] = (c < r) ? (double)Mo[sig[q]][sig[c]] : 0.0;
    }
    if (tid == 0) {
        int q = 0;
        for (int t = 0; t < r;) {
            if (bt[t] == 1) {
                dd[lo + q] = bx[t]; de[lo + q] = 0.0;
                q += 1; t += 1;
            } else {
                dd[lo + q] = 0.0; de[lo + q] = bx[t];
                dd[lo + q + 1] = by[t]; de[lo + q + 1] = 0.0;
                q += 2; t += 2;
            }
        }
        for (; q < s; ++q) { dd[lo + q] = 0.0; de[lo + q] = 0.0; }
        *rank_out = r;
    }
    __syncthreads();
    if (tid < s) {
        W[(lo + tid) * ld + lo + tid] = dd[lo + tid];
        sig_out[tid] = sig[tid];
    }
}

// ===========================================================================
// Rank-profile-revealing PLDUQ of one tile (Sections 4.2 and 5 pivoting):
// rows = positions [a0, a0+m) (m <= 32), columns = positions [c0, c0+nc)
// (nc <= 256), Y[i][j] = W[c0+j][a0+i] (Y is stored transposed below the
// diagonal of W).  Rows are processed in order; a row's pivot is the first
// nonzero of its reduced row among non-pivot columns; a zero row is skipped.
// Right-looking over the tile's rows with delayed reduction (the tile sits in
// registers: thread t owns column t%256 of rows 8*(t/256) .. +8).
// The LU pack is written back in the ORIGINAL (unpermuted) coordinates; the
// driver then applies the row permutation rsig and column permutation csig.
// ===========================================================================
__global__ __launch_bounds__(1024) void k_plduq_leaf(double* W, int64_t ld, int64_t a0, int m, int64_t c0,
                                                     int nc, Field F, int32_t* rsig, int32_t* csig,
                                                     int32_t* rank_out) {
    __shared__ double rowI[256];
    __shared__ double fvec[32];
    __shared__ int ispc[256];
    __shared__ int prow[32], pcol[32];
    __shared__ double pinvx[32];
    __shared__ int wmin[4];
    __shared__ int sh_c;
    __shared__ double sh_xi;
    const int tid = threadIdx.x, col = tid & 255, rg = tid >> 8;  // rows rg*8 .. rg*8+7
    double y[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        int i = rg * 8 + a;
        y[a] = (i < m && col < nc) ? W[(c0 + col) * ld + a0 + i] : 0.0;
    }
    if (tid < 256) ispc[tid] = 0;
    __syncthreads();
    int r = 0;
    for (int i = 0; i < m; ++i) {
        if (rg == (i >> 3)) rowI[col] = (col < nc && !ispc[col]) ? fred(y[i & 7], F) : 0.0;
        __syncthreads();
        if (tid < 256) {
            bool pr = rowI[tid] != 0.0;
            unsigned long long bal = __ballot(pr);
            if ((tid & 63) == 0) wmin[tid >> 6] = bal ? (tid + __ffsll((long long)bal) - 1) : 1 << 30;
        }
        __syncthreads();
        if (tid == 0) {
            int c = min(min(wmin[0], wmin[1]), min(wmin[2], wmin[3]));
            if (c >= (1 << 30)) c = -1;
            sh_c = c;
            if (c >= 0) {
                double x = rowI[c];
                double xi = finv(x, F);
                sh_xi = xi;
                prow[r] = i; pcol[r] = c; pinvx[r] = xi; ispc[c] = 1;
            }
        }
        __syncthreads();
        const int c = sh_c;
        if (c < 0) continue;
        // multipliers of the rows below for this pivot: f = Y[i'][c] / x
        if (col == c) {
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                int ii = rg * 8 + a;
                if (ii < 32) fvec[ii] = (ii > i && ii < m) ? fcen(fmulm(fred(y[a], F), sh_xi, F), F) : 0.0;
            }
        }
        __syncthreads();
        const double rv = fcen(rowI[col], F);
#pragma unroll
        for (int a = 0; a < 8; ++a) y[a] = fma(-fvec[rg * 8 + a], rv, y[a]);
        // the pivot column now stores the multipliers (L) of the rows below
        if (col == c) {
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                int ii = rg * 8 + a;
                if (ii > i && ii < m) y[a] = fcan(fvec[ii], F);
            }
        }
        ++r;
        __syncthreads();
    }
    // ---- output orders
    __shared__ int rord[32], cord[256], rpos[32], cpos[256];
    if (tid == 0) {
        int a = 0;
        for (int t = 0; t < r; ++t) rord[a++] = prow[t];
        for (int i = 0; i < m; ++i) {
            bool piv = false;
            for (int t = 0; t < r; ++t) piv |= (prow[t] == i);
            if (!piv) rord[a++] = i;
        }
        int b = 0;
        for (int t = 0; t < r; ++t) cord[b++] = pcol[t];
        for (int j = 0; j < nc; ++j)
            if (!ispc[j]) cord[b++] = j;
        for (int t = 0; t < m; ++t) rpos[rord[t]] = t;
        for (int t = 0; t < nc; ++t) cpos[cord[t]] = t;
        *rank_out = r;
    }
    __syncthreads();
    if (tid < m) rsig[tid] = rord[tid];
    if (tid < nc) csig[tid] = cord[tid];
    // pack entry LU[a][b] (a = rpos[i], b = cpos[j]) at W[c0 + j][a0 + i] (old coordinates)
    if (col < nc) {
        const int b = cpos[col];
#pragma unroll
        for (int aa = 0; aa < 8; ++aa) {
            int i = rg * 8 + aa;
            if (i >= m) continue;
            int a = rpos[i];
            double v = fred(y[aa], F);
            double out;
            if (a == b && a < r) out = v;                          // D
            else if (b < a && b < r) out = v;                      // L / M (stored multipliers)
            else if (a < b && a < r) out = fmulm(v, pinvx[a], F);  // U / V
            else out = 0.0;
            W[(c0 + col) * ld + a0 + i] = out;
        }
    }
}

// ===========================================================================
// TRSS leaf (Problem 1) of order r <= 64, one wave: X upper with
// X^T U + U^T X = C, solved column by column from the defining equations
// (entry (i, j), i < j, determines X[i][j] through U[i][i] = 1; the diagonal
// entry gives 2 X[j][j]; in characteristic 2 X[j][j] = 0).
// C (lower) at W[s0..s0+r)^2, U[a][b] = W[s0+b][u0+a] (a < b).  X^T is
// written over C's lower triangle.
// ===========================================================================
__global__ __launch_bounds__(64) void k_trss_leaf(double* W, int64_t ld, int64_t s0, int64_t u0, int r, Field F) {
    __shared__ double X[64][65];  // X[t][j]
    __shared__ double U[64][65];  // U[t][j], unit upper
    __shared__ double C[64][65];  // symmetric C
    const int lane = threadIdx.x;
    for (int e = lane; e < r * r; e += 64) {
        int a = e / r, b = e % r;
        U[a][b] = (a == b) ? 1.0 : (a < b ? fcen(W[(s0 + b) * ld + u0 + a], F) : 0.0);
        C[a][b] = (a >= b) ? W[(s0 + a) * ld + s0 + b] : W[(s0 + b) * ld + s0 + a];
        X[a][b] = 0.0;
    }
    __syncthreads();
    for (int j = 0; j < r; ++j) {
        // b_i = C_ij - sum_{t<=i} X[t][i] U[t][j]   (i < j; lane i)
        double bi = 0.0;
        if (lane < j) {
            double s = C[lane][j];
            for (int t = 0; t <= lane; ++t) s = fma(-X[t][lane], U[t][j], s);
            bi = fred(s, F);
        }
        // solve sum_{t<=i} U[t][i] X[t][j] = b_i, U unit: forward substitution
        for (int i = 0; i < j; ++i) {
            double xi = __shfl(bi, i);
            xi = fcen(fred(xi, F), F);
            if (lane == i) X[i][j] = fcan(xi, F);
            if (lane > i && lane < j) bi = fma(-U[i][lane], xi, bi);
        }
        __syncthreads();
        if (lane == 0) {
            if (F.ip == 2) X[j][j] = 0.0;
            else {
                double s = 0.0;
                for (int t = 0; t < j; ++t) s = fma(fcen(X[t][j], F), U[t][j], s);
                X[j][j] = fcan(fred(fmulm(C[j][j], F.inv2, F) - fred(s, F), F), F);
            }
        }
        __syncthreads();
    }
    for (int e = lane; e < r * r; e += 64) {
        int a = e / r, b = e % r;
        if (b <= a) W[(s0 + a) * ld + s0 + b] = X[b][a];
    }
}

// ===========================================================================
// Triangular solve leaves (Section 3, TRSM) with unit triangular T of order
// r <= 64, delayed reduction over at most 63 products.
// ===========================================================================
// B (m x r, row-major) <- B T^{-1}, T unit upper; one workgroup per 64 rows.
__global__ __launch_bounds__(256) void k_trsm_ru_leaf(double* B, int64_t ld, int64_t m, int r, MatV T, Field F) {
    __shared__ double Ts[64][65];
    __shared__ double Bs[64][65];
    const int tid = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int rows = (int)min((int64_t)64, m - i0);
    for (int e = tid; e < r * r; e += 256) {
        int a = e / r, b = e - a * r;
        Ts[a][b] = (a < b) ? fcen(T.p[a * T.rs + b * T.cs], F) : 0.0;
    }
    for (int e = tid; e < rows * r; e += 256) {
        int i = e / r, j = e - i * r;
        Bs[i][j] = B[(i0 + i) * ld + j];
    }
    __syncthreads();
    for (int j = 0; j < r; ++j) {
        if (tid < rows) Bs[tid][j] = fcen(fred(Bs[tid][j], F), F);
        __syncthreads();
        const int w = r - j - 1;
        if (w > 0)
            for (int e = tid; e < rows * w; e += 256) {
                int i = e / w, jj = j + 1 + (e - (e / w) * w);
                Bs[i][jj] = fma(-Bs[i][j], Ts[j][jj], Bs[i][jj]);
            }
        __syncthreads();
    }
    for (int e = tid; e < rows * r; e += 256) {
        int i = e / r, j = e - i * r;
        B[(i0 + i) * ld + j] = fcan(Bs[i][j], F);
    }
}

// B (r x ncols, row-major) <- T^{-1} B, T unit lower; one workgroup per 64 columns.
__global__ __launch_bounds__(256) void k_trsm_ll_leaf(double* B, int64_t ld, int64_t ncols, int r, MatV T, Field F) {
    __shared__ double Ts[64][65];
    __shared__ double Bs[64][65];
    const int tid = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    const int cols = (int)min((int64_t)64, ncols - j0);
    for (int e = tid; e < r * r; e += 256) {
        int a = e / r, b = e - a * r;
        Ts[a][b] = (a > b) ? fcen(T.p[a * T.rs + b * T.cs], F) : 0.0;
    }
    for (int e = tid; e < r * cols; e += 256) {
        int i = e / cols, c = e - i * cols;
        Bs[i][c] = B[i * ld + j0 + c];
    }
    __syncthreads();
    for (int i = 0; i < r; ++i) {
        if (tid < cols) Bs[i][tid] = fcen(fred(Bs[i][tid], F), F);
        __syncthreads();
        const int h = r - i - 1;
        if (h > 0)
            for (int e = tid; e < h * cols; e += 256) {
                int ii = i + 1 + e / cols, c = e - (e / cols) * cols;
                Bs[ii][c] = fma(-Ts[ii][i], Bs[i][c], Bs[ii][c]);
            }
        __syncthreads();
    }
    for (int e = tid; e < r * cols; e += 256) {
        int i = e / cols, c = e - i * cols;
        B[i * ld + j0 + c] = fcan(Bs[i][c], F);
    }
}

// ===========================================================================
// Symmetric permutation of the position range [lo, hi) (new lo+q <- old
// lo+sig[q]), through a temporary: part 0 rows [lo,hi) x cols [0,lo);
// part 1 the lower block; part 2 rows [hi,n) x cols [lo,hi); part 3 orig.
// Gather into tmp (blockIdx.z = part), then scatter back.
// ===========================================================================
__global__ __launch_bounds__(256) void k_perm_gather(const double* W, int64_t ld, int64_t n, int64_t lo,
                                                     int64_t hi, const int32_t* sig, double* tmp,
                                                     const int32_t* orig, int32_t* tmpo, int parts) {
    const int64_t s = hi - lo;
    const int part = blockIdx.z;
    if (!((parts >> part) & 1)) return;
    const int64_t row = blockIdx.y;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    // a sigma entry outside [0, s) is a bug upstream: clamp it so no access leaves the range
    auto sg = [&](int64_t q) -> int64_t { int64_t v = sig[q]; return (v < 0 || v >= s) ? 0 : v; };
    if (part == 0) {
        if (row >= s || c >= lo) return;
        tmp[row * lo + c] = W[(lo + sg(row)) * ld + c];
    } else if (part == 1) {
        if (row >= s || c > row) return;
        int64_t a = lo + sg(row), b = lo + sg(c);
        tmp[s * lo + row * s + c] = (a >= b) ? W[a * ld + b] : W[b * ld + a];
    } else if (part == 2) {
        if (row >= n - hi || c >= s) return;
        tmp[s * lo + s * s + row * s + c] = W[(hi + row) * ld + lo + sg(c)];
    } else {
        if (row != 0 || c >= s) return;
        tmpo[c] = orig[lo + sg(c)];
    }
}

__global__ __launch_bounds__(256) void k_perm_scatter(double* W, int64_t ld, int64_t n, int64_t lo, int64_t hi,
                                                      const double* tmp, int32_t* orig, const int32_t* tmpo,
                                                      int parts) {
    const int64_t s = hi - lo;
    const int part = blockIdx.z;
    if (!((parts >> part) & 1)) return;
    const int64_t row = blockIdx.y;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (part == 0) {
        if (row >= s || c >= lo) return;
        W[(lo + row) * ld + c] = tmp[row * lo + c];
    } else if (part == 1) {
        if (row >= s || c > row) return;
        W[(lo + row) * ld + lo + c] = tmp[s * lo + row * s + c];
    } else if (part == 2) {
        if (row >= n - hi || c >= s) return;
        W[(hi + row) * ld + lo + c] = tmp[s * lo + s * s + row * s + c];
    } else {
        if (row != 0 || c >= s) return;
        orig[lo + c] = tmpo[c];
    }
}

// sigma of the rotation [len1 | len2] -> [len2 | len1]
__global__ void k_sigma_rotate(int32_t* sig, int64_t len1, int64_t len2) {
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= len1 + len2) return;
    sig[q] = (int32_t)(q < len2 ? len1 + q : q - len2);
}

// Merge two runs of positions [a, a+n1) and [a+n1, a+n1+n2), each sorted by
// original index, into one sorted run: sig[rank] = local index.
__global__ void k_sigma_merge(const int32_t* orig, int64_t a, int64_t n1, int64_t n2, int32_t* sig) {
    int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n1 + n2) return;
    const int32_t* A = orig + a;
    const int32_t* B = orig + a + n1;
    int32_t v;
    int64_t lo = 0, hi;
    if (t < n1) {
        v = A[t]; hi = n2;
        while (lo < hi) { int64_t md = (lo + hi) / 2; if (B[md] < v) lo = md + 1; else hi = md; }
        sig[t + lo] = (int32_t)t;
    } else {
        int64_t u = t - n1;
        v = B[u]; hi = n1;
        while (lo < hi) { int64_t md = (lo + hi) / 2; if (A[md] < v) lo = md + 1; else hi = md; }
        sig[u + lo] = (int32_t)t;
    }
}

// ===========================================================================
// D^{-1} bookkeeping.  For positions [lo, lo+r) of a finished pivot range:
// xinv[q] = x^{-1} of q's block; yy[q] = -y/x^2 at the first position of a
// relaxed block [[0,x],[x,y]] (0 otherwise); kind[q] = 1 (1x1), 2 (first of a
// 2x2 block), 3 (second).
// ===========================================================================
__global__ void k_block_dinv(const double* dd, const double* de, int64_t lo, int64_t r, Field F, double* xinv,
                             double* yy, int8_t* kind) {
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= r) return;
    int k;
    double x, y = 0.0;
    if (de[lo + q] != 0.0) { k = 2; x = de[lo + q]; y = dd[lo + q + 1]; }
    else if (q > 0 && de[lo + q - 1] != 0.0) { k = 3; x = de[lo + q - 1]; }
    else { k = 1; x = dd[lo + q]; }
    double xi = finv(x, F);
    xinv[q] = xi;
    yy[q] = (k == 2 && y != 0.0) ? fcan(-fmulm(y, fmulm(xi, xi, F), F), F) : 0.0;
    kind[q] = (int8_t)k;
}

// SCAL (Algorithm 2): T <- X (copy), X <- X D^{-1} for the rows x r matrix X
// (row-major).  Row vector v D^{-1}: 1x1: v_q/x; 2x2 [[0,x],[x,y]]:
// (v_{q+1}/x - y v_q/x^2, v_q/x).
__global__ void k_scal_dinv(double* X, int64_t ldx, int64_t rows, int64_t r, const double* xinv, const double* yy,
                            const int8_t* kind, double* T, int64_t ldt, Field F) {
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t i = blockIdx.y;
    if (q >= r || i >= rows) return;
    int k = kind[q];
    if (k == 3) return;
    double* x = X + i * ldx;
    if (k == 1) {
        double v = x[q];
        T[i * ldt + q] = v;
        x[q] = fmulm(v, xinv[q], F);
    } else {
        double v0 = x[q], v1 = x[q + 1];
        T[i * ldt + q] = v0; T[i * ldt + q + 1] = v1;
        x[q] = fred(fmulm(v1, xinv[q], F) + fmulm(v0, yy[q], F), F);
        x[q + 1] = fmulm(v0, xinv[q], F);
    }
}

// Inverses of the diagonal of a PLDUQ pack: dinv[k] = 1 / W[c0+k][a0+k].
__global__ void k_pack_dinv(const double* W, int64_t ld, int64_t c0, int64_t a0, int64_t r, Field F, double* dinv) {
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= r) return;
    dinv[k] = finv(W[(c0 + k) * ld + a0 + k], F);
}

// X[k][j] *= dinv[k]  (rows x cols block, row k scaled)   -- by_row = 1
// X[j][k] *= dinv[k]  (column k scaled)                   -- by_row = 0
__global__ void k_scale_by(double* X, int64_t ld, int64_t rows, int64_t cols, const double* dinv, int by_row,
                           Field F) {
    int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t i = blockIdx.y;
    if (j >= cols || i >= rows) return;
    double d = by_row ? dinv[i] : dinv[j];
    X[i * ld + j] = fmulm(X[i * ld + j], d, F);
}

// out[i][k] = X[i][k] * dinv[k] for k < kmax(i) (lower: k <= i) -- G1, G2 of Algorithm 3
__global__ void k_mul_cols(const double* X, int64_t ldx, int64_t rows, int64_t cols, const double* dinv, int lower,
                           double* out, int64_t ldo, Field F) {
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t i = blockIdx.y;
    if (k >= cols || i >= rows) return;
    out[i * ldo + k] = (lower && k > i) ? 0.0 : fmulm(X[i * ldx + k], dinv[k], F);
}

// Plain 2-D copy (row-major both sides).
__global__ void k_copy2d(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t rows, int64_t cols) {
    int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t i = blockIdx.y;
    if (j >= cols || i >= rows) return;
    dst[i * ldd + j] = src[i * lds + j];
}

// ===========================================================================
// Algorithm 3 assembly.  Range [lo, hi): R = [lo, lo+mz) (zero rows), with
// its rY pivot rows first; S = [lo+mz, hi) with its rY pivot columns first.
// New order: pairs (R pivot k, S pivot k) interleaved (P_i of the paper), then
// the rest of S (Z), then the non-pivot rows of R.  The new lower block:
//   pair block: L1 (from the pack), G1 (temporary), U1^T (pack); zeros;
//   Z rows x pair columns: G2 (temporary) and V1^T (pack); Z x Z unchanged;
//   R non-pivot rows x pair columns: M1 (pack) and 0; zeros elsewhere.
// The block is built in tmp (N x N lower), copied back by the caller.
// ===========================================================================
__global__ void k_zlp_assemble(const double* W, int64_t ld, int64_t lo, int64_t mz, int64_t hi, int64_t rY,
                               const double* G1, int64_t ldg1, const double* G2, int64_t ldg2, double* tmp) {
    const int64_t N = hi - lo, s0 = lo + mz, nz = hi - s0 - rY;
    int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t q = blockIdx.y;
    if (q >= N || c > q) return;
    // old position of a new position
    auto oldp = [&](int64_t t) -> int64_t {
        if (t < 2 * rY) return (t & 1) ? s0 + (t >> 1) : lo + (t >> 1);
        if (t < 2 * rY + nz) return s0 + rY + (t - 2 * rY);
        return lo + rY + (t - 2 * rY - nz);
    };
    double v;
    if (c < 2 * rY) {
        const int64_t k = c >> 1;
        const bool codd = c & 1;
        if (q < 2 * rY) {
            const int64_t k2 = q >> 1;
            const bool qodd = q & 1;
            if (q == c) v = 0.0;  // diagonal: D is set separately
            else if (!qodd && !codd) v = W[(s0 + k) * ld + lo + k2];          // L1[k2][k]
            else if (qodd && !codd) v = G1[k2 * ldg1 + k];                     // G1[k2][k]
            else if (qodd && codd) v = W[(s0 + k2) * ld + lo + k];             // U1^T[k2][k]
            else v = 0.0;
        } else if (q < 2 * rY + nz) {
            const int64_t z = q - 2 * rY;
            v = codd ? W[(s0 + rY + z) * ld + lo + k] : G2[z * ldg2 + k];     // V1^T / G2
        } else {
            const int64_t t = q - 2 * rY - nz;
            v = codd ? 0.0 : W[(s0 + k) * ld + lo + rY + t];                  // M1[t][k]
        }
    } else {
        int64_t a = oldp(q), b = oldp(c);
        v = (a >= b) ? W[a * ld + b] : W[b * ld + a];
    }
    tmp[q * N + c] = v;
}

// new lo+q <- old lo+oldp(q): orig of the assembly, plus D of the pairs
__global__ void k_zlp_orig_d(int32_t* orig, int32_t* tmpo, int64_t lo, int64_t mz, int64_t hi, int64_t rY,
                             const double* W, int64_t ld, const double* delta, double* dd, double* de, int phase) {
    const int64_t N = hi - lo, s0 = lo + mz, nz = hi - s0 - rY;
    int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= N) return;
    if (phase == 0) {
        int64_t o;
        if (t < 2 * rY) o = (t & 1) ? s0 + (t >> 1) : lo + (t >> 1);
        else if (t < 2 * rY + nz) o = s0 + rY + (t - 2 * rY);
        else o = lo + rY + (t - 2 * rY - nz);
        tmpo[t] = orig[o];
    } else if (phase == 1) {
        orig[lo + t] = tmpo[t];
    } else {
        // phase 2 (after the block copy-back): D for the pairs; the pack's
        // diagonal d_k must be read before the copy-back, so it is passed in delta[rY + k]
        if (t < 2 * rY) {
            int64_t k = t >> 1;
            if (!(t & 1)) { de[lo + t] = delta[rY + k]; dd[lo + t] = 0.0; }
            else { de[lo + t] = 0.0; dd[lo + t] = delta[k]; }
        }
    }
}

// d_k = W[s0+k][lo+k] saved next to Delta before the assembly overwrites the pack
__global__ void k_save_pack_diag(const double* W, int64_t ld, int64_t s0, int64_t lo, int64_t rY, double* out) {
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= rY) return;
    out[k] = W[(s0 + k) * ld + lo + k];
}

// ===========================================================================
// Characteristic-2 extras of Algorithm 3.
// Delta_ii = C'_ii - sum_{j<i} Delta_jj U_ji^2  (Section 4.1.2), by a forward
// sweep (one workgroup): after Delta_i is final, c_k -= Delta_i U_ik^2, k > i.
// U[j][i] = W[s0+i][u0+j] (j < i).
// ===========================================================================
__global__ __launch_bounds__(1024) void k_delta(const double* W, int64_t ld, int64_t s0, int64_t u0, int64_t r,
                                                Field F, double* delta) {
    extern __shared__ double cvec[];
    for (int64_t k = threadIdx.x; k < r; k += blockDim.x) cvec[k] = W[(s0 + k) * ld + s0 + k];
    __syncthreads();
    for (int64_t i = 0; i < r; ++i) {
        if (threadIdx.x == 0) cvec[i] = fred(cvec[i], F);
        __syncthreads();
        const double di = fcen(cvec[i], F);
        for (int64_t k = i + 1 + threadIdx.x; k < r; k += blockDim.x) {
            double u = fcen(W[(s0 + k) * ld + u0 + i], F);
            cvec[k] = fred(cvec[k] - di * fmulm(fcan(u, F), fcan(u, F), F), F);
        }
        __syncthreads();
    }
    for (int64_t k = threadIdx.x; k < r; k += blockDim.x) delta[k] = fred(cvec[k], F);
}

// UT = U1^T as a clean unit lower matrix; UTD = UT * Delta (column scaling).
__global__ void k_u1t_delta(const double* W, int64_t ld, int64_t s0, int64_t u0, int64_t r, const double* delta,
                            double* UT, double* UTD, Field F) {
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t i = blockIdx.y;
    if (k >= r || i >= r) return;
    double u = (i == k) ? 1.0 : (i > k ? W[(s0 + i) * ld + u0 + k] : 0.0);
    UT[i * r + k] = u;
    UTD[i * r + k] = fmulm(u, delta[k], F);
}

// DADD: X <- X + Delta U1, on X^T stored lower at W[s0..)^2: X^T[j][i] += Delta_i U1^T[j][i] (j >= i)
__global__ void k_dadd(double* W, int64_t ld, int64_t s0, int64_t u0, int64_t r, const double* delta, Field F) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t j = blockIdx.y;
    if (i > j || j >= r) return;
    double u = (i == j) ? 1.0 : W[(s0 + j) * ld + u0 + i];
    double* x = W + (s0 + j) * ld + s0 + i;
    *x = fred(*x + fmulm(delta[i], u, F), F);
}

// out = V (rows x r, row-major view in W) * Delta (column scaling)
__global__ void k_mul_delta(const double* V, int64_t ldv, int64_t rows, int64_t r, const double* delta, double* out,
                            Field F) {
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t i = blockIdx.y;
    if (k >= r || i >= rows) return;
    out[i * r + k] = fmulm(V[i * ldv + k], delta[k], F);
}

// ===========================================================================
// Input / output.
// ===========================================================================
template <typename T>
__global__ void k_load_input(const T* A, int64_t lda, double* W, int64_t ld, int64_t n, Field F, int32_t* err) {
    int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t i = blockIdx.y;
    if (i >= n || j > i) return;
    double v = (double)A[i * lda + j];
    if (!(v >= 0.0 && v < F.p && v == floor(v))) { atomicExch(err, 1); v = 0.0; }
    W[i * ld + j] = v;
}

template <typename T>
__global__ void k_store_output(T* A, int64_t lda, const double* W, int64_t ld, int64_t n, const double* dd,
                               const double* de, T* e, const int32_t* orig, int32_t* perm) {
    int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t i = blockIdx.y;
    if (i >= n || j > i) return;
    A[i * lda + j] = (T)(j == i ? dd[i] : W[i * ld + j]);
    if (j == 0) { e[i] = (T)de[i]; perm[i] = orig[i]; }
}

// rpm from the block structure: R = P Psi P^T (pivoting matrix, Section 2.1)
__global__ void k_rpm(const int32_t* orig, const double* de, int64_t n, int64_t r, int32_t* rpm) {
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    if (q >= r) { rpm[orig[q]] = -1; return; }
    if (de[q] != 0.0) { rpm[orig[q]] = orig[q + 1]; rpm[orig[q + 1]] = orig[q]; return; }
    if (q > 0 && de[q - 1] != 0.0) return;
    rpm[orig[q]] = orig[q];
}

// Characteristic 2, Section 2.3: for every relaxed block (q, q+1) with d = D[q+1][q+1] != 0,
// P~ = P P_J, L~ = (P_J^T L P_J) L_J, D~ block = diag(d, c^2/d).  Phase 0 gathers the
// conjugated L (lower) into tmp, phase 1 copies it back and applies L_J, phase 2 fixes P, D.
__device__ __forceinline__ int64_t c2_swap(const double* dd, const double* de, int64_t n, int64_t t) {
    if (t + 1 < n && de[t] != 0.0 && dd[t + 1] != 0.0) return t + 1;
    if (t > 0 && de[t - 1] != 0.0 && dd[t] != 0.0) return t - 1;
    return t;
}
__global__ void k_char2_std(double* W, int64_t ld, int64_t n, double* dd, double* de, int32_t* orig, double* tmp,
                            int phase) {
    int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t q = blockIdx.y;
    if (phase == 0) {
        if (q >= n || c >= q) return;
        int64_t a = c2_swap(dd, de, n, q), b = c2_swap(dd, de, n, c);
        // L[a][b] in position coordinates; a < b cannot occur below the diagonal except inside a block (0)
        tmp[q * n + c] = (a > b) ? W[a * ld + b] : 0.0;
    } else if (phase == 1) {
        if (q >= n || c >= q) return;
        double v = tmp[q * n + c];
        // column c of a relaxed block start: += (c_/d) column c+1 (over F_2, c_ = d = 1)
        if (c + 1 < n && de[c] != 0.0 && dd[c + 1] != 0.0) {
            double add = (q == c + 1) ? 1.0 : tmp[q * n + c + 1];
            v = fmod(v + add, 2.0);
        }
        W[q * ld + c] = v;
    } else {
        if (q != 0 || c >= n) return;
        if (c + 1 < n && de[c] != 0.0 && dd[c + 1] != 0.0) {
            int32_t t = orig[c]; orig[c] = orig[c + 1]; orig[c + 1] = t;
            dd[c] = 1.0; dd[c + 1] = 1.0; de[c] = 0.0;
        }
    }
}

// ===========================================================================
// Small helpers of the driver and of the standalone building-block calls.
// ===========================================================================
__global__ void k_iota(int32_t* a, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = (int32_t)i;
}

// sigma (local old index) of the Algorithm 3 assembly order
__global__ void k_zlp_sigma(int32_t* sig, int64_t mz, int64_t nc, int64_t rY) {
    const int64_t N = mz + nc, nz = nc - rY;
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= N) return;
    int64_t o;
    if (q < 2 * rY) o = (q & 1) ? mz + (q >> 1) : (q >> 1);
    else if (q < 2 * rY + nz) o = mz + rY + (q - 2 * rY);
    else o = rY + (q - 2 * rY - nz);
    sig[q] = (int32_t)o;
}

// out = A D (n x k), D block diagonal given by (dd, de)
__global__ void k_apply_d(const double* A, int64_t lda, int64_t n, int64_t k, const double* dd, const double* de,
                          double* out, Field F) {
    int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t i = blockIdx.y;
    if (c >= k || i >= n) return;
    const double* a = A + i * lda;
    double t = fmulm(a[c], dd[c], F);
    if (c + 1 < k) t = fred(t + fmulm(a[c + 1], de[c], F), F);
    if (c > 0) t = fred(t + fmulm(a[c - 1], de[c - 1], F), F);
    out[i * k + c] = t;
}

// TRSS standalone layout in a 2n x 2n W: U^T strictly lower at W[n.., 0..], C lower at W[n.., n..]
__global__ void k_trss_pack(const double* U, int64_t ldu, const double* C, int64_t ldc, double* W, int64_t ldw,
                            int64_t n, int32_t* info, int check_char2) {
    int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t i = blockIdx.y;
    if (i >= n || j > i) return;
    if (j < i) W[(n + i) * ldw + j] = U[j * ldu + i];
    W[(n + i) * ldw + n + j] = C[i * ldc + j];
    if (check_char2 && j == i && C[i * ldc + i] != 0.0) atomicExch(info, 1);
}
__global__ void k_trss_unpack(const double* W, int64_t ldw, int64_t n, double* X, int64_t ldx) {
    int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t a = blockIdx.y;
    if (a >= n || b >= n) return;
    X[a * ldx + b] = (a <= b) ? W[(n + b) * ldw + n + a] : 0.0;
}

// PLDUQ standalone layout in an (m+n) x (m+n) W: Y^T at W[m.., 0..m)
__global__ void k_plduq_pack(const double* Y, int64_t ldy, int64_t m, int64_t n, double* W, int64_t ldw) {
    int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t i = blockIdx.y;
    if (i >= m || j >= n) return;
    W[(m + j) * ldw + i] = Y[i * ldy + j];
}
__global__ void k_plduq_unpack(const double* W, int64_t ldw, int64_t m, int64_t n, double* Y, int64_t ldy,
                               const int32_t* orig, int32_t* rows, int32_t* cols) {
    int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t a = blockIdx.y;
    if (a >= m) return;
    if (b < n) Y[a * ldy + b] = W[(m + b) * ldw + a];
    if (b == 0) rows[a] = orig[a];
    if (a == 0 && b < n) cols[b] = orig[m + b] - (int32_t)m;
}

// ===========================================================================
// Explicit instantiations used by the driver.
// ===========================================================================
template __global__ void k_load_input<uint32_t>(const uint32_t*, int64_t, double*, int64_t, int64_t, Field, int32_t*);
template __global__ void k_load_input<double>(const double*, int64_t, double*, int64_t, int64_t, Field, int32_t*);
template __global__ void k_store_output<uint32_t>(uint32_t*, int64_t, const double*, int64_t, int64_t, const double*,
                                                  const double*, uint32_t*, const int32_t*, int32_t*);
template __global__ void k_store_output<double>(double*, int64_t, const double*, int64_t, int64_t, const double*,
                                                const double*, double*, const int32_t*, int32_t*);

}  // namespace pldl
