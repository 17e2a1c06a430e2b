// plduq.hip -- the leaf of the rank-profile-revealing PLDUQ (Sections 4.2 and 5
// pivoting): one row slab of Y (at most 64 rows, any width) in one launch.
//
// Y is held as its compact transpose T (Y[i][j] = T[j][i], leading dimension
// ld), so Y column j is T row j and the slab's rows a0 .. a0+m-1 are m
// contiguous doubles of every T row.
//
// Pivoting.  Columns are cut into chunks of PS_CHUNK; chunk b belongs to
// workgroup b.  The pivots are taken chunk by chunk from left to right, and
// inside a chunk in increasing row order: a row's pivot is the first nonzero of
// its reduced row among the chunk's columns that are not yet pivot columns.
// A pivot eliminates the rows that have no pivot yet; rows with a pivot keep
// their values (their U part).  This is a lexicographic search: a row takes
// a pivot in chunk b only when it is zero on every earlier chunk, so
// elimination by pivots of later chunks never changes what an earlier chunk
// saw, and the pivot set is the rank profile matrix of the slab.
//
// Elimination is fraction free: pivot (i, c) with value x turns an active row t
// into x y_t - y_t[c] y_i.  Every active row is then scaled by the same factor
// (the product S_s of the pivots taken before pivot s), which changes no zero
// pattern, and no inverse is needed while searching.  At the end, with
// x_s the scaled pivot values: multiplier of row t for pivot s = y_t[c_s] / x_s,
// U entry of pivot row s = y / x_s, D_s = x_s / S_s.
//
// Chain.  Workgroup b loads its chunk into registers (lane = slab row, each
// wave PS_CPW columns), applies the pivots of chunks 0 .. b-1 in order as they
// are published (no barrier: wave shuffles only), searches its own chunk (one
// workgroup barrier per pivot), then publishes its pivots (slab row, column,
// x, and the scaled pivot column of multipliers) and raises its flag.  Once
// the last chunk has published, every workgroup writes its chunk to its final
// place: pivot rows first in pivot order, then the other rows in their previous
// order; pivot columns first (T rows c0 .. c0+R) in pivot order, then the other
// columns in increasing order.  Every workgroup has read its chunk before it
// publishes, so no write lands on data still to be read.  pR / pC (original
// row / column indices) follow the same orders.
//
// The chain needs every workgroup of the grid resident at once (at most
// PS_MAXCH workgroups, one per compute unit suffices).  Each wait is bounded:
// after PS_SPIN polls a wave marks the launch aborted, every waiting wave
// leaves, and the host reports the error instead of hanging.
#include <type_traits>

#include "kernels.h"

namespace pldl {

namespace {

__device__ __forceinline__ double rdlane(double v, int l) {
    const long long w = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(w & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(w >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Waits for chunk flag *flag to carry generation gen and returns it (base and
// count in its low word).  0: the launch was aborted (or this wait timed out and
// aborted it).  Relaxed polls; one agent-scope acquire fence once it is seen.
__device__ uint64_t ps_wait(const uint64_t* flag, int32_t gen, int32_t* abort_word, int32_t* herr) {
    for (int it = 0;; ++it) {
        const uint64_t v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((int32_t)(v >> 32) == gen) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return v;
        }
        if ((it & 31) == 31 &&
            __hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen)
            return 0;
        if (it >= PS_SPIN) {
            __hip_atomic_store(abort_word, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (herr) __hip_atomic_store(herr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            return 0;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}
__device__ __forceinline__ int flag_base(uint64_t v) { return (int)((v >> 8) & 0xff); }
__device__ __forceinline__ int flag_cnt(uint64_t v) { return (int)(v & 0xff); }

}  // namespace

__global__ __launch_bounds__(PS_THREADS) void k_plduq_slab(PsArgs g) {
    constexpr int CPW = PS_CPW, NW = PS_THREADS / 64;
    static_assert(NW * CPW == PS_CHUNK && CPW <= 32, "chunk geometry");
    __shared__ int offer[2][NW];
    __shared__ double offer_col[2][NW][64];
    __shared__ int colpiv[PS_CHUNK];     // chunk column -> slab pivot index (-1: none)
    __shared__ int rowpiv[64];           // slab row -> slab pivot index (-1: none)
    __shared__ double xinv_l[64], dval_l[64];
    __shared__ int newpos[64];
    __shared__ unsigned long long cmask[PS_CHUNK / 64];
    __shared__ int okw, rtot;
    __shared__ uint64_t flagw;

    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const Field F = g.F;
    PsShared* sh = g.sh;
    const int m = g.m;
    const int64_t cb = g.c0 + (int64_t)b * PS_CHUNK;           // first T row of the chunk
    const int64_t wc = cb + (int64_t)wave * CPW;               // first T row of this wave
    const int nw = (int)max((int64_t)0, min((int64_t)CPW, g.c1 - wc));
    const int lr = min(lane, max(m - 1, 0));

    // ---- the chunk into registers (row = lane), the old index vectors
    double y[CPW];
    if (nw > 0) {
        const double* src = g.T + wc * g.ld + g.a0 + lr;
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
            const double v = src[(int64_t)min(k, nw - 1) * g.ld];
            y[k] = (k < nw && lane < m) ? fcen(v, F) : 0.0;
        }
    } else {
#pragma unroll
        for (int k = 0; k < CPW; ++k) y[k] = 0.0;
    }
    const int pc_old = (lane < nw) ? g.pC[wc + lane] : 0;
    const int pr_old = (b == 0 && lane < m) ? g.pR[g.a0 + lane] : 0;
    for (int e = tid; e < PS_CHUNK; e += PS_THREADS) colpiv[e] = -1;
    bool active = lane < m;
    uint32_t live = nw >= 32 ? 0xffffffffu : ((1u << nw) - 1u);

    // eliminate the active rows other than i with pivot (i, x) and scaled column f (this lane's row).
    // A row left as it is takes x = 1, f = 0: 1 * y - 0 * u = y, which the reduction keeps
    // (y is a reduced centered residue).  The live-column mask is the same in every lane
    // of the wave, so the column tests are scalar branches.
    // all_live: no column of the chunk is a pivot column yet (the pivots of the chunks to
    // the left), so every column is updated (the padding columns past the edge hold 0
    // in every row and stay 0).
    auto apply = [&](int i, double x, double f, auto all_live) {
        const bool upd = active && lane != i;
        const double xl = upd ? x : 1.0, fl = upd ? f : 0.0;
        const uint32_t lv = __builtin_amdgcn_readfirstlane(live);
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
            if (decltype(all_live)::value || __builtin_expect((lv >> k) & 1u, 1u)) {
                const double u = rdlane(y[k], i);
                y[k] = fredc(fma(xl, y[k], -fl * u), F);
            }
        }
        if (lane == i) active = false;
    };
    using AllLive = std::true_type;
    using SomeDead = std::false_type;

    // ---- pivots of the chunks to the left, in order, as they are published:
    // wave 0 polls the flag (one poller per workgroup), the others wait at a barrier
    bool ok = true;
    int base = 0;
    for (int bp = 0; bp < b && ok; ++bp) {
        if (wave == 0) {
            const uint64_t fv = ps_wait(&sh->flag[bp * PS_FLAG_STRIDE], g.gen, &sh->abort_gen, g.hout + 1);
            if (lane == 0) flagw = fv;
        }
        __syncthreads();
        const uint64_t fv = flagw;
        ok = fv != 0;
        if (!ok) break;
        const int bb = __builtin_amdgcn_readfirstlane(flag_base(fv));
        const int bc = __builtin_amdgcn_readfirstlane(flag_cnt(fv));
        // the records of up to four pivots in flight at once
        for (int s0 = bb; s0 < bb + bc; s0 += 4) {
            int ri[4];
            double rx[4], rf[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int s = min(s0 + q, bb + bc - 1);
                ri[q] = sh->prow[s];
                rx[q] = sh->px[s];
                rf[q] = sh->pf[s * 64 + lane];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (s0 + q < bb + bc) apply(__builtin_amdgcn_readfirstlane(ri[q]), rx[q], rf[q], AllLive{});
        }
        base = bb + bc;
        __syncthreads();   // flagw is rewritten for the next chunk
    }
    if (!ok) return;   // (uniform: every wave read the same flag)

    // ---- own search: the first active row with a nonzero on a live column, its first such
    // column.  Each wave offers a candidate (its first such row, that row's first such
    // column among the wave's columns, packed row << 16 | column, and the column's values
    // in every row); the smallest packed value wins, so one barrier per pivot suffices.
    // The offers are double-buffered: a wave that runs ahead writes the other buffer.
    int r = 0;
    for (;; ++r) {
        const int ob = r & 1;
        const uint32_t lv = __builtin_amdgcn_readfirstlane(live);
        uint32_t nzb = 0;
#pragma unroll
        for (int k = 0; k < CPW; ++k) nzb |= (((lv >> k) & 1u) && y[k] != 0.0) ? (1u << k) : 0u;
        if (!active) nzb = 0;
        const unsigned long long bal = __ballot(nzb != 0);
        int cw = 0x7fffffff;
        if (bal) {
            const int iw = __ffsll((long long)bal) - 1;
            const int kw = __ffs(__builtin_amdgcn_readlane((int)nzb, iw)) - 1;
            cw = (iw << 16) | (wave * CPW + kw);
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < CPW; ++k) v = (k == kw) ? y[k] : v;
            offer_col[ob][wave][lane] = v;
        }
        if (lane == 0) offer[ob][wave] = cw;
        __syncthreads();
        int best = 0x7fffffff;
#pragma unroll
        for (int w = 0; w < NW; ++w) best = min(best, offer[ob][w]);
        if (best == 0x7fffffff) break;
        const int i = best >> 16, c = best & 0xffff;
        const int wo = c / CPW, ko = c - wo * CPW;
        const double x = offer_col[ob][wo][i];
        const double fv = offer_col[ob][wo][lane];
        const double f = (active && lane != i) ? fv : 0.0;
        const int sp = base + r;
        if (wave == wo) {
            sh->pf[sp * 64 + lane] = f;
            if (lane == 0) {
                sh->px[sp] = x;
                sh->prow[sp] = i;
                sh->pcol[sp] = (int32_t)(cb + c);
                colpiv[c] = sp;
            }
            live &= ~(1u << ko);   // the column keeps D (row i), multipliers (active rows), U (pivot rows)
        }
        apply(i, x, f, SomeDead{});
    }

    // ---- publish: the barrier puts every wave's record stores in the (shared)
    // L2, thread 0's agent-scope release writes them back with the flag
    __syncthreads();
    if (tid == 0) {
        const uint64_t fv = ((uint64_t)(uint32_t)g.gen << 32) | ((uint64_t)base << 8) | (uint64_t)r;
        __hip_atomic_store(&sh->flag[b * PS_FLAG_STRIDE], fv, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }

    // ---- every chunk published: final values, final places
    if (tid < 64) {
        const uint64_t fv = ps_wait(&sh->flag[(g.nch - 1) * PS_FLAG_STRIDE], g.gen, &sh->abort_gen, g.hout + 1);
        if (tid == 0) { okw = fv != 0; rtot = flag_base(fv) + flag_cnt(fv); }
    }
    __syncthreads();
    if (!okw) return;
    const int R = rtot;
    if (wave == 0) {
        // 1/x_s, the exclusive prefix products of 1/x (1/S_s) and D_s = x_s / S_s
        rowpiv[lane] = -1;
        const double x = lane < R ? fcan(sh->px[lane], F) : 1.0;
        const double xi = lane < R ? (g.itab ? (double)g.itab[(int)x] : finv(x, F)) : 1.0;
        double pre = xi;   // inclusive scan of the inverses
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double o = __shfl_up(pre, off);
            if (lane >= off) pre = fmulm(pre, o, F);
        }
        double sinv = __shfl_up(pre, 1);
        if (lane == 0) sinv = 1.0;
        xinv_l[lane] = xi;
        dval_l[lane] = fmulm(x, sinv, F);
    }
    // this chunk's pivot columns as a bit mask (PS_CHUNK bits)
    if (tid < PS_CHUNK) {
        const unsigned long long cm = __ballot(colpiv[tid] >= 0);
        if (lane == 0) cmask[tid >> 6] = cm;
    }
    __syncthreads();
    if (wave == 0 && lane < R) rowpiv[sh->prow[lane]] = lane;
    __syncthreads();
    if (wave == 0) {
        const bool isp = lane < m && rowpiv[lane] >= 0;
        const unsigned long long pm = __ballot(isp);
        const int before = lane - __popcll(pm & ((1ull << lane) - 1ull));   // non-pivot rows before this one
        newpos[lane] = isp ? rowpiv[lane] : R + before;
        if (b == 0 && lane < m) {
            g.pR[g.a0 + newpos[lane]] = pr_old;
            g.srcR[newpos[lane]] = lane;
        }
    }
    __syncthreads();
    if (nw > 0) {
        const int rp = lane < m ? rowpiv[lane] : -1;
        const double xr = rp >= 0 ? xinv_l[rp] : 0.0;   // U scale of this row
        const int np = newpos[lr];
        // pivot columns of this chunk before the wave's first column
        const int c00 = wave * CPW;
        int pbefore = 0;
#pragma unroll
        for (int q = 0; q < PS_CHUNK / 64; ++q) {
            const int lo = q * 64;
            if (lo + 64 <= c00) pbefore += __popcll(cmask[q]);
            else if (lo < c00) pbefore += __popcll(cmask[q] & ((1ull << (c00 - lo)) - 1ull));
        }
#pragma unroll
        for (int k = 0; k < CPW; ++k) {
            if (k < nw) {
                const int c = wave * CPW + k;
                const int s = colpiv[c];
                int64_t dest;
                double v;
                if (s >= 0) {
                    dest = g.c0 + s;
                    if (rp == s) v = dval_l[s];
                    else if (rp >= 0 && rp < s) v = fmulm(y[k], xr, F);
                    else v = fmulm(y[k], xinv_l[s], F);
                } else {
                    dest = g.c0 + R + (cb - g.c0 + c) - base - pbefore;
                    v = rp >= 0 ? fmulm(y[k], xr, F) : 0.0;
                }
                if (lane < m) g.T[dest * g.ld + g.a0 + np] = v;
                const int pco = __shfl(pc_old, k);
                if (lane == 0) {
                    g.pC[dest] = pco;
                    g.srcC[dest - g.c0] = (int32_t)(cb - g.c0 + c);
                }
                pbefore += s >= 0;
            }
        }
    }
    if (b == g.nch - 1 && tid == 0) {
        g.rdev[0] = R;
        g.hout[0] = R;
        // the host polls this word instead of waiting for the launch to end
        __threadfence_system();
        __hip_atomic_store(g.hflag, g.hgen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace pldl
