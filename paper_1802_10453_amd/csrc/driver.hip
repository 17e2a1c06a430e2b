// driver.hip -- host side of the library: workspace, the recursive algorithms of
// Section 4 (Algorithm 2 RECALL, Algorithm 3 ZLP with the PLDUQ it starts with,
// Algorithm 1 TRSS), the cascade to the base case of Section 5, and the C-ABI.
//
// Data layout (device): W is an n x n FP64 matrix, row-major, leading dimension
// n, of which only the lower triangle is meaningful.  Each recursive call owns a
// contiguous range [lo, hi) of positions; on entry W[lo:hi, lo:hi] holds the
// symmetric Schur complement of the range, W[lo:hi, 0:lo] the rows of L computed
// so far, W[hi:n, lo:hi] the coupling with the positions after the range.  A call
// permutes its range symmetrically (all three parts), leaves L (strict lower)
// and D (dd, de) for its pivots, its rank pivots first and its non-pivots last in
// increasing original index.  `orig` maps positions to original indices.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <chrono>
#include <immintrin.h>
#include <fstream>
#include <random>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/pldl.h"
#include "common.h"
#include "kernels.h"

namespace pldl {

Field make_field(uint32_t p) {
    Field F;
    F.p = (double)p;
    F.pinv = 1.0 / (double)p;
    F.half = (double)(p / 2);
    F.inv2 = (double)((p + 1) / 2);
    F.ip = (int32_t)p;
    double mh = (double)((p - 1) / 2);
    double lim = 9007199254740992.0 - (double)p;
    int64_t k = (mh > 0.0) ? (int64_t)(lim / (mh * mh)) : ((int64_t)1 << 30);
    if (k > ((int64_t)1 << 30)) k = (int64_t)1 << 30;
    k = (k / 16) * 16;
    F.kred = (int32_t)std::max<int64_t>(16, k);
    return F;
}

struct Err : std::runtime_error {
    int code;
    Err(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) throw Err(PLDL_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)
#define REQUIRE(c)                                                                                         \
    do {                                                                                                   \
        if (!(c)) throw Err(PLDL_EINTERNAL, std::string("internal check failed: ") + #c + " at line " +   \
                                                std::to_string(__LINE__));                                 \
    } while (0)

static inline unsigned nblk(int64_t x, int b = 256) { return (unsigned)((x + b - 1) / b); }
// mapped host words written by the PLDUQ slab launch: rank, abort flag
constexpr int HW_SLAB = 256;
// mapped host word a leaf launch raises to its generation once its results are written
constexpr int HW_FLAG = 512;
// device word of ws.info that a PLDUQ slab writes its rank to
constexpr int INFO_SLAB_RANK = 16;
// "no column left of the range is read later" (see Engine::recall)
constexpr int64_t AL_NONE = INT64_MAX;

// ---------------------------------------------------------------------------
// Profiling: HIP events around each launch, harvested at host synchronisations.
struct Prof {
    bool on = false;
    bool light = false;      // product launches timed in-kernel, nothing else recorded
    uint32_t mask = 0x1FFu;  // classes recorded while on
    pldl_stats tot{};
    struct Rec { hipEvent_t a, b; int cls; double flops, bytes, ops8; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t open_a = nullptr;
    int open_cls = -1;
    double open_f = 0.0, open_b = 0.0, open_o = 0.0;
    // in-kernel stamps: NTS slots of (start, end) wall-clock ticks
    static constexpr int NTS = 16384;
    unsigned long long *ts0 = nullptr, *ts1 = nullptr;
    int nts = 0;
    double wall_khz = 0.0;
    hipStream_t ts_stream = nullptr;
    struct TRec { int cls; double flops, bytes, ops8; };
    std::vector<TRec> trecs;
    // counts of the current call (pldl_schedule): dispatches queued, host waits, products per path
    int64_t n_launch = 0, n_wait = 0, n_f64 = 0, n_i8 = 0, n_wino = 0;
    void reset_counts() { n_launch = n_wait = n_f64 = n_i8 = n_wino = 0; }

    hipEvent_t ev() {
        if (pool.empty()) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            return e;
        }
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    // Starts recording one launch of class c; in light mode returns the stamp slot
    // the launch must fill (product classes only) instead of recording events.
    Stamp begin(hipStream_t st, int c, double flops = 0.0, double bytes = 0.0, double ops8 = 0.0) {
        if (!on || !((mask >> c) & 1u)) return Stamp{};
        if (light) return stamp(st, c, flops, bytes, ops8);
        open_a = ev();
        HIPCHK(hipEventRecord(open_a, st));
        open_cls = c; open_f = flops; open_b = bytes; open_o = ops8;
        return Stamp{};
    }
    void end(hipStream_t st) {
        if (!on || open_cls < 0) return;
        hipEvent_t b = ev();
        HIPCHK(hipEventRecord(b, st));
        recs.push_back(Rec{open_a, b, open_cls, open_f, open_b, open_o});
        open_cls = -1;
    }
    Stamp stamp(hipStream_t st, int c, double flops, double bytes, double ops8) {
        if (!ts0) {
            int dev = 0, khz = 0;
            HIPCHK(hipGetDevice(&dev));
            HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
            wall_khz = (double)khz;
            HIPCHK(hipMalloc((void**)&ts0, NTS * sizeof(unsigned long long)));
            HIPCHK(hipMalloc((void**)&ts1, NTS * sizeof(unsigned long long)));
            reset_stamps(st);
        }
        if (nts == NTS || (ts_stream && ts_stream != st)) harvest_stamps();
        ts_stream = st;
        trecs.push_back(TRec{c, flops, bytes, ops8});
        const int k = nts++;
        return Stamp{ts0 + k, ts1 + k};
    }
    void reset_stamps(hipStream_t st) {
        HIPCHK(hipMemsetAsync(ts0, 0xFF, NTS * sizeof(unsigned long long), st));
        HIPCHK(hipMemsetAsync(ts1, 0x00, NTS * sizeof(unsigned long long), st));
    }
    // waits for the stamped launches, folds them into the totals, re-arms the slots
    void harvest_stamps() {
        if (nts == 0) return;
        HIPCHK(hipStreamSynchronize(ts_stream));
        std::vector<unsigned long long> a(nts), b(nts);
        HIPCHK(hipMemcpy(a.data(), ts0, nts * sizeof(unsigned long long), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(b.data(), ts1, nts * sizeof(unsigned long long), hipMemcpyDeviceToHost));
        for (int k = 0; k < nts; ++k) {
            pldl_kstat& s = tot.cls[trecs[k].cls];
            s.launches += 1; s.flops += trecs[k].flops; s.bytes += trecs[k].bytes; s.ops8 += trecs[k].ops8;
            if (b[k] > a[k]) s.ms += (double)(b[k] - a[k]) / wall_khz;
        }
        nts = 0;
        trecs.clear();
        reset_stamps(ts_stream);
        HIPCHK(hipStreamSynchronize(ts_stream));
    }
    void harvest() {
        for (Rec& r : recs) {
            HIPCHK(hipEventSynchronize(r.b));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
            pldl_kstat& k = tot.cls[r.cls];
            k.launches += 1; k.flops += r.flops; k.bytes += r.bytes; k.ops8 += r.ops8; k.ms += ms;
            pool.push_back(r.a); pool.push_back(r.b);
        }
        recs.clear();
        harvest_stamps();
    }
    void host_wait(double ms) {
        if (!on || light || !((mask >> PLDL_CLASS_HOST_SYNC) & 1u)) return;
        tot.cls[PLDL_CLASS_HOST_SYNC].launches += 1;
        tot.cls[PLDL_CLASS_HOST_SYNC].ms += ms;
    }
    ~Prof() {
        for (Rec& r : recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        if (ts0) (void)hipFree(ts0);
        if (ts1) (void)hipFree(ts1);
    }
};

#define LAUNCH(CLS, KERNEL, GRID, BLOCK, SHM, STREAM, ...)                  \
    do {                                                                   \
        prof->begin(STREAM, CLS);                                          \
        prof->n_launch++;                                                  \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, __VA_ARGS__); \
        prof->end(STREAM);                                                 \
    } while (0)

// ---------------------------------------------------------------------------
// Workspace: device buffers sized for order n (grown monotonically).
struct Workspace {
    int64_t cap = -1;
    double *W = nullptr, *tmp1 = nullptr, *tmp2 = nullptr, *dd = nullptr, *de = nullptr;
    double *xinv = nullptr, *yy = nullptr, *dvec = nullptr;
    double* tinv = nullptr;   // N_k = I - T_kk^{-1} of the diagonal blocks of a TRSM (64 x 64 each)
    int64_t tinv_rows = 0;    // tinv holds tinv_rows / 64 blocks
    int8_t* kind = nullptr;
    int32_t *orig = nullptr, *sig = nullptr, *tmpo = nullptr, *info = nullptr, *pidx = nullptr;
    int32_t* ipool = nullptr;          // stack of PLDUQ orders and orig snapshots, then scratch
    int64_t ipool_len = 0;             // ints of the stack part
    int32_t* ipool_scratch = nullptr;  // two halves: inverse map, reorder source
    int64_t ipool_scratch_len = 0;
    int32_t* colblk = nullptr;     // per column: block id once it stops moving with its rows, else -1
    int32_t* dinv = nullptr;       // per block: position of each original index when it stopped (n each)
    int64_t dinv_blocks = 0;       // capacity of dinv in blocks
    PsShared* ps = nullptr;        // words shared by the workgroups of a PLDUQ slab launch
    int32_t ps_gen = 0;            // generation of the last slab launch (flags compare equal to it)
    int32_t* hinfo = nullptr;      // pinned host words (rank, error flag, sigma, pivot columns)
    int32_t hgen = 0;              // last generation raised in hinfo[HW_FLAG]
    int32_t* hinfo_dev = nullptr;  // the same words as seen from the device: leaves write them directly
    void release() {
        double* ds[] = {W, tmp1, tmp2, dd, de, xinv, yy, dvec, tinv};
        for (double* p : ds) if (p) (void)hipFree(p);
        if (kind) (void)hipFree(kind);
        int32_t* is[] = {orig, sig, tmpo, info, pidx, ipool, colblk, dinv};
        for (int32_t* p : is) if (p) (void)hipFree(p);
        if (ps) (void)hipFree(ps);
        if (hinfo) (void)hipHostFree(hinfo);
        *this = Workspace();
    }
    void ensure(int64_t n) {
        if (n <= cap) return;
        release();
        int64_t m = std::max<int64_t>(n, 1);
        size_t nn = (size_t)m * (size_t)m;
        auto dalloc = [&](double** p, size_t cnt) {
            if (hipMalloc((void**)p, cnt * sizeof(double)) != hipSuccess) {
                (void)hipGetLastError();
                release();
                throw Err(PLDL_ENOMEM, "device allocation of " + std::to_string(cnt * 8) + " bytes failed");
            }
        };
        dalloc(&W, nn);
        dalloc(&tmp1, nn + 256);
        dalloc(&tmp2, 2 * nn + 256);
        dalloc(&dd, m + 1);
        dalloc(&de, m + 1);
        dalloc(&xinv, m + 1);
        dalloc(&yy, m + 1);
        dalloc(&dvec, 2 * m + 2);
        dalloc(&tinv, 64 * (size_t)(m + 64));
        tinv_rows = m + 64;
        if (hipMalloc((void**)&kind, m + 1) != hipSuccess) { release(); throw Err(PLDL_ENOMEM, "alloc"); }
        int32_t** ips[] = {&orig, &sig, &tmpo, &pidx, &colblk};
        for (int32_t** p : ips)
            if (hipMalloc((void**)p, (2 * m + 1024) * sizeof(int32_t)) != hipSuccess) {
                release();
                throw Err(PLDL_ENOMEM, "alloc");
            }
        if (hipMalloc((void**)&info, 1024 * sizeof(int32_t)) != hipSuccess) { release(); throw Err(PLDL_ENOMEM, "alloc"); }
        // stack: the row and column orders of both halves of a PLDUQ row split (at most
        // 4 segments of m entries per level, <= 11 levels for m <= 65535), the orig
        // snapshots of the ranges that move the rows under them at their end (at most 2m
        // along one recursion path), then the scratch (inverse map and source, m + 64 each)
        ipool_len = 44 * (m + 64);
        ipool_scratch_len = 2 * (m + 64);
        if (hipMalloc((void**)&ipool, (ipool_len + ipool_scratch_len) * sizeof(int32_t)) != hipSuccess) {
            release();
            throw Err(PLDL_ENOMEM, "alloc");
        }
        ipool_scratch = ipool + ipool_len;
        dinv_blocks = 2 * ((m + 63) / 64) + 16;
        if (hipMalloc((void**)&dinv, (size_t)dinv_blocks * (size_t)m * sizeof(int32_t)) != hipSuccess) {
            (void)hipGetLastError();
            release();
            throw Err(PLDL_ENOMEM, "alloc");
        }
        if (hipMalloc((void**)&ps, sizeof(PsShared)) != hipSuccess || hipMemset(ps, 0, sizeof(PsShared)) != hipSuccess) {
            (void)hipGetLastError();
            release();
            throw Err(PLDL_ENOMEM, "alloc");
        }
        ps_gen = 0;
        if (hipHostMalloc((void**)&hinfo, 1024 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
            hipHostGetDevicePointer((void**)&hinfo_dev, hinfo, 0) != hipSuccess) {
            (void)hipGetLastError();
            release();
            throw Err(PLDL_ENOMEM, "pinned alloc");
        }
        std::memset(hinfo, 0, 1024 * sizeof(int32_t));
        hgen = 0;
        cap = n;
    }
};

// ---------------------------------------------------------------------------
// Limb planes of the INT8-split products (grown on demand; see gemm_i8.hip).
struct GrowBuf {
    int8_t* p = nullptr;
    size_t cap = 0;
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    // returns true when it had to wait for the stream (a larger buffer)
    bool ensure(size_t bytes, hipStream_t st) {
        if (bytes <= cap) return false;
        HIPCHK(hipStreamSynchronize(st));   // the old planes may still be read
        release();
        size_t want = std::max(bytes, cap + cap / 2);
        if (hipMalloc((void**)&p, want) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            throw Err(PLDL_ENOMEM, "device allocation of " + std::to_string(want) + " bytes failed");
        }
        cap = want;
        return true;
    }
};

struct Engine {
    hipStream_t st;
    Field F;
    int64_t n, ld;
    int t_leaf;
    Workspace& ws;
    double* W;
    Prof* prof;
    const uint32_t* itab = nullptr;  // x -> x^{-1} mod p table (device), or NULL
    int path = PLDL_PATH_F64;         // products on FP64 or INT8-split matrix cores
    GrowBuf* i8 = nullptr;
    double i8_min_flops = 0.0;        // smaller products stay on FP64 (split passes would dominate)
    GrowBuf* wg = nullptr;            // temporaries of the Winograd products (a stack)
    int64_t wino_min = 0;             // products with m, n, k all >= this take a Winograd level (0: off)
    size_t wg_top = 0;                // doubles in use on the Winograd stack
    Engine(Workspace& w, hipStream_t s, uint32_t p, int64_t n_, int t, Prof* pr)
        : st(s), F(make_field(p)), n(n_), ld(std::max<int64_t>(n_, 1)), t_leaf(t), ws(w), W(w.W), prof(pr) {}

    // bounds of a view inside W (every view the algorithms form lies in W's lower triangle)
    void chk(int64_t r0, int64_t c0, int64_t rows, int64_t cols) const {
        REQUIRE(r0 >= 0 && c0 >= 0 && rows >= 0 && cols >= 0 && r0 + rows <= n && c0 + cols <= n);
    }
    MatV vrow(int64_t r0, int64_t c0) { return MatV{W + r0 * ld + c0, ld, 1}; }  // W[r0+i][c0+j]
    MatV vcol(int64_t r0, int64_t c0) { return MatV{W + r0 * ld + c0, 1, ld}; }  // W[r0+j][c0+i]

    // words the device wrote into `info` (device memory): copied back after the queued work
    int32_t* read_info(int cnt, int off = 0) {
        HIPCHK(hipMemcpyAsync(ws.hinfo, ws.info + off, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        prof->n_launch++;
        return read_host();
    }
    // A leaf launch writes its results straight into the pinned host words and then
    // raises HW_FLAG to its generation (system-scope release): the host polls that
    // word and queues the next launches while the leaf's last waves drain, instead
    // of waiting for the launch to end.  A launch that ends without raising it (an
    // aborted PLDUQ slab) is caught by the stream query.  With per-launch events on,
    // the plain wait keeps their harvest as it was.
    int32_t next_hgen() {
        ws.hgen = ws.hgen == INT32_MAX ? 1 : ws.hgen + 1;
        return ws.hgen;
    }
    int32_t* wait_leaf(int32_t gen) {
        if (prof->on && !prof->light) return read_host();
        for (uint32_t it = 1;; ++it) {
            if (__atomic_load_n(ws.hinfo + HW_FLAG, __ATOMIC_ACQUIRE) == gen) break;
            if ((it & 255u) == 0) {
                const hipError_t e = hipStreamQuery(st);
                if (e == hipSuccess) break;
                if (e != hipErrorNotReady) HIPCHK(e);
            }
            _mm_pause();
        }
        prof->n_wait++;
        return ws.hinfo;
    }
    // words the device wrote straight into the pinned host words: only a wait
    int32_t* read_host() {
        auto t0 = std::chrono::steady_clock::now();
        HIPCHK(hipStreamSynchronize(st));
        prof->n_wait++;
        if (prof->on && !prof->light) {   // (stamps are collected when their slots run out, or at pldl_profile)
            prof->host_wait(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
            prof->harvest();
        }
        return ws.hinfo;
    }

    void gemm(double* C, int64_t m, int64_t nn, GemmSeg s0, GemmSeg s1 = GemmSeg{MatV{nullptr, 0, 1}, MatV{nullptr, 0, 1}, 0},
              bool lower = false, bool b_upper = false) {
        if (m <= 0 || nn <= 0 || (s0.k <= 0 && s1.k <= 0)) return;
        GemmSeg segs[2] = {s0, s1};
        if (s0.k > 0 && s1.k > 0) REQUIRE((s0.A.cs == 1) == (s1.A.cs == 1) && (s0.B.cs == 1) == (s1.B.cs == 1));
        double kk = (double)std::max<int64_t>(s0.k, 0) + (double)std::max<int64_t>(s1.k, 0);
        double outs = lower ? (double)m * (double)(m + 1) / 2.0 : (double)m * (double)nn;
        double flops = 2.0 * outs * kk;
        if (b_upper && s0.k > 0 && !lower) {
            // segment 0's B is upper triangular: output column j sums min(j + 1, k) products
            const double k0 = (double)s0.k, nc = (double)nn;
            const double tri = nc <= k0 ? nc * (nc + 1) / 2.0 : k0 * (k0 + 1) / 2.0 + (nc - k0) * k0;
            flops -= 2.0 * (double)m * (nc * k0 - tri);
        }
        mm(C, ld, m, nn, segs, 2, lower, b_upper, flops);
    }
    // one product on the selected matrix cores
    // (the limb split is timed as class OTHER, the INT8 product as class GEMM).  flops: the
    // useful work recorded by the profile (structural zeros of a triangular operand left
    // out); the path is chosen on the work the matrix cores do (every product of the tiles).
    void mm(double* C, int64_t ldc, int64_t m, int64_t nn, const GemmSeg* segs, int nseg, bool lower, bool b_upper,
            double flops) {
        if (wino_min > 0 && !lower && !b_upper && segs[0].k >= wino_min && (nseg < 2 || segs[1].k <= 0) &&
            m >= wino_min && nn >= wino_min) {
            winograd(C, ldc, m, nn, segs[0].A, segs[0].B, segs[0].k);
            return;
        }
        double opnd = 0.0;   // operand elements, each read once
        double ksum = 0.0;
        for (int q = 0; q < nseg; ++q)
            if (segs[q].k > 0) {
                opnd += (double)segs[q].k * ((double)m + (double)nn);
                ksum += (double)segs[q].k;
            }
        const double outs = lower ? (double)m * (double)(m + 1) / 2.0 : (double)m * (double)nn;
        if (path == PLDL_PATH_I8 && 2.0 * outs * ksum >= i8_min_flops) {
            if (i8->ensure(i8_workspace_bytes((uint32_t)F.ip, m, nn, segs, nseg), st)) prof->n_wait++;
            I8Product pr;
            prof->begin(st, PLDL_CLASS_OTHER);
            const bool ok = i8_prepare(st, F, m, nn, segs, nseg, b_upper, i8->p, i8->cap, &pr);
            prof->end(st);
            if (ok) {
                const int L = pr.L;
                const Stamp sp = prof->begin(st, PLDL_CLASS_GEMM_I8, flops, (double)L * opnd + 16.0 * outs,
                                             flops * (double)(L * L));
                i8_run(st, F, pr, C, ldc, lower, sp);
                prof->end(st);
                prof->n_launch += 2;   // the limb split of every operand, the product
                prof->n_i8++;
                return;
            }
        }
        const Stamp sp = prof->begin(st, PLDL_CLASS_GEMM, flops, 8.0 * opnd + 16.0 * outs);
        launch_gemm(st, F, m, nn, C, ldc, segs, nseg, lower, b_upper, sp);
        prof->end(st);
        prof->n_launch++;
        prof->n_f64++;
    }

    // One level of Winograd's variant of Strassen's product (exact over F_p: the
    // seven half-size products and the fifteen sums are all taken mod p) on the
    // leading 2mh x 2nh x 2kh part of C -= A B, the halves rounded down to
    // multiples of 64; the strips outside it are plain products.  With
    // S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2,
    // T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12, T4 = T2 - B21 and
    // P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4, P5 = S1 T1,
    // P6 = S2 T2, P7 = S3 T3, U2 = P1 + P6, U3 = U2 + P7, U4 = U2 + P5:
    // C11 -= P1 + P2, C12 -= U4 + P3, C21 -= U3 - P4, C22 -= U3 + P5.
    // The product kernel subtracts, so the temporaries hold -P1, -U2, ...
    // Sub-products go through mm again (another level when they are still large).
    double* wpush(size_t cnt) {
        REQUIRE(wg_top + cnt <= wg->cap / sizeof(double));
        double* p = (double*)wg->p + wg_top;
        wg_top += (cnt + 31) / 32 * 32;
        return p;
    }
    void winograd(double* C, int64_t ldc, int64_t m, int64_t nn, MatV A, MatV B, int64_t k) {
        const int64_t mh = (m / 2) / 64 * 64, nh = (nn / 2) / 64 * 64, kh = (k / 2) / 64 * 64;
        REQUIRE(mh > 0 && nh > 0 && kh > 0);
        const size_t need = (size_t)(2 * mh * kh + 2 * kh * nh + 4 * mh * nh);
        if (wg_top == 0) {   // outermost level: room for every nested level (each a quarter of its parent's)
            if (wg->ensure(2 * (need + 1024) * sizeof(double), st)) prof->n_wait++;
        }
        prof->n_wino++;
        const size_t top0 = wg_top;
        double* S = wpush(mh * kh);
        double* S4 = wpush(mh * kh);
        double* Tt = wpush(kh * nh);
        double* T34 = wpush(kh * nh);
        double* Qa = wpush(mh * nh);
        double* Qb = wpush(mh * nh);
        double* Qc = wpush(mh * nh);
        double* Qd = wpush(mh * nh);
        auto blk = [](MatV X, int64_t r0, int64_t c0) { return MatV{X.p + r0 * X.rs + c0 * X.cs, X.rs, X.cs}; };
        const MatV Cv{C, ldc, 1}, none{nullptr, 0, 0};
        const MatV A11 = blk(A, 0, 0), A12 = blk(A, 0, kh), A21 = blk(A, mh, 0), A22 = blk(A, mh, kh);
        const MatV B11 = blk(B, 0, 0), B12 = blk(B, 0, nh), B21 = blk(B, kh, 0), B22 = blk(B, kh, nh);
        const MatV C11 = blk(Cv, 0, 0), C12 = blk(Cv, 0, nh), C21 = blk(Cv, mh, 0), C22 = blk(Cv, mh, nh);
        const MatV vS{S, kh, 1}, vS4{S4, kh, 1}, vT{Tt, nh, 1}, vT34{T34, nh, 1};
        const MatV vQa{Qa, nh, 1}, vQb{Qb, nh, 1}, vQc{Qc, nh, 1}, vQd{Qd, nh, 1};
        auto ew = [&](MatV D, int64_t rows, int64_t cols, MatV X, int sx, MatV Y, int sy, MatV Z, int sz) {
            LAUNCH(PLDL_CLASS_OTHER, k_ew3, dim3(nblk(cols), (unsigned)rows), dim3(256), 0, st, D, X, Y, Z, rows, cols,
                   sx, sy, sz, F);
        };
        auto prod = [&](MatV Cq, int64_t pm, int64_t pn, MatV X, MatV Y, int64_t pk) {   // Cq -= X Y
            if (pm <= 0 || pn <= 0 || pk <= 0) return;
            GemmSeg sg{X, Y, pk};
            mm(Cq.p, Cq.rs, pm, pn, &sg, 1, false, false, 2.0 * (double)pm * (double)pn * (double)pk);
        };
        REQUIRE(mh <= 65535 && kh <= 65535);
        ew(vQa, mh, nh, none, 0, none, 0, none, 0);        // Qa = 0
        prod(vQa, mh, nh, A11, B11, kh);                   // Qa = -P1
        prod(C11, mh, nh, A12, B21, kh);                   // C11 -= P2
        ew(C11, mh, nh, C11, 1, vQa, 1, none, 0);          // C11 -= P1
        ew(vS, mh, kh, A21, 1, A22, 1, none, 0);           // S1
        ew(vT, kh, nh, B12, 1, B11, -1, none, 0);          // T1
        ew(vQc, mh, nh, none, 0, none, 0, none, 0);
        prod(vQc, mh, nh, vS, vT, kh);                     // Qc = -P5
        ew(vS, mh, kh, vS, 1, A11, -1, none, 0);           // S2
        ew(vT, kh, nh, B22, 1, vT, -1, none, 0);           // T2
        prod(vQa, mh, nh, vS, vT, kh);                     // Qa = -U2
        ew(vS4, mh, kh, A12, 1, vS, -1, none, 0);          // S4
        ew(vQb, mh, nh, vQa, 1, none, 0, none, 0);         // Qb = -U2
        ew(vS, mh, kh, A11, 1, A21, -1, none, 0);          // S3
        ew(vT34, kh, nh, B22, 1, B12, -1, none, 0);        // T3
        prod(vQb, mh, nh, vS, vT34, kh);                   // Qb = -U3
        ew(C22, mh, nh, C22, 1, vQb, 1, vQc, 1);           // C22 -= U3 + P5
        ew(vQa, mh, nh, vQa, 1, vQc, 1, none, 0);          // Qa = -U4
        prod(vQa, mh, nh, vS4, B22, kh);                   // Qa = -(U4 + P3)
        ew(C12, mh, nh, C12, 1, vQa, 1, none, 0);          // C12 -= U4 + P3
        ew(vT34, kh, nh, vT, 1, B21, -1, none, 0);         // T4
        ew(vQd, mh, nh, none, 0, none, 0, none, 0);
        prod(vQd, mh, nh, A22, vT34, kh);                  // Qd = -P4
        ew(C21, mh, nh, C21, 1, vQb, 1, vQd, -1);          // C21 -= U3 - P4
        wg_top = top0;
        prod(C11, 2 * mh, 2 * nh, blk(A, 0, 2 * kh), blk(B, 2 * kh, 0), k - 2 * kh);
        prod(blk(Cv, 2 * mh, 0), m - 2 * mh, nn, blk(A, 2 * mh, 0), B, k);
        prod(blk(Cv, 0, 2 * nh), 2 * mh, nn - 2 * nh, A, blk(B, 0, 2 * nh), k);
    }

    // Columns left of every range still to be permuted that no later step reads
    // before the output stop moving with their rows (see `al` below): columns
    // [dead_upto, upto) are marked now, with where each original index sits,
    // and the output reads them from there.
    int64_t dead_upto = 0;
    int32_t dead_blocks = 0;
    bool track_dead = false;   // pldl_factor only: its output step gathers the stopped columns
    void stop_columns(int64_t upto) {
        if (!track_dead || upto <= dead_upto) return;
        REQUIRE(dead_blocks < ws.dinv_blocks);
        LAUNCH(PLDL_CLASS_PERM, k_dead_snapshot, dim3(nblk(n)), dim3(256), 0, st, ws.orig, dead_upto, upto, n,
               dead_blocks, ws.colblk, ws.dinv + (int64_t)dead_blocks * n);
        ++dead_blocks;
        dead_upto = upto;
    }
    // Symmetric permutation of [lo, hi): new lo+q <- old lo+sig[q].
    // parts: 1 = rows x [al, lo), 2 = block, 4 = rows [hi, below) x range, 8 = orig.
    // al: the first column left of the range that a later step still reads
    // (AL_NONE: none of them; every column left of min(al, lo) stops moving).
    // below: the rows under the range that take the new column order now; the
    // rows past it take it later, composed with the enclosing range's own order
    // (see recall).
    int64_t n_perms = 0;   // symmetric permutations applied so far
    // skip_ident: sig may be the identity (a leaf's, queued before the host has seen
    // it); the kernels then move nothing.
    void perm_sym(int64_t lo, int64_t hi, const int32_t* sig, int parts, int64_t al, int64_t below,
                  bool skip_ident = false) {
        const int64_t s = hi - lo;
        if (s <= 1) return;
        REQUIRE(below >= hi && below <= n);
        ++n_perms;
        REQUIRE(lo >= 0 && hi <= n && sig);
        REQUIRE(lo >= dead_upto);   // no stopped column lies in a range that still moves
        const int64_t c0 = (parts & 1) ? (track_dead ? std::min(std::max<int64_t>(al, 0), lo) : 0) : lo;
        if (parts & 1) stop_columns(c0);
        // rows below in one pass through LDS when a row segment fits
        const bool below1 = (parts & 4) && below > hi && s <= SEG_PERM_LDS;
        PermGeom g{};
        g.n = n; g.lo = lo; g.hi = hi; g.s = s; g.c0 = c0; g.parts = parts; g.skip_ident = skip_ident ? 1 : 0;
        g.nb0 = nblk(std::max<int64_t>(lo - c0, 1), 256 * PERM_EPT);
        g.nb1 = nblk(s, 256 * PERM_EPT);
        g.B0 = ((parts & 1) && lo > c0) ? s * g.nb0 : 0;
        g.B1 = (parts & 2) ? s * g.nb1 : 0;
        g.B2 = ((parts & 4) && below > hi && !below1) ? (below - hi) * g.nb1 : 0;
        g.B3 = (parts & 8) ? g.nb1 : 0;
        const int64_t blocks = g.B0 + g.B1 + g.B2 + g.B3;
        REQUIRE(blocks < ((int64_t)1 << 31));
        double elems = (double)(g.B0 ? s * (lo - c0) : 0) + (double)(g.B1 ? s * (s + 1) / 2 : 0) +
                       (double)(((parts & 4) && below > hi) ? s * (below - hi) : 0);
        if (elems == 0.0 && blocks == 0) return;
        prof->begin(st, PLDL_CLASS_PERM, 0.0, 16.0 * elems);
        if (blocks > 0) {
            hipLaunchKernelGGL(k_perm_sym, dim3((unsigned)blocks), dim3(256), 0, st, W, ld, g, sig, ws.tmp1, ws.orig, ws.tmpo, 0);
            hipLaunchKernelGGL(k_perm_sym, dim3((unsigned)blocks), dim3(256), 0, st, W, ld, g, sig, ws.tmp1, ws.orig, ws.tmpo, 1);
            prof->n_launch += 2;
        }
        if (below1) {
            const int rpw = (int)std::max<int64_t>(1, SEG_PERM_ROWS_LDS / s);
            const int64_t nwg = (below - hi + rpw - 1) / rpw;
            REQUIRE(nwg < ((int64_t)1 << 31));
            hipLaunchKernelGGL(k_seg_perm, dim3((unsigned)nwg), dim3(256), (size_t)rpw * s * sizeof(double), st, W, ld,
                               lo, s, hi, below, sig, rpw, skip_ident ? 1 : 0);
            prof->n_launch += 1;
        }
        prof->end(st);
    }

    // ---- TRSM (Section 3) ---------------------------------------------------
    // A triangle of order <= 64 is one substitution launch (k_trsm_small).
    // Larger ones: the inverses of all 64 x 64 diagonal blocks come from one
    // launch; then recursive halving (on multiples of 64) down to orders <= 256,
    // each solved in one launch (k_trsm_stripe: stripes of independent rows, or
    // columns of a left solve, take the 64-blocks in order), with the updates
    // between halves as products.
    static unsigned ts_grid(int64_t nrhs) {
        const int64_t per = (int64_t)TS_COLS * (TS_THREADS / 64);
        return (unsigned)((nrhs + per - 1) / per);
    }
    // B (m x r, row-major) <- B T^{-1}, T unit upper (view)
    void trsm_ru(MatV B, int64_t m, int64_t r, MatV T) {
        if (m <= 0 || r <= 0) return;
        if (r <= 64) {   // one block: substitution, no inverse
            LAUNCH(PLDL_CLASS_TRSM_LEAF, k_trsm_small, dim3(ts_grid(m)), dim3(TS_THREADS), 0, st, B.p, B.rs, m, (int)r, T,
                   1, F);
            return;
        }
        const int64_t nb = (r + 63) / 64;
        ensure_tinv(nb * 64);
        LAUNCH(PLDL_CLASS_TRSM_LEAF, k_trinv_blocks, dim3((unsigned)nb), dim3(1024), 0, st, T, r, 0, ws.tinv, F);
        trsm_ru_rec(B, m, r, T, ws.tinv);
    }
    void trsm_ru_rec(MatV B, int64_t m, int64_t r, MatV T, double* Nb) {
        if (r <= TS_MAXR) {   // one launch: row stripes, 64-column blocks in order
            REQUIRE((m + TSR - 1) / TSR < ((int64_t)1 << 31));
            LAUNCH(PLDL_CLASS_TRSM_LEAF, k_trsm_stripe, dim3((unsigned)((m + TSR - 1) / TSR)), dim3(256), 0, st, B, m,
                   (int)r, T, Nb, 0, F);
            return;
        }
        int64_t r1 = std::max<int64_t>(64, (r / 2) / 64 * 64);
        trsm_ru_rec(B, m, r1, T, Nb);
        gemm_ld(B.p + r1, B.rs, m, r - r1, GemmSeg{MatV{B.p, B.rs, 1}, MatV{T.p + r1 * T.cs, T.rs, T.cs}, r1});
        trsm_ru_rec(MatV{B.p + r1, B.rs, 1}, m, r - r1, MatV{T.p + r1 * (T.rs + T.cs), T.rs, T.cs}, Nb + (r1 / 64) * 4096);
    }
    // B (r x ncols, row-major) <- T^{-1} B, T unit lower (view)
    void trsm_ll(MatV B, int64_t r, int64_t ncols, MatV T) {
        if (r <= 0 || ncols <= 0) return;
        if (r <= 64) {   // one block: substitution, no inverse
            LAUNCH(PLDL_CLASS_TRSM_LEAF, k_trsm_small, dim3(ts_grid(ncols)), dim3(TS_THREADS), 0, st, B.p, B.rs, ncols,
                   (int)r, T, 0, F);
            return;
        }
        const int64_t nb = (r + 63) / 64;
        ensure_tinv(nb * 64);
        LAUNCH(PLDL_CLASS_TRSM_LEAF, k_trinv_blocks, dim3((unsigned)nb), dim3(1024), 0, st, T, r, 1, ws.tinv, F);
        trsm_ll_rec(B, r, ncols, T, ws.tinv);
    }
    void trsm_ll_rec(MatV B, int64_t r, int64_t ncols, MatV T, double* Nb) {
        if (r <= TS_MAXR) {   // one launch, on the transposed views: X^T = B^T T^{-T}
            REQUIRE((ncols + TSR - 1) / TSR < ((int64_t)1 << 31));
            LAUNCH(PLDL_CLASS_TRSM_LEAF, k_trsm_stripe, dim3((unsigned)((ncols + TSR - 1) / TSR)), dim3(256), 0, st,
                   MatV{B.p, B.cs, B.rs}, ncols, (int)r, MatV{T.p, T.cs, T.rs}, Nb, 1, F);
            return;
        }
        int64_t r1 = std::max<int64_t>(64, (r / 2) / 64 * 64);
        trsm_ll_rec(B, r1, ncols, T, Nb);
        gemm_ld(B.p + r1 * B.rs, B.rs, r - r1, ncols, GemmSeg{MatV{T.p + r1 * T.rs, T.rs, T.cs}, MatV{B.p, B.rs, 1}, r1});
        trsm_ll_rec(MatV{B.p + r1 * B.rs, B.rs, 1}, r - r1, ncols, MatV{T.p + r1 * (T.rs + T.cs), T.rs, T.cs},
                    Nb + (r1 / 64) * 4096);
    }
    // the block inverses of a triangle of order `rows` (grown after the queued work is done)
    void ensure_tinv(int64_t rows) {
        if (rows <= ws.tinv_rows) return;
        HIPCHK(hipStreamSynchronize(st));
        prof->n_wait++;
        HIPCHK(hipFree(ws.tinv));
        ws.tinv = nullptr;
        ws.tinv_rows = 0;
        if (hipMalloc((void**)&ws.tinv, 64 * (size_t)rows * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            ws.tinv = nullptr;
            throw Err(PLDL_ENOMEM, "device allocation of the triangle inverses failed");
        }
        ws.tinv_rows = rows;
    }
    // flops < 0: the dense count 2 m nn k (else the useful flops of a structured operand)
    void gemm_ld(double* C, int64_t ldc, int64_t m, int64_t nn, GemmSeg s0, double flops = -1.0) {
        if (m <= 0 || nn <= 0 || s0.k <= 0) return;
        mm(C, ldc, m, nn, &s0, 1, false, false,
           flops >= 0.0 ? flops : 2.0 * (double)m * (double)nn * (double)s0.k);
    }

    // ---- base case (Section 5) ------------------------------------------------
    // below: the rows under the range that take its column order now (see recall)
    int64_t bc(int64_t lo, int64_t hi, int64_t al, int64_t below) {
        int s = (int)(hi - lo);
        REQUIRE(s >= 1 && s <= 128);
        const int32_t gen = next_hgen();
        LAUNCH(PLDL_CLASS_BASE_CASE, k_bc_leaf, dim3(1), dim3(BC_THREADS), 0, st, W, ld, lo, s, F, itab, ws.dd, ws.de, ws.sig,
               ws.hinfo_dev, ws.hinfo_dev + 1, ws.hinfo_dev + HW_FLAG, gen);
        // the leaf's order applied to the rows left of and below it, queued behind the leaf
        // before the host waits for its rank (the kernels skip an identity order)
        perm_sym(lo, hi, ws.sig, 1 | 4 | 8, al, below, true);
        int32_t* h = wait_leaf(gen);
        return h[0];
    }

    // ---- Algorithm 2 -----------------------------------------------------------
    // al: the first column left of lo that a later step still reads: the start
    // of the highest enclosing range whose first half contains this one (its
    // TRSM and GEMM read that half's L block once the half is done); AL_NONE
    // when there is none.  The first half of this range inherits min(al, lo);
    // the second part inherits al (this range reads nothing after it).
    //
    // below: the rows under the range that must hold its columns in their final
    // order when it returns.  A range with al != AL_NONE moves the rows under it
    // only once, at its end: its permutations update the rows inside it at once
    // and leave the rows in [hi, below) alone, and its end applies the order of
    // its columns relative to its start (from a snapshot of orig) to those rows.
    // This is sound because no step inside the range reads rows below hi, and
    // no column of the range stops moving meanwhile (every permutation inside
    // keeps the columns from min(al, ...) <= al <= lo on moving).  A range with
    // al == AL_NONE updates every row under its permutations at once (its own
    // steps stop columns inside it).
    int64_t recall(int64_t lo, int64_t hi, int64_t al, int64_t below) {
        int64_t N = hi - lo;
        if (N <= 0) return 0;
        if (N <= t_leaf) return bc(lo, hi, al, below);
        const bool defer = al != AL_NONE && below > hi;
        const int64_t inner = al == AL_NONE ? n : hi;   // bound the parts of this range pass down
        const int64_t ip_save = ip_top;
        const int32_t* snap = defer ? snapshot(ws.orig + lo, N) : nullptr;
        const int64_t perms0 = n_perms;
        int64_t m = N / 2;
        if (m >= 128) m = m / 64 * 64;
        int64_t r1 = recall(lo, lo + m, std::min(al, lo), inner);
        int64_t s = lo + m, n2 = hi - s;
        if (r1 > 0 && n2 > 0) {
            chk(s, lo, n2, m);
            // X^T = B'1^T L1^{-T}:  right solve with T = L1^T, T[a][b] = W[lo+b][lo+a]
            trsm_ru(vrow(s, lo), n2, r1, vcol(lo, lo));
            // Y^T = B'2^T - X^T M1^T, M1 = W[lo+r1 : lo+m, lo : lo+r1]
            if (m > r1) gemm(W + s * ld + lo + r1, n2, m - r1, GemmSeg{vrow(s, lo), vcol(lo + r1, lo), r1});
            // SCAL: T <- X^T, G = X^T D1^{-1} in place
            LAUNCH(PLDL_CLASS_OTHER, k_block_dinv, dim3(nblk(r1)), dim3(256), 0, st, ws.dd, ws.de, lo, r1, F, ws.xinv, ws.yy, ws.kind);
            LAUNCH(PLDL_CLASS_OTHER, k_scal_dinv, dim3(nblk(r1), (unsigned)n2), dim3(256), 0, st, W + s * ld + lo, ld, n2, r1,
                               ws.xinv, ws.yy, ws.kind, ws.tmp2, r1, F);
            // SYRDK: Z = C - G D1 G^T = lower(C - G X)
            gemm(W + s * ld + s, n2, n2, GemmSeg{vrow(s, lo), MatV{ws.tmp2, 1, r1}, r1}, GemmSeg{MatV{nullptr, 0, 1}, MatV{nullptr, 0, 1}, 0}, true);
        }
        const int64_t r = r1 + zlp(lo + r1, m - r1, hi, al, inner);
        if (defer && n_perms != perms0) perm_sym(lo, hi, reorder_src(snap, ws.orig + lo, N), 4, al, below);
        ip_top = ip_save;
        return r;
    }

    // ---- Algorithm 3 -----------------------------------------------------------
    // below: as in recall, for the rows under hi (the enclosing recall's bound)
    int64_t zlp(int64_t lo, int64_t mz, int64_t hi, int64_t al, int64_t below) {
        int64_t s0 = lo + mz, nc = hi - s0;
        if (mz == 0) return recall(lo, hi, al, below);
        if (nc == 0) return 0;
        // PLDUQ of Y on a compact copy of Y^T; then C' = Q C Q^T and the pack back into W
        REQUIRE(nc <= 65535 && mz <= 65535);
        T = ws.tmp2; ldT = mz; TR = nc; TC = mz; pR = ws.pidx; pC = ws.pidx + mz;
        LAUNCH(PLDL_CLASS_OTHER, k_copy2d, dim3(nblk(mz), (unsigned)nc), dim3(256), 0, st, T, mz, W + s0 * ld + lo, ld, nc, mz);
        LAUNCH(PLDL_CLASS_OTHER, k_iota2, dim3(nblk(std::max(mz, nc))), dim3(256), 0, st, pR, mz, pC, nc);
        int64_t rY = plduq_all(mz, nc);
        if (rY > 0) {
            perm_sym(s0, hi, pC, 2, al, hi);
            LAUNCH(PLDL_CLASS_OTHER, k_copy2d, dim3(nblk(mz), (unsigned)nc), dim3(256), 0, st, W + s0 * ld + lo, ld, T, mz, nc, mz);
        }
        int64_t nz = nc - rY, nr = mz - rY, N = hi - lo;
        double* G1 = ws.tmp2;
        double* G2 = ws.tmp2 + rY * rY;
        double* UT = G2 + nz * rY;        // characteristic-2 temporaries
        double* UTD = UT + rY * rY;
        double* VD = UTD + rY * rY;
        double* delta = ws.dvec;          // Delta (rY) then the pack diagonal d (rY)
        if (rY > 0) {
            HIPCHK(hipMemsetAsync(delta, 0, rY * sizeof(double), st));
            prof->n_launch++;
            LAUNCH(PLDL_CLASS_OTHER, k_save_pack_diag, dim3(nblk(rY)), dim3(256), 0, st, W, ld, s0, lo, rY, delta + rY);
            if (F.ip == 2) {
                REQUIRE(rY <= 8192);
                LAUNCH(PLDL_CLASS_OTHER, k_delta, dim3(1), dim3(1024), rY * sizeof(double), st, W, ld, s0, lo, rY, F, delta);
                LAUNCH(PLDL_CLASS_OTHER, k_u1t_delta, dim3(nblk(rY), (unsigned)rY), dim3(256), 0, st, W, ld, s0, lo, rY, delta, UT, UTD, F);
                // C'1 <- C'1 - U1^T Delta U1 (lower)
                gemm(W + s0 * ld + s0, rY, rY, GemmSeg{MatV{UTD, rY, 1}, MatV{UT, 1, rY}, rY},
                     GemmSeg{MatV{nullptr, 0, 1}, MatV{nullptr, 0, 1}, 0}, true);
            }
            trss(s0, rY, lo);
            // G1 = X^T D1^{-1} (lower)
            LAUNCH(PLDL_CLASS_OTHER, k_pack_dinv, dim3(nblk(rY)), dim3(256), 0, st, W, ld, s0, lo, rY, F, ws.xinv);
            LAUNCH(PLDL_CLASS_OTHER, k_mul_cols, dim3(nblk(rY), (unsigned)rY), dim3(256), 0, st, W + s0 * ld + s0, ld, rY, rY, ws.xinv, 1, G1, rY, F);
            if (F.ip == 2)
                LAUNCH(PLDL_CLASS_OTHER, k_dadd, dim3(nblk(rY), (unsigned)rY), dim3(256), 0, st, W, ld, s0, lo, rY, delta, F);
            if (nz > 0) {
                chk(s0 + rY, lo, nz, mz + rY);
                // C''2^T = C'2^T - V1^T X   (X upper = transpose of the stored X^T)
                gemm(W + (s0 + rY) * ld + s0, nz, rY, GemmSeg{vrow(s0 + rY, lo), vcol(s0, s0), rY},
                     GemmSeg{MatV{nullptr, 0, 1}, MatV{nullptr, 0, 1}, 0}, false, true);
                // Y2^T = C''2^T U1^{-1},  U1[a][b] = W[s0+b][lo+a]
                trsm_ru(vrow(s0 + rY, s0), nz, rY, vcol(s0, lo));
                // Z = C'3 - (Y2^T V1 + V1^T Y2)   (SYRD2K, lower)
                gemm(W + (s0 + rY) * ld + s0 + rY, nz, nz, GemmSeg{vrow(s0 + rY, s0), vcol(s0 + rY, lo), rY},
                     GemmSeg{vrow(s0 + rY, lo), vcol(s0 + rY, s0), rY}, true);
                if (F.ip == 2) {
                    // Z <- Z - V1^T Delta V1
                    LAUNCH(PLDL_CLASS_OTHER, k_mul_delta, dim3(nblk(rY), (unsigned)nz), dim3(256), 0, st, W + (s0 + rY) * ld + lo, ld, nz, rY, delta, VD, F);
                    gemm(W + (s0 + rY) * ld + s0 + rY, nz, nz, GemmSeg{MatV{VD, rY, 1}, vcol(s0 + rY, lo), rY},
                         GemmSeg{MatV{nullptr, 0, 1}, MatV{nullptr, 0, 1}, 0}, true);
                }
                // G2 = Y2^T D1^{-1}
                LAUNCH(PLDL_CLASS_OTHER, k_mul_cols, dim3(nblk(rY), (unsigned)nz), dim3(256), 0, st, W + (s0 + rY) * ld + s0, ld, nz, rY, ws.xinv, 0, G2, rY, F);
            }
        }
        // ---- assembly: [pairs (P_i interleave) | Z | non-pivot rows of the zero block]
        REQUIRE(N <= 65535);
        LAUNCH(PLDL_CLASS_PERM, k_zlp_assemble, dim3(nblk(N), (unsigned)N), dim3(256), 0, st, W, ld, lo, mz, hi, rY, G1,
                           std::max<int64_t>(rY, 1), G2, std::max<int64_t>(rY, 1), ws.tmp1);
        LAUNCH(PLDL_CLASS_PERM, k_copy2d, dim3(nblk(N), (unsigned)N), dim3(256), 0, st, W + lo * ld + lo, ld, ws.tmp1, N, N, N);
        // the assembly order composed with PLDUQ's maps, for the L part, the rows below and orig
        if (rY > 0)
            LAUNCH(PLDL_CLASS_OTHER, k_zlp_sigma_total, dim3(nblk(N)), dim3(256), 0, st, ws.sig, mz, nc, rY, pR, pC);
        else
            LAUNCH(PLDL_CLASS_OTHER, k_zlp_sigma, dim3(nblk(N)), dim3(256), 0, st, ws.sig, mz, nc, rY);
        perm_sym(lo, hi, ws.sig, 1 | 4 | 8, al, below);
        if (rY > 0)
            LAUNCH(PLDL_CLASS_OTHER, k_zlp_orig_d, dim3(nblk(N)), dim3(256), 0, st, ws.orig, ws.tmpo, lo, mz, hi, rY, W, ld, delta, ws.dd, ws.de, 2);
        int64_t rz = recall(lo + 2 * rY, lo + 2 * rY + nz, al, below);
        // non-pivots of Z and of the zero block, merged by original index
        int64_t a = lo + 2 * rY + rz, n1 = nz - rz;
        if (n1 > 0 && nr > 0) {
            LAUNCH(PLDL_CLASS_OTHER, k_sigma_merge, dim3(nblk(n1 + nr)), dim3(256), 0, st, ws.orig, a, n1, nr, ws.sig);
            perm_sym(a, hi, ws.sig, 1 | 4 | 8, al, below);
        }
        return 2 * rY + rz;
    }

    // ---- PLDUQ revealing the rank profile, on a compact transposed copy -------
    // T (TR x TC, leading dimension ldT) holds Y^T: Y[i][j] = T[j][i].  pR / pC
    // give the original row / column index at each position of Y.  A call on rows
    // [a0, a1) and columns [c0, c1) reorders rows and columns of that submatrix
    // only, keeps pR[a0 .. a1) and pC[c0 .. c1) up to date and returns the row
    // and column orders it applied; its caller carries them to the other parts
    // of the matrix that hold data, so no step moves the whole width of Y.  The
    // caller of the whole PLDUQ applies pC to W once.
    double* T = nullptr;
    int64_t ldT = 0, TR = 0, TC = 0;
    int32_t *pR = nullptr, *pC = nullptr;
    int64_t ip_top = 0;   // stack pointer in ws.ipool

    int32_t* ipush(int64_t cnt) {
        REQUIRE(ip_top + cnt + 64 <= ws.ipool_len);
        int32_t* p = ws.ipool + ip_top;
        ip_top += (cnt + 63) / 64 * 64;
        return p;
    }
    int32_t* snapshot(const int32_t* src, int64_t len) {
        int32_t* p = ipush(std::max<int64_t>(len, 1));
        if (len > 0) {
            HIPCHK(hipMemcpyAsync(p, src, len * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
            prof->n_launch++;
        }
        return p;
    }
    // src[q] = old position of the entry now at q, from a snapshot of an index segment
    int32_t* reorder_src(const int32_t* snap, const int32_t* cur, int64_t len) {
        int32_t* inv = ws.ipool_scratch;   // indexed by original index (< max(TR, TC))
        int32_t* src = ws.ipool_scratch + ws.ipool_scratch_len / 2;
        if (len <= 16384) {
            LAUNCH(PLDL_CLASS_OTHER, k_reorder_src_1wg, dim3(1), dim3(1024), 0, st, snap, cur, len, inv, src);
        } else {
            LAUNCH(PLDL_CLASS_OTHER, k_inv_scatter, dim3(nblk(len)), dim3(256), 0, st, snap, len, inv);
            LAUNCH(PLDL_CLASS_OTHER, k_src_gather, dim3(nblk(len)), dim3(256), 0, st, cur, len, inv, src);
        }
        return src;
    }
    // reorder T rows [j0, j0+len) (Y columns) by src, in T columns [i0, i0+ni) (Y rows)
    // skip_zero: a device word; nothing moves when it holds 0 (see plduq_t)
    void tcolperm(int64_t j0, int64_t len, const int32_t* src, int64_t i0, int64_t ni,
                  const int32_t* skip_zero = nullptr) {
        if (len <= 1 || ni <= 0) return;
        REQUIRE(len <= 65535 && len * ni <= ws.cap * ws.cap);
        dim3 g(nblk(ni, 256 * PERM_EPT), (unsigned)len);
        prof->begin(st, PLDL_CLASS_PERM, 0.0, 16.0 * (double)len * (double)ni);
        hipLaunchKernelGGL(k_tcolperm, g, dim3(256), 0, st, T, ldT, j0, len, src, i0, ni, ws.tmp1, 0, skip_zero);
        hipLaunchKernelGGL(k_tcolperm, g, dim3(256), 0, st, T, ldT, j0, len, src, i0, ni, ws.tmp1, 1, skip_zero);
        prof->end(st);
        prof->n_launch += 2;
    }
    // reorder T columns [i0, i0+len) (Y rows) by src, within T rows [j0, j0+nj)
    void trowperm(int64_t j0, int64_t nj, int64_t i0, int64_t len, const int32_t* src) {
        if (len <= 1 || nj <= 0) return;
        REQUIRE(nj <= 65535 && len * nj <= ws.cap * ws.cap);
        prof->begin(st, PLDL_CLASS_PERM, 0.0, 16.0 * (double)len * (double)nj);
        if (len <= SEG_PERM_LDS) {   // one pass: each T row segment through LDS
            const int rpw = (int)std::max<int64_t>(1, SEG_PERM_ROWS_LDS / len);
            const int64_t nwg = (nj + rpw - 1) / rpw;
            hipLaunchKernelGGL(k_seg_perm, dim3((unsigned)nwg), dim3(256), (size_t)rpw * len * sizeof(double), st, T,
                               ldT, i0, len, j0, j0 + nj, src, rpw, 0);
            prof->n_launch += 1;
        } else {
            dim3 g(nblk(len), (unsigned)nj);
            hipLaunchKernelGGL(k_trowperm, g, dim3(256), 0, st, T, ldT, j0, nj, i0, len, src, ws.tmp1, 0);
            hipLaunchKernelGGL(k_trowperm, g, dim3(256), 0, st, T, ldT, j0, nj, i0, len, src, ws.tmp1, 1);
            prof->n_launch += 2;
        }
        prof->end(st);
    }
    // idx[a + q] <- idx[a + src[q]]
    void idx_reorder(int32_t* idx, int64_t a, int64_t len, const int32_t* src) {
        if (len <= 1) return;
        if (len <= 16384) {
            LAUNCH(PLDL_CLASS_OTHER, k_idx_reorder_1wg, dim3(1), dim3(1024), 0, st, idx, a, len, src);
            return;
        }
        LAUNCH(PLDL_CLASS_OTHER, k_idx_gather, dim3(nblk(len)), dim3(256), 0, st, idx, a, len, src, ws.tmpo);
        LAUNCH(PLDL_CLASS_OTHER, k_idx_copy, dim3(nblk(len)), dim3(256), 0, st, idx, a, len, ws.tmpo);
    }

    // rows [a0, a1) and columns [c0, c1) of Y.  Row slabs of <= 64 rows; the
    // bottom half of a row split is updated with the top half's pivots (TRSM,
    // GEMM) and continues on the columns the top half left.  On return row a0 + q
    // holds the row that was at a0 + srcR[q], column c0 + q the column that was at
    // c0 + srcC[q] (the caller carries these orders to the parts it holds); when
    // *moved is false nothing moved and the orders (the identity) are not written.
    int64_t plduq_t(int64_t a0, int64_t a1, int64_t c0, int64_t c1, int32_t* srcR, int32_t* srcC, bool* moved) {
        const int64_t m = a1 - a0;
        *moved = m > 0 && c1 > c0;
        if (!*moved) return 0;
        REQUIRE(a1 <= TC && c1 <= TR);
        if (m <= 64) return plduq_slab_wait(plduq_slab_launch(a0, a1, c0, c1, srcR, srcC), m);
        const int64_t ip_save = ip_top;
        const int64_t am = a0 + std::max<int64_t>(64, (m / 2) / 64 * 64);
        const int64_t h = am - a0, mb = a1 - am, len = c1 - c0;
        int32_t* sRt = ipush(h);
        int32_t* sCt = ipush(len);
        bool tmv = false, bmv = false;
        int64_t r1;
        const bool top_slab = h <= 64;
        if (top_slab) {
            // The bottom rows take the top slab's column order: queued behind the slab
            // before the host waits for its rank (skipped on the device when it is 0).
            const int32_t gen = plduq_slab_launch(a0, am, c0, c1, sRt, sCt);
            tmv = true;
            tcolperm(c0, len, sCt, am, mb, ws.info + INFO_SLAB_RANK);
            r1 = plduq_slab_wait(gen, h);
        } else {
            r1 = plduq_t(a0, am, c0, c1, sRt, sCt, &tmv);
        }
        if (r1 > 0) {
            const int64_t ncr = len - r1;
            // the bottom rows take the top half's column order
            if (!top_slab) tcolperm(c0, len, sCt, am, mb);
            // Wb^T = U_t^{-T} Y_b1^T  (U_t^T unit lower at T[c0.., a0..])
            trsm_ll(MatV{T + c0 * ldT + am, ldT, 1}, r1, mb, MatV{T + c0 * ldT + a0, ldT, 1});
            // Y_b2^T -= V_t^T Wb^T
            if (ncr > 0)
                gemm_ld(T + (c0 + r1) * ldT + am, ldT, ncr, mb,
                        GemmSeg{MatV{T + (c0 + r1) * ldT + a0, ldT, 1}, MatV{T + c0 * ldT + am, ldT, 1}, r1});
            // L_b^T = D_t^{-1} Wb^T
            LAUNCH(PLDL_CLASS_OTHER, k_scale_pack, dim3(nblk(mb), (unsigned)r1), dim3(256), 0, st, T + c0 * ldT + am, ldT, r1, mb,
                   T + c0 * ldT + a0, ldT, 1, itab, F);
        }
        int32_t* sRb = ipush(mb);
        int32_t* sCb = ipush(std::max<int64_t>(len - r1, 1));
        // a bottom half that is one slab: the top rows' reorder by its column order is
        // queued the same way, before the host waits for its rank
        const bool bot_slab = mb <= 64 && len > r1;
        int64_t r2;
        if (bot_slab) {
            const int32_t gen = plduq_slab_launch(am, a1, c0 + r1, c1, sRb, sCb);
            bmv = true;
            tcolperm(c0 + r1, len - r1, sCb, a0, h, ws.info + INFO_SLAB_RANK);
            r2 = plduq_slab_wait(gen, mb);
        } else {
            r2 = plduq_t(am, a1, c0 + r1, c1, sRb, sCb, &bmv);
        }
        if (r2 > 0) {
            // the top rows take the bottom half's column order, the bottom rows' multipliers its row order
            if (!bot_slab) tcolperm(c0 + r1, len - r1, sCb, a0, h);
            if (r1 > 0) trowperm(c0, r1, am, mb, sRb);
            // pivot rows of both halves first: rotate the top non-pivots behind the bottom pivots
            if (h > r1) {
                const int64_t rl = am + r2 - (a0 + r1);
                int32_t* src = ws.ipool_scratch + ws.ipool_scratch_len / 2;
                LAUNCH(PLDL_CLASS_OTHER, k_rot_src, dim3(nblk(rl)), dim3(256), 0, st, rl, h - r1, src);
                trowperm(c0, len, a0 + r1, rl, src);
                idx_reorder(pR, a0 + r1, rl, src);
            }
        }
        // this call's orders, composed from its halves' (a half on which nothing moved: null)
        LAUNCH(PLDL_CLASS_OTHER, k_compose, dim3(nblk(std::max(len, m))), dim3(256), 0, st, srcC, tmv ? sCt : nullptr,
               bmv ? sCb : nullptr, len, srcR, tmv ? sRt : nullptr, bmv ? sRb : nullptr, h, m, r1, r2);
        ip_top = ip_save;
        return r1 + r2;
    }
    // the whole of T: the orders go to scratch on the stack
    int64_t plduq_all(int64_t rows, int64_t cols) {
        const int64_t ip_save = ip_top;
        int32_t* sR = ipush(rows);
        int32_t* sC = ipush(cols);
        bool moved = false;
        const int64_t r = plduq_t(0, rows, 0, cols, sR, sC, &moved);
        ip_top = ip_save;
        return r;
    }

    // A slab (<= 64 rows) in one launch (k_plduq_slab): chunks of PS_CHUNK
    // columns, one workgroup each, pivots chunk by chunk from left to right and
    // in row order inside a chunk; on return the slab's pivot rows and pivot
    // columns come first (pivot order), pR / pC updated.  The host reads the
    // slab's rank from mapped host words (one wait per slab).
    int32_t plduq_slab_launch(int64_t a0, int64_t a1, int64_t c0, int64_t c1, int32_t* srcR, int32_t* srcC) {
        const int64_t m = a1 - a0;
        const int64_t nch = (c1 - c0 + PS_CHUNK - 1) / PS_CHUNK;
        REQUIRE(m >= 1 && m <= 64 && nch >= 1 && nch <= PS_MAXCH);
        PsArgs g{};
        g.T = T; g.ld = ldT; g.a0 = a0; g.m = (int)m; g.nch = (int)nch; g.c0 = c0; g.c1 = c1;
        g.F = F; g.itab = itab; g.pR = pR; g.pC = pC; g.sh = ws.ps;
        g.srcR = srcR; g.srcC = srcC;
        g.rdev = ws.info + INFO_SLAB_RANK;
        g.gen = ++ws.ps_gen;
        g.hout = ws.hinfo_dev + HW_SLAB;   // (the base case uses words 0 .. 128)
        g.hflag = ws.hinfo_dev + HW_FLAG;
        g.hgen = next_hgen();
        ws.hinfo[HW_SLAB + 1] = 0;
        LAUNCH(PLDL_CLASS_PLDUQ_LEAF, k_plduq_slab, dim3((unsigned)nch), dim3(PS_THREADS), 0, st, g);
        return g.hgen;
    }
    // the rank of the slab launched with generation gen (m rows), once it has written it
    int64_t plduq_slab_wait(int32_t gen, int64_t m) {
        const int32_t* h = wait_leaf(gen);
        if (h[HW_SLAB + 1]) throw Err(PLDL_EINTERNAL, "PLDUQ slab: a chunk waited too long for its predecessor (launch aborted)");
        const int64_t R = h[HW_SLAB];
        REQUIRE(R >= 0 && R <= m);
        return R;
    }

    // ---- Algorithm 1 (TRSS): C at W[s0..s0+r)^2, U[a][b] = W[s0+b][u0+a] -----
    void trss(int64_t s0, int64_t r, int64_t u0) {
        if (r <= 0) return;
        if (r <= 64) {
            LAUNCH(PLDL_CLASS_TRSS_LEAF, k_trss_leaf, dim3(1), dim3(256), 0, st, W, ld, s0, u0, (int)r, F);
            return;
        }
        int64_t h = std::max<int64_t>(64, (r / 2) / 64 * 64);
        trss(s0, h, u0);
        // D2^T = C2^T - U2^T X1
        gemm(W + (s0 + h) * ld + s0, r - h, h, GemmSeg{vrow(s0 + h, u0), vcol(s0, s0), h},
             GemmSeg{MatV{nullptr, 0, 1}, MatV{nullptr, 0, 1}, 0}, false, true);
        // X2^T = D2^T U11^{-1}
        trsm_ru(vrow(s0 + h, s0), r - h, h, vcol(s0, u0));
        // D3 = C3 - (X2^T U2 + U2^T X2)
        gemm(W + (s0 + h) * ld + s0 + h, r - h, r - h, GemmSeg{vrow(s0 + h, s0), vcol(s0 + h, u0), h},
             GemmSeg{vrow(s0 + h, u0), vcol(s0 + h, s0), h}, true);
        trss(s0 + h, r - h, u0 + h);
    }
};

}  // namespace pldl

// ===========================================================================
// C-ABI
// ===========================================================================
using namespace pldl;

struct pldl_ctx {
    int device = 0;
    Workspace ws;
    Prof prof;
    std::string err;
    uint32_t* itab = nullptr;  // inverse table of modulus itab_p
    uint32_t itab_p = 0;
    int path = PLDL_PATH_AUTO; // matrix cores of the products (pldl_set_path)
    GrowBuf i8;
    GrowBuf wbuf;              // Winograd temporaries
    int64_t wino_min = 0;      // pldl_set_winograd
    // autotuned base-case thresholds: (p, n, threshold); pldl_factor takes the entry of
    // the same p (else any p) nearest to its n on a log scale, else 128
    struct Tune { uint32_t p; int64_t n; int t; };
    std::vector<Tune> tune;
    int tuned_threshold(uint32_t p, int64_t n) const {
        int best = 128;
        double bd = 1e300;
        for (int pass = 0; pass < 2 && bd == 1e300; ++pass)
            for (const Tune& e : tune) {
                if (pass == 0 && e.p != p) continue;
                const double dist = std::fabs(std::log((double)std::max<int64_t>(n, 1) / (double)e.n));
                if (dist < bd) { bd = dist; best = e.t; }
            }
        return best;
    }
    // Online threshold (the introspective refinement suggested at the end of
    // Section 6): per (p, order rounded to a power of two), the wall time of
    // every pldl_factor call made with threshold = PLDL_THRESHOLD_ONLINE.  Each
    // candidate is tried once, then the fastest is used; every 16th call
    // re-times the candidate with the oldest measurement, so the choice follows
    // changes of the running instances (load, other processes).
    static constexpr int N_ONLINE = 3;
    static constexpr int online_cand[N_ONLINE] = {128, 96, 64};
    struct Online { double ms[N_ONLINE]; int64_t when[N_ONLINE]; int64_t calls; };
    std::vector<std::pair<std::pair<uint32_t, int>, Online>> online;
    Online& online_slot(uint32_t p, int64_t n) {
        int lg = 0;
        while (((int64_t)1 << (lg + 1)) <= n) ++lg;
        for (auto& e : online)
            if (e.first.first == p && e.first.second == lg) return e.second;
        Online o{};
        for (int c = 0; c < N_ONLINE; ++c) { o.ms[c] = -1.0; o.when[c] = -1; }
        online.push_back({{p, lg}, o});
        return online.back().second;
    }
    int online_pick(uint32_t p, int64_t n, int* slot) {
        Online& o = online_slot(p, n);
        int pick = -1;
        for (int c = 0; c < N_ONLINE && pick < 0; ++c)
            if (o.ms[c] < 0.0) pick = c;
        if (pick < 0 && o.calls % 16 == 15) {   // re-time the oldest measurement
            pick = 0;
            for (int c = 1; c < N_ONLINE; ++c)
                if (o.when[c] < o.when[pick]) pick = c;
        }
        if (pick < 0) {
            pick = 0;
            for (int c = 1; c < N_ONLINE; ++c)
                if (o.ms[c] < o.ms[pick]) pick = c;
        }
        *slot = pick;
        return online_cand[pick];
    }
    void online_record(uint32_t p, int64_t n, int slot, double ms) {
        Online& o = online_slot(p, n);
        o.ms[slot] = ms;
        o.when[slot] = o.calls;
        ++o.calls;
    }
    void* bws = nullptr;       // batched factorizations: one slot per persistent workgroup
    int bslots = 0;
    int32_t* bqueue = nullptr;
    int32_t* border = nullptr;   // the batch's matrix order (largest first), grown to the largest batch
    int64_t border_cap = 0;
    // an Engine on this context's workspace, products on `path`
    void setup(Engine& E, int pth, double i8_min) {
        E.path = pth;
        E.i8 = &i8;
        E.i8_min_flops = i8_min;
        E.wg = &wbuf;
        E.wino_min = wino_min;
    }
    // table x -> x^{-1} mod p, built on the device the first time p is used
    const uint32_t* inv_table(uint32_t p, hipStream_t st) {
        if (itab_p == p && itab) return itab;
        if (itab) { HIPCHK(hipStreamSynchronize(st)); HIPCHK(hipFree(itab)); itab = nullptr; itab_p = 0; }
        if (hipMalloc((void**)&itab, (size_t)p * sizeof(uint32_t)) != hipSuccess) {
            (void)hipGetLastError();
            itab = nullptr;
            throw Err(PLDL_ENOMEM, "inverse table allocation failed");
        }
        Field F = make_field(p);
        hipLaunchKernelGGL(k_inv_table, dim3(nblk(p)), dim3(256), 0, st, itab, F);
        HIPCHK(hipGetLastError());
        itab_p = p;
        return itab;
    }
};

namespace {
int fail(pldl_ctx* c, int code, const std::string& m) {
    if (c) c->err = m;
    return code;
}
hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }
bool bad_p(uint32_t p) { return p < 2 || p >= (1u << 24); }

template <typename Fn>
int guarded(pldl_ctx* ctx, Fn&& fn) {
    try {
        HIPCHK(hipSetDevice(ctx->device));
        fn();
        if ((ctx->prof.on && !ctx->prof.light) || !ctx->prof.recs.empty()) ctx->prof.harvest();
        ctx->err.clear();
        return PLDL_OK;
    } catch (const Err& e) {
        return fail(ctx, e.code, e.what());
    } catch (const std::bad_alloc&) {
        return fail(ctx, PLDL_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(ctx, PLDL_EINTERNAL, e.what());
    }
}
}  // namespace

extern "C" {

int pldl_create(pldl_ctx** ctx, int device) {
    if (!ctx) return -1;
    int cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess || device < 0 || device >= cnt) return -2;
    // the allocation-free entry point's array, resolved on this device
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return PLDL_EHIP;
    const bool na = noalloc_init(device);
    (void)hipSetDevice(prev);
    if (!na) return PLDL_EHIP;
    pldl_ctx* c = new (std::nothrow) pldl_ctx();
    if (!c) return PLDL_ENOMEM;
    c->device = device;
    *ctx = c;
    return PLDL_OK;
}

int pldl_destroy(pldl_ctx* ctx) {
    if (!ctx) return PLDL_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->ws.release();
    ctx->i8.release();
    ctx->wbuf.release();
    if (ctx->bws) (void)hipFree(ctx->bws);
    if (ctx->bqueue) (void)hipFree(ctx->bqueue);
    if (ctx->border) (void)hipFree(ctx->border);
    if (ctx->itab) (void)hipFree(ctx->itab);
    delete ctx;
    return PLDL_OK;
}

const char* pldl_last_error(const pldl_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int pldl_factor(pldl_ctx* ctx, uint32_t p, int64_t n, void* A, int64_t lda, int32_t dtype, void* e, int32_t* perm,
                int32_t* rpm, int64_t* rank, const pldl_opts* opts, pldl_schedule* sched_out, void* stream) {
    if (!ctx) return -1;
    if (bad_p(p)) return fail(ctx, PLDL_EUNSUPPORTED_P, "p must satisfy 2 <= p < 2^24");
    if (n < 0 || n > 65535) return fail(ctx, -3, "n out of range [0, 65535]");
    if (n > 0 && !A) return fail(ctx, -4, "A is NULL");
    if (lda < std::max<int64_t>(1, n)) return fail(ctx, -5, "lda < max(1, n)");
    if (dtype != PLDL_U32 && dtype != PLDL_F64) return fail(ctx, -6, "unknown dtype");
    if (n > 0 && !e) return fail(ctx, -7, "e is NULL");
    if (n > 0 && !perm) return fail(ctx, -8, "perm is NULL");
    if (n > 0 && !rpm) return fail(ctx, -9, "rpm is NULL");
    if (!rank) return fail(ctx, -10, "rank is NULL");
    pldl_opts o{PLDL_PATH_AUTO, 0, 0, 1};
    if (opts) o = *opts;
    if (o.path != PLDL_PATH_AUTO && o.path != PLDL_PATH_F64 && o.path != PLDL_PATH_I8)
        return fail(ctx, -11, "unknown path");
    if (o.threshold < PLDL_THRESHOLD_ONLINE || o.threshold > 128)
        return fail(ctx, -11, "threshold must be PLDL_THRESHOLD_ONLINE or in [0, 128]");
    int online_slot = -1;
    int t = o.threshold > 0 ? o.threshold
          : o.threshold == 0 ? ctx->tuned_threshold(p, n)
          : (n > 0 ? ctx->online_pick(p, n, &online_slot) : 128);
    const auto t_call = std::chrono::steady_clock::now();
    // PLDL_PATH_AUTO: the INT8 split wherever its limbs cover the residues (p < 2^23)
    int path_used = o.path == PLDL_PATH_AUTO ? ctx->path : o.path;
    if (path_used == PLDL_PATH_AUTO) path_used = p < (1u << 23) ? PLDL_PATH_I8 : PLDL_PATH_F64;
    ctx->prof.reset_counts();
    auto fill_sched = [&]() {
        if (!sched_out) return;
        pldl_schedule sc{};
        sc.threshold_used = t;
        sc.split_rule = 64;
        sc.path_used = path_used;
        sc.i8_min_log2_flops = (int32_t)std::lround(std::log2(I8_MIN_FLOPS));
        sc.products_f64 = ctx->prof.n_f64;
        sc.products_i8 = ctx->prof.n_i8;
        sc.launches = ctx->prof.n_launch;
        sc.host_waits = ctx->prof.n_wait;
        sc.products_winograd = ctx->prof.n_wino;
        *sched_out = sc;
    };
    if (n == 0) { *rank = 0; fill_sched(); return PLDL_OK; }
    hipStream_t st = as_stream(stream);
    const int rc = guarded(ctx, [&]() {
        ctx->ws.ensure(n);
        Engine E(ctx->ws, st, p, n, t, &ctx->prof);
        ctx->setup(E, path_used, I8_MIN_FLOPS);
        E.itab = ctx->inv_table(p, st);
        Prof* prof = &ctx->prof;
        Workspace& ws = ctx->ws;
        HIPCHK(hipMemsetAsync(ws.info, 0, sizeof(int32_t) * 4, st));
        prof->n_launch++;
        dim3 g(nblk(n), (unsigned)n);
        if (dtype == PLDL_U32)
            LAUNCH(PLDL_CLASS_OTHER, k_load_input<uint32_t>, g, dim3(256), 0, st, (const uint32_t*)A, lda, ws.W, E.ld, n, E.F, ws.info + 2);
        else
            LAUNCH(PLDL_CLASS_OTHER, k_load_input<double>, g, dim3(256), 0, st, (const double*)A, lda, ws.W, E.ld, n, E.F, ws.info + 2);
        if (o.check_range) {
            int32_t* h = E.read_info(3);
            if (h[2]) throw Err(PLDL_ERANGE, "input entry outside [0, p)");
        }
        LAUNCH(PLDL_CLASS_OTHER, k_iota, dim3(nblk(n)), dim3(256), 0, st, ws.orig, n);
        HIPCHK(hipMemsetAsync(ws.dd, 0, sizeof(double) * n, st));
        HIPCHK(hipMemsetAsync(ws.de, 0, sizeof(double) * n, st));
        HIPCHK(hipMemsetAsync(ws.colblk, 0xFF, sizeof(int32_t) * n, st));
        prof->n_launch += 3;
        E.track_dead = true;
        int64_t r = E.recall(0, n, AL_NONE, n);
        const bool gathered = E.dead_blocks > 0;
        LAUNCH(PLDL_CLASS_OTHER, k_rpm, dim3(nblk(n)), dim3(256), 0, st, ws.orig, ws.de, n, r, rpm);
        if (o.standard_form && p == 2) {
            dim3 g2(nblk(n), (unsigned)n);
            if (gathered) {   // the transform works on W in the final row order
                LAUNCH(PLDL_CLASS_PERM, k_dead_gather, g2, dim3(256), 0, st, ws.W, E.ld, n, ws.orig, ws.colblk, ws.dinv, ws.tmp1);
                LAUNCH(PLDL_CLASS_PERM, k_copy2d, g2, dim3(256), 0, st, ws.W, E.ld, ws.tmp1, E.ld, n, n);
                E.dead_blocks = 0;
            }
            LAUNCH(PLDL_CLASS_OTHER, k_char2_std, g2, dim3(256), 0, st, ws.W, E.ld, n, ws.dd, ws.de, ws.orig, ws.tmp1, 0);
            LAUNCH(PLDL_CLASS_OTHER, k_char2_std, g2, dim3(256), 0, st, ws.W, E.ld, n, ws.dd, ws.de, ws.orig, ws.tmp1, 1);
            LAUNCH(PLDL_CLASS_OTHER, k_char2_std, dim3(nblk(n)), dim3(256), 0, st, ws.W, E.ld, n, ws.dd, ws.de, ws.orig, ws.tmp1, 2);
        }
        if (dtype == PLDL_U32)
            LAUNCH(PLDL_CLASS_OTHER, k_store_output<uint32_t>, g, dim3(256), 0, st, (uint32_t*)A, lda, ws.W, E.ld, n, ws.dd, ws.de, (uint32_t*)e, ws.orig, perm,
                   E.dead_blocks > 0 ? ws.colblk : nullptr, ws.dinv);
        else
            LAUNCH(PLDL_CLASS_OTHER, k_store_output<double>, g, dim3(256), 0, st, (double*)A, lda, ws.W, E.ld, n, ws.dd, ws.de, (double*)e, ws.orig, perm,
                   E.dead_blocks > 0 ? ws.colblk : nullptr, ws.dinv);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        prof->n_wait++;
        *rank = r;
    });
    if (rc == PLDL_OK && online_slot >= 0)
        ctx->online_record(p, n, online_slot,
                           std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_call).count());
    if (rc == PLDL_OK) fill_sched();
    return rc;
}

int pldl_gemm(pldl_ctx* ctx, uint32_t p, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, int32_t transA,
              const double* B, int64_t ldb, int32_t transB, double* C, int64_t ldc, int32_t lower_only, void* stream) {
    if (!ctx) return -1;
    if (bad_p(p)) return fail(ctx, PLDL_EUNSUPPORTED_P, "p must satisfy 2 <= p < 2^24");
    if (m < 0) return fail(ctx, -3, "m < 0");
    if (n < 0) return fail(ctx, -4, "n < 0");
    if (k < 0) return fail(ctx, -5, "k < 0");
    if (m > 0 && k > 0 && !A) return fail(ctx, -6, "A is NULL");
    if (lda < std::max<int64_t>(1, transA ? m : k)) return fail(ctx, -7, "lda too small");
    if (n > 0 && k > 0 && !B) return fail(ctx, -9, "B is NULL");
    if (ldb < std::max<int64_t>(1, transB ? k : n)) return fail(ctx, -10, "ldb too small");
    if (m > 0 && n > 0 && !C) return fail(ctx, -12, "C is NULL");
    if (ldc < std::max<int64_t>(1, n)) return fail(ctx, -13, "ldc too small");
    if (lower_only && m != n) return fail(ctx, -14, "lower_only needs m == n");
    hipStream_t st = as_stream(stream);
    return guarded(ctx, [&]() {
        GemmSeg s{transA ? MatV{(double*)A, 1, lda} : MatV{(double*)A, lda, 1},
                  transB ? MatV{(double*)B, 1, ldb} : MatV{(double*)B, ldb, 1}, k};
        Engine E(ctx->ws, st, p, 0, 128, &ctx->prof);
        ctx->setup(E, ctx->path == PLDL_PATH_I8 ? PLDL_PATH_I8 : PLDL_PATH_F64, 0.0);
        double outs = lower_only ? (double)m * (double)(m + 1) / 2.0 : (double)m * (double)n;
        if (m > 0 && n > 0 && k > 0) E.mm(C, ldc, m, n, &s, 1, lower_only != 0, false, 2.0 * outs * (double)k);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
    });
}

int pldl_trsm(pldl_ctx* ctx, uint32_t p, int32_t lower, int64_t m, int64_t n, const double* T, int64_t ldt, double* B,
              int64_t ldb, void* stream) {
    if (!ctx) return -1;
    if (bad_p(p)) return fail(ctx, PLDL_EUNSUPPORTED_P, "p must satisfy 2 <= p < 2^24");
    if (m < 0) return fail(ctx, -4, "m < 0");
    if (n < 0) return fail(ctx, -5, "n < 0");
    int64_t tord = lower ? m : n;
    if (tord > 0 && !T) return fail(ctx, -6, "T is NULL");
    if (ldt < std::max<int64_t>(1, tord)) return fail(ctx, -7, "ldt too small");
    if (m > 0 && n > 0 && !B) return fail(ctx, -8, "B is NULL");
    if (ldb < std::max<int64_t>(1, n)) return fail(ctx, -9, "ldb too small");
    hipStream_t st = as_stream(stream);
    return guarded(ctx, [&]() {
        ctx->ws.ensure(1);
        Engine E(ctx->ws, st, p, 0, 128, &ctx->prof);
        ctx->setup(E, ctx->path == PLDL_PATH_I8 ? PLDL_PATH_I8 : PLDL_PATH_F64, 0.0);
        if (lower) E.trsm_ll(MatV{B, ldb, 1}, m, n, MatV{(double*)T, ldt, 1});
        else E.trsm_ru(MatV{B, ldb, 1}, m, n, MatV{(double*)T, ldt, 1});
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
    });
}

int pldl_syrdk(pldl_ctx* ctx, uint32_t p, int64_t n, int64_t k, const double* A, int64_t lda, const double* B,
               int64_t ldb, const double* dd, const double* de, double* C, int64_t ldc, void* stream) {
    if (!ctx) return -1;
    if (bad_p(p)) return fail(ctx, PLDL_EUNSUPPORTED_P, "p must satisfy 2 <= p < 2^24");
    if (n < 0) return fail(ctx, -3, "n < 0");
    if (k < 0) return fail(ctx, -4, "k < 0");
    if (n > 0 && k > 0 && !A) return fail(ctx, -5, "A is NULL");
    if (lda < std::max<int64_t>(1, k)) return fail(ctx, -6, "lda too small");
    if (B && ldb < std::max<int64_t>(1, k)) return fail(ctx, -8, "ldb too small");
    if (k > 0 && (!dd || !de)) return fail(ctx, -9, "dd/de is NULL");
    if (n > 0 && !C) return fail(ctx, -11, "C is NULL");
    if (ldc < std::max<int64_t>(1, n)) return fail(ctx, -12, "ldc too small");
    hipStream_t st = as_stream(stream);
    return guarded(ctx, [&]() {
        if (n == 0 || k == 0) return;
        ctx->ws.ensure(std::max(n, k));
        Field F = make_field(p);
        Prof* prof = &ctx->prof;
        double* AD = ctx->ws.tmp2;
        double* BD = ctx->ws.tmp2 + n * k;
        LAUNCH(PLDL_CLASS_OTHER, k_apply_d, dim3(nblk(k), (unsigned)n), dim3(256), 0, st, A, lda, n, k, dd, de, AD, F);
        GemmSeg s0{MatV{AD, k, 1}, B ? MatV{(double*)B, 1, ldb} : MatV{(double*)A, 1, lda}, k};
        GemmSeg s1{MatV{nullptr, 0, 1}, MatV{nullptr, 0, 1}, 0};
        if (B) {
            LAUNCH(PLDL_CLASS_OTHER, k_apply_d, dim3(nblk(k), (unsigned)n), dim3(256), 0, st, B, ldb, n, k, dd, de, BD, F);
            s1 = GemmSeg{MatV{BD, k, 1}, MatV{(double*)A, 1, lda}, k};
        }
        GemmSeg segs[2] = {s0, s1};
        Engine E(ctx->ws, st, p, 0, 128, &ctx->prof);
        ctx->setup(E, ctx->path == PLDL_PATH_I8 ? PLDL_PATH_I8 : PLDL_PATH_F64, 0.0);
        E.mm(C, ldc, n, n, segs, 2, true, false, 2.0 * (double)n * (double)(n + 1) / 2.0 * (double)(B ? 2 * k : k));
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
    });
}

int pldl_syrdk_noalloc(pldl_ctx* ctx, uint32_t p, int64_t n, int64_t k, const double* A, int64_t lda, const double* B,
                       int64_t ldb, const double* dd, const double* de, double* C, int64_t ldc, void* stream) {
    if (!ctx) return -1;
    if (bad_p(p)) return fail(ctx, PLDL_EUNSUPPORTED_P, "p must satisfy 2 <= p < 2^24");
    if (n < 0) return fail(ctx, -3, "n < 0");
    if (k < 0) return fail(ctx, -4, "k < 0");
    if (n > 0 && k > 0 && !A) return fail(ctx, -5, "A is NULL");
    if (lda < std::max<int64_t>(1, k)) return fail(ctx, -6, "lda too small");
    if (B && ldb < std::max<int64_t>(1, k)) return fail(ctx, -8, "ldb too small");
    if (k > 0 && (!dd || !de)) return fail(ctx, -9, "dd/de is NULL");
    if (n > 0 && !C) return fail(ctx, -11, "C is NULL");
    if (ldc < std::max<int64_t>(1, n)) return fail(ctx, -12, "ldc too small");
    if (n > 0 && k > 0 && (double)n * (double)k * (B ? 2.0 : 1.0) > (double)PLDL_NOALLOC_SCRATCH_DOUBLES)
        return fail(ctx, PLDL_ETOOBIG, "n * k (2 n k with B) exceeds the allocation-free scratch of " +
                                           std::to_string(PLDL_NOALLOC_SCRATCH_DOUBLES) + " doubles");
    if (n == 0 || k == 0) return PLDL_OK;
    double* sp = noalloc_scratch(ctx->device);
    if (!sp) return fail(ctx, PLDL_EINTERNAL, "the allocation-free scratch was not resolved on this device");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, PLDL_EHIP, "hipSetDevice failed");
    hipStream_t st = as_stream(stream);
    const Field F = make_field(p);
    double* AD = sp;
    double* BD = sp + n * k;
    hipLaunchKernelGGL(k_apply_d, dim3(nblk(k), (unsigned)n), dim3(256), 0, st, A, lda, n, k, dd, de, AD, F);
    GemmSeg segs[2] = {GemmSeg{MatV{AD, k, 1}, B ? MatV{(double*)B, 1, ldb} : MatV{(double*)A, 1, lda}, k},
                       GemmSeg{MatV{nullptr, 0, 1}, MatV{nullptr, 0, 1}, 0}};
    if (B) {
        hipLaunchKernelGGL(k_apply_d, dim3(nblk(k), (unsigned)n), dim3(256), 0, st, B, ldb, n, k, dd, de, BD, F);
        segs[1] = GemmSeg{MatV{BD, k, 1}, MatV{(double*)A, 1, lda}, k};
    }
    launch_gemm(st, F, n, n, C, ldc, segs, 2, true, false);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, PLDL_EHIP, std::string("launch failed: ") + hipGetErrorString(e));
    ctx->err.clear();
    return PLDL_OK;
}

int pldl_solve(pldl_ctx* ctx, uint32_t p, int64_t n, const void* F, int64_t lda, int32_t dtype, const void* e,
               const int32_t* perm, int64_t rank, double* B, int64_t ldb, int64_t nrhs, int32_t* consistent,
               void* stream) {
    if (!ctx) return -1;
    if (bad_p(p)) return fail(ctx, PLDL_EUNSUPPORTED_P, "p must satisfy 2 <= p < 2^24");
    if (n < 0 || n > 65535) return fail(ctx, -3, "n out of range [0, 65535]");
    if (n > 0 && !F) return fail(ctx, -4, "F is NULL");
    if (lda < std::max<int64_t>(1, n)) return fail(ctx, -5, "lda < max(1, n)");
    if (dtype != PLDL_U32 && dtype != PLDL_F64) return fail(ctx, -6, "unknown dtype");
    if (n > 0 && !e) return fail(ctx, -7, "e is NULL");
    if (n > 0 && !perm) return fail(ctx, -8, "perm is NULL");
    if (rank < 0 || rank > n) return fail(ctx, -9, "rank outside [0, n]");
    if (nrhs < 0) return fail(ctx, -12, "nrhs < 0");
    if (n > 0 && nrhs > 0 && !B) return fail(ctx, -10, "B is NULL");
    if (ldb < std::max<int64_t>(1, nrhs)) return fail(ctx, -11, "ldb < max(1, nrhs)");
    if (n == 0 || nrhs == 0) return PLDL_OK;
    hipStream_t st = as_stream(stream);
    return guarded(ctx, [&]() {
        ctx->ws.ensure(n);
        Workspace& ws = ctx->ws;
        Engine E(ws, st, p, n, 128, &ctx->prof);
        ctx->setup(E, ctx->path == PLDL_PATH_I8 ? PLDL_PATH_I8 : PLDL_PATH_F64, 0.0);
        E.itab = ctx->inv_table(p, st);
        Prof* prof = &ctx->prof;
        const Field Fl = E.F;
        dim3 g(nblk(n), (unsigned)n);
        // L (strict lower part of F) into W, and M^T = (J L J)^T into tmp1 for the L^T solve
        HIPCHK(hipMemsetAsync(ws.info, 0, sizeof(int32_t) * 4, st));
        prof->n_launch++;
        if (dtype == PLDL_U32)
            LAUNCH(PLDL_CLASS_OTHER, k_load_input<uint32_t>, g, dim3(256), 0, st, (const uint32_t*)F, lda, ws.W, E.ld, n, Fl, ws.info + 2);
        else
            LAUNCH(PLDL_CLASS_OTHER, k_load_input<double>, g, dim3(256), 0, st, (const double*)F, lda, ws.W, E.ld, n, Fl, ws.info + 2);
        LAUNCH(PLDL_CLASS_OTHER, k_solve_revlt, g, dim3(256), 0, st, F, lda, dtype, n, ws.tmp1, E.ld);
        if (consistent) {
            LAUNCH(PLDL_CLASS_OTHER, k_fill_i32, dim3(nblk(nrhs)), dim3(256), 0, st, consistent, nrhs, 1);
        }
        // column blocks of at most n right-hand sides (two n x nb buffers in tmp2)
        for (int64_t k0 = 0; k0 < nrhs; k0 += n) {
            const int64_t nb = std::min(n, nrhs - k0);
            double* Y = ws.tmp2;
            double* U = ws.tmp2 + n * nb;
            dim3 gb(nblk(nb), (unsigned)n);
            LAUNCH(PLDL_CLASS_OTHER, k_solve_gather, gb, dim3(256), 0, st, B + k0, ldb, perm, n, nb, Y);
            E.trsm_ll(MatV{Y, nb, 1}, n, nb, MatV{ws.W, E.ld, 1});                  // L^{-1} P^T b
            LAUNCH(PLDL_CLASS_OTHER, k_solve_dblock, gb, dim3(256), 0, st, Y, n, nb, rank, F, lda, dtype, e, E.itab, Fl,
                   consistent ? consistent + k0 : nullptr, U);                        // D^+, reversed
            E.trsm_ll(MatV{U, nb, 1}, n, nb, MatV{ws.tmp1, E.ld, 1});                // (M^T)^{-1} J u = J L^{-T} u
            LAUNCH(PLDL_CLASS_OTHER, k_solve_scatter, gb, dim3(256), 0, st, U, n, nb, perm, B + k0, ldb);   // x = P w
        }
        HIPCHK(hipGetLastError());
        int32_t* h = E.read_info(3);
        if (h[2]) throw Err(PLDL_ERANGE, "an entry of the factorization is not in [0, p)");
    });
}

int pldl_invariants(pldl_ctx* ctx, uint32_t p, int64_t n, const void* F, int64_t lda, int32_t dtype, const void* e,
                    int64_t rank, int64_t* out, void* stream) {
    if (!ctx) return -1;
    if (bad_p(p)) return fail(ctx, PLDL_EUNSUPPORTED_P, "p must satisfy 2 <= p < 2^24");
    if (n < 0 || n > 65535) return fail(ctx, -3, "n out of range [0, 65535]");
    if (n > 0 && !F) return fail(ctx, -4, "F is NULL");
    if (lda < std::max<int64_t>(1, n)) return fail(ctx, -5, "lda < max(1, n)");
    if (dtype != PLDL_U32 && dtype != PLDL_F64) return fail(ctx, -6, "unknown dtype");
    if (n > 0 && !e) return fail(ctx, -7, "e is NULL");
    if (rank < 0 || rank > n) return fail(ctx, -8, "rank outside [0, n]");
    if (!out) return fail(ctx, -9, "out is NULL");
    hipStream_t st = as_stream(stream);
    return guarded(ctx, [&]() {
        ctx->ws.ensure(std::max<int64_t>(n, 1));
        Prof* prof = &ctx->prof;
        int64_t* dout = reinterpret_cast<int64_t*>(ctx->ws.info + 16);   // 8-byte aligned words of info
        LAUNCH(PLDL_CLASS_OTHER, k_invariants, dim3(1), dim3(1024), 0, st, F, lda, dtype, e, n, rank, make_field(p), dout);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(out + 1, dout, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        out[0] = rank;
    });
}

int pldl_trss(pldl_ctx* ctx, uint32_t p, int64_t n, const double* U, int64_t ldu, const double* C, int64_t ldc,
              double* X, int64_t ldx, void* stream) {
    if (!ctx) return -1;
    if (bad_p(p)) return fail(ctx, PLDL_EUNSUPPORTED_P, "p must satisfy 2 <= p < 2^24");
    if (n < 0 || 2 * n > 65535) return fail(ctx, -3, "n out of range");
    if (n > 0 && !U) return fail(ctx, -4, "U is NULL");
    if (ldu < std::max<int64_t>(1, n)) return fail(ctx, -5, "ldu too small");
    if (n > 0 && !C) return fail(ctx, -6, "C is NULL");
    if (ldc < std::max<int64_t>(1, n)) return fail(ctx, -7, "ldc too small");
    if (n > 0 && !X) return fail(ctx, -8, "X is NULL");
    if (ldx < std::max<int64_t>(1, n)) return fail(ctx, -9, "ldx too small");
    hipStream_t st = as_stream(stream);
    int bad_diag = 0;
    int rc = guarded(ctx, [&]() {
        if (n == 0) return;
        int64_t N2 = 2 * n;
        ctx->ws.ensure(N2);
        Engine E(ctx->ws, st, p, N2, 128, &ctx->prof);
        ctx->setup(E, ctx->path == PLDL_PATH_I8 ? PLDL_PATH_I8 : PLDL_PATH_F64, 0.0);
        Prof* prof = &ctx->prof;
        Workspace& ws = ctx->ws;
        HIPCHK(hipMemsetAsync(ws.info, 0, sizeof(int32_t) * 4, st));
        LAUNCH(PLDL_CLASS_OTHER, k_trss_pack, dim3(nblk(n), (unsigned)n), dim3(256), 0, st, U, ldu, C, ldc, ws.W, N2, n, ws.info, p == 2 ? 1 : 0);
        if (p == 2) {
            int32_t* h = E.read_info(1);
            if (h[0]) { bad_diag = 1; return; }
        }
        E.trss(n, n, 0);
        LAUNCH(PLDL_CLASS_OTHER, k_trss_unpack, dim3(nblk(n), (unsigned)n), dim3(256), 0, st, ws.W, N2, n, X, ldx);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
    });
    if (rc == PLDL_OK && bad_diag) return fail(ctx, -6, "characteristic 2: C must have a zero diagonal");
    return rc;
}

int pldl_plduq(pldl_ctx* ctx, uint32_t p, int64_t m, int64_t n, double* Y, int64_t ldy, int32_t* rows, int32_t* cols,
               int64_t* rank, void* stream) {
    if (!ctx) return -1;
    if (bad_p(p)) return fail(ctx, PLDL_EUNSUPPORTED_P, "p must satisfy 2 <= p < 2^24");
    if (m < 0 || m > 65535) return fail(ctx, -3, "m out of range");
    if (n < 0 || n > 65535) return fail(ctx, -4, "n out of range");
    if (m > 0 && n > 0 && !Y) return fail(ctx, -5, "Y is NULL");
    if (ldy < std::max<int64_t>(1, n)) return fail(ctx, -6, "ldy too small");
    if (m > 0 && !rows) return fail(ctx, -7, "rows is NULL");
    if (n > 0 && !cols) return fail(ctx, -8, "cols is NULL");
    if (!rank) return fail(ctx, -9, "rank is NULL");
    hipStream_t st = as_stream(stream);
    return guarded(ctx, [&]() {
        if (m == 0 || n == 0) {
            Prof* prof = &ctx->prof;
            if (m > 0) LAUNCH(PLDL_CLASS_OTHER, k_iota, dim3(nblk(m)), dim3(256), 0, st, rows, m);
            if (n > 0) LAUNCH(PLDL_CLASS_OTHER, k_iota, dim3(nblk(n)), dim3(256), 0, st, cols, n);
            HIPCHK(hipStreamSynchronize(st));
            *rank = 0;
            return;
        }
        ctx->ws.ensure(std::max(m, n));
        Engine E(ctx->ws, st, p, std::max(m, n), 128, &ctx->prof);
        ctx->setup(E, ctx->path == PLDL_PATH_I8 ? PLDL_PATH_I8 : PLDL_PATH_F64, 0.0);
        E.itab = ctx->inv_table(p, st);
        Prof* prof = &ctx->prof;
        Workspace& ws = ctx->ws;
        E.T = ws.tmp2; E.ldT = m; E.TR = n; E.TC = m; E.pR = ws.pidx; E.pC = ws.pidx + m;
        LAUNCH(PLDL_CLASS_OTHER, k_transpose, dim3(nblk(n), (unsigned)m), dim3(256), 0, st, E.T, m, Y, ldy, m, n);
        LAUNCH(PLDL_CLASS_OTHER, k_iota2, dim3(nblk(std::max(m, n))), dim3(256), 0, st, E.pR, m, E.pC, n);
        int64_t r = E.plduq_all(m, n);
        LAUNCH(PLDL_CLASS_OTHER, k_transpose, dim3(nblk(m), (unsigned)n), dim3(256), 0, st, Y, ldy, E.T, m, n, m);
        HIPCHK(hipMemcpyAsync(rows, E.pR, m * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(cols, E.pC, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        *rank = r;
    });
}

int pldl_factor_batched(pldl_ctx* ctx, uint32_t p, int64_t batch, const int64_t* n, void* const* A, const int64_t* lda,
                        int32_t dtype, void* const* e, int32_t* const* perm, int32_t* const* rpm, int64_t* rank,
                        int32_t* status, const pldl_opts* opts, void* stream) {
    if (!ctx) return -1;
    if (bad_p(p)) return fail(ctx, PLDL_EUNSUPPORTED_P, "p must satisfy 2 <= p < 2^24");
    if (batch < 0 || batch > ((int64_t)1 << 30)) return fail(ctx, -3, "batch out of range");
    if (batch > 0 && !n) return fail(ctx, -4, "n is NULL");
    if (batch > 0 && !A) return fail(ctx, -5, "A is NULL");
    if (batch > 0 && !lda) return fail(ctx, -6, "lda is NULL");
    if (dtype != PLDL_U32 && dtype != PLDL_F64) return fail(ctx, -7, "unknown dtype");
    if (batch > 0 && !e) return fail(ctx, -8, "e is NULL");
    if (batch > 0 && !perm) return fail(ctx, -9, "perm is NULL");
    if (batch > 0 && !rpm) return fail(ctx, -10, "rpm is NULL");
    if (batch > 0 && !rank) return fail(ctx, -11, "rank is NULL");
    if (batch > 0 && !status) return fail(ctx, -12, "status is NULL");
    pldl_opts o{PLDL_PATH_AUTO, 0, 0, 1};
    if (opts) o = *opts;
    if (o.standard_form) return fail(ctx, -13, "standard_form is not available in batched mode");
    if (batch == 0) return PLDL_OK;
    hipStream_t st = as_stream(stream);
    return guarded(ctx, [&]() {
        if (!ctx->bws) {
            hipDeviceProp_t prop;
            HIPCHK(hipGetDeviceProperties(&prop, ctx->device));
            const int slots = std::max(1, batched_wg_per_cu() * prop.multiProcessorCount);
            if (hipMalloc((void**)&ctx->bws, (size_t)slots * batched_slot_bytes()) != hipSuccess ||
                hipMalloc((void**)&ctx->bqueue, 256) != hipSuccess) {
                (void)hipGetLastError();
                if (ctx->bws) (void)hipFree(ctx->bws);
                ctx->bws = nullptr;
                throw Err(PLDL_ENOMEM, "batched workspace allocation failed");
            }
            ctx->bslots = slots;
        }
        if (batch > ctx->border_cap) {   // (at least 65536 entries; a larger batch than that allocates)
            const int64_t cap = std::max<int64_t>(batch, (int64_t)1 << 16);
            if (ctx->border) {
                HIPCHK(hipStreamSynchronize(st));
                (void)hipFree(ctx->border);
            }
            ctx->border = nullptr;
            ctx->border_cap = 0;
            if (hipMalloc((void**)&ctx->border, (size_t)cap * sizeof(int32_t)) != hipSuccess) {
                (void)hipGetLastError();
                ctx->border = nullptr;
                throw Err(PLDL_ENOMEM, "batched order allocation failed");
            }
            ctx->border_cap = cap;
        }
        const uint32_t* itab = ctx->inv_table(p, st);
        Field F = make_field(p);
        ctx->prof.begin(st, PLDL_CLASS_BASE_CASE);
        launch_factor_batched(st, F, itab, batch, n, A, lda, dtype, e, perm, rpm, rank, status, o.check_range,
                              ctx->bws, ctx->bslots, ctx->bqueue, ctx->border);
        ctx->prof.end(st);
        HIPCHK(hipGetLastError());
    });
}

int pldl_char2_to_standard(pldl_ctx* ctx, int64_t n, void* A, int64_t lda, int32_t dtype, void* e, int32_t* perm,
                           void* stream) {
    if (!ctx) return -1;
    if (n < 0 || n > 65535) return fail(ctx, -2, "n out of range [0, 65535]");
    if (n > 0 && !A) return fail(ctx, -3, "A is NULL");
    if (lda < std::max<int64_t>(1, n)) return fail(ctx, -4, "lda < max(1, n)");
    if (dtype != PLDL_U32 && dtype != PLDL_F64) return fail(ctx, -5, "unknown dtype");
    if (n > 0 && !e) return fail(ctx, -6, "e is NULL");
    if (n > 0 && !perm) return fail(ctx, -7, "perm is NULL");
    if (n == 0) return PLDL_OK;
    hipStream_t st = as_stream(stream);
    return guarded(ctx, [&]() {
        ctx->ws.ensure(n);
        Workspace& ws = ctx->ws;
        Prof* prof = &ctx->prof;
        Field F = make_field(2);
        const int64_t ld = n;
        HIPCHK(hipMemsetAsync(ws.info, 0, sizeof(int32_t) * 4, st));
        dim3 g(nblk(n), (unsigned)n);
        if (dtype == PLDL_U32) {
            LAUNCH(PLDL_CLASS_OTHER, k_load_input<uint32_t>, g, dim3(256), 0, st, (const uint32_t*)A, lda, ws.W, ld, n, F, ws.info + 2);
            LAUNCH(PLDL_CLASS_OTHER, k_load_factors<uint32_t>, dim3(nblk(n)), dim3(256), 0, st, ws.W, ld, n, (const uint32_t*)e, perm, ws.dd, ws.de, ws.orig);
        } else {
            LAUNCH(PLDL_CLASS_OTHER, k_load_input<double>, g, dim3(256), 0, st, (const double*)A, lda, ws.W, ld, n, F, ws.info + 2);
            LAUNCH(PLDL_CLASS_OTHER, k_load_factors<double>, dim3(nblk(n)), dim3(256), 0, st, ws.W, ld, n, (const double*)e, perm, ws.dd, ws.de, ws.orig);
        }
        LAUNCH(PLDL_CLASS_OTHER, k_char2_std, g, dim3(256), 0, st, ws.W, ld, n, ws.dd, ws.de, ws.orig, ws.tmp1, 0);
        LAUNCH(PLDL_CLASS_OTHER, k_char2_std, g, dim3(256), 0, st, ws.W, ld, n, ws.dd, ws.de, ws.orig, ws.tmp1, 1);
        LAUNCH(PLDL_CLASS_OTHER, k_char2_std, dim3(nblk(n)), dim3(256), 0, st, ws.W, ld, n, ws.dd, ws.de, ws.orig, ws.tmp1, 2);
        if (dtype == PLDL_U32)
            LAUNCH(PLDL_CLASS_OTHER, k_store_output<uint32_t>, g, dim3(256), 0, st, (uint32_t*)A, lda, ws.W, ld, n, ws.dd, ws.de, (uint32_t*)e, ws.orig, perm,
                   nullptr, nullptr);
        else
            LAUNCH(PLDL_CLASS_OTHER, k_store_output<double>, g, dim3(256), 0, st, (double*)A, lda, ws.W, ld, n, ws.dd, ws.de, (double*)e, ws.orig, perm,
                   nullptr, nullptr);
        HIPCHK(hipGetLastError());
        int32_t bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, ws.info + 2, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (bad) throw Err(PLDL_ERANGE, "an entry of the factorization is not in [0, 2)");
    });
}

int pldl_autotune(pldl_ctx* ctx, uint32_t p, const int64_t* n_list, int64_t count, const char* table_path,
                  void* stream) {
    if (!ctx) return -1;
    if (bad_p(p)) return fail(ctx, PLDL_EUNSUPPORTED_P, "p must satisfy 2 <= p < 2^24");
    if (count < 0) return fail(ctx, -4, "count < 0");
    if (count > 0 && !n_list) return fail(ctx, -3, "n_list is NULL");
    for (int64_t k = 0; k < count; ++k)
        if (n_list[k] < 1 || n_list[k] > 16384) return fail(ctx, -3, "every n must lie in [1, 16384]");
    if (count == 0) {   // load a table written by an earlier call
        if (!table_path) return fail(ctx, -5, "nothing to tune and no table to read");
        std::ifstream in(table_path);
        if (!in) return fail(ctx, -5, std::string("cannot read ") + table_path);
        std::string line;
        while (std::getline(in, line)) {
            if (line.empty() || line[0] == '#') continue;
            std::istringstream ls(line);
            uint32_t tp; int64_t tn; int tt;
            if (ls >> tp >> tn >> tt && tt >= 1 && tt <= 128 && tn >= 1) ctx->tune.push_back({tp, tn, tt});
        }
        return PLDL_OK;
    }
    hipStream_t st = as_stream(stream);
    static const int cand[] = {32, 48, 64, 96, 128};
    std::vector<std::string> rows;
    int rc = guarded(ctx, [&]() {
        for (int64_t k = 0; k < count; ++k) {
            const int64_t n = n_list[k];
            const size_t nn = (size_t)n * (size_t)n;
            double *A0 = nullptr, *A1 = nullptr, *Aw = nullptr, *Lb = nullptr, *Bb = nullptr, *ev = nullptr, *sc = nullptr;
            int32_t *perm = nullptr, *rpm = nullptr, *rr = nullptr;
            auto cleanup = [&]() {
                double* ds[] = {A0, A1, Aw, Lb, Bb, ev, sc};
                for (double* q : ds) if (q) (void)hipFree(q);
                int32_t* is[] = {perm, rpm, rr};
                for (int32_t* q : is) if (q) (void)hipFree(q);
            };
            try {
                HIPCHK(hipMalloc((void**)&A0, nn * 8));
                HIPCHK(hipMalloc((void**)&A1, nn * 8));
                HIPCHK(hipMalloc((void**)&Aw, nn * 8));
                HIPCHK(hipMalloc((void**)&Lb, nn * 8));
                HIPCHK(hipMalloc((void**)&Bb, nn * 8));
                HIPCHK(hipMalloc((void**)&ev, n * 8));
                HIPCHK(hipMalloc((void**)&sc, n * 8));
                HIPCHK(hipMalloc((void**)&perm, n * 4));
                HIPCHK(hipMalloc((void**)&rpm, n * 4));
                HIPCHK(hipMalloc((void**)&rr, n * 4));
                Field F = make_field(p);
                dim3 g2(nblk(n), (unsigned)n);
                const uint64_t seed = 0x243F6A8885A308D3ull ^ (uint64_t)n;
                // class 1: uniform symmetric (generic rank profile)
                hipLaunchKernelGGL(k_fill_uniform_sym, g2, dim3(256), 0, st, A0, n, p, seed);
                // class 2: A = L R L^T, R a random symmetric rook placement of rank about n/2
                std::mt19937_64 rng(seed);
                std::vector<int32_t> hr(n, -1);
                std::vector<double> hs(n, 0.0);
                std::vector<int64_t> idx(n);
                for (int64_t i = 0; i < n; ++i) idx[i] = i;
                std::shuffle(idx.begin(), idx.end(), rng);
                const int64_t f = n / 4, c = n / 8;
                for (int64_t i = 0; i < f; ++i) { hr[idx[i]] = (int32_t)idx[i]; hs[idx[i]] = (double)(1 + rng() % (p - 1)); }
                for (int64_t i = 0; i < c; ++i) {
                    const int64_t a = idx[f + 2 * i], b = idx[f + 2 * i + 1];
                    const double s = (double)(1 + rng() % (p - 1));
                    hr[a] = (int32_t)b; hr[b] = (int32_t)a; hs[a] = s; hs[b] = s;
                }
                HIPCHK(hipMemcpyAsync(rr, hr.data(), n * 4, hipMemcpyHostToDevice, st));
                HIPCHK(hipMemcpyAsync(sc, hs.data(), n * 8, hipMemcpyHostToDevice, st));
                hipLaunchKernelGGL(k_fill_unit_lower, g2, dim3(256), 0, st, Lb, n, p, seed + 1);
                hipLaunchKernelGGL(k_fill_neg_rlt, g2, dim3(256), 0, st, Bb, Lb, n, rr, sc, F);
                HIPCHK(hipMemsetAsync(A1, 0, nn * 8, st));
                GemmSeg sg{MatV{Lb, n, 1}, MatV{Bb, n, 1}, n};
                launch_gemm(st, F, n, n, A1, n, &sg, 1, true, false);
                HIPCHK(hipGetLastError());
                HIPCHK(hipStreamSynchronize(st));
                double best = 1e300, bu = 0.0, br = 0.0;
                int bt = 128;
                for (int t : cand) {
                    if (t > n && t != cand[0]) continue;
                    double ms[2];
                    for (int cls = 0; cls < 2; ++cls) {
                        ms[cls] = 1e300;
                        for (int rep = 0; rep < 2; ++rep) {
                            HIPCHK(hipMemcpyAsync(Aw, cls ? A1 : A0, nn * 8, hipMemcpyDeviceToDevice, st));
                            HIPCHK(hipStreamSynchronize(st));
                            pldl_opts o{PLDL_PATH_AUTO, t, 0, 0};
                            int64_t rk = 0;
                            const auto t0 = std::chrono::steady_clock::now();
                            const int frc = pldl_factor(ctx, p, n, Aw, n, PLDL_F64, ev, perm, rpm, &rk, &o, nullptr, stream);
                            const double el = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                            if (frc != PLDL_OK) throw Err(frc, "factorization during tuning failed: " + ctx->err);
                            ms[cls] = std::min(ms[cls], el);
                        }
                    }
                    if (ms[0] + ms[1] < best) { best = ms[0] + ms[1]; bt = t; bu = ms[0]; br = ms[1]; }
                }
                ctx->tune.erase(std::remove_if(ctx->tune.begin(), ctx->tune.end(),
                                               [&](const pldl_ctx::Tune& e) { return e.p == p && e.n == n; }),
                                ctx->tune.end());
                ctx->tune.push_back({p, n, bt});
                char buf[160];
                std::snprintf(buf, sizeof buf, "%u %lld %d %.3f %.3f", p, (long long)n, bt, bu, br);
                rows.push_back(buf);
            } catch (...) {
                (void)hipStreamSynchronize(st);
                cleanup();
                throw;
            }
            HIPCHK(hipStreamSynchronize(st));
            cleanup();
        }
    });
    if (rc == PLDL_OK && table_path) {
        std::ofstream out(table_path);
        if (!out) return fail(ctx, -5, std::string("cannot write ") + table_path);
        out << "# pldl_autotune: p n threshold ms_uniform ms_rank_profile\n";
        for (const std::string& r : rows) out << r << "\n";
    }
    return rc;
}

int pldl_set_winograd(pldl_ctx* ctx, int64_t min_order) {
    if (!ctx) return -1;
    if (min_order != 0 && (min_order < 256 || min_order > 65535))
        return fail(ctx, -2, "min_order must be 0 (off) or in [256, 65535]");
    ctx->wino_min = min_order;
    return PLDL_OK;
}

int pldl_set_path(pldl_ctx* ctx, int32_t path) {
    if (!ctx) return -1;
    if (path != PLDL_PATH_AUTO && path != PLDL_PATH_F64 && path != PLDL_PATH_I8)
        return fail(ctx, -2, "path must be PLDL_PATH_AUTO, PLDL_PATH_F64 or PLDL_PATH_I8");
    ctx->path = path;
    return PLDL_OK;
}

int pldl_profile(pldl_ctx* ctx, int32_t mode, pldl_stats* out) {
    if (!ctx) return -1;
    if (mode < 0 || mode > 3) return fail(ctx, -2, "mode must be 0, 1, 2 or 3");
    return guarded(ctx, [&]() {
        ctx->prof.harvest();
        if (mode == 1 || mode == 3) {
            ctx->prof.tot = pldl_stats{};
            ctx->prof.on = true;
            ctx->prof.light = (mode == 3);
            ctx->prof.mask = (mode == 1) ? 0x1FFu : ((1u << PLDL_CLASS_GEMM) | (1u << PLDL_CLASS_GEMM_I8));
        }
        if (mode == 0) ctx->prof.on = false;
        if (out) *out = ctx->prof.tot;
    });
}

}  // extern "C"
