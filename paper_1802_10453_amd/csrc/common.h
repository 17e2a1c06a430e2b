// common.h -- device arithmetic over F_p held in FP64, matrix views, kernel
// launch declarations shared by the HIP sources of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pldl {

// ---------------------------------------------------------------------------
// Field parameters.  Residues are integers held exactly in doubles; every
// kernel keeps W canonical ([0, p)).  Products of two centered residues are
// below p^2/4 (< 2^44 for p < 2^23, < 2^46 for p < 2^24), so a double
// accumulates `kred` of them (plus one carried residue) before the 2^53
// exactness limit: 496 at p = 8388593, 128 at p = 16777213.
struct Field {
    double p;       // modulus
    double pinv;    // 1/p rounded
    double half;    // floor(p/2): centered representative threshold
    double inv2;    // (p+1)/2 = 1/2 mod p (unused for p = 2)
    int32_t ip;     // p as an integer
    int32_t kred;   // products accumulated between two reductions (multiple of 16)
};

Field make_field(uint32_t p);

// v mod p in [0, p) for any integer-valued |v| < 2^53.  q may be off by one
// from floor(v/p) because of the rounded reciprocal; the two corrections bring
// the exact remainder (computed by one fma) back into range.
__device__ __forceinline__ double fred(double v, const Field& F) {
    double q = floor(v * F.pinv);
    double r = fma(-q, F.p, v);
    r = (r < 0.0) ? r + F.p : r;
    r = (r >= F.p) ? r - F.p : r;
    return r;
}
// Centered reduction in three dependent operations: q = rint(v/p) is the
// nearest integer quotient up to one unit when v/p lies within rounding error
// of a half-integer, where both choices leave |r| ~ p/2; hence |r| <= p/2 + 2
// for every integer-valued |v| < 2^53.  Used on the latency-bound paths.
__device__ __forceinline__ double fredc(double v, const Field& F) {
    return fma(-rint(v * F.pinv), F.p, v);
}
// centered representative of a canonical residue: (-p/2, p/2]
__device__ __forceinline__ double fcen(double v, const Field& F) { return v > F.half ? v - F.p : v; }
// canonical representative of a residue in (-p, p)
__device__ __forceinline__ double fcan(double v, const Field& F) { return v < 0.0 ? v + F.p : v; }
__device__ __forceinline__ double fmulm(double a, double b, const Field& F) { return fred(a * b, F); }

// Inverse by the extended Euclidean algorithm on 32-bit integers.
__device__ __forceinline__ double finv(double a, const Field& F) {
    int r0 = F.ip, r1 = (int)a, s0 = 0, s1 = 1;
    while (r1 != 0) {
        int q = r0 / r1, t;
        t = r0 - q * r1; r0 = r1; r1 = t;
        t = s0 - q * s1; s0 = s1; s1 = t;
    }
    if (s0 < 0) s0 += F.ip;
    return (double)s0;
}

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Strided matrix view: element (i, j) at p[i*rs + j*cs].  One of the strides
// is 1 for every view the library forms (row-major: cs = 1; column-major: rs = 1).
struct MatV {
    double* p;
    int64_t rs, cs;
};

// ---------------------------------------------------------------------------
// In-kernel launch timing: the earliest workgroup start and the latest
// workgroup end of one launch on the device's constant-rate wall clock, folded
// into a slot with atomicMin / atomicMax (null pointers: off).  It adds no
// launch and no queue marker, so a timed run is not perturbed by it.
struct Stamp {
    unsigned long long* t0 = nullptr;
    unsigned long long* t1 = nullptr;
};
__device__ __forceinline__ void stamp_begin(const Stamp& s) {
    if (s.t0 && threadIdx.x == 0) atomicMin(s.t0, (unsigned long long)wall_clock64());
}
// every thread of the workgroup calls it (one barrier when timing is on)
__device__ __forceinline__ void stamp_end(const Stamp& s) {
    if (s.t1) {
        __syncthreads();
        if (threadIdx.x == 0) atomicMax(s.t1, (unsigned long long)wall_clock64());
    }
}

// ---------------------------------------------------------------------------
// Launchers (host functions; each validates nothing -- callers check bounds).
struct GemmSeg {
    MatV A, B;     // A: m x k, B: k x n
    int64_t k;
};
// C (row-major, ldc) <- C - sum_seg A_seg B_seg   (mod p)
//   lower_c: only entries j <= i of C (m == n);  b_upper: B[t][j] taken as 0 for t > j (segment 0)
void launch_gemm(hipStream_t s, const Field& F, int64_t m, int64_t n, double* C, int64_t ldc,
                 const GemmSeg* segs, int nseg, bool lower_c, bool b_upper, Stamp stamp = Stamp{});

// The same product on the INT8 matrix cores with residues split into signed
// bytes (gemm_i8.hip), in two launches: i8_prepare writes the operands' limb
// planes into ws (ws_bytes) and fills `out`; it returns false, having queued
// nothing, when the workspace is too small or a K exceeds the INT32
// accumulation bound (the caller then uses launch_gemm).  i8_run is the product.
struct I8Product {
    int64_t m = 0, n = 0;
    int L = 0;
    const int8_t* A[2] = {nullptr, nullptr};
    const int8_t* B[2] = {nullptr, nullptr};
    int64_t Kp[2] = {0, 0};
};
int i8_limbs(uint32_t p);
size_t i8_workspace_bytes(uint32_t p, int64_t m, int64_t n, const GemmSeg* segs, int nseg);
bool i8_prepare(hipStream_t s, const Field& F, int64_t m, int64_t n, const GemmSeg* segs, int nseg, bool b_upper,
                int8_t* ws, size_t ws_bytes, I8Product* out);
void i8_run(hipStream_t s, const Field& F, const I8Product& pr, double* C, int64_t ldc, bool lower_c,
            Stamp stamp = Stamp{});
// Batched factorizations (batched.hip): one persistent launch, one workgroup
// per matrix at a time (slots workgroups, each with a private slot of
// batched_slot_bytes() in ws); queue is a device counter the launch resets.
int batched_nb_max();
int batched_wg_per_cu();
size_t batched_slot_bytes();
void launch_factor_batched(hipStream_t s, const Field& F, const uint32_t* itab, int64_t batch, const int64_t* n,
                           void* const* A, const int64_t* lda, int32_t dtype, void* const* e, int32_t* const* perm,
                           int32_t* const* rpm, int64_t* rank, int32_t* status, int check_range, void* ws,
                           int slots, int32_t* queue,
                           int32_t* order);

// Longest K (summed over the segments of one product) the INT8 split accumulates
// exactly in INT32: a shift class gains at most 2^15 per k, 65535 * 2^15 < 2^31.
constexpr int64_t I8_MAX_KTOT = 65535;
// The allocation-free entry point's device array (noalloc.hip): resolved per
// device by noalloc_init (the device current), read back by noalloc_scratch.
bool noalloc_init(int device);
double* noalloc_scratch(int device);
// Products below this many flops stay on FP64 inside a factorization.
constexpr double I8_MIN_FLOPS = 134217728.0;   // 2^27: below it the limb split costs more than it saves

}  // namespace pldl
