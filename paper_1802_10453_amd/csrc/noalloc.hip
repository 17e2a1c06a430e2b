// noalloc.hip -- SYRDK / SYRD2K (Section 3) with no device allocation in the
// call: the A D (and B D) operands go to a file-scope device array instead of
// the context's workspace.
//
// The array is one per GPU the library runs on (each device holds its own
// copy, at its own address, until the process ends).  pldl_create resolves its
// address once per device with that device current (noalloc_init); host code
// only ever passes that resolved address, never the array's name.  Every call
// on one GPU shares the array: calls that overlap on one GPU (two streams,
// two threads) race.  Nothing in it needs clearing: a call writes the part it
// reads first.
#include <mutex>

#include "../../include/pldl.h"
#include "common.h"
#include "kernels.h"

namespace pldl {

static __device__ __align__(256) double scratch[PLDL_NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
double* g_scratch[kMaxDevices] = {};   // the array's address on each device
std::mutex g_mu;
}  // namespace

// Resolves the array's address on `device` (made current by the caller).
// Returns false when the address cannot be taken.
bool noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return true;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return false;
    }
    g_scratch[device] = static_cast<double*>(ptr);
    return true;
}

double* noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_scratch[device];
}

}  // namespace pldl
