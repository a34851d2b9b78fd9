// k_noalloc.hip -- the fixed device work area of fmm_evaluate_noalloc.
//
// Callers that cannot allocate device memory (code under stream capture,
// serving loops, harnesses that forbid allocation) evaluate on a work area
// the library holds from the moment its code object is loaded on a device
// until the process ends: a file-scope __device__ array.  In host code the
// array's name is only a host-side stand-in, never a device address; the
// device address of each device's copy is looked up once per device with
// hipGetSymbolAddress (at context creation, with that device current) and
// only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fmm_internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[fmm::kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

}  // namespace

namespace fmm {

hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[device]) return hipSuccess;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[device] = ptr;
    return hipSuccess;
}

void* noalloc_area(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_scratch[device];
}

}  // namespace fmm
