// qq_static.hip -- the fixed device array behind qq_evaluate_static (the entry point for callers
// that cannot allocate device memory).
//
// `scratch` is a file-scope device array of QQ_STATIC_SCRATCH_BYTES; every GPU the library runs on
// holds its own copy at its own address until the process ends.  In host code the name `scratch` is
// only a host-side stand-in for the symbol, so its device address is taken here, once per device
// with that device current, through hipGetSymbolAddress, and only that address is ever handed to
// kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "qq_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[QQ_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

}  // namespace

namespace qq {

hipError_t static_scratch(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices || !ptr) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!a) return hipErrorInvalidSymbol;
        g_addr[device] = a;
    }
    *ptr = g_addr[device];
    return hipSuccess;
}

}  // namespace qq
