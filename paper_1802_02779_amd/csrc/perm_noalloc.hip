// Allocation-free complex solve: the layer tables and the packed matrix live
// in one file-scope device array, `scratch`, instead of a caller-supplied
// workspace (part of the device translation unit perm_device.hip).
//
// Host code never passes the array's name to a kernel or a copy: its
// address on the current device comes from hipGetSymbolAddress, taken once
// per device and kept (each device holds its own copy of the array).
#include <mutex>

#include "perm.h"

namespace permgpu {

static_assert(PERM_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");

static __device__ __align__(256) unsigned char scratch[PERM_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64];  // device address of `scratch`, per device

hipError_t noalloc_scratch(void **ptr, size_t *bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    *bytes = PERM_NOALLOC_SCRATCH_BYTES;
    return hipSuccess;
}

}  // namespace permgpu
