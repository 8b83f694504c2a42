// Fixed device workspace of the allocation-free query entry point
// (gr_sssp_noalloc).  The array is part of the code object: every GPU that
// loads the library holds its own copy, at its own address, until the process
// ends.  Host code never passes the array's name to a kernel (in host code it
// is a host-side stand-in); it passes the device address that
// hipGetSymbolAddress returns for the current device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gr_noalloc.h"

namespace gr {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void **ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace gr
