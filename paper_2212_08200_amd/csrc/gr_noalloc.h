// Allocation-free entry point (gr_noalloc.hip): a fixed per-device array of
// kNoAllocScratchBytes holds the frontier workspace of gr_sssp_noalloc.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace gr {

constexpr size_t kNoAllocScratchBytes = size_t(96) << 20;
static_assert(kNoAllocScratchBytes == (96u << 20), "matches GR_NOALLOC_SCRATCH_BYTES in gr.h");

// Device address of the array on the current device, looked up once per
// device with hipGetSymbolAddress.
hipError_t noalloc_scratch(void **ptr);

}  // namespace gr
