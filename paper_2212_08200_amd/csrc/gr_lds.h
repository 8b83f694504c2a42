// Single-workgroup loop for small graphs: one workgroup holds the whole query
// in LDS (declarations; see gr_lds.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gr {

// LDS budget of the loop (words of 4 bytes) and its layout for n vertices and
// m arcs: distances (n), row offsets (n + 1), packed arcs (m: head << 16 |
// weight, or the head alone for unit steps), next-list membership bits
// (ceil(n / 32)), two frontier lists of 16-bit vertex ids (n each).
constexpr int kLdsWords = 39936;  // 156 KiB of the 160 KiB of a compute unit
constexpr int32_t kLdsMaxN = 65536;
int64_t lds_words(int32_t n, int32_t m);
inline bool lds_fits(int32_t n, int32_t m) { return n >= 1 && n <= kLdsMaxN && lds_words(n, m) <= kLdsWords; }

// Statistics words the kernel writes to stat[0..3]: rounds, status (1 done,
// 2 round cap reached), arcs relaxed, vertex expansions.
constexpr int kLdsStatWords = 4;

// wt: 0 uint32 weights (every weight below 2^16), 2 unit steps.  The graph's
// CSR (ro, adj as (head, weight bits)) stays in device memory; it is copied
// into LDS by the kernel.  Writes dist_out[0..n) and stat (device memory or
// pinned host memory: written with system-scope stores).
hipError_t launch_lds(int32_t n, int32_t m, int wt, const int32_t *ro, const uint2 *adj, int32_t src,
                      uint32_t *dist_out, int64_t max_rounds, unsigned long long *stat, hipStream_t st);

}  // namespace gr
