// Single-workgroup loop for small graphs: one workgroup holds the whole query
// in LDS (declarations; see gr_lds.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gr {

// LDS budget of the loop (words of 4 bytes) and its layout for n vertices and
// m arcs: distances with a free bit each (n), row offsets (n + 1), packed
// arcs (m: head << 16 | weight, or the head alone for unit steps), two
// frontier lists of 16-bit vertex ids (n each).
constexpr int kLdsWords = 39936;  // 156 KiB of the 160 KiB of a compute unit
constexpr int32_t kLdsMaxN = 65536;
int64_t lds_words(int32_t n, int32_t m);
// Distances are kept in 31 bits: a graph that fits has n < kLdsWords / 3
// vertices, so every path, and every offer one arc beyond one, stays below
// 2^31 - 1 with 16-bit weights.
static_assert((int64_t)(kLdsWords / 3) * 65535 < 0x7FFFFFFF, "31-bit distances");
inline bool lds_fits(int32_t n, int32_t m) { return n >= 1 && n <= kLdsMaxN && lds_words(n, m) <= kLdsWords; }

// Statistics words the kernel writes to stat[0..3]: rounds, status (1 done,
// 2 round cap reached), arcs relaxed, vertex expansions.
constexpr int kLdsStatWords = 4;

// One workgroup per source, up to kLdsMaxBatch sources in one launch.
constexpr int kLdsMaxBatch = 64;

// wt: 0 uint32 weights (every weight below 2^16), 2 unit steps.  The graph's
// CSR (ro, adj as (head, weight bits)) stays in device memory; it is copied
// into LDS by each workgroup.  srcs: host array of k sources, 1 <= k <=
// kLdsMaxBatch; workgroup b writes row b of dist_out (k x n, row-major) and
// stat[4 b .. 4 b + 3] (device memory or pinned host memory: written with
// system-scope stores).
hipError_t launch_lds(int32_t n, int32_t m, int wt, const int32_t *ro, const uint2 *adj, const int32_t *srcs,
                      int32_t k, uint32_t *dist_out, int64_t max_rounds, unsigned long long *stat, hipStream_t st);

}  // namespace gr
