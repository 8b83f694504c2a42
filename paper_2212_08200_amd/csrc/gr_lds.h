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

// One workgroup per query, up to kLdsMaxBatch queries in one launch.
constexpr int kLdsMaxBatch = 64;

// A query: its graph's CSR in device memory (ro[n + 1], adj[m] as (head,
// weight bits)), its source and its output row dist[n] (device memory).
struct LdsJob {
    const int32_t *ro;
    const uint2 *adj;
    uint32_t *dist;
    int32_t n, m, src;
};

// wt: 0 uint32 weights (every weight below 2^16), 2 unit steps, for every
// job.  jobs: host array of k jobs, 1 <= k <= kLdsMaxBatch, each graph
// fitting (lds_fits); workgroup b copies job b's graph into its LDS, writes
// its dist row and stat[4 b .. 4 b + 3] (device memory or pinned host
// memory: written with system-scope stores).
hipError_t launch_lds(const LdsJob *jobs, int32_t k, int wt, int64_t max_rounds, unsigned long long *stat,
                      hipStream_t st);

}  // namespace gr
