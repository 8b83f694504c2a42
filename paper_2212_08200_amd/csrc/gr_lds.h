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
// ell (optional): the same arcs padded to 2^ell_lg slots per vertex, packed
// head << 16 | weight, empty slots kLdsNoArc (see lds_ell_fits); when every
// job of a launch has one with the same ell_lg, the launch uses it.
struct LdsJob {
    const int32_t *ro;
    const uint2 *adj;
    const uint32_t *ell;
    uint32_t *dist;
    int32_t n, m, src, ell_lg;
};

// Padded layout in LDS: distances (n), the padded arcs (n << lg), two lists
// (n 16-bit ids each).  At most 16 slots per vertex.
constexpr uint32_t kLdsNoArc = 0xFFFFFFFFu;
constexpr int kLdsEllMaxLg = 4;
inline int64_t lds_ell_words(int32_t n, int lg) { return (int64_t)n + ((int64_t)n << lg) + (n + 1) / 2 * 2; }
inline bool lds_ell_fits(int32_t n, int lg) {
    return n >= 1 && n <= kLdsMaxN && lg >= 0 && lg <= kLdsEllMaxLg && lds_ell_words(n, lg) <= kLdsWords;
}

// wt: 0 uint32 weights (every weight below 2^16), 2 unit steps, for every
// job.  jobs: host array of k jobs, 1 <= k <= kLdsMaxBatch, each graph
// fitting the layout the launch takes (the padded one when every job has it
// with the same ell_lg, else lds_fits); workgroup b copies job b's graph into its LDS, writes
// its dist row and stat[4 b .. 4 b + 3] (device memory or pinned host
// memory: written with system-scope stores).
hipError_t launch_lds(const LdsJob *jobs, int32_t k, int wt, int64_t max_rounds, unsigned long long *stat,
                      hipStream_t st);

}  // namespace gr
