// Internal declarations shared by the host runtime (gr_api.cpp) and the HIP
// kernels (gr_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gr {

constexpr uint32_t kInfU32 = 0xFFFFFFFFu;
constexpr uint32_t kInfF32 = 0x7F7FFFFFu;  // FLT_MAX bits

// Frontier bitmaps are grouped in blocks of 4096 vertices (64 words of 64
// bits); a summary bitmap holds one bit per group so that the filter skips
// empty groups without reading them.
constexpr int kGroupShift = 12;
constexpr int kGroupVerts = 1 << kGroupShift;
constexpr int kGroupWords = kGroupVerts / 64;

inline int64_t groups_for(int64_t n) { return (n + kGroupVerts - 1) / kGroupVerts; }

// Device view of a graph: CSR for push, CSC (or the same CSR when the graph
// is symmetric) for pull.  Arcs are interleaved (destination, weight bits) so
// that one 8-byte load fetches both.
struct DevGraph {
    int32_t n;
    int32_t m;
    int32_t wt;  // 0 = uint32, 1 = binary32
    const int32_t *ro;
    const uint2 *adj;
    const int32_t *ro_in;
    const uint2 *adj_in;
};

// Per-query frontier workspace (device memory).
//   bits[p], sum[p]   frontier bitmap and its group summary, parity p
//   q[p], s[p]        sparse frontier (vertex ids) and the exclusive prefix
//                     sum of their out-degrees, parity p
//   ctl[0..1]         packed counters per parity: low 32 bits = frontier
//                     size F, high 32 bits = sum of out-degrees E
//   ctl[2]            filter blocks-done counter
//   ctl[3..]          device-loop state (barrier, iteration, stats)
struct Frontier {
    uint64_t *bits[2];
    uint64_t *sum[2];
    int32_t *q[2];
    int32_t *s[2];
    unsigned long long *ctl;
    int64_t nwords;   // words per bitmap (multiple of kGroupWords)
    int64_t nsumw;    // words per summary bitmap
    int32_t ngroups;
};

constexpr int kCtlWords = 64;

// Device-driven loop state, at ctl + 8.
struct LoopState {
    unsigned long long bar_count;   // grid barrier arrivals
    unsigned long long bar_gen;     // grid barrier generation
    unsigned long long iter;        // iterations done
    unsigned long long status;      // 0 running, 1 done, 2 iteration cap
    unsigned long long edges_pushed;
    unsigned long long arcs_pulled;
    unsigned long long frontier_sum;
    unsigned long long frontier_max;
    unsigned long long pull_iters;
};

size_t frontier_bytes(int64_t n);
void frontier_carve(Frontier &f, void *base, int64_t n);

// ---- launch wrappers (gr_kernels.hip) -------------------------------------
hipError_t launch_init(const DevGraph &g, uint32_t *dist, int32_t src, const Frontier &f, hipStream_t st);
hipError_t launch_push(const DevGraph &g, uint32_t *dist, const Frontier &f, int parity, int32_t F, int32_t E,
                       int num_cu, hipStream_t st);
hipError_t launch_pull(const DevGraph &g, uint32_t *dist, const Frontier &f, int parity, hipStream_t st);
hipError_t launch_filter(const DevGraph &g, const Frontier &f, int parity, hipStream_t st);

// Device-driven loop (cooperative launch).
struct PersistentCfg {
    int32_t max_iters;
    int32_t alpha_x16;
    int32_t direction;  // gr_direction
    int32_t grid;       // blocks (co-resident)
};
hipError_t launch_persistent(const DevGraph &g, uint32_t *dist, int32_t src, const Frontier &f,
                             const PersistentCfg &cfg, hipStream_t st);
int persistent_max_blocks_per_cu();

// Graph build helpers.
hipError_t launch_pack_arcs(const int32_t *col, const uint32_t *w, int32_t m, uint2 *adj, hipStream_t st);
hipError_t launch_validate(int32_t n, int32_t m, const int32_t *ro, const int32_t *col, const uint32_t *w, int wt,
                           unsigned int *err, hipStream_t st);
hipError_t launch_csc_build(int32_t n, int32_t m, const int32_t *ro, const uint2 *adj, int32_t *ro_in,
                            uint2 *adj_in, int32_t *scratch_cnt, hipStream_t st);
hipError_t launch_symmetry_check(int32_t n, const int32_t *ro, const uint2 *adj, unsigned int *not_sym,
                                 hipStream_t st);

// Batched multi-source.
struct BatchWs {
    uint32_t *dist;     // n x 64 vertex-major (lane = source slot)
    uint64_t *mask[2];  // per-vertex active-source masks, parity
    uint64_t *bits[2];  // any-source frontier bitmap
    uint64_t *sum[2];
    int32_t *q[2];
    int32_t *s[2];
    unsigned long long *ctl;
    int64_t nwords, nsumw;
    int32_t ngroups;
};
size_t batch_bytes(int64_t n);
void batch_carve(BatchWs &b, void *base, int64_t n);
hipError_t launch_batch_init(const DevGraph &g, const BatchWs &b, const int32_t *srcs_dev, int32_t k,
                             hipStream_t st);
hipError_t launch_batch_push(const DevGraph &g, const BatchWs &b, int parity, int32_t F, int32_t E, int num_cu,
                             hipStream_t st);
hipError_t launch_batch_filter(const DevGraph &g, const BatchWs &b, int parity, hipStream_t st);
hipError_t launch_batch_output(const DevGraph &g, const BatchWs &b, int32_t k, uint32_t *dist_out, hipStream_t st);

}  // namespace gr
