// Internal declarations shared by the host runtime (gr_api.cpp) and the HIP
// kernels (gr_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gr {

constexpr uint32_t kInfU32 = 0xFFFFFFFFu;
constexpr uint32_t kInfF32 = 0x7F7FFFFFu;  // FLT_MAX bits

// The filter works on groups of 4096 vertices.
constexpr int kGroupShift = 12;
constexpr int kGroupVerts = 1 << kGroupShift;

// Push layouts: the arcs are split by destination into kMaxParts contiguous
// vertex ranges ("partitions"), stored partition-major.  Push blocks are
// assigned to partitions round-robin, matching the round-robin placement of
// workgroups on the 8 XCDs, so each XCD's L2 only holds its slice of the
// distance array.  A one-partition layout is the plain CSR.
constexpr int kMaxParts = 8;

inline int64_t groups_for(int64_t n) { return (n + kGroupVerts - 1) / kGroupVerts; }

// Device view of a graph.
//   ro/adj        CSR, arcs interleaved as (destination, weight bits)
//   ro_in/adj_in  transposed copy for pull (== ro/adj when symmetric)
//   pro/padj      push layout with np partitions: arcs of u into partition k
//                 are padj[pro[u*np+k] .. pro[(u+1)*np+k]) (arcs stored
//                 partition-major, offsets vertex-major); for np == 1 these
//                 alias ro/adj
struct DevGraph {
    int32_t n;
    int32_t m;
    int32_t wt;  // 0 = uint32, 1 = binary32
    const int32_t *ro;
    const uint2 *adj;
    const int32_t *ro_in;
    const uint2 *adj_in;
    int32_t np;     // 1 or kMaxParts
    int32_t psize;  // vertices per partition
    const int32_t *pro;
    const uint2 *padj;
    int32_t cap[kMaxParts];  // max frontier entries per partition
    // Members of partition k: the vertices u with arcs into it, in increasing
    // order, as mem_u[i] = u and mem_sd[i] = (first arc, arc count), for
    // i in [mem_off[k], mem_off[k+1]).  Used by the streaming filter.
    const int32_t *mem_u;
    const uint2 *mem_sd;
    int64_t mem_off[kMaxParts + 1];
};

// Per-query frontier workspace (device memory).
//   flags[2]         frontier as one byte per vertex (current / next, by
//                    iteration parity), padded to whole groups
//   far[2]           near-far split: one byte per vertex that was improved
//                    but held back because its distance is not below the
//                    current threshold (read / written by iteration parity)
//   qse[k], qs[k]    sparse frontier of partition k: entries (first arc, u)
//                    and the exclusive prefix sum of their arc counts
//   cand[2]          queued loop: candidate lists (improved vertices, with
//                    repeats) that let small rounds skip the flag scan
//   ctl              3 slots of kSlotWords counters, rotated over three
//                    iterations so that a slot is cleared one iteration after
//                    its last use: word k * kCtrStride (k < 8) packs F_k (low
//                    32 bits) and E_k (high 32 bits) of partition k, word
//                    kFarCountWord counts held-back vertices and word
//                    kFarMaxInvWord holds the max of ~dist over them;
//                    then the device-driven loop state
struct Frontier {
    uint8_t *flags[2];
    uint32_t *bits;  // the frontier as one bit per vertex (word w: vertices 32w .. 32w + 31), written by
                     // the filter for the next round and by init; read by pull

    uint8_t *far[2];
    int32_t *cand[2];  // candidate lists of the small rounds (queued loop)
    unsigned long long *ccount;  // their counters: 3 rounds x kCandRegions
    unsigned long long *rstat;   // small-round statistics (kStatWords)
    uint32_t *bound;             // per-vertex upper bound on dist that filters relaxations (see relax_bound)
    int32_t cand_cap;
    uint2 *qse[kMaxParts];
    int32_t *qs[kMaxParts];
    unsigned long long *ctl;
    int64_t nflag;  // bytes per flag array (multiple of kGroupVerts)
    int32_t ngroups;
    int32_t np;
};

constexpr int kCandRegions = 64;  // regions of a small-round candidate list
constexpr int kCtlSlots = 3;
// Counters that many blocks update at once each sit on a 256-byte line of
// their own: memory-side atomics to one line are serialised.
constexpr int kCtrStride = 32;                    // words from one counter to the next
constexpr int kFarCountWord = 8 * kCtrStride;     // within a slot
constexpr int kFarMaxInvWord = 9 * kCtrStride;    // within a slot: max of ~dist[u] over held-back u
constexpr int kSlotWords = 10 * kCtrStride;       // partition k's counter at word k * kCtrStride
constexpr int kLoopStateWord = 3 * kSlotWords;    // LoopState after the 3 slots
constexpr int kCtlWords = kLoopStateWord + 32;
// Untuned default: streaming filter when |frontier| >= n / 8 (measured against
// 64: grid 2048^2 131 -> 115 ms, road-like 7.7 -> 7.2 ms, R-MAT 20 2.16 -> 2.11
// ms, R-MAT 22 within 1%).  Batched queries keep n / 64.
constexpr int32_t kDenseRatio = 8;
constexpr int32_t kBatchDenseRatio = 64;

// Device-driven loop state.
struct LoopState {
    unsigned long long bar_count;  // grid barrier arrivals
    unsigned long long bar_gen;    // grid barrier generation
    unsigned long long iter;       // iterations done
    unsigned long long status;     // 0 running, 1 done, 2 iteration cap, 3 barrier wait timed out
    unsigned long long edges_pushed;
    unsigned long long arcs_pulled;
    unsigned long long frontier_sum;
    unsigned long long frontier_max;
    unsigned long long pull_iters;
    unsigned long long push_frontier_sum;
    unsigned long long threshold;  // near-far: distances below it are pushed now
    unsigned long long st_round[2];  // queued loop state machine, by launch parity: round ...
    unsigned long long st_phase[2];  // ... and phase the launch runs
    unsigned long long small_rounds;
    unsigned long long last_pull[2];  // queued loop: whether the advance of round r pulled, at r & 1
                                      // (direction hysteresis; read one round later)
};
static_assert(kLoopStateWord + sizeof(LoopState) / 8 <= kCtlWords, "loop state fits the control block");
// Small-round statistics by candidate region: expanded vertices with arcs in
// rounds r mod 3 (3 x kCandRegions), then running totals of expanded vertices
// and of their arcs (kCandRegions each).
constexpr int kStatFrontier = 3 * kCandRegions;
constexpr int kStatEdges = 4 * kCandRegions;
constexpr int kStatWords = 5 * kCandRegions;
static_assert(kCtlSlots * kSlotWords <= kLoopStateWord, "counter slots fit below the loop state");

// Optional parts of a query's workspace: the held-back flags of the near-far
// split and the bound array of the relaxation filter (absent parts take no
// space and their pointers are NULL).
struct WsParts {
    bool far;
    bool bound;
};
size_t frontier_bytes(const DevGraph &g, WsParts w);
void frontier_carve(Frontier &f, void *base, const DevGraph &g, WsParts w);

// Totals of one frontier as read back from the counters.
struct FrontierCounts {
    int32_t F[kMaxParts];
    int32_t E[kMaxParts];
    int64_t far_count;  // held-back vertices (near-far split)
    uint32_t far_min;   // their smallest distance (bits)
    int64_t Fsum() const;
    int64_t Esum() const;
};
void read_counts(const unsigned long long *slot, FrontierCounts *c);

// Near-far threshold after the near frontier ran empty: far_min (+) delta in
// the weight type, and always above far_min so that the smallest held-back
// vertex is released.
uint32_t next_threshold(uint32_t far_min, uint32_t delta, int wt);

// ---- launch wrappers (gr_kernels.hip) -------------------------------------
// threshold: first near-far threshold (kInfU32 when the split is off); with
// use_far the held-back flags are cleared too.
hipError_t launch_init(const DevGraph &g, uint32_t *dist, int32_t src, const Frontier &f, uint32_t threshold,
                       bool use_far, hipStream_t st);
hipError_t launch_push(const DevGraph &g, uint32_t *dist, const Frontier &f, int64_t iter, const FrontierCounts &c,
                       int num_cu, hipStream_t st);
// Pull over the partitioned layout when the graph is symmetric (arcs into a
// destination range from sources in partition k are read by blocks on XCD k),
// else over the transposed copy.
// level (breadth-first search): the depth of every vertex of the frontier
// when the caller knows it (the pull then reads no source depth), else
// kInfU32.
hipError_t launch_pull(const DevGraph &g, uint32_t *dist, const Frontier &f, int64_t iter, hipStream_t st,
                       uint32_t level = kInfU32);
// The pull that launch_pull runs: 1 partitioned, 0 over the transposed copy.
bool pull_partitioned(const DevGraph &g);
// zmask: optional per-vertex 64-bit masks (batched queries) cleared by the filter.
// dense: stream the membership lists (large frontiers) instead of visiting
// the 4096-vertex groups that hold flags (small frontiers).
// use_far: near-far split at `threshold` (needs dist): flagged or held-back
// vertices below it join the frontier, the others are held back.
hipError_t launch_filter(const DevGraph &g, const Frontier &f, int64_t iter, uint64_t *zmask, bool dense,
                         const uint32_t *dist, bool use_far, uint32_t threshold, hipStream_t st);
// Device address of the counter slot filled by the filter of iteration `iter`.
unsigned long long *counters_after(const Frontier &f, int64_t iter);

// Device-driven loop (cooperative launch).
struct PersistentCfg {
    int32_t max_iters;
    int32_t alpha_x16;
    int32_t beta;         // pull -> push when |frontier| * beta < n
    int32_t direction;    // gr_direction
    int32_t filter;       // 0 auto, 1 group, 2 streaming
    int32_t dense_ratio;  // auto filter: streaming when |frontier| * dense_ratio >= n
    int32_t grid;         // co-resident blocks, a multiple of kMaxParts
    uint64_t spin_ticks;  // grid-barrier wait bound, in wall_clock64 ticks
    uint32_t delta;       // near-far split width (weight-type bits); 0 = off
    int32_t small;        // queued loop: rounds from a short candidate list may skip the filter
    int32_t local_hops;   // small rounds: hops a block expands before appending (1 = none)
};
// Largest co-resident grid for the graph's layout (0 if none).
int persistent_grid(const DevGraph &g, int num_cu);
hipError_t launch_persistent(const DevGraph &g, uint32_t *dist, const Frontier &f, const PersistentCfg &cfg,
                             hipStream_t st);
// Queued loop: launch number `launch` of the step kernel (cfg.grid blocks),
// which runs the phase the loop state names (advance, filter or a small
// round) and does nothing once the query has ended.
// phase_log (optional, timing): one byte per launch, what it ran: 1 advance,
// 2 filter, 3 small round, 4 nothing.
hipError_t launch_step(const DevGraph &g, uint32_t *dist, const Frontier &f, const PersistentCfg &cfg, int64_t launch,
                       int8_t *phase_log, int64_t phase_log_cap, hipEvent_t ev_begin, hipEvent_t ev_end,
                       hipStream_t st);

// Graph build helpers.
hipError_t launch_pack_arcs(const int32_t *col, const uint32_t *w, int32_t m, uint2 *adj, hipStream_t st);
hipError_t launch_canon_negzero(uint2 *adj, int32_t m, hipStream_t st);
hipError_t launch_validate(int32_t n, int32_t m, const int32_t *ro, const int32_t *col, const uint32_t *w, int wt,
                           unsigned int *err, hipStream_t st);
size_t scan_tmp_ints(int64_t len);
hipError_t launch_csc_build(int32_t n, int32_t m, const int32_t *ro, const uint2 *adj, int32_t *ro_in,
                            uint2 *adj_in, int32_t *scratch, hipStream_t st);
hipError_t launch_symmetry_check(int32_t n, const int32_t *ro, const uint2 *adj, unsigned int *not_sym,
                                 hipStream_t st);
// Partitioned push layout: pro needs (n+1)*np ints; cnt and pm np*(n+1)+1
// ints each, tmp scan_tmp_ints(np*(n+1)+1).
hipError_t launch_partition_build(int32_t n, int32_t m, const int32_t *ro, const uint2 *adj, int32_t np,
                                  int32_t psize, int32_t *pro, uint2 *padj, int32_t *cnt, int32_t *pm, int32_t *tmp,
                                  unsigned long long *caps, hipStream_t st);
// Membership lists of a push layout (see DevGraph): cnt needs np*(n+1)+1 ints,
// pos the same, tmp scan_tmp_ints(np*(n+1)+1); mem_u / mem_sd hold
// sum(cap) entries; off receives np + 1 offsets (device, int64).
hipError_t launch_members(int32_t n, int32_t np, const int32_t *pro, int32_t *cnt, int32_t *pos, int32_t *tmp,
                          int32_t *mem_u, uint2 *mem_sd, long long *off, hipStream_t st);
// Fraction numerator for the locality test: arcs with |u - v| < span.
hipError_t launch_locality(int32_t n, const int32_t *ro, const uint2 *adj, int32_t span, unsigned long long *near,
                           hipStream_t st);

// Asynchronous loop (gr_async.hip).  Its worklist and counters live in a
// buffer of async_bytes(n) bytes; the frontier workspace's two flag arrays
// serve as the in-queue and spill bytes.  Counter words (each hot one on its
// own 256-byte line): status (0 running or done, 3 a wait timed out), the
// expanded-vertex and arc totals, then the list's head, tail and done counts.
constexpr int kAsyncStatus = 0;
constexpr int kAsyncStatItems = 1;
constexpr int kAsyncStatArcs = 2;
constexpr int kAsyncHead = 32;
constexpr int kAsyncTail = 64;
constexpr int kAsyncDone = 96;
constexpr int kAsyncCtlWords = 128;
int64_t async_capacity(int32_t n);  // default list entries: 4 n + 1024
size_t async_bytes(int64_t cap);    // list of cap entries + counters
unsigned long long *async_ctl(int64_t cap, void *ws);
// dist, flags, list {src} and counters for a new query.
hipError_t launch_async_init(const DevGraph &g, uint32_t *dist, int32_t src, const Frontier &f, void *ws, int64_t cap,
                             hipStream_t st);
// Default block count of the asynchronous kernel for a graph.
int async_blocks(const DevGraph &g, int num_cu);
// One phase with `blocks` blocks: runs until the list is drained or a wait
// exceeds spin_ticks.  Appends past the list's capacity are spilled: tail -
// cap of them.
hipError_t launch_async(const DevGraph &g, uint32_t *dist, const Frontier &f, void *ws, int64_t cap, int blocks,
                        uint64_t spin_ticks, hipStream_t st);
// Restarts the list with the spilled vertices (those past cap stay spilled).
hipError_t launch_async_relist(const DevGraph &g, const Frontier &f, void *ws, int64_t cap, hipStream_t st);

// Batched multi-source queries: up to kBatchLanes sources, one per wave lane
// (gr_multi.hip).
constexpr int kBatchLanes = 64;

}  // namespace gr
