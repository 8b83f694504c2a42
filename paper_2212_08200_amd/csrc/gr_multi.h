// Multi-query engine: up to kMqSlots independent single-source queries, on
// one graph or on several graphs of different sizes, advance together.  Each
// round is two kernel launches over the union of the queries' frontiers:
//   k_mq_push    every out-arc of every queued (slot, vertex) entry is relaxed
//                in that slot's distance array (Section IV-D, Listing 4); an
//                improved vertex is marked in its slot's next-frontier bytes
//                and the 4096-vertex group holding it is marked dirty;
//   k_mq_filter  the dirty groups of every live slot are compacted into the
//                next union queue (entries (first arc, vertex), the slot, and
//                the exclusive prefix sum of arc counts for the load-balanced
//                search), clearing the marks.
// Kernel arguments never change during a session (all round state is read
// from a control block in device memory), so a chunk of rounds is captured
// once as a HIP graph and replayed; the host reads the control block once per
// chunk, and admits new queries between chunks (continuous batching).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gr_internal.h"

namespace gr {

constexpr int kMqSlots = 64;

// One query, as the kernels see it (written on the device by k_mq_update).
struct MqSlot {
    const int32_t *ro;   // the graph's CSR offsets
    const uint2 *adj;    // its arcs (destination, weight bits)
    uint32_t *dist;      // working distances = the query's output
    uint8_t *flags;      // 2 x nflag bytes: next-frontier marks, by round parity
    uint8_t *dirty;      // 2 x ngroups bytes: group holds marks, by round parity
    int32_t n;
    int32_t wt;          // 0 uint32, 1 binary32, 2 unit steps (BFS)
    int32_t ngroups;     // groups of kGroupVerts vertices
    int32_t nflag;       // bytes per flag array (ngroups * kGroupVerts)
    int32_t light;       // 1: every vertex has at most kMqLight out-arcs (local hops apply)
    int32_t pad;
};

// Local hops (MqBufs::local_hops > 1): a push block keeps up to kMqLocalCap of
// the vertices it improved in queries on light graphs, with the candidate
// distance that improved them, and expands them again itself, one thread per
// vertex, for up to local_hops - 1 further hops; only the improvements it does
// not expand are marked for the next round.  Expanding v with its own
// candidate c relaxes a real path (dist[v] <= c once the atomic executed); a
// relaxation that lowered dist[v] further marked or expanded v itself, so every
// decrease is still followed by an expansion with that value or a smaller one.
constexpr int kMqLight = 8;
constexpr int kMqLocalCap = 1024;

// Control block of a session (device memory, cleared at session start).
// Counters that many blocks update sit on 256-byte lines of their own.
struct MqCtl {
    unsigned long long cnt[3][32];         // queue of round r: cnt[r % 3][0] = F | E << 32
    unsigned long long slot_cnt[3][kMqSlots];  // entries of each slot in the queue of round r
    unsigned long long st_round[2];        // round of the next launch, by launch parity
    unsigned long long rounds;             // non-empty rounds run
    unsigned long long edges;              // arcs expanded
    unsigned long long frontier;           // queue entries expanded
    unsigned long long pairs;              // batched same-graph queries: (arc, active source) relaxations
    unsigned long long pad0[2];
    unsigned long long slot_rounds[kMqSlots];  // non-empty rounds of each slot's query
    int32_t nlive;                         // live slots, their ids, and the exclusive
    int32_t live[kMqSlots];                // prefix sum of their group counts
    int32_t gpre[kMqSlots + 1];
    MqSlot slot[kMqSlots];
};

// Session buffers.
struct MqBufs {
    MqCtl *ctl;
    uint2 *qse[2];      // union queue by round parity: (first arc, vertex)
    int32_t *qs[2];     // exclusive prefix sums of arc counts
    uint8_t *qslot[2];  // slot of each entry
    int64_t qcap;       // entries per queue
    uint64_t *mask[2];  // batched same-graph queries: per-vertex active-source masks by round
                        // parity, cleared by the filter for the round's entries (NULL otherwise)
    int32_t local_hops; // multi-query push: see kMqLocalCap (1 = none)
};

// Batched same-graph queries (up to kBatchLanes sources, one per wave lane):
// distances vertex-major, D[v * kBatchLanes + lane], one 256-byte row per
// vertex; the union queue holds each frontier vertex once (slot 0), with the
// sources active at it in its mask.
struct MqBatchSrc {
    int32_t k;
    int32_t src[kBatchLanes];
};
struct MqOutRows {
    uint32_t *row[kBatchLanes];
};

// Admission and slot-set update, applied on the device between chunks.
struct MqUpdate {
    int32_t nadmit;
    int32_t admit_slot[16];
    int32_t admit_src[16];
    MqSlot admit[16];
    int32_t nlive;  // the live set after this update (-1: unchanged)
    uint8_t live[kMqSlots];
    int32_t gpre[kMqSlots + 1];
};
static_assert(sizeof(MqUpdate) <= 3072, "update fits the kernel-argument buffer");

size_t mq_ctl_bytes();
// Clears the control block (a kernel: safe in captured graphs too).
hipError_t mq_reset(const MqBufs &b, hipStream_t st);
// Writes admitted slots, initialises their distances and marks, appends their
// sources to the current round's queue, and installs the live set.
hipError_t mq_update(const MqBufs &b, const MqUpdate &u, hipStream_t st);
// One round: push then filter.  The push reads its round
// from st_round[0] and writes it to st_round[1]; the filter reads st_round[1]
// and writes the next round to st_round[0]; so no launch writes a word that
// another block of the same launch reads.
hipError_t mq_round(const MqBufs &b, int push_grid, int filter_grid, hipStream_t st);

// Batched same-graph queries on slot 0 (graph s, workspace D and b.mask):
// initialisation (after mq_reset), one round, and the k x n output.
hipError_t mq_batch_init(const MqBufs &b, const MqSlot &s, uint32_t *D, const MqBatchSrc &src, hipStream_t st);
hipError_t mq_batch_round(const MqBufs &b, uint32_t *D, int wt, int push_grid, int filter_grid, hipStream_t st);
hipError_t mq_batch_output(const uint32_t *D, int32_t n, int32_t k, const MqOutRows &rows, hipStream_t st);

}  // namespace gr
