// HIP kernels for frontier-driven SSSP on gfx950 (MI355X).
//
// Operators (Osama et al., Section IV-C) on a CSR graph (Section IV-A) and a
// frontier kept as byte marks (written by push), a dense bitmap (one bit per
// vertex, read by pull) and sparse queues (Section IV-B):
//   k_init    dist = INF, dist[src] = 0, frontier = {src} (Listing 4 set-up)
//   k_push    advance, push direction (Listing 3, with Listing 4's condition):
//             every out-edge of the sparse frontier is relaxed with an atomic
//             min, and the destination joins the next bitmap iff the new value
//             is strictly smaller than the old one.  Edges are spread evenly
//             over blocks by a load-balanced search over the prefix sum of
//             frontier out-degrees, so a hub's edges are shared by many blocks
//             and consecutive lanes read consecutive arcs.
//   k_pull    advance, pull direction over the transposed graph
//             (Section III-C): each vertex takes the min over its in-arcs from
//             active vertices; one owner per vertex, no global atomics on dist.
//   k_filter  deduplicated, compacted next frontier from the flags, written
//             as per-partition queues of (first arc, u) plus the prefix sum of
//             arc counts, and the totals the convergence test reads.
//
// Partitioned push layout: arcs are grouped by destination range into up to
// eight partitions; block b of the push works on partition b % 8.  Workgroups
// are placed on the eight XCDs round-robin, so each XCD's L2 only sees one
// eighth of the distance array (2 MB at 4M vertices), which then stays
// resident and the per-edge pre-read of dist[v] hits in L2.
//
// Distances are 32-bit patterns; binary32 values are non-negative, so their
// bit patterns order like the values and one uint32 atomic min serves both
// weight types.
#include "gr_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

namespace gr {


// The next frontier is a byte per vertex, set by plain stores: every writer
// stores the same value, so concurrent marks need no atomics (distinct bytes
// are distinct memory locations, so marks of neighbouring vertices by other
// blocks are never lost).
template <bool O32 = false>
__device__ __forceinline__ void mark(uint8_t *flags, uint32_t v) { *elem<O32>(flags, v) = 1; }

// Relaxation of one edge (Listing 4) is split in two so that a thread can
// issue the loads of several edges before any of their atomics:
//   new = du (+) w; old = plain read of dist[v]; then, if new < old, an atomic
//   min and a mark of v for the next frontier.
// The old value is taken from the plain read instead of from the atomic's
// return, so the atomic needs no reply.  The read may be stale, i.e. older and
// hence larger or equal: if new >= read, no update is needed; if new < read,
// then either the atomic lowers dist[v] or dist[v] was already lowered since
// the read was cached, during this advance -- either way v improved in this
// round, so the marked set is exactly the set of improved vertices.
template <bool O32 = false>
__device__ __forceinline__ void relax_commit(uint32_t *dist, uint8_t *nflags, uint32_t v, uint32_t nd) {
    __hip_atomic_fetch_min(elem<O32>(dist, v), nd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    mark<O32>(nflags, v);
}

// Relaxation filter with the bound array: the pre-read comes from `bound`, a
// per-vertex upper bound on dist kept with plain stores.  A relaxation that
// passes it issues its atomic min and then stores its candidate into the
// bound: once that atomic has executed (at the latest when the launch ends)
// dist <= candidate, and dist never rises within a query, so every value the
// bound has held is an upper bound on dist by the end of the launch that
// wrote it, and a candidate not below the value read can be dropped.  Racing
// stores may leave a larger candidate than another one that passed: still an
// upper bound.  Every issuer marks its vertex, so every decrease of dist is
// marked.  Within a round a vertex's bound line stays in the L2 of the die
// that relaxes it (the partitioned layout sends all arcs into one destination
// range to one XCD) and is kept current there by the stores, and the
// pre-reads no longer touch the lines that the atomics (executed beyond the
// L2) are working on.  Measured on R-MAT graphs: the same number of atomics
// and L2 hits, 10-25% less time per query; slower on road-like graphs.
template <bool O32>
__device__ __forceinline__ void relax_bound(uint32_t *dist, uint32_t *bound, uint8_t *nflags, uint32_t v,
                                            uint32_t nd) {
    relax_commit<O32>(dist, nflags, v, nd);
    *elem<O32>(bound, v) = nd;
}

// ---------------------------------------------------------------------------
// init: dist, bitmaps, summaries, counters and the one-vertex frontier.

struct InitArgs {
    uint32_t *dist;
    int32_t n;
    int32_t np;
    uint32_t inf;
    int32_t src;
    const int32_t *pro;
    uint8_t *flags0, *flags1;
    uint32_t *bits;        // frontier bitmap
    uint8_t *far0, *far1;  // NULL when the near-far split is off
    unsigned long long *ccount;  // candidate-list counters (queued loop), NULL if absent
    uint32_t *bound;             // relaxation filter (see relax_bound), NULL if off
    unsigned long long *rstat;   // small-round statistics, NULL if absent
    int64_t nflag;  // bytes per flag array (multiple of 16)
    uint2 *qse[kMaxParts];
    int32_t *qs[kMaxParts];
    unsigned long long *ctl;
    uint32_t threshold;
};

__global__ __launch_bounds__(kBlk) void k_init(InitArgs a) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int32_t src = a.src;
    for (int64_t v = tid; v < a.n; v += stride) {
        a.dist[v] = (v == src) ? 0u : a.inf;
        if (a.bound) a.bound[v] = (v == src) ? 0u : a.inf;
    }
    const int64_t sw = src >> 4;
    for (int64_t w = tid; w < a.nflag / 16; w += stride) {
        uint4 z = make_uint4(0u, 0u, 0u, 0u);
        reinterpret_cast<uint4 *>(a.flags1)[w] = z;
        if (a.far0) {
            reinterpret_cast<uint4 *>(a.far0)[w] = z;
            reinterpret_cast<uint4 *>(a.far1)[w] = z;
        }
        if (w == sw) reinterpret_cast<uint32_t *>(&z)[(src >> 2) & 3] = 1u << ((src & 3) * 8);
        reinterpret_cast<uint4 *>(a.flags0)[w] = z;
    }
    for (int64_t w = tid; w < a.nflag / 32; w += stride) a.bits[w] = (w == (src >> 5)) ? 1u << (src & 31) : 0u;
    if (blockIdx.x == 0) {
        for (int t = threadIdx.x; t < kCtlWords; t += kBlk) a.ctl[t] = 0ull;
        __syncthreads();
        if (threadIdx.x == 0) reinterpret_cast<LoopState *>(a.ctl + kLoopStateWord)->threshold = a.threshold;
        if (a.ccount && threadIdx.x < 3 * kCandRegions) a.ccount[threadIdx.x] = 0ull;
        if (a.rstat)
            for (int t = threadIdx.x; t < kStatWords; t += kBlk) a.rstat[t] = 0ull;
        if (threadIdx.x < a.np) {
            const int k = threadIdx.x;
            const int32_t st = a.pro[(int64_t)src * a.np + k];
            const int32_t d = a.pro[(int64_t)(src + 1) * a.np + k] - st;
            if (d > 0) {
                a.qse[k][0] = make_uint2((uint32_t)st, (uint32_t)src);
                a.qs[k][0] = 0;
                a.ctl[k * kCtrStride] = 1ull | ((unsigned long long)d << 32);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// push advance with load-balanced search.
//
// Partition k's frontier has F entries (first arc, u) with exclusive arc
// count prefix sums s[0..F) (strictly increasing: the filter drops entries
// without arcs) and E arcs in total.  Block j of partition k relaxes arc ranks
// [j*per, min(E, (j+1)*per)).  It finds the entry holding its first rank with
// a 256-way search, then walks windows of up to kWin consecutive entries
// staged in LDS; each lane maps its rank to an entry by binary search in LDS.
constexpr int kPushItems = 16;
// Smallest arc range a block of the device-sized advance takes (one pass of
// its 256 lanes x kPushItems items).
constexpr int32_t kMinChunk = kBlk * kPushItems;

struct PushArgs {
    const uint2 *padj;
    uint32_t *dist;
    const uint2 *qse[kMaxParts];
    const int32_t *qs[kMaxParts];
    int32_t F[kMaxParts];
    int32_t E[kMaxParts];
    int32_t per[kMaxParts];
    uint8_t *nflags;
    uint32_t *bound;  // relaxation filter (NULL: pre-read dist)
};

// Candidate list of the small-frontier rounds: the vertices a round
// improved, appended in any order and with repeats; the flag bytes decide
// which copy is expanded.  A wave reserves room for all its lanes' appends
// with one atomic add; appends past the capacity are dropped but still
// counted, so an overflowing count tells the next round to scan the flags.
struct CandOut {
    int32_t *list;              // NULL: no appends
    unsigned long long *count;
    int32_t cap;
};

// All threads of the block call this (convergent); thread t appends the
// values vals[i] with take[i] set.  One atomic add per block reserves the
// room; values past cap are dropped (the count still grows).
template <int N>
__device__ __forceinline__ void block_append(const CandOut &o, const uint32_t (&vals)[N], const bool (&take)[N]) {
    __shared__ int32_t sWave[kBlk / 64];
    __shared__ unsigned long long sBase;
    int32_t c = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) c += take[i] ? 1 : 0;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t inc = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t t = __shfl_up(inc, off, 64);
        if (lane >= off) inc += t;
    }
    if (lane == 63) sWave[wid] = inc;
    __syncthreads();
    int32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kBlk / 64; ++w) {
        before += w < wid ? sWave[w] : 0;
        total += sWave[w];
    }
    if (threadIdx.x == 0 && total > 0) sBase = atomicAdd(o.count, (unsigned long long)total);
    __syncthreads();
    if (total == 0) return;
    int64_t pos = (int64_t)sBase + before + (inc - c);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if (take[i]) {
            if (pos < o.cap) o.list[pos] = (int32_t)vals[i];
            ++pos;
        }
    }
}

// Arc ranks [j*per, min(E, (j+1)*per)) of one partition's frontier
// (F entries (first arc, u) with arc-count prefix sums s), by one block.
// With cand.list set, improved vertices are also appended to the candidate
// list (small rounds follow when it stays short).  O32: 32-bit offsets for
// the arc and distance accesses (arcs * 8 and n * 4 below 2^32).
template <int WT, bool O32>
__device__ __forceinline__ void push_range(const uint2 *__restrict__ padj, uint32_t *__restrict__ dist,
                                           const uint2 *__restrict__ qse, const int32_t *__restrict__ s,
                                           int32_t F, int32_t E, int32_t per, int64_t j,
                                           uint8_t *__restrict__ nflags, const CandOut &cand, uint32_t *bound) {
    __shared__ int32_t sS[kWin + 1];
    __shared__ uint32_t sRow[kWin];
    __shared__ uint32_t sDu[kWin];

    const int64_t beg64 = j * per;
    if (F <= 0 || beg64 >= E) return;
    const int32_t beg = (int32_t)beg64;
    const int32_t end = (int32_t)min<int64_t>(beg64 + per, E);

    int32_t i0 = find_entry(s, F, beg);
    int32_t e = beg;
    while (e < end) {
        const int32_t cnt = min(kWin, F - i0);
        // dist[u] is read now rather than when the filter ran: a value lowered
        // since then (earlier in this advance) saves relaxations -- on R-MAT
        // 22, 420M instead of 540M per query with the filter's snapshot.
        for (int t = threadIdx.x; t < cnt; t += kBlk) {
            const uint2 q = qse[i0 + t];
            sS[t] = s[i0 + t];
            sRow[t] = q.x;
            sDu[t] = *elem<O32>(dist, q.y);
        }
        // sS[cnt] bounds the window's ranks; entries past it are padded with
        // INT32_MAX so that the search below needs no bounds test.
        for (int t = cnt + threadIdx.x; t <= kWin; t += kBlk)
            sS[t] = (t == cnt) ? ((i0 + cnt < F) ? s[i0 + cnt] : E) : INT32_MAX;
        __syncthreads();
        const int32_t wend = min(end, sS[cnt]);
        // The pass loop is uniform over the block (x0b), so the waves stay
        // convergent for the candidate appends.
        for (int32_t x0b = e; x0b < wend; x0b += kBlk * kPushItems) {
            const int32_t x0 = x0b + (int32_t)threadIdx.x;
            // Ranks past the window end are clamped to its last rank, so every
            // item does the same unconditional LDS reads and loads (keeping them
            // batched); only the commit is predicated.
            int32_t xr[kPushItems], pos[kPushItems];
#pragma unroll
            for (int it = 0; it < kPushItems; ++it) {
                xr[it] = min(x0 + it * kBlk, wend - 1);
                pos[it] = 0;
            }
            // entry of each rank: largest j with sS[j] <= rank, by branch-free
            // binary lifting (sS is strictly increasing, then padded)
#pragma unroll
            for (int b = kWin / 2; b >= 1; b >>= 1) {
#pragma unroll
                for (int it = 0; it < kPushItems; ++it) {
                    const int32_t p = pos[it] + b;
                    pos[it] = (sS[p] <= xr[it]) ? p : pos[it];
                }
            }
            uint2 arc[kPushItems];
            uint32_t du[kPushItems];
#pragma unroll
            for (int it = 0; it < kPushItems; ++it) {
                du[it] = sDu[pos[it]];
                arc[it] = load_arc(elem<O32>(padj, sRow[pos[it]] + (uint32_t)(xr[it] - sS[pos[it]])));
            }
            uint32_t nd[kPushItems], cur[kPushItems];
#pragma unroll
            for (int it = 0; it < kPushItems; ++it) {
                nd[it] = plus<WT>(du[it], arc[it].y);
                cur[it] = *elem<O32>(bound ? bound : dist, arc[it].x);
            }
            bool take[kPushItems];
            uint32_t vv[kPushItems];
            if (bound) {  // two loops: a branch inside the unrolled one measured 5% slower
#pragma unroll
                for (int it = 0; it < kPushItems; ++it) {
                    take[it] = x0 + it * kBlk < wend && nd[it] < cur[it];
                    vv[it] = arc[it].x;
                    if (take[it]) relax_bound<O32>(dist, bound, nflags, arc[it].x, nd[it]);
                }
            } else {
#pragma unroll
                for (int it = 0; it < kPushItems; ++it) {
                    take[it] = x0 + it * kBlk < wend && nd[it] < cur[it];
                    vv[it] = arc[it].x;
                    if (take[it]) relax_commit<O32>(dist, nflags, arc[it].x, nd[it]);
                }
            }
            if (cand.list) block_append<kPushItems>(cand, vv, take);
        }
        i0 += cnt;
        e = wend;
        __syncthreads();  // window reuse
    }
}

template <int WT, int NP, bool O32>
__global__ __launch_bounds__(kBlk) void k_push(PushArgs a) {
    const int k = (NP == 1) ? 0 : (int)(blockIdx.x % NP);
    const int64_t j = (NP == 1) ? blockIdx.x : blockIdx.x / NP;
    push_range<WT, O32>(a.padj, a.dist, a.qse[k], a.qs[k], a.F[k], a.E[k], a.per[k], j, a.nflags,
                        CandOut{nullptr, nullptr, 0}, a.bound);
}

// ---------------------------------------------------------------------------
// pull advance: block owns vertices [v0, v0 + kBlk); its in-arcs are the
// contiguous CSC range [ro_in[v0], ro_in[v0 + kBlk]).  Lanes stride over that
// range, map each arc to its owner by binary search in LDS, and fold the
// candidates dist[u] (+) w of active u (bit u of the frontier bitmap) into an
// LDS min per owner.  Then each owner compares with dist[v], stores the
// improvement (it is the only writer of dist[v] in this launch) and marks v.
constexpr int kPullItems = 8;

__device__ __forceinline__ bool in_frontier(const uint32_t *__restrict__ bits, uint32_t u) {
    return (bits[u >> 5] >> (u & 31)) & 1u;
}

template <int WT>
__device__ __forceinline__ void pull_block(int32_t n, const int32_t *__restrict__ ro_in,
                                           const uint2 *__restrict__ adj_in, uint32_t *__restrict__ dist,
                                           const uint32_t *__restrict__ cbits, uint8_t *__restrict__ nflags,
                                           uint32_t *__restrict__ bound, int64_t vb) {
    __shared__ int32_t sOff[kBlk + 1];
    __shared__ uint32_t sMin[kBlk];
    const int32_t v0 = (int32_t)(vb * kBlk);
    const int32_t nv = min(kBlk, n - v0);
    // sOff[0..nv] are the owners' arc offsets; entries past nv are padded with
    // INT32_MAX so that the owner search needs no bounds test.
    for (int t = threadIdx.x; t <= kBlk; t += kBlk) sOff[t] = (t <= nv) ? ro_in[v0 + t] : INT32_MAX;
    sMin[threadIdx.x] = kInfU32;
    __syncthreads();
    const int32_t a0 = sOff[0], a1 = sOff[nv];
    const uint32_t inf = WT == 0 ? kInfU32 : kInfF32;
    for (int32_t x0 = a0 + threadIdx.x; x0 < a1; x0 += kBlk * kPullItems) {
        // arcs past the range end are clamped to its last arc (loads stay
        // unconditional and batched); only the fold is predicated
        int32_t xr[kPullItems];
        uint2 arc[kPullItems];
#pragma unroll
        for (int it = 0; it < kPullItems; ++it) {
            xr[it] = min(x0 + it * kBlk, a1 - 1);
            arc[it] = load_arc(adj_in + xr[it]);
        }
        bool fl[kPullItems];
#pragma unroll
        for (int it = 0; it < kPullItems; ++it) fl[it] = in_frontier(cbits, arc[it].x);
        // distances only of active in-neighbours (the loads stay batched:
        // each one is predicated on its own lane's flag)
        uint32_t du[kPullItems];
#pragma unroll
        for (int it = 0; it < kPullItems; ++it) du[it] = fl[it] ? dist[arc[it].x] : inf;
        int32_t pos[kPullItems];
#pragma unroll
        for (int it = 0; it < kPullItems; ++it) pos[it] = 0;
#pragma unroll
        for (int b = kBlk / 2; b >= 1; b >>= 1) {
#pragma unroll
            for (int it = 0; it < kPullItems; ++it) {
                const int32_t p = pos[it] + b;
                pos[it] = (sOff[p] <= xr[it]) ? p : pos[it];
            }
        }
#pragma unroll
        for (int it = 0; it < kPullItems; ++it) {
            const bool act = (x0 + it * kBlk < a1) && du[it] != inf;
            if (act) atomicMin(&sMin[pos[it]], plus<WT>(du[it], arc[it].y));
        }
    }
    __syncthreads();
    const int32_t v = v0 + threadIdx.x;
    if (threadIdx.x < nv) {
        const uint32_t cand = sMin[threadIdx.x];
        const uint32_t cur = dist[v];
        if (cand < cur) {
            dist[v] = cand;
            if (bound) bound[v] = cand;  // keeps push's relaxation filter tight
            mark(nflags, (uint32_t)v);
        }
    }
}

// Breadth-first pull (unit weights): a vertex that already has a depth keeps
// it (depths only shrink from INF once), so only the in-arcs of the block's
// unreached vertices are scanned -- the saving that makes pull pay in the
// middle levels.  Their arcs are laid out by an LDS prefix sum over the
// unreached owners and searched like the push's windows.
__device__ __forceinline__ void pull_block_bfs(int32_t n, const int32_t *__restrict__ ro_in,
                                               const uint2 *__restrict__ adj_in, uint32_t *__restrict__ dist,
                                               const uint32_t *__restrict__ cbits, uint8_t *__restrict__ nflags,
                                               uint32_t *__restrict__ bound, int64_t vb, uint32_t level) {
    __shared__ int32_t sPre[kBlk + 1];
    __shared__ int32_t sStart[kBlk];
    __shared__ uint32_t sMin[kBlk];
    const int32_t v0 = (int32_t)(vb * kBlk);
    const int32_t nv = min(kBlk, n - v0);
    const int t = threadIdx.x;
    int32_t deg = 0;
    if (t < nv && dist[v0 + t] == kInfU32) {
        sStart[t] = ro_in[v0 + t];
        deg = ro_in[v0 + t + 1] - sStart[t];
    }
    int32_t x[1] = {deg}, tot[1];
    block_scan<1>(x, tot);
    sPre[t] = x[0];
    if (t == 0) sPre[kBlk] = INT32_MAX;
    sMin[t] = kInfU32;
    __syncthreads();
    const int32_t H = tot[0];
    for (int32_t x0b = 0; x0b < H; x0b += kBlk * kPullItems) {
        int32_t xr[kPullItems], pos[kPullItems];
#pragma unroll
        for (int it = 0; it < kPullItems; ++it) {
            xr[it] = min(x0b + t + it * kBlk, H - 1);
            pos[it] = 0;
        }
        // owner of each rank: largest p with sPre[p] <= rank (owners without
        // arcs to scan repeat the next prefix and are never chosen)
#pragma unroll
        for (int b = kBlk / 2; b >= 1; b >>= 1) {
#pragma unroll
            for (int it = 0; it < kPullItems; ++it) {
                const int32_t p = pos[it] + b;
                pos[it] = (sPre[p] <= xr[it]) ? p : pos[it];
            }
        }
        uint2 arc[kPullItems];
#pragma unroll
        for (int it = 0; it < kPullItems; ++it) arc[it] = load_arc(adj_in + sStart[pos[it]] + (xr[it] - sPre[pos[it]]));
        bool fl[kPullItems];
#pragma unroll
        for (int it = 0; it < kPullItems; ++it) fl[it] = in_frontier(cbits, arc[it].x);
        // level: the depth of every frontier vertex when the caller knows it
        // (level-synchronous rounds of the host-driven loop), so no source
        // depth is read; else kInfU32 and each active source's depth is read
        uint32_t du[kPullItems];
        if (level != kInfU32) {
#pragma unroll
            for (int it = 0; it < kPullItems; ++it) du[it] = fl[it] ? level : kInfU32;
        } else {
#pragma unroll
            for (int it = 0; it < kPullItems; ++it) du[it] = fl[it] ? dist[arc[it].x] : kInfU32;
        }
#pragma unroll
        for (int it = 0; it < kPullItems; ++it)
            if (x0b + t + it * kBlk < H && du[it] != kInfU32) atomicMin(&sMin[pos[it]], du[it] + 1u);
    }
    __syncthreads();
    if (t < nv) {
        const uint32_t cand = sMin[t];
        if (cand < dist[v0 + t]) {
            dist[v0 + t] = cand;
            if (bound) bound[v0 + t] = cand;
            mark(nflags, (uint32_t)(v0 + t));
        }
    }
}

// Partitioned pull (symmetric graphs with the partitioned layout): the
// in-arcs of v are its out-arcs, and those from sources in partition k are
// the contiguous run padj[pro[v*8 + k] .. pro[(v+1)*8 + k]) -- so block b,
// placed on XCD b % 8 like the push's blocks, takes partition k = b % 8 and
// the 256 destinations of chunk b / 8, and its gathers of the frontier bits
// and distances of the sources stay in that XCD's slice (a 64 KB bitmap
// slice and a 2 MB distance slice at n = 4M), the same locality the
// partitioned push gets for its destinations.  Each block folds its
// candidates into an LDS min per destination; the eight blocks of a chunk
// then combine theirs with an atomic min, issued only when the candidate is
// below the distance read (the same rule as push's relaxation).
template <int WT>
__device__ __forceinline__ void pull_part_block(int32_t n, const int32_t *__restrict__ pro,
                                                const uint2 *__restrict__ padj, uint32_t *__restrict__ dist,
                                                const uint32_t *__restrict__ cbits, uint8_t *__restrict__ nflags,
                                                uint32_t *__restrict__ bound, int64_t vb) {
    __shared__ int32_t sOff[kBlk + 1];
    __shared__ uint32_t sMin[kBlk];
    const int k = (int)(vb % kMaxParts);
    const int32_t v0 = (int32_t)((vb / kMaxParts) * kBlk);
    const int32_t nv = min(kBlk, n - v0);
    for (int t = threadIdx.x; t <= kBlk; t += kBlk)
        sOff[t] = (t <= nv) ? pro[(int64_t)(v0 + t) * kMaxParts + k] : INT32_MAX;
    sMin[threadIdx.x] = kInfU32;
    __syncthreads();
    const int32_t a0 = sOff[0], a1 = sOff[nv];
    const uint32_t inf = WT == 0 ? kInfU32 : kInfF32;
    for (int32_t x0 = a0 + threadIdx.x; x0 < a1; x0 += kBlk * kPullItems) {
        int32_t xr[kPullItems];
        uint2 arc[kPullItems];
#pragma unroll
        for (int it = 0; it < kPullItems; ++it) {
            xr[it] = min(x0 + it * kBlk, a1 - 1);
            arc[it] = load_arc(padj + xr[it]);
        }
        bool fl[kPullItems];
#pragma unroll
        for (int it = 0; it < kPullItems; ++it) fl[it] = in_frontier(cbits, arc[it].x);
        uint32_t du[kPullItems];
#pragma unroll
        for (int it = 0; it < kPullItems; ++it) du[it] = fl[it] ? dist[arc[it].x] : inf;
        int32_t pos[kPullItems];
#pragma unroll
        for (int it = 0; it < kPullItems; ++it) pos[it] = 0;
#pragma unroll
        for (int b = kBlk / 2; b >= 1; b >>= 1) {
#pragma unroll
            for (int it = 0; it < kPullItems; ++it) {
                const int32_t p = pos[it] + b;
                pos[it] = (sOff[p] <= xr[it]) ? p : pos[it];
            }
        }
#pragma unroll
        for (int it = 0; it < kPullItems; ++it) {
            const bool act = (x0 + it * kBlk < a1) && du[it] != inf;
            if (act) atomicMin(&sMin[pos[it]], plus<WT>(du[it], arc[it].y));
        }
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        const uint32_t v = (uint32_t)(v0 + threadIdx.x);
        const uint32_t cand = sMin[threadIdx.x];
        if (cand < (bound ? bound[v] : dist[v])) {
            if (bound) relax_bound<false>(dist, bound, nflags, v, cand);
            else relax_commit<false>(dist, nflags, v, cand);
        }
    }
}

template <int WT>
__global__ __launch_bounds__(kBlk) void k_pull(int32_t n, const int32_t *__restrict__ ro_in,
                                               const uint2 *__restrict__ adj_in, uint32_t *__restrict__ dist,
                                               const uint32_t *__restrict__ cbits, uint8_t *__restrict__ nflags,
                                               uint32_t *__restrict__ bound, uint32_t level) {
    if constexpr (WT == 2) pull_block_bfs(n, ro_in, adj_in, dist, cbits, nflags, bound, blockIdx.x, level);
    else pull_block<WT>(n, ro_in, adj_in, dist, cbits, nflags, bound, blockIdx.x);
}

template <int WT>
__global__ __launch_bounds__(kBlk) void k_pull_part(int32_t n, const int32_t *__restrict__ pro,
                                                    const uint2 *__restrict__ padj, uint32_t *__restrict__ dist,
                                                    const uint32_t *__restrict__ cbits, uint8_t *__restrict__ nflags,
                                                    uint32_t *__restrict__ bound) {
    pull_part_block<WT>(n, pro, padj, dist, cbits, nflags, bound, blockIdx.x);
}

// ---------------------------------------------------------------------------
// filter: one block per group of 4096 vertices.  Thread t owns vertices
// [base + 16 t, base + 16 t + 16), so each queue slice is in vertex order.  A
// block reserves its slice of partition k's queue and of that queue's arc
// prefix sum with one 64-bit atomic add of (count | arcs << 32) per partition.
// It also clears the group's current flags (so they can hold the frontier
// after next); block 0 clears the counter slot that was last used one
// iteration ago.
constexpr int kVpt = kGroupVerts / kBlk;  // 16

struct FilterArgs {
    int32_t np;
    const int32_t *pro;
    uint64_t *zmask;  // when set (batched queries): per-vertex masks cleared by partition-0 blocks
    const uint32_t *dist;  // distances, read by the near-far split (NULL for batched queries)
    const uint8_t *nflags;
    uint8_t *cflags;
    const uint8_t *far_cur;  // near-far split (NULL: off): held-back flags read ...
    uint8_t *far_next;       // ... and written
    uint32_t threshold;
    uint16_t *nbits;         // the next frontier's bitmap, 16 vertices per granule (NULL: not kept)
    uint2 *qse[kMaxParts];
    int32_t *qs[kMaxParts];
    unsigned long long *ctl_next;
    unsigned long long *ctl_zero;
};

// Bytes of a 16-byte flag word that are non-zero, as 16 bits.
__device__ __forceinline__ uint32_t nonzero_bytes(uint4 w) {
    uint32_t m = 0;
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        const uint32_t word = b < 4 ? w.x : b < 8 ? w.y : b < 12 ? w.z : w.w;
        m |= (((word >> ((b & 3) * 8)) & 0xFFu) != 0u ? 1u : 0u) << b;
    }
    return m;
}

// The inverse: byte b of the word is 1 when bit b is set.
__device__ __forceinline__ uint4 bytes_of_bits(uint32_t m) {
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        w[q] = 0u;
#pragma unroll
        for (int b = 0; b < 4; ++b) w[q] |= ((m >> (q * 4 + b)) & 1u) << (b * 8);
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Near-far split of 16 consecutive vertices from base: of the candidates
// (bits of cand), those at or above the threshold are held back (returned).
// The 16 distances are loaded before any is tested, each non-candidate slot
// reading the first candidate's (a vertex below n): loads guarded one by one
// ran one round trip at a time.
__device__ __forceinline__ uint32_t held_back(const uint32_t *__restrict__ dist, int64_t base, uint32_t cand,
                                              uint32_t T, uint32_t *cnt, uint32_t *inv) {
    if (cand == 0u) return 0u;
    const uint32_t b0 = (uint32_t)__builtin_ctz(cand);
    uint32_t d[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        uint32_t o = ((cand >> b) & 1u) ? (uint32_t)b : b0;
        asm volatile("" : "+v"(o));  // keeps the select: no load-or-copy branch
        d[b] = dist[base + o];
    }
    uint32_t held = 0;
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        if (((cand >> b) & 1u) && d[b] >= T) {
            held |= 1u << b;
            *cnt += 1u;
            *inv = max(*inv, ~d[b]);
        }
    }
    return held;
}

// Offsets of u's arcs in every partition: first[k] = pro[u*NP + k], and
// end[k] = pro[(u+1)*NP + k] (rows of NP ints, 32-byte aligned for NP = 8).
template <int NP>
__device__ __forceinline__ void arc_rows(const int32_t *__restrict__ pro, int64_t u, int32_t (&first)[NP],
                                         int32_t (&end)[NP]) {
    if constexpr (NP == 8) {
        const uint4 *r = reinterpret_cast<const uint4 *>(pro + u * 8);
        const uint4 a0 = r[0], a1 = r[1], b0 = r[2], b1 = r[3];
        first[0] = a0.x; first[1] = a0.y; first[2] = a0.z; first[3] = a0.w;
        first[4] = a1.x; first[5] = a1.y; first[6] = a1.z; first[7] = a1.w;
        end[0] = b0.x; end[1] = b0.y; end[2] = b0.z; end[3] = b0.w;
        end[4] = b1.x; end[5] = b1.y; end[6] = b1.z; end[7] = b1.w;
    } else {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            first[k] = pro[u * NP + k];
            end[k] = pro[(u + 1) * NP + k];
        }
    }
}

// Group filter: block g takes the 4096 vertices of group g for every
// partition.  Thread t owns vertices g*4096 + 16t .. +15: it reads their flag
// bytes as one 16-byte word, clears the matching word of the current flags
// and, for each flagged vertex, reads its offset rows once; one block-wide
// scan of the per-partition counts (entries, arcs) and one atomic per
// partition reserve the block's slices of the partition queues.
// a: the iteration-independent arguments (kernel-argument resident); the
// flags, held-back flags, threshold and counter slots of the iteration are
// passed separately.
constexpr int kFilterBatch = 4;

template <int NP>
__device__ __forceinline__ void filter_group(const FilterArgs &a, int64_t g, const uint8_t *__restrict__ nflags,
                                             uint8_t *__restrict__ cflags, unsigned long long *ctl_next,
                                             unsigned long long *ctl_zero, const uint8_t *__restrict__ far_cur,
                                             uint8_t *__restrict__ far_next, uint32_t T) {
    __shared__ unsigned long long sh_base[NP];
    __shared__ uint32_t sh_far_cnt, sh_far_inv;
    if (g == 0)
        for (int t = threadIdx.x; t < kSlotWords; t += kBlk) ctl_zero[t] = 0ull;
    if (a.zmask)
        for (int t = threadIdx.x; t < kGroupVerts; t += kBlk) a.zmask[g * kGroupVerts + t] = 0ull;
    const int64_t base = g * kGroupVerts + threadIdx.x * kVpt;
    uint32_t mask16 = nonzero_bytes(reinterpret_cast<const uint4 *>(nflags)[base >> 4]);
    reinterpret_cast<uint4 *>(cflags)[base >> 4] = make_uint4(0u, 0u, 0u, 0u);
    if (far_cur) {
        // near-far split: candidates are the flagged and the held-back
        // vertices; those below T join the frontier, the others are held back
        // again (each thread writes the next held-back flags of its 16)
        if (threadIdx.x == 0) {
            sh_far_cnt = 0u;
            sh_far_inv = 0u;
        }
        mask16 |= nonzero_bytes(reinterpret_cast<const uint4 *>(far_cur)[base >> 4]);
        uint32_t cnt = 0u, inv = 0u;
        const uint32_t held = held_back(a.dist, base, mask16, T, &cnt, &inv);
        mask16 &= ~held;
        reinterpret_cast<uint4 *>(far_next)[base >> 4] = bytes_of_bits(held);
        __syncthreads();
        if (cnt) {
            atomicAdd(&sh_far_cnt, cnt);
            atomicMax(&sh_far_inv, inv);
        }
        __syncthreads();
        if (threadIdx.x == 0 && sh_far_cnt) {
            atomicAdd(ctl_next + kFarCountWord, (unsigned long long)sh_far_cnt);
            atomicMax(ctl_next + kFarMaxInvWord, (unsigned long long)sh_far_inv);
        }
    }
    if (a.nbits) a.nbits[base >> 4] = (uint16_t)mask16;
    if (!__syncthreads_or(mask16 != 0)) return;  // uniform per block

    // x[k] = entries of partition k, x[NP + k] = their arcs.  The offset rows
    // of up to kFilterBatch flagged vertices are loaded together (a slot past
    // the last flagged vertex repeats its row and is not counted): one row at
    // a time made a chain of round trips per thread.
    int32_t x[2 * NP], tot[2 * NP];
#pragma unroll
    for (int i = 0; i < 2 * NP; ++i) x[i] = 0;
    for (uint32_t mm = mask16; mm;) {
        int b[kFilterBatch];
        bool on[kFilterBatch];
#pragma unroll
        for (int q = 0; q < kFilterBatch; ++q) {
            on[q] = mm != 0u;
            b[q] = on[q] ? __builtin_ctz(mm) : b[q > 0 ? q - 1 : 0];
            mm = on[q] ? (mm & (mm - 1)) : mm;
        }
        int32_t f[kFilterBatch][NP], e[kFilterBatch][NP];
#pragma unroll
        for (int q = 0; q < kFilterBatch; ++q) arc_rows<NP>(a.pro, base + b[q], f[q], e[q]);
#pragma unroll
        for (int q = 0; q < kFilterBatch; ++q) {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const int32_t d = on[q] ? e[q][k] - f[q][k] : 0;
                x[k] += d > 0 ? 1 : 0;
                x[NP + k] += d;
            }
        }
    }
    block_scan<2 * NP>(x, tot);
    if (threadIdx.x < NP) {
        const int k = threadIdx.x;
        sh_base[k] = tot[k] ? atomicAdd(ctl_next + k * kCtrStride, (unsigned long long)tot[k] |
                                                          ((unsigned long long)tot[NP + k] << 32))
                            : 0ull;
    }
    __syncthreads();
    int32_t pos[NP], spos[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        pos[k] = (int32_t)(sh_base[k] & 0xFFFFFFFFull) + x[k];
        spos[k] = (int32_t)(sh_base[k] >> 32) + x[NP + k];
    }
    for (uint32_t mm = mask16; mm;) {
        int b[kFilterBatch];
        bool on[kFilterBatch];
#pragma unroll
        for (int q = 0; q < kFilterBatch; ++q) {
            on[q] = mm != 0u;
            b[q] = on[q] ? __builtin_ctz(mm) : b[q > 0 ? q - 1 : 0];
            mm = on[q] ? (mm & (mm - 1)) : mm;
        }
        int32_t f[kFilterBatch][NP], e[kFilterBatch][NP];
#pragma unroll
        for (int q = 0; q < kFilterBatch; ++q) arc_rows<NP>(a.pro, base + b[q], f[q], e[q]);
#pragma unroll
        for (int q = 0; q < kFilterBatch; ++q) {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const int32_t d = e[q][k] - f[q][k];
                if (on[q] && d > 0) {
                    a.qse[k][pos[k]] = make_uint2((uint32_t)f[q][k], (uint32_t)(base + b[q]));
                    a.qs[k][pos[k]] = spos[k];
                    ++pos[k];
                    spos[k] += d;
                }
            }
        }
    }
}

template <int NP>
__global__ __launch_bounds__(kBlk) void k_filter(FilterArgs a) {
    filter_group<NP>(a, blockIdx.x, a.nflags, a.cflags, a.ctl_next, a.ctl_zero, a.far_cur, a.far_next, a.threshold);
}

// Streaming filter for large frontiers: block b works on partition b % np and
// on chunk b / np of that partition's membership list (kDenseChunk members,
// in vertex order).  Each member whose frontier flag is set becomes an entry
// (first arc, u); one atomic per block reserves the slice.  Every block also
// clears its share of the current frontier's flags.
constexpr int kDenseItems = 8;
constexpr int kDenseChunk = kBlk * kDenseItems;

struct DenseFilterArgs {
    int32_t np;
    int32_t chunks;  // chunks of the longest list
    const int32_t *mem_u;
    const uint2 *mem_sd;
    long long off[kMaxParts + 1];
    const uint8_t *nflags;
    uint8_t *cflags;
    int64_t clear16;  // uint4 words of flags each block clears
    int64_t nflag16;
    uint64_t *zmask;  // when set: per-vertex masks to clear (same share as the flags)
    const uint32_t *dist;  // as in FilterArgs
    const uint8_t *far_cur;  // as in FilterArgs
    uint8_t *far_next;
    uint32_t threshold;
    uint16_t *nbits;         // as in FilterArgs
    uint2 *qse[kMaxParts];
    int32_t *qs[kMaxParts];
    unsigned long long *ctl_next;
    unsigned long long *ctl_zero;
};

__device__ __forceinline__ void filter_dense(const DenseFilterArgs &a, int64_t vb, const uint8_t *__restrict__ nflags,
                                             uint8_t *__restrict__ cflags, uint64_t *zmask,
                                             unsigned long long *ctl_next, unsigned long long *ctl_zero,
                                             const uint8_t *__restrict__ far_cur, uint8_t *__restrict__ far_next,
                                             uint32_t T) {
    __shared__ unsigned long long sh_base;
    __shared__ uint32_t sh_far_cnt, sh_far_inv;
    const int np = a.np;
    const int k = (int)(vb % np);
    const int64_t j = vb / np;
    if (vb == 0)
        for (int t = threadIdx.x; t < kSlotWords; t += kBlk) ctl_zero[t] = 0ull;
    {
        // this block's share of the flags: clear the current ones and, with
        // the near-far split, write the next held-back flags of the share
        const int64_t c0 = vb * a.clear16;
        const int64_t c1 = min(c0 + a.clear16, a.nflag16);
        uint32_t cnt = 0u, inv = 0u;
        if (far_cur && threadIdx.x == 0) {
            sh_far_cnt = 0u;
            sh_far_inv = 0u;
        }
        for (int64_t w = c0 + threadIdx.x; w < c1; w += kBlk) {
            reinterpret_cast<uint4 *>(cflags)[w] = make_uint4(0u, 0u, 0u, 0u);
            if (zmask)
                for (int q = 0; q < 16; ++q) zmask[w * 16 + q] = 0ull;
            uint32_t nb = (far_cur || a.nbits) ? nonzero_bytes(reinterpret_cast<const uint4 *>(nflags)[w]) : 0u;
            if (far_cur) {
                const uint32_t cand = nb | nonzero_bytes(reinterpret_cast<const uint4 *>(far_cur)[w]);
                const uint32_t held = held_back(a.dist, w * 16, cand, T, &cnt, &inv);
                reinterpret_cast<uint4 *>(far_next)[w] = bytes_of_bits(held);
                nb = cand & ~held;
            }
            if (a.nbits) a.nbits[w] = (uint16_t)nb;
        }
        if (far_cur) {
            __syncthreads();
            if (cnt) {
                atomicAdd(&sh_far_cnt, cnt);
                atomicMax(&sh_far_inv, inv);
            }
            __syncthreads();
            if (threadIdx.x == 0 && sh_far_cnt) {
                atomicAdd(ctl_next + kFarCountWord, (unsigned long long)sh_far_cnt);
                atomicMax(ctl_next + kFarMaxInvWord, (unsigned long long)sh_far_inv);
            }
        }
    }
    const int64_t lo = a.off[k] + j * kDenseChunk;
    const int64_t hi = min((int64_t)a.off[k + 1], lo + kDenseChunk);
    if (lo >= hi) return;  // uniform per block
    // item it of thread t is member lo + it*kBlk + t: consecutive lanes read
    // consecutive members (and nearby flag bytes), one cache line per 32 lanes
    int32_t u[kDenseItems];
    uint2 sd[kDenseItems];
    bool on[kDenseItems];
#pragma unroll
    for (int it = 0; it < kDenseItems; ++it) {
        const int64_t m = min(lo + (int64_t)it * kBlk + threadIdx.x, hi - 1);
        u[it] = a.mem_u[m];
    }
    int32_t x[2] = {0, 0}, tot[2];
    uint32_t du[kDenseItems];
    // the flag bytes of all items are loaded before any is tested (a test
    // between the loads made each load wait for the previous one)
    uint32_t fl[kDenseItems];
#pragma unroll
    for (int it = 0; it < kDenseItems; ++it) fl[it] = nflags[u[it]];
    if (far_cur) {
#pragma unroll
        for (int it = 0; it < kDenseItems; ++it) fl[it] |= far_cur[u[it]];
    }
#pragma unroll
    for (int it = 0; it < kDenseItems; ++it) on[it] = (lo + (int64_t)it * kBlk + threadIdx.x < hi) && fl[it] != 0u;
    // arc ranges only of the members in the frontier (R-MAT 20: 2.25 -> 2.17 ms)
#pragma unroll
    for (int it = 0; it < kDenseItems; ++it)
        sd[it] = on[it] ? a.mem_sd[min(lo + (int64_t)it * kBlk + threadIdx.x, hi - 1)] : make_uint2(0u, 0u);
#pragma unroll
    for (int it = 0; it < kDenseItems; ++it) {
        if (far_cur) {
            du[it] = a.dist[u[it]];  // u[it] is a member (a vertex below n) even when off
            on[it] = on[it] && du[it] < T;
        }
        if (on[it]) {
            x[0] += 1;
            x[1] += (int32_t)sd[it].y;
        }
    }
    block_scan<2>(x, tot);
    if (threadIdx.x == 0)
        sh_base = tot[0] ? atomicAdd(ctl_next + k * kCtrStride, (unsigned long long)tot[0] | ((unsigned long long)tot[1] << 32))
                         : 0ull;
    __syncthreads();
    int32_t pos = (int32_t)(sh_base & 0xFFFFFFFFull) + x[0];
    int32_t spos = (int32_t)(sh_base >> 32) + x[1];
#pragma unroll
    for (int it = 0; it < kDenseItems; ++it) {
        if (on[it]) {
            a.qse[k][pos] = make_uint2(sd[it].x, (uint32_t)u[it]);
            a.qs[k][pos] = spos;
            ++pos;
            spos += (int32_t)sd[it].y;
        }
    }
}

__global__ __launch_bounds__(kBlk) void k_filter_dense(DenseFilterArgs a) {
    filter_dense(a, blockIdx.x, a.nflags, a.cflags, a.zmask, a.ctl_next, a.ctl_zero, a.far_cur, a.far_next,
                 a.threshold);
}

// ---------------------------------------------------------------------------
// Device-driven loop: one cooperative launch runs every iteration (advance,
// grid barrier, filter, grid barrier, convergence test) without returning to
// the host.  All blocks are co-resident (cooperative launch), block b stays
// on XCD b % 8 for the whole query, so its partition's distances stay in
// that XCD's L2 across iterations.

// Grid barrier: arrival counter + generation.  Thread 0 of each block
// publishes the block's writes with an agent-scope fence, arrives, and waits
// for the generation to move; the last arrival resets the counter and moves
// it.  The wait is bounded: after spin_ticks of the constant-rate clock the
// block marks the loop failed (status 3) and moves the generation itself, so
// that every block leaves instead of waiting forever.  Returns false once the
// loop has failed.
__device__ __forceinline__ bool grid_sync(LoopState *ls, unsigned nblocks, uint64_t spin_ticks) {
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long g = __hip_atomic_load(&ls->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned long long arrived =
            __hip_atomic_fetch_add(&ls->bar_count, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1ull;
        if (arrived == nblocks) {
            __hip_atomic_store(&ls->bar_count, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ls->bar_gen, g + 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(&ls->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                if (wall_clock64() - t0 > spin_ticks) {
                    __hip_atomic_store(&ls->status, 3ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&ls->bar_gen, g + 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __threadfence();
        ok = __hip_atomic_load(&ls->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 3ull;
    }
    __syncthreads();
    return ok != 0;
}

struct PersistArgs {
    FilterArgs fg;        // iteration-independent filter arguments
    DenseFilterArgs fd;
    const uint2 *padj;
    uint32_t *dist;
    const int32_t *ro_in;
    const uint2 *adj_in;
    uint8_t *flags[2];
    uint8_t *far[2];      // NULL when the near-far split is off
    unsigned long long *ctl;
    int32_t n, m, ngroups;
    int32_t max_iters, alpha_x16, beta, direction, filter, dense_ratio;
    const uint32_t *bits;  // the current frontier's bitmap (pull)
    int32_t part_pull;     // pull over the partitioned layout (symmetric graphs)
    uint32_t delta;
    uint64_t spin_ticks;
    // queued loop, small rounds: the CSR as given, the candidate lists (in
    // kCandRegions regions of cand_region entries) and their counters
    const int32_t *ro;
    const uint2 *adj;
    int32_t *cand[2];
    unsigned long long *ccount;  // 3 rounds x kCandRegions
    unsigned long long *rstat;   // small-round statistics by region (see kStat*)
    uint32_t *bound;             // relaxation filter (NULL: pre-read dist)
    int32_t cand_region;
    int32_t small;
    int32_t local_hops;  // small rounds: hops expanded inside the block before appending (1 = none)
    int8_t *phase_log;  // timing: phase each launch ran (NULL: off)
    int64_t phase_log_cap;
};

// Totals of the frontier in a counter slot, and partition kb's share.
struct SlotTotals {
    int64_t Fs, Es, far_cnt;
    int32_t Fk, Ek;
    uint32_t far_min;
};

template <int NP>
__device__ __forceinline__ SlotTotals slot_totals(const unsigned long long *cur, int kb) {
    SlotTotals t{0, 0, 0, 0, 0, 0u};
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const unsigned long long c = __hip_atomic_load(cur + k * kCtrStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t f = (int32_t)(c & 0xFFFFFFFFull), e = (int32_t)(c >> 32);
        t.Fs += f;
        t.Es += e;
        if (k == kb) {
            t.Fk = f;
            t.Ek = e;
        }
    }
    t.far_cnt = (int64_t)__hip_atomic_load(cur + kFarCountWord, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    t.far_min = ~(uint32_t)__hip_atomic_load(cur + kFarMaxInvWord, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return t;
}

template <int WT>
__device__ __forceinline__ uint32_t next_threshold_dev(uint32_t far_min, uint32_t delta) {
    const uint32_t t = plus<WT>(far_min, delta);
    return t > far_min ? t : far_min + 1u;
}

// Direction of round iter.  AUTO: push -> pull when the frontier's out-arcs
// reach m / alpha (Es * alpha_x16 >= 16 m); pull -> push when the frontier
// holds fewer than n / beta vertices (the two switching rules of Beamer et
// al., with hysteresis: prev is the direction of the previous round).
__device__ __forceinline__ bool pick_pull(const PersistArgs &a, int64_t iter, int64_t Es, int64_t Fs, bool prev) {
    switch (a.direction) {
        case 1: return false;
        case 2: return true;
        case 3: return (iter & 1) != 0;
        default:
            if (a.alpha_x16 <= 0) return false;
            if (prev) return Fs * a.beta >= (int64_t)a.n;
            return Es * a.alpha_x16 >= (int64_t)16 * a.m;
    }
}

// One block's share of a pull round (blocks vb of nvb = pull_blocks()).
template <int WT, int NP>
__device__ __forceinline__ void pull_share(const PersistArgs &a, uint8_t *nf, int64_t vb) {
    if constexpr (WT == 2) {
        pull_block_bfs(a.n, a.ro_in, a.adj_in, a.dist, a.bits, nf, a.bound, vb, kInfU32);
    } else if constexpr (NP == kMaxParts) {
        if (a.part_pull) pull_part_block<WT>(a.n, a.fg.pro, a.padj, a.dist, a.bits, nf, a.bound, vb);
        else pull_block<WT>(a.n, a.ro_in, a.adj_in, a.dist, a.bits, nf, a.bound, vb);
    } else {
        pull_block<WT>(a.n, a.ro_in, a.adj_in, a.dist, a.bits, nf, a.bound, vb);
    }
}

template <int WT, int NP>
__device__ __forceinline__ int64_t pull_blocks(const PersistArgs &a) {
    const int64_t chunks = ((int64_t)a.n + kBlk - 1) / kBlk;
    return (WT != 2 && NP == kMaxParts && a.part_pull) ? chunks * kMaxParts : chunks;
}

template <int WT, int NP>
__global__ __launch_bounds__(kBlk) void k_persistent(PersistArgs a) {
    LoopState *ls = reinterpret_cast<LoopState *>(a.ctl + kLoopStateWord);
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int kb = (int)(b % NP);
    const int64_t jb = b / NP, B = G / NP;
    bool prev_pull = false;  // every block takes the same decisions from the same counters
    for (int64_t iter = 0;; ++iter) {
        const SlotTotals t = slot_totals<NP>(a.ctl + (iter % kCtlSlots) * kSlotWords, kb);
        if ((t.Fs == 0 && t.far_cnt == 0) || iter >= a.max_iters) {
            if (b == 0 && threadIdx.x == 0) {
                ls->status = t.Fs == 0 && t.far_cnt == 0 ? 1ull : 2ull;
                ls->iter = (unsigned long long)iter;
            }
            break;
        }
        // An empty frontier with held-back vertices: this round only raises
        // the near-far threshold and filters.
        const bool idle = t.Fs == 0;
        const bool pull = !idle && pick_pull(a, iter, t.Es, t.Fs, prev_pull);
        prev_pull = pull;
        uint8_t *cf = a.flags[iter & 1];
        uint8_t *nf = a.flags[(iter + 1) & 1];
        if (idle) {
            if (b == 0 && threadIdx.x == 0)
                __hip_atomic_store(&ls->threshold, (unsigned long long)next_threshold_dev<WT>(t.far_min, a.delta),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (pull) {
            const int64_t nvb = pull_blocks<WT, NP>(a);
            for (int64_t vb = b; vb < nvb; vb += G) pull_share<WT, NP>(a, nf, vb);
        } else {
            const int32_t per = (int32_t)max<int64_t>(kMinChunk, ((int64_t)t.Ek + B - 1) / B);
            push_range<WT, false>(a.padj, a.dist, a.fg.qse[kb], a.fg.qs[kb], t.Fk, t.Ek, per, jb, nf,
                                  CandOut{nullptr, nullptr, 0}, a.bound);
        }
        if (!grid_sync(ls, (unsigned)G, a.spin_ticks)) break;
        unsigned long long *cn = a.ctl + ((iter + 1) % kCtlSlots) * kSlotWords;
        unsigned long long *cz = a.ctl + ((iter + 2) % kCtlSlots) * kSlotWords;
        const uint32_t T =
            (uint32_t)__hip_atomic_load(&ls->threshold, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint8_t *fc = a.far[0] ? a.far[iter & 1] : nullptr;
        uint8_t *fn = a.far[0] ? a.far[(iter + 1) & 1] : nullptr;
        const bool dense = a.filter == 2 || (a.filter == 0 && t.Fs * a.dense_ratio >= a.n);
        if (dense) {
            const int64_t nvb = (int64_t)a.fd.chunks * NP;
            for (int64_t vb = b; vb < nvb; vb += G) filter_dense(a.fd, vb, nf, cf, nullptr, cn, cz, fc, fn, T);
        } else {
            for (int64_t vb = b; vb < a.ngroups; vb += G) filter_group<NP>(a.fg, vb, nf, cf, cn, cz, fc, fn, T);
        }
        if (b == 0 && threadIdx.x == 0 && !idle) {
            ls->frontier_sum += (unsigned long long)t.Fs;
            if ((unsigned long long)t.Fs > ls->frontier_max) ls->frontier_max = (unsigned long long)t.Fs;
            if (pull) {
                ls->arcs_pulled += (unsigned long long)a.m;
                ls->pull_iters += 1ull;
            } else {
                ls->edges_pushed += (unsigned long long)t.Es;
                ls->push_frontier_sum += (unsigned long long)t.Fs;
            }
        }
        if (!grid_sync(ls, (unsigned)G, a.spin_ticks)) break;
    }
}

// ---------------------------------------------------------------------------
// Queued loop: the host enqueues launches of one step kernel ahead of the
// device, in chunks, without waiting for frontier sizes.  The step kernel is
// a small state machine kept in the loop state: each launch runs one phase of
// the round it finds there and writes the phase the next launch runs (by
// launch parity, so blocks of one launch never see the next launch's state).
// The kernel boundary orders the phases (no grid barrier).  Once some phase
// finds the frontier empty (or the cap reached) it ends the query, after
// which the launches still queued return at once.
//
// Phases of round r:
//   advance      push (or pull) from the round's queues; then filter
//   filter       the flag scan that builds the next round's queues
//   after-small  round r - 1 was a small round: if its candidate list did not
//                overflow, round r is another small round (advance and filter
//                in one launch); otherwise this launch runs round r - 1's
//                filter and round r continues with a normal advance
// A round's candidate list is split into kCandRegions regions with their own
// counters (block b appends to region b % kCandRegions), so that appends do
// not all contend for one counter.

__device__ __forceinline__ unsigned long long loop_status(const LoopState *ls) {
    return __hip_atomic_load(&ls->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

enum : int { kPhaseAdvance = 0, kPhaseFilter = 1, kPhaseAfterSmall = 2 };
// phase log entries (timing): what a launch ran
enum : int8_t { kRanAdvance = 1, kRanFilter = 2, kRanSmall = 3, kRanIdle = 4 };

// Candidate regions of one round, summed by a block: sPre[r] = candidates in
// regions before r (each region capped at its size), sPre[kCandRegions] = N.
// Returns the uncapped total; *ovf = some region overflowed.
__device__ __forceinline__ int64_t cand_prefix(const unsigned long long *cnt, int32_t rsize, int32_t *sPre,
                                               int *sOvf) {
    __shared__ unsigned long long sTot;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const unsigned long long c = cnt[lane];
        const int32_t cc = (int32_t)min(c, (unsigned long long)rsize);
        int32_t inc = cc;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t t = __shfl_up(inc, off, 64);
            if (lane >= off) inc += t;
        }
        sPre[lane] = inc - cc;
        if (lane == 63) sPre[64] = inc;
        const unsigned long long any = __ballot(c > (unsigned long long)rsize);
        unsigned long long tot = c;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) tot += __shfl_xor(tot, off, 64);
        if (lane == 0) {
            *sOvf = any != 0ull;
            sTot = tot;
        }
    }
    __syncthreads();
    return (int64_t)sTot;
}

// Small round r (push only): the frontier is the candidate list of round
// r - 1.  Each candidate is claimed by an atomic clear of its flag byte (so
// repeats expand once, and the flags of the round are left clear); a claimed
// vertex with at most kLight arcs is expanded by its own thread
// (thread-mapped), the others are gathered in LDS and expanded by the whole
// block over the prefix sum of their degrees (block-mapped, the push's
// search).  Improved vertices are marked in the next flags and appended to
// the next candidate list.  Used only on graphs whose largest degree is small
// (see run_queued), so one block's share stays bounded.
//
// Local hops (local_hops > 1): the light vertices a block improves are not
// all handed to the next round; up to kLocalCap of them are kept in LDS with
// the candidate distance that improved them and expanded again by the same
// block, for up to local_hops - 1 further hops, before the improvements of
// the last hop (and any that do not fit) are appended.  Expanding v with its
// own candidate c is a relaxation from a real path (dist[v] <= c once the
// atomic has executed); if another relaxation lowered dist[v] further, that
// one marked and appended (or expanded) v itself, so every decrease is still
// followed by an expansion with that value or a smaller one.  The marks of
// locally expanded vertices stay set, which only costs a repeated expansion
// if a flag scan follows.  On bounded-degree graphs of long diameter this
// takes several hops of the wavefront per launch instead of one.
constexpr int kLight = 8;
constexpr int kLocalCap = 1024;

// Thread-mapped expansion of up to kLight arcs of v (first arc st, deg arcs)
// with distance du: take[it] says arc it improved its destination vv[it] to
// nd[it] (atomic min and mark issued).
template <int WT, bool O32>
__device__ __forceinline__ void expand_light(const PersistArgs &a, uint8_t *nf, bool on, int32_t st, int32_t deg,
                                             uint32_t du, uint32_t (&vv)[kLight], uint32_t (&nd)[kLight],
                                             bool (&take)[kLight]) {
    uint2 arc[kLight];
    uint32_t cur[kLight];
#pragma unroll
    for (int it = 0; it < kLight; ++it)
        arc[it] = (on && it < deg) ? load_arc(elem<O32>(a.adj, (uint32_t)(st + it))) : make_uint2(0u, 0u);
#pragma unroll
    for (int it = 0; it < kLight; ++it) {
        nd[it] = plus<WT>(du, arc[it].y);
        // unguarded: an item past the degree reads vertex 0 (its arc is (0, 0));
        // a guarded load with a default value made each item wait for the last
        cur[it] = *elem<O32>(a.bound ? a.bound : a.dist, arc[it].x);
    }
#pragma unroll
    for (int it = 0; it < kLight; ++it) {
        take[it] = on && it < deg && nd[it] < cur[it];
        vv[it] = arc[it].x;
        if (take[it]) {
            if (a.bound)
                relax_bound<O32>(a.dist, a.bound, nf, arc[it].x, nd[it]);
            else
                relax_commit<O32>(a.dist, nf, arc[it].x, nd[it]);
        }
    }
}

// Routes a thread's improvements: into the block's LDS list for the next
// local hop while there is room (glob[it] = false), else to the global
// candidate list (glob[it] = true).
__device__ __forceinline__ void route_local(bool keep, const uint32_t (&vv)[kLight], const uint32_t (&nd)[kLight],
                                            const bool (&take)[kLight], bool (&glob)[kLight], uint32_t *lv,
                                            uint32_t *ld, int32_t *ln) {
#pragma unroll
    for (int it = 0; it < kLight; ++it) {
        glob[it] = take[it];
        if (take[it] && keep) {
            const int32_t p = atomicAdd(ln, 1);
            if (p < kLocalCap) {
                lv[p] = vv[it];
                ld[p] = nd[it];
                glob[it] = false;
            }
        }
    }
}

template <int WT, bool O32>
__device__ __forceinline__ void small_round(const PersistArgs &a, int64_t r, LoopState *ls, const int32_t *sPre) {
    __shared__ int32_t hS[kBlk + 1];
    __shared__ int32_t hStart[kBlk];
    __shared__ int32_t hDeg[kBlk];
    __shared__ uint32_t hDu[kBlk];
    __shared__ int32_t hCount;
    __shared__ uint32_t lV[2][kLocalCap], lD[2][kLocalCap];
    __shared__ int32_t lN[2];
    const int hops = a.local_hops > 1 ? a.local_hops : 1;
    const int64_t nin = sPre[kCandRegions];
    const int32_t R = a.cand_region;
    const int32_t *__restrict__ cin = a.cand[r & 1];
    const int region = (int)(blockIdx.x % kCandRegions);
    const CandOut co{a.cand[(r + 1) & 1] + (int64_t)region * R, a.ccount + ((r + 1) % 3) * kCandRegions + region, R};
    unsigned int *curw = reinterpret_cast<unsigned int *>(a.flags[r & 1]);
    uint8_t *nf = a.flags[(r + 1) & 1];
    int32_t st_win = 0, st_arcs = 0;
    // candidates are dealt evenly over the blocks (at most one pass of 256
    // each when they fit), so that a short list still spreads over many
    // blocks -- with local hops each block then grows a small local frontier
    const int64_t per = (nin + gridDim.x - 1) / gridDim.x;
    const int64_t cbeg = (int64_t)blockIdx.x * per, cend = min(nin, cbeg + per);
    for (int64_t j0 = cbeg; j0 < cend; j0 += kBlk) {
        if (threadIdx.x == 0) {
            hCount = 0;
            lN[0] = 0;
        }
        __syncthreads();
        const int64_t j = j0 + threadIdx.x;
        int32_t v = -1;
        if (j < cend) {
            int q = 0;  // region of j: largest q with sPre[q] <= j
#pragma unroll
            for (int b = kCandRegions / 2; b >= 1; b >>= 1) q = (sPre[q + b] <= j) ? q + b : q;
            v = cin[(int64_t)q * R + (j - sPre[q])];
        }
        bool win = false;
        if (v >= 0) {
            const unsigned int m = 0xFFu << ((v & 3) * 8);
            win = (atomicAnd(curw + (v >> 2), ~m) & m) != 0u;
        }
        int32_t st = 0, deg = 0;
        uint32_t du = 0;
        if (win) {
            st = a.ro[v];
            deg = a.ro[v + 1] - st;
            du = a.dist[v];
            st_win += deg > 0 ? 1 : 0;  // as the filter, which drops vertices without arcs
            st_arcs += deg;
        }
        const bool light = win && deg <= kLight;
        if (win && !light) {
            const int h = atomicAdd(&hCount, 1);
            hStart[h] = st;
            hDeg[h] = deg;
            hDu[h] = du;
        }
        {  // thread-mapped expansion
            uint32_t nd[kLight], vv[kLight];
            bool take[kLight], glob[kLight];
            expand_light<WT, O32>(a, nf, light, st, deg, du, vv, nd, take);
            route_local(hops > 1, vv, nd, take, glob, lV[0], lD[0], &lN[0]);
            block_append<kLight>(co, vv, glob);
        }
        __syncthreads();
        const int hc = hCount;
        if (hc > 0) {  // block-mapped expansion of the heavier vertices
            int32_t x[1] = {(int)threadIdx.x < hc ? hDeg[threadIdx.x] : 0}, tot[1];
            block_scan<1>(x, tot);
            if ((int)threadIdx.x < hc) hS[threadIdx.x] = x[0];
            for (int t = hc + threadIdx.x; t <= kBlk; t += kBlk) hS[t] = (t == hc) ? tot[0] : INT32_MAX;
            __syncthreads();
            const int32_t H = tot[0];
            for (int32_t x0b = 0; x0b < H; x0b += kBlk * kPushItems) {
                int32_t xr[kPushItems], pos[kPushItems];
#pragma unroll
                for (int it = 0; it < kPushItems; ++it) {
                    xr[it] = min(x0b + (int32_t)threadIdx.x + it * kBlk, H - 1);
                    pos[it] = 0;
                }
#pragma unroll
                for (int b = kBlk / 2; b >= 1; b >>= 1) {
#pragma unroll
                    for (int it = 0; it < kPushItems; ++it) {
                        const int32_t p = pos[it] + b;
                        pos[it] = (hS[p] <= xr[it]) ? p : pos[it];
                    }
                }
                uint2 arc[kPushItems];
#pragma unroll
                for (int it = 0; it < kPushItems; ++it)
                    arc[it] = load_arc(elem<O32>(a.adj, (uint32_t)(hStart[pos[it]] + (xr[it] - hS[pos[it]]))));
                uint32_t nd[kPushItems], cur[kPushItems], vv[kPushItems];
                bool take[kPushItems];
#pragma unroll
                for (int it = 0; it < kPushItems; ++it) {
                    nd[it] = plus<WT>(hDu[pos[it]], arc[it].y);
                    cur[it] = *elem<O32>(a.bound ? a.bound : a.dist, arc[it].x);
                }
#pragma unroll
                for (int it = 0; it < kPushItems; ++it) {
                    take[it] = x0b + (int32_t)threadIdx.x + it * kBlk < H && nd[it] < cur[it];
                    vv[it] = arc[it].x;
                    if (take[it]) {
                        if (a.bound)
                            relax_bound<O32>(a.dist, a.bound, nf, arc[it].x, nd[it]);
                        else
                            relax_commit<O32>(a.dist, nf, arc[it].x, nd[it]);
                    }
                }
                block_append<kPushItems>(co, vv, take);
            }
        }
        __syncthreads();  // LDS reuse
        // local hops over the light vertices this block improved
        for (int h = 1; h < hops; ++h) {
            const int sp = (h - 1) & 1, dp = h & 1;
            const int32_t nloc = min(lN[sp], kLocalCap);
            if (nloc == 0) break;  // uniform: LDS read after a barrier
            if (threadIdx.x == 0) lN[dp] = 0;
            __syncthreads();
            const bool last = h == hops - 1;
            for (int32_t i0 = 0; i0 < nloc; i0 += kBlk) {
                const int32_t i = i0 + (int32_t)threadIdx.x;
                int32_t lst = 0, ldeg = 0;
                uint32_t lv = 0, lc = 0;
                if (i < nloc) {
                    lv = lV[sp][i];
                    lc = lD[sp][i];
                    lst = a.ro[lv];
                    ldeg = a.ro[lv + 1] - lst;
                }
                const bool lon = i < nloc && ldeg > 0 && ldeg <= kLight;
                st_win += lon ? 1 : 0;
                st_arcs += lon ? ldeg : 0;
                uint32_t nd[kLight], vv[kLight];
                bool take[kLight], glob[kLight];
                expand_light<WT, O32>(a, nf, lon, lst, ldeg, lc, vv, nd, take);
                route_local(!last, vv, nd, take, glob, lV[dp], lD[dp], &lN[dp]);
                // a heavier vertex is expanded by the next round: it is already
                // marked (its improvement marked it); append it
                uint32_t hv[1] = {lv};
                bool hb[1] = {i < nloc && ldeg > kLight};
                block_append<kLight>(co, vv, glob);
                block_append<1>(co, hv, hb);
            }
            __syncthreads();
        }
    }
    // statistics per region (so that blocks rarely share an address): the
    // round's expanded vertices, and running totals folded in at the end
    int32_t x[2] = {st_win, st_arcs}, tot[2];
    block_scan<2>(x, tot);
    if (threadIdx.x == 0 && tot[0] > 0) {
        atomicAdd(a.rstat + (r % 3) * kCandRegions + region, (unsigned long long)tot[0]);
        atomicAdd(a.rstat + kStatFrontier + region, (unsigned long long)tot[0]);
        atomicAdd(a.rstat + kStatEdges + region, (unsigned long long)tot[1]);
    }
}

// Query end (lead thread): fold the small rounds' regional totals into the
// loop state, then publish the status.
__device__ __forceinline__ void end_query(const PersistArgs &a, LoopState *ls, int64_t iter, unsigned long long st) {
    if (a.rstat) {
        unsigned long long f = 0, e = 0;
        for (int q = 0; q < kCandRegions; ++q) {
            f += a.rstat[kStatFrontier + q];
            e += a.rstat[kStatEdges + q];
        }
        ls->frontier_sum += f;
        ls->push_frontier_sum += f;
        ls->edges_pushed += e;
    }
    ls->iter = (unsigned long long)iter;
    __hip_atomic_store(&ls->status, st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Normal filter of round r (flag scan), shared by the filter phase and the
// after-small phase.  Fs: the size estimate of the next frontier.
template <int NP>
__device__ __forceinline__ void step_filter(const PersistArgs &a, int64_t r, const LoopState *ls, int64_t Fs) {
    const int64_t G = gridDim.x, b = blockIdx.x;
    uint8_t *cf = a.flags[r & 1];
    uint8_t *nf = a.flags[(r + 1) & 1];
    unsigned long long *cn = a.ctl + ((r + 1) % kCtlSlots) * kSlotWords;
    unsigned long long *cz = a.ctl + ((r + 2) % kCtlSlots) * kSlotWords;
    const uint32_t T = (uint32_t)ls->threshold;
    const uint8_t *fc = a.far[0] ? a.far[r & 1] : nullptr;
    uint8_t *fn = a.far[0] ? a.far[(r + 1) & 1] : nullptr;
    const bool dense = a.filter == 2 || (a.filter == 0 && Fs * a.dense_ratio >= a.n);
    if (dense) {
        const int64_t nvb = (int64_t)a.fd.chunks * NP;
        for (int64_t vb = b; vb < nvb; vb += G) filter_dense(a.fd, vb, nf, cf, nullptr, cn, cz, fc, fn, T);
    } else {
        for (int64_t vb = b; vb < a.ngroups; vb += G) filter_group<NP>(a.fg, vb, nf, cf, cn, cz, fc, fn, T);
    }
}

template <int WT, int NP, bool O32>
__global__ __launch_bounds__(kBlk) void k_step(PersistArgs a, int64_t launch) {
    __shared__ int32_t sPre[kCandRegions + 1];
    __shared__ int sOvf;
    LoopState *ls = reinterpret_cast<LoopState *>(a.ctl + kLoopStateWord);
    if (loop_status(ls) != 0ull) return;
    const int par = (int)(launch & 1);
    const int64_t r = (int64_t)ls->st_round[par];
    const int phase = (int)ls->st_phase[par];
    const int64_t G = gridDim.x, b = blockIdx.x;
    const bool lead = b == 0 && threadIdx.x == 0;
    int8_t ran = kRanIdle;
    int64_t next_r = r;
    int next_phase = -1;  // -1: the query ended in this launch
    const int32_t R = a.cand_region;
    if (phase == kPhaseAfterSmall) {
        const int64_t total = cand_prefix(a.ccount + (r % 3) * kCandRegions, R, sPre, &sOvf);
        if (total == 0) {
            // round r - 1 improved nothing: the query ends; round r - 1 counts
            // if some vertex it claimed had arcs
            if (lead) {
                unsigned long long act = 0;
                for (int q = 0; q < kCandRegions; ++q) act += a.rstat[((r - 1) % 3) * kCandRegions + q];
                end_query(a, ls, act ? r : r - 1, 1ull);
            }
        } else if (!sOvf && r < a.max_iters) {
            if (b == 0 && threadIdx.x < kCandRegions)  // expanded-vertex counters of round r + 1
                a.rstat[((r + 1) % 3) * kCandRegions + threadIdx.x] = 0ull;
            if (b == 0 && threadIdx.x < kCandRegions) a.ccount[((r + 2) % 3) * kCandRegions + threadIdx.x] = 0ull;
            // the queue counter slot a filter of round r would clear (a filter of
            // round r + 1 may run later and add into it)
            if (b == 0)
                for (int t = threadIdx.x; t < kSlotWords; t += kBlk) a.ctl[((r + 2) % kCtlSlots) * kSlotWords + t] = 0ull;
            if (lead) {
                ls->small_rounds += 1ull;
                ls->last_pull[r & 1] = 0ull;
            }
            small_round<WT, O32>(a, r, ls, sPre);
            ran = kRanSmall;
            next_r = r + 1;
            next_phase = kPhaseAfterSmall;
        } else if (r >= a.max_iters) {
            if (lead) end_query(a, ls, r, 2ull);
        } else {
            // too many candidates: round r - 1's filter, then a normal round r
            step_filter<NP>(a, r - 1, ls, total);
            ran = kRanFilter;
            next_phase = kPhaseAdvance;
        }
    } else if (phase == kPhaseAdvance) {
        const int kb = (int)(b % NP);
        const int64_t jb = b / NP, B = G / NP;
        const SlotTotals t = slot_totals<NP>(a.ctl + (r % kCtlSlots) * kSlotWords, kb);
        if ((t.Fs == 0 && t.far_cnt == 0) || r >= a.max_iters) {
            if (lead) end_query(a, ls, r, t.Fs == 0 && t.far_cnt == 0 ? 1ull : 2ull);
        } else {
            next_phase = kPhaseFilter;
            // counters of round r + 2's list (last read when round r - 1 began)
            if (b == 0 && threadIdx.x < kCandRegions) a.ccount[((r + 2) % 3) * kCandRegions + threadIdx.x] = 0ull;
            if (t.Fs == 0) {  // held-back vertices only: raise the threshold, the filter releases them
                if (lead) {
                    ls->threshold = next_threshold_dev<WT>(t.far_min, a.delta);
                    ls->last_pull[r & 1] = 0ull;
                }
            } else {
                const bool pull = pick_pull(a, r, t.Es, t.Fs, ls->last_pull[(r + 1) & 1] != 0ull);
                if (lead) {
                    ls->last_pull[r & 1] = pull ? 1ull : 0ull;
                    ls->frontier_sum += (unsigned long long)t.Fs;
                    if ((unsigned long long)t.Fs > ls->frontier_max) ls->frontier_max = (unsigned long long)t.Fs;
                    if (pull) {
                        ls->arcs_pulled += (unsigned long long)a.m;
                        ls->pull_iters += 1ull;
                    } else {
                        ls->edges_pushed += (unsigned long long)t.Es;
                        ls->push_frontier_sum += (unsigned long long)t.Fs;
                    }
                }
                uint8_t *nf = a.flags[(r + 1) & 1];
                if (pull) {
                    const int64_t nvb = pull_blocks<WT, NP>(a);
                    for (int64_t vb = b; vb < nvb; vb += G) pull_share<WT, NP>(a, nf, vb);
                } else {
                    // Candidate appends only when this round cannot improve many
                    // more vertices than the list holds (a too-long list just
                    // sends the next round to the flag scan).
                    const bool app = a.small && t.Es <= 4 * (int64_t)R * kCandRegions;
                    const int region = (int)(b % kCandRegions);
                    const CandOut co{app ? a.cand[(r + 1) & 1] + (int64_t)region * R : nullptr,
                                     a.ccount + ((r + 1) % 3) * kCandRegions + region, R};
                    // at least kMinChunk arcs per block: small frontiers use few blocks
                    const int32_t per = (int32_t)max<int64_t>(kMinChunk, ((int64_t)t.Ek + B - 1) / B);
                    push_range<WT, O32>(a.padj, a.dist, a.fg.qse[kb], a.fg.qs[kb], t.Fk, t.Ek, per, jb, nf, co,
                                        a.bound);
                    if (a.small && !app && lead) a.ccount[((r + 1) % 3) * kCandRegions] = (unsigned long long)R + 1ull;
                }
            }
            ran = kRanAdvance;
        }
    } else {  // kPhaseFilter
        const int64_t Fs = slot_totals<NP>(a.ctl + (r % kCtlSlots) * kSlotWords, 0).Fs;
        step_filter<NP>(a, r, ls, Fs);
        ran = kRanFilter;
        next_r = r + 1;
        next_phase = kPhaseAdvance;
        if (a.small && b == 0) {
            // the next round takes the candidate list if it did not overflow
            // and is not empty (block 0 reads the counters after its share of
            // the filter; the push that appended ended with the last launch)
            const int64_t total = cand_prefix(a.ccount + ((r + 1) % 3) * kCandRegions, R, sPre, &sOvf);
            if (!sOvf && total > 0) {
                next_phase = kPhaseAfterSmall;
                if (threadIdx.x < kCandRegions)  // expanded-vertex counters of round r + 1
                    a.rstat[((r + 1) % 3) * kCandRegions + threadIdx.x] = 0ull;
            }
        }
    }
    if (lead) {
        if (a.phase_log && launch < a.phase_log_cap) a.phase_log[launch] = ran;
        if (next_phase >= 0) {
            ls->st_round[par ^ 1] = (unsigned long long)next_r;
            ls->st_phase[par ^ 1] = (unsigned long long)next_phase;
        }
    }
}

// Membership lists: flag[k*(n+1)+u] = 1 when u has arcs into partition k.
__global__ void k_member_flags(int32_t n, int32_t np, const int32_t *__restrict__ pro, int32_t *__restrict__ cnt) {
    const int64_t total = (int64_t)np * n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int64_t k = i / n, u = i % n;
        cnt[k * ((int64_t)n + 1) + u] = pro[(u + 1) * np + k] > pro[u * np + k] ? 1 : 0;
    }
}

__global__ void k_member_scatter(int32_t n, int32_t np, const int32_t *__restrict__ pro,
                                 const int32_t *__restrict__ cnt, const int32_t *__restrict__ pos,
                                 int32_t *__restrict__ mem_u, uint2 *__restrict__ mem_sd, long long *off) {
    const int64_t total = (int64_t)np * n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int64_t k = i / n, u = i % n;
        const int64_t c = k * ((int64_t)n + 1) + u;
        if (cnt[c]) {
            const int32_t st = pro[u * np + k];
            mem_u[pos[c]] = (int32_t)u;
            mem_sd[pos[c]] = make_uint2((uint32_t)st, (uint32_t)(pro[(u + 1) * np + k] - st));
        }
    }
    if (blockIdx.x == 0 && threadIdx.x <= np) off[threadIdx.x] = pos[(int64_t)threadIdx.x * ((int64_t)n + 1)];
}

// ---------------------------------------------------------------------------
// graph build helpers

__global__ void k_pack_arcs(const int32_t *__restrict__ col, const uint32_t *__restrict__ w, int32_t m,
                            uint2 *__restrict__ adj) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        adj[e] = make_uint2((uint32_t)col[e], w[e]);
    }
}

// err bits: 1 = offsets, 2 = column out of range, 4 = bad binary32 weight
__global__ void k_validate(int32_t n, int32_t m, const int32_t *__restrict__ ro, const int32_t *__restrict__ col,
                           const uint32_t *__restrict__ w, int wt, unsigned int *err) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned int e = 0;
    for (int64_t v = tid; v <= n; v += stride) {
        if (v == 0 && ro[0] != 0) e |= 1u;
        if (v == n && ro[n] != m) e |= 1u;
        if (v < n && ro[v + 1] < ro[v]) e |= 1u;
    }
    for (int64_t i = tid; i < m; i += stride) {
        if (col[i] < 0 || col[i] >= n) e |= 2u;
        if (wt == 1) {
            const uint32_t b = w[i];
            if ((b & 0x80000000u) && b != 0x80000000u) e |= 4u;  // negative (-0 is allowed)
            if ((b & 0x7F800000u) == 0x7F800000u) e |= 4u;       // inf / NaN
        }
    }
    if (e) atomicOr(err, e);
}

__global__ void k_canon_negzero(uint2 *adj, int32_t m) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        if (adj[e].y == 0x80000000u) adj[e].y = 0u;
    }
}

__global__ void k_count_in(const uint2 *__restrict__ adj, int32_t m, int32_t *__restrict__ cnt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride)
        atomicAdd(cnt + adj[e].x, 1);
}

// Exclusive scan, one level: each block scans 1024 items (4 per thread) of
// in[0..len) into out, and writes its total to bsum[blockIdx.x].
constexpr int kScanItems = 4;
constexpr int kScanChunk = kBlk * kScanItems;

__global__ __launch_bounds__(kBlk) void k_scan_level(const int32_t *__restrict__ in, int64_t len,
                                                     int32_t *__restrict__ out, int32_t *__restrict__ bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t t = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < len) ? in[base + k] : 0;
        t += v[k];
    }
    int32_t x[1] = {t}, tot[1];
    block_scan<1>(x, tot);
    int32_t ex = x[0];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < len) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0 && bsum) bsum[blockIdx.x] = tot[0];
}

__global__ void k_scan_add(int32_t *__restrict__ out, int64_t len, const int32_t *__restrict__ boff) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) out[i] += boff[i / kScanChunk];
}

// One wave per row (grid-stride over rows).
#define FOR_EACH_ROW_BY_WAVE(u, n)                                                   \
    for (int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64; u < (n); \
         u += ((int64_t)gridDim.x * blockDim.x) / 64)

__global__ __launch_bounds__(kBlk) void k_scatter_in(int32_t n, const int32_t *__restrict__ ro,
                                                     const uint2 *__restrict__ adj,
                                                     const int32_t *__restrict__ ro_in, int32_t *__restrict__ fill,
                                                     uint2 *__restrict__ adj_in) {
    const int lane = threadIdx.x & 63;
    FOR_EACH_ROW_BY_WAVE(u, n) {
        for (int32_t e = ro[u] + lane; e < ro[u + 1]; e += 64) {
            const uint2 a = adj[e];
            const int32_t p = atomicAdd(fill + a.x, 1);
            adj_in[ro_in[a.x] + p] = make_uint2((uint32_t)u, a.y);
        }
    }
}

// Symmetric iff every row is strictly increasing and each arc u -> v of
// weight w has a reverse arc v -> u of the same weight bits.
__global__ __launch_bounds__(kBlk) void k_symmetry(int32_t n, const int32_t *__restrict__ ro,
                                                   const uint2 *__restrict__ adj, unsigned int *not_sym) {
    const int lane = threadIdx.x & 63;
    bool bad = false;
    FOR_EACH_ROW_BY_WAVE(u, n) {
        const int32_t r1 = ro[u + 1];
        for (int32_t e = ro[u] + lane; e < r1; e += 64) {
            const uint2 a = adj[e];
            if (e + 1 < r1 && adj[e + 1].x <= a.x) bad = true;
            int32_t lo = ro[a.x], hi = ro[a.x + 1];
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if ((int64_t)adj[mid].x < u) lo = mid + 1;
                else hi = mid;
            }
            if (lo >= ro[a.x + 1] || (int64_t)adj[lo].x != u || adj[lo].y != a.y) bad = true;
        }
    }
    if (__ballot(bad) && lane == 0) atomicOr(not_sym, 1u);
}

// Arcs with |u - v| < span (locality test for the push layout choice).
__global__ __launch_bounds__(kBlk) void k_locality(int32_t n, const int32_t *__restrict__ ro,
                                                   const uint2 *__restrict__ adj, int32_t span,
                                                   unsigned long long *near) {
    const int lane = threadIdx.x & 63;
    unsigned long long c = 0;
    FOR_EACH_ROW_BY_WAVE(u, n) {
        for (int32_t e = ro[u] + lane; e < ro[u + 1]; e += 64) {
            const int64_t d = (int64_t)adj[e].x - u;
            c += (d < span && d > -span) ? 1 : 0;
        }
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if (lane == 0 && c) atomicAdd(near, c);
}

// Partition layout: count the arcs of each row per destination partition.
__global__ __launch_bounds__(kBlk) void k_part_count(int32_t n, const int32_t *__restrict__ ro,
                                                     const uint2 *__restrict__ adj, int32_t np, int32_t psize,
                                                     int32_t *__restrict__ cnt) {
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)n + 1;
    FOR_EACH_ROW_BY_WAVE(u, n) {
        int32_t c[kMaxParts] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int32_t e0 = ro[u]; e0 < ro[u + 1]; e0 += 64) {
            const int32_t e = e0 + lane;
            const int p = (e < ro[u + 1]) ? (int)(adj[e].x / (uint32_t)psize) : -1;
#pragma unroll
            for (int k = 0; k < kMaxParts; ++k) c[k] += __popcll(__ballot(p == k));
        }
        if (lane < np) {
            int32_t mine = 0;
#pragma unroll
            for (int k = 0; k < kMaxParts; ++k)
                if (k == lane) mine = c[k];
            cnt[lane * stride + u] = mine;
        }
    }
}

// Vertices with at least one arc into partition k (queue capacity).
__global__ __launch_bounds__(kBlk) void k_part_caps(int32_t n, int32_t np, const int32_t *__restrict__ cnt,
                                                    unsigned long long *caps) {
    __shared__ unsigned int sc[kMaxParts];
    if (threadIdx.x < kMaxParts) sc[threadIdx.x] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)n + 1;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
        for (int k = 0; k < np; ++k)
            if (cnt[k * stride + u] > 0) atomicAdd(&sc[k], 1u);
    __syncthreads();
    if (threadIdx.x < np && sc[threadIdx.x]) atomicAdd(caps + threadIdx.x, (unsigned long long)sc[threadIdx.x]);
}

// Scatter arcs into the partition-major layout, keeping their order in the row.
__global__ __launch_bounds__(kBlk) void k_part_scatter(int32_t n, const int32_t *__restrict__ ro,
                                                       const uint2 *__restrict__ adj, int32_t psize,
                                                       const int32_t *__restrict__ pro, uint2 *__restrict__ padj) {
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)n + 1;
    const uint64_t lanemask_lt = (1ull << lane) - 1ull;
    FOR_EACH_ROW_BY_WAVE(u, n) {
        int32_t run[kMaxParts] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int32_t e0 = ro[u]; e0 < ro[u + 1]; e0 += 64) {
            const int32_t e = e0 + lane;
            const bool ok = e < ro[u + 1];
            const uint2 a = ok ? adj[e] : make_uint2(0u, 0u);
            const int p = ok ? (int)(a.x / (uint32_t)psize) : -1;
#pragma unroll
            for (int k = 0; k < kMaxParts; ++k) {
                const uint64_t msk = __ballot(p == k);
                if (p == k) padj[pro[k * stride + u] + run[k] + __popcll(msk & lanemask_lt)] = a;
                run[k] += __popcll(msk);
            }
        }
    }
}

// Partition-major offsets (k, u) -> vertex-major (u, k), so that the filter
// reads one contiguous record per frontier vertex.
__global__ void k_part_transpose(int32_t n, int32_t np, const int32_t *__restrict__ pm, int32_t *__restrict__ vm) {
    const int64_t total = ((int64_t)n + 1) * np;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int64_t u = i / np, k = i % np;
        vm[i] = pm[k * ((int64_t)n + 1) + u];
    }
}

// ---------------------------------------------------------------------------
// launch wrappers

static inline int grid_for(int64_t items, int per_block, int cap) {
    int64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

static hipError_t scan_exclusive(const int32_t *in, int64_t len, int32_t *out, int32_t *tmp, hipStream_t st);

// 32-bit byte offsets reach every arc, distance and flag of the graph.
static inline bool offsets32(const DevGraph &g) {
    return (uint64_t)std::max(g.m, 1) * sizeof(uint2) < (1ull << 32) && (uint64_t)g.n * sizeof(uint32_t) < (1ull << 32);
}

static inline int slot_of(int64_t i) { return (int)(((i % kCtlSlots) + kCtlSlots) % kCtlSlots); }

unsigned long long *counters_after(const Frontier &f, int64_t iter) { return f.ctl + slot_of(iter + 1) * kSlotWords; }

void read_counts(const unsigned long long *h, FrontierCounts *c) {
    for (int k = 0; k < kMaxParts; ++k) {
        c->F[k] = (int32_t)(h[k * kCtrStride] & 0xFFFFFFFFull);
        c->E[k] = (int32_t)(h[k * kCtrStride] >> 32);
    }
    c->far_count = (int64_t)h[kFarCountWord];
    c->far_min = ~(uint32_t)h[kFarMaxInvWord];
}

uint32_t next_threshold(uint32_t far_min, uint32_t delta, int wt) {
    uint32_t t;
    if (wt == 1) {
        float a, d;
        std::memcpy(&a, &far_min, 4);
        std::memcpy(&d, &delta, 4);
        float r = a + d;
        if (!(r <= 3.40282347e38f)) r = 3.40282347e38f;
        std::memcpy(&t, &r, 4);
    } else {
        const uint64_t r = (uint64_t)far_min + delta;
        t = r >= 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)r;
    }
    return t > far_min ? t : far_min + 1u;
}

int64_t FrontierCounts::Fsum() const {
    int64_t s = 0;
    for (int k = 0; k < kMaxParts; ++k) s += F[k];
    return s;
}

int64_t FrontierCounts::Esum() const {
    int64_t s = 0;
    for (int k = 0; k < kMaxParts; ++k) s += E[k];
    return s;
}

hipError_t launch_init(const DevGraph &g, uint32_t *dist, int32_t src, const Frontier &f, uint32_t threshold,
                       bool use_far, hipStream_t st) {
    InitArgs a;
    a.dist = dist;
    a.n = g.n;
    a.np = g.np;
    a.inf = g.wt == 1 ? kInfF32 : kInfU32;
    a.src = src;
    a.pro = g.pro;
    a.flags0 = f.flags[0];
    a.flags1 = f.flags[1];
    a.bits = f.bits;
    a.ccount = f.ccount;
    a.rstat = f.rstat;
    a.bound = f.bound;
    a.far0 = use_far ? f.far[0] : nullptr;
    a.far1 = use_far ? f.far[1] : nullptr;
    a.threshold = threshold;
    a.nflag = f.nflag;
    for (int k = 0; k < kMaxParts; ++k) {
        a.qse[k] = f.qse[k];
        a.qs[k] = f.qs[k];
    }
    a.ctl = f.ctl;
    const int grid = grid_for(g.n, kBlk * 4, 8192);
    hipLaunchKernelGGL(k_init, dim3(grid), dim3(kBlk), 0, st, a);
    return hipGetLastError();
}

template <int WT>
static void push_dispatch(const DevGraph &g, dim3 gd, dim3 bd, hipStream_t st, const PushArgs &a) {
    if (offsets32(g)) {
        if (g.np == 1) hipLaunchKernelGGL((k_push<WT, 1, true>), gd, bd, 0, st, a);
        else hipLaunchKernelGGL((k_push<WT, kMaxParts, true>), gd, bd, 0, st, a);
    } else {
        if (g.np == 1) hipLaunchKernelGGL((k_push<WT, 1, false>), gd, bd, 0, st, a);
        else hipLaunchKernelGGL((k_push<WT, kMaxParts, false>), gd, bd, 0, st, a);
    }
}

hipError_t launch_push(const DevGraph &g, uint32_t *dist, const Frontier &f, int64_t iter, const FrontierCounts &c,
                       int num_cu, hipStream_t st) {
    const int64_t E = c.Esum();
    if (E <= 0) return hipSuccess;
    // about 16 blocks per CU: four waves of resident blocks, which run
    // roughly in rank order (R-MAT 22: 3.50 ms per query against 3.65 with 8
    // per CU and 3.99 with 4)
    int64_t target = (E + (int64_t)num_cu * 16 - 1) / ((int64_t)num_cu * 16);
    if (target < kMinChunk) target = kMinChunk;
    int64_t emax = 0;
    for (int k = 0; k < g.np; ++k) emax = c.E[k] > emax ? c.E[k] : emax;
    const int64_t B = (emax + target - 1) / target;
    PushArgs a;
    a.padj = g.padj;
    a.dist = dist;
    for (int k = 0; k < kMaxParts; ++k) {
        a.qse[k] = f.qse[k];
        a.qs[k] = f.qs[k];
        a.F[k] = k < g.np ? c.F[k] : 0;
        a.E[k] = k < g.np ? c.E[k] : 0;
        a.per[k] = (int32_t)((a.E[k] + B - 1) / B);
        if (a.per[k] < 1) a.per[k] = 1;
    }
    a.nflags = f.flags[(iter + 1) & 1];
    a.bound = f.bound;
    const int grid = (int)(B * g.np);
    const dim3 gd((unsigned)grid), bd(kBlk);
    switch (g.wt) {
        case 1: push_dispatch<1>(g, gd, bd, st, a); break;
        case 2: push_dispatch<2>(g, gd, bd, st, a); break;
        default: push_dispatch<0>(g, gd, bd, st, a);
    }
    return hipGetLastError();
}

bool pull_partitioned(const DevGraph &g) { return g.np == kMaxParts && g.ro_in == g.ro && g.adj_in == g.adj; }

template <int WT>
static void pull_dispatch(const DevGraph &g, uint32_t *dist, const Frontier &f, int64_t iter, uint32_t level,
                          hipStream_t st) {
    const int p = (int)(iter & 1), np1 = p ^ 1;
    const int64_t chunks = (g.n + kBlk - 1) / kBlk;
    if (WT != 2 && pull_partitioned(g))
        hipLaunchKernelGGL(k_pull_part<WT>, dim3((unsigned)(chunks * kMaxParts)), dim3(kBlk), 0, st, g.n, g.pro,
                           g.padj, dist, f.bits, f.flags[np1], f.bound);
    else
        hipLaunchKernelGGL(k_pull<WT>, dim3((unsigned)chunks), dim3(kBlk), 0, st, g.n, g.ro_in, g.adj_in, dist, f.bits,
                           f.flags[np1], f.bound, level);
    (void)p;
}

hipError_t launch_pull(const DevGraph &g, uint32_t *dist, const Frontier &f, int64_t iter, hipStream_t st,
                       uint32_t level) {
    if (g.wt == 1) pull_dispatch<1>(g, dist, f, iter, level, st);
    else if (g.wt == 2) pull_dispatch<2>(g, dist, f, iter, level, st);
    else pull_dispatch<0>(g, dist, f, iter, level, st);
    return hipGetLastError();
}

hipError_t launch_filter(const DevGraph &g, const Frontier &f, int64_t iter, uint64_t *zmask, bool dense,
                         const uint32_t *dist, bool use_far, uint32_t threshold, hipStream_t st) {
    if (use_far && (!dist || !f.far[0])) return hipErrorInvalidValue;
    const int p = (int)(iter & 1);
    if (dense) {
        DenseFilterArgs a;
        a.np = g.np;
        int64_t maxlen = 0;
        for (int k = 0; k < g.np; ++k) maxlen = std::max<int64_t>(maxlen, g.mem_off[k + 1] - g.mem_off[k]);
        a.chunks = (int32_t)std::max<int64_t>(1, (maxlen + kDenseChunk - 1) / kDenseChunk);
        const int64_t blocks = (int64_t)a.chunks * g.np;
        a.mem_u = g.mem_u;
        a.mem_sd = g.mem_sd;
        for (int k = 0; k <= kMaxParts; ++k) a.off[k] = k <= g.np ? g.mem_off[k] : g.mem_off[g.np];
        a.nflags = f.flags[p ^ 1];
        a.cflags = f.flags[p];
        a.nflag16 = f.nflag / 16;
        a.clear16 = (a.nflag16 + blocks - 1) / blocks;
        a.zmask = zmask;
        a.dist = dist;
        for (int k = 0; k < kMaxParts; ++k) {
            a.qse[k] = f.qse[k];
            a.qs[k] = f.qs[k];
        }
        a.ctl_next = f.ctl + slot_of(iter + 1) * kSlotWords;
        a.ctl_zero = f.ctl + slot_of(iter + 2) * kSlotWords;
        a.far_cur = use_far ? f.far[p] : nullptr;
        a.far_next = use_far ? f.far[p ^ 1] : nullptr;
        a.threshold = threshold;
        a.nbits = reinterpret_cast<uint16_t *>(f.bits);
        hipLaunchKernelGGL(k_filter_dense, dim3((unsigned)blocks), dim3(kBlk), 0, st, a);
        return hipGetLastError();
    }
    FilterArgs a;
    a.np = g.np;
    a.pro = g.pro;
    a.zmask = zmask;
    a.dist = dist;
    a.nflags = f.flags[p ^ 1];
    a.cflags = f.flags[p];
    for (int k = 0; k < kMaxParts; ++k) {
        a.qse[k] = f.qse[k];
        a.qs[k] = f.qs[k];
    }
    a.ctl_next = f.ctl + slot_of(iter + 1) * kSlotWords;
    a.ctl_zero = f.ctl + slot_of(iter + 2) * kSlotWords;
    a.far_cur = use_far ? f.far[p] : nullptr;
    a.far_next = use_far ? f.far[p ^ 1] : nullptr;
    a.threshold = threshold;
    a.nbits = reinterpret_cast<uint16_t *>(f.bits);
    if (g.np == 1) hipLaunchKernelGGL(k_filter<1>, dim3(f.ngroups), dim3(kBlk), 0, st, a);
    else hipLaunchKernelGGL(k_filter<kMaxParts>, dim3(f.ngroups), dim3(kBlk), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_members(int32_t n, int32_t np, const int32_t *pro, int32_t *cnt, int32_t *pos, int32_t *tmp,
                          int32_t *mem_u, uint2 *mem_sd, long long *off, hipStream_t st) {
    const int64_t len = (int64_t)np * (n + 1) + 1;
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)len, st);
    if (e != hipSuccess) return e;
    const int grid = grid_for((int64_t)np * n, kBlk * 4, 16384);
    hipLaunchKernelGGL(k_member_flags, dim3(grid), dim3(kBlk), 0, st, n, np, pro, cnt);
    e = scan_exclusive(cnt, len, pos, tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_member_scatter, dim3(grid), dim3(kBlk), 0, st, n, np, pro, cnt, pos, mem_u, mem_sd, off);
    return hipGetLastError();
}

hipError_t launch_pack_arcs(const int32_t *col, const uint32_t *w, int32_t m, uint2 *adj, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_arcs, dim3(grid_for(m, kBlk * 8, 16384)), dim3(kBlk), 0, st, col, w, m, adj);
    return hipGetLastError();
}

hipError_t launch_validate(int32_t n, int32_t m, const int32_t *ro, const int32_t *col, const uint32_t *w, int wt,
                           unsigned int *err, hipStream_t st) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for((int64_t)n + m + 1, kBlk * 8, 16384)), dim3(kBlk), 0, st, n, m,
                       ro, col, w, wt, err);
    return hipGetLastError();
}

static hipError_t scan_exclusive(const int32_t *in, int64_t len, int32_t *out, int32_t *tmp, hipStream_t st) {
    // out[0..len) = exclusive scan of in; tmp holds scan_tmp_ints(len) ints.
    const int64_t nb = (len + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_level, dim3((unsigned)nb), dim3(kBlk), 0, st, in, len, out, tmp);
    if (nb > 1) {
        hipError_t e = scan_exclusive(tmp, nb, tmp + nb, tmp + 2 * nb, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((len + kBlk - 1) / kBlk)), dim3(kBlk), 0, st, out, len,
                           tmp + nb);
    }
    return hipGetLastError();
}

size_t scan_tmp_ints(int64_t len) {
    size_t t = 0;
    int64_t l = len;
    while (true) {
        const int64_t nb = (l + kScanChunk - 1) / kScanChunk;
        t += 2 * nb;
        if (nb <= 1) break;
        l = nb;
    }
    return t + 16;
}

static inline int row_grid(int32_t n) { return grid_for((int64_t)n, kBlk / 64, 16384); }

hipError_t launch_csc_build(int32_t n, int32_t m, const int32_t *ro, const uint2 *adj, int32_t *ro_in,
                            uint2 *adj_in, int32_t *scratch, hipStream_t st) {
    // scratch: n + 1 ints (counts) + n ints (fill) + scan temporaries.
    int32_t *cnt = scratch;
    int32_t *fill = scratch + (n + 1);
    int32_t *tmp = fill + n;
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)(2 * (int64_t)n + 1), st);
    if (e != hipSuccess) return e;
    if (m > 0) hipLaunchKernelGGL(k_count_in, dim3(grid_for(m, kBlk * 8, 16384)), dim3(kBlk), 0, st, adj, m, cnt);
    e = scan_exclusive(cnt, (int64_t)n + 1, ro_in, tmp, st);
    if (e != hipSuccess) return e;
    if (m > 0)
        hipLaunchKernelGGL(k_scatter_in, dim3(row_grid(n)), dim3(kBlk), 0, st, n, ro, adj, ro_in, fill, adj_in);
    return hipGetLastError();
}

hipError_t launch_symmetry_check(int32_t n, const int32_t *ro, const uint2 *adj, unsigned int *not_sym,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_symmetry, dim3(row_grid(n)), dim3(kBlk), 0, st, n, ro, adj, not_sym);
    return hipGetLastError();
}

hipError_t launch_locality(int32_t n, const int32_t *ro, const uint2 *adj, int32_t span, unsigned long long *near,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_locality, dim3(row_grid(n)), dim3(kBlk), 0, st, n, ro, adj, span, near);
    return hipGetLastError();
}

hipError_t launch_partition_build(int32_t n, int32_t m, const int32_t *ro, const uint2 *adj, int32_t np,
                                  int32_t psize, int32_t *pro, uint2 *padj, int32_t *cnt, int32_t *pm, int32_t *tmp,
                                  unsigned long long *caps, hipStream_t st) {
    // cnt, pm: np * (n + 1) + 1 ints.  In partition-major order the entries
    // k*(n+1)+n and the last stay 0, so the exclusive scan gives
    // pm[k*(n+1)+n] = pm[(k+1)*(n+1)] (end of partition k's arcs).  The result
    // pro is vertex-major: pro[u*np + k], u in [0, n].
    const int64_t len = (int64_t)np * (n + 1) + 1;
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)len, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_part_count, dim3(row_grid(n)), dim3(kBlk), 0, st, n, ro, adj, np, psize, cnt);
    hipLaunchKernelGGL(k_part_caps, dim3(grid_for(n, kBlk * 16, 4096)), dim3(kBlk), 0, st, n, np, cnt, caps);
    e = scan_exclusive(cnt, len, pm, tmp, st);
    if (e != hipSuccess) return e;
    if (m > 0)
        hipLaunchKernelGGL(k_part_scatter, dim3(row_grid(n)), dim3(kBlk), 0, st, n, ro, adj, psize, pm, padj);
    hipLaunchKernelGGL(k_part_transpose, dim3(grid_for(((int64_t)n + 1) * np, kBlk * 4, 16384)), dim3(kBlk), 0, st,
                       n, np, pm, pro);
    return hipGetLastError();
}

hipError_t launch_canon_negzero(uint2 *adj, int32_t m, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_canon_negzero, dim3(grid_for(m, kBlk * 8, 16384)), dim3(kBlk), 0, st, adj, m);
    return hipGetLastError();
}

template <int WT, int NP>
static hipError_t coop_launch(const PersistArgs &a, int grid, hipStream_t st) {
    void *args[] = {const_cast<PersistArgs *>(&a)};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_persistent<WT, NP>), dim3(grid), dim3(kBlk),
                                      args, 0, st);
}

int persistent_grid(const DevGraph &g, int num_cu) {
    int nb = 0;
    hipError_t e;
    if (g.np == 1) e = g.wt == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<1, 1>, kBlk, 0)
                                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<0, 1>, kBlk, 0);
    else
        e = g.wt == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<1, kMaxParts>, kBlk, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<0, kMaxParts>, kBlk, 0);
    if (e != hipSuccess || nb < 1) return 0;
    nb = std::min(nb, 8);
    int grid = nb * num_cu;
    grid -= grid % kMaxParts;  // whole rounds of the 8 XCDs
    return grid;
}

static void persist_args(const DevGraph &g, uint32_t *dist, const Frontier &f, const PersistentCfg &cfg,
                         PersistArgs &a) {
    FilterArgs &fg = a.fg;
    fg.np = g.np;
    fg.pro = g.pro;
    fg.zmask = nullptr;
    fg.dist = dist;
    fg.far_cur = nullptr;
    fg.far_next = nullptr;
    fg.threshold = 0u;
    fg.nbits = reinterpret_cast<uint16_t *>(f.bits);
    fg.nflags = nullptr;
    fg.cflags = nullptr;
    fg.ctl_next = nullptr;
    fg.ctl_zero = nullptr;
    DenseFilterArgs &fd = a.fd;
    fd.np = g.np;
    int64_t maxlen = 0;
    for (int k = 0; k < g.np; ++k) maxlen = std::max<int64_t>(maxlen, g.mem_off[k + 1] - g.mem_off[k]);
    fd.chunks = (int32_t)std::max<int64_t>(1, (maxlen + kDenseChunk - 1) / kDenseChunk);
    fd.mem_u = g.mem_u;
    fd.mem_sd = g.mem_sd;
    for (int k = 0; k <= kMaxParts; ++k) fd.off[k] = k <= g.np ? g.mem_off[k] : g.mem_off[g.np];
    fd.nflags = nullptr;
    fd.cflags = nullptr;
    fd.nflag16 = f.nflag / 16;
    fd.clear16 = (fd.nflag16 + (int64_t)fd.chunks * g.np - 1) / ((int64_t)fd.chunks * g.np);
    fd.zmask = nullptr;
    fd.dist = dist;
    fd.far_cur = nullptr;
    fd.far_next = nullptr;
    fd.threshold = 0u;
    fd.nbits = reinterpret_cast<uint16_t *>(f.bits);
    fd.ctl_next = nullptr;
    fd.ctl_zero = nullptr;
    for (int k = 0; k < kMaxParts; ++k) {
        fg.qse[k] = fd.qse[k] = f.qse[k];
        fg.qs[k] = fd.qs[k] = f.qs[k];
    }
    a.padj = g.padj;
    a.dist = dist;
    a.ro_in = g.ro_in;
    a.adj_in = g.adj_in;
    a.flags[0] = f.flags[0];
    a.flags[1] = f.flags[1];
    a.ro = g.ro;
    a.adj = g.adj;
    a.cand[0] = f.cand[0];
    a.cand[1] = f.cand[1];
    a.ccount = f.ccount;
    a.rstat = f.rstat;
    a.bound = f.bound;
    a.cand_region = f.cand_cap / kCandRegions;
    a.small = cfg.small && f.cand[0] != nullptr ? 1 : 0;
    a.local_hops = cfg.local_hops > 1 ? cfg.local_hops : 1;
    a.phase_log = nullptr;
    a.phase_log_cap = 0;
    a.far[0] = cfg.delta ? f.far[0] : nullptr;
    a.far[1] = cfg.delta ? f.far[1] : nullptr;
    a.delta = cfg.delta;
    a.ctl = f.ctl;
    a.n = g.n;
    a.m = g.m;
    a.ngroups = f.ngroups;
    a.max_iters = cfg.max_iters;
    a.alpha_x16 = cfg.alpha_x16;
    a.beta = cfg.beta > 0 ? cfg.beta : 24;
    a.bits = f.bits;
    a.part_pull = pull_partitioned(g) ? 1 : 0;
    a.direction = cfg.direction;
    a.filter = cfg.filter;
    a.dense_ratio = cfg.dense_ratio;
    a.spin_ticks = cfg.spin_ticks;
}

hipError_t launch_persistent(const DevGraph &g, uint32_t *dist, const Frontier &f, const PersistentCfg &cfg,
                             hipStream_t st) {
    PersistArgs a;
    persist_args(g, dist, f, cfg, a);
    if (g.np == 1) return g.wt == 1 ? coop_launch<1, 1>(a, cfg.grid, st) : coop_launch<0, 1>(a, cfg.grid, st);
    return g.wt == 1 ? coop_launch<1, kMaxParts>(a, cfg.grid, st) : coop_launch<0, kMaxParts>(a, cfg.grid, st);
}

template <int WT>
static void step_dispatch(const DevGraph &g, dim3 grid, dim3 blk, hipStream_t st, const PersistArgs &a, int64_t launch) {
    if (offsets32(g)) {
        if (g.np == 1) hipLaunchKernelGGL((k_step<WT, 1, true>), grid, blk, 0, st, a, launch);
        else hipLaunchKernelGGL((k_step<WT, kMaxParts, true>), grid, blk, 0, st, a, launch);
    } else {
        if (g.np == 1) hipLaunchKernelGGL((k_step<WT, 1, false>), grid, blk, 0, st, a, launch);
        else hipLaunchKernelGGL((k_step<WT, kMaxParts, false>), grid, blk, 0, st, a, launch);
    }
}

hipError_t launch_step(const DevGraph &g, uint32_t *dist, const Frontier &f, const PersistentCfg &cfg, int64_t launch,
                       int8_t *phase_log, int64_t phase_log_cap, hipEvent_t ev_begin, hipEvent_t ev_end,
                       hipStream_t st) {
    PersistArgs a;
    persist_args(g, dist, f, cfg, a);
    a.phase_log = phase_log;
    a.phase_log_cap = phase_log_cap;
    const dim3 grid((unsigned)cfg.grid), blk(kBlk);
    if (ev_begin) (void)hipEventRecord(ev_begin, st);
    switch (g.wt) {
        case 1: step_dispatch<1>(g, grid, blk, st, a, launch); break;
        case 2: step_dispatch<2>(g, grid, blk, st, a, launch); break;
        default: step_dispatch<0>(g, grid, blk, st, a, launch);
    }
    if (ev_end) (void)hipEventRecord(ev_end, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// frontier workspace layout

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Candidate-list capacity: a multiple of kCandRegions, up to 2^18 vertices
// (1 MiB per list).
static inline int32_t cand_capacity(int32_t n) {
    return kCandRegions * std::max(1, std::min(n, 1 << 18) / kCandRegions);
}

size_t frontier_bytes(const DevGraph &g, WsParts w) {
    const int64_t ng = groups_for(g.n);
    size_t b = 0;
    b += (w.far ? 4 : 2) * align256((size_t)ng * kGroupVerts);  // flags, held-back flags
    b += align256((size_t)ng * kGroupVerts / 8);                 // frontier bitmap
    b += 2 * align256(sizeof(int32_t) * (size_t)cand_capacity(g.n));
    b += align256(sizeof(unsigned long long) * 3 * kCandRegions);
    b += align256(sizeof(unsigned long long) * kStatWords);
    if (w.bound) b += align256(sizeof(uint32_t) * (size_t)std::max(g.n, 1));
    for (int k = 0; k < g.np; ++k) {
        const size_t c = (size_t)(g.cap[k] > 0 ? g.cap[k] : 1);
        b += align256(c * 8) + align256(c * 4);
    }
    b += align256(kCtlWords * 8);
    return b;
}

void frontier_carve(Frontier &f, void *base, const DevGraph &g, WsParts w) {
    const int64_t ng = groups_for(g.n);
    f.ngroups = (int32_t)ng;
    f.nflag = ng * kGroupVerts;
    f.np = g.np;
    char *p = static_cast<char *>(base);
    for (int i = 0; i < 2; ++i) {
        f.flags[i] = reinterpret_cast<uint8_t *>(p);
        p += align256((size_t)f.nflag);
    }
    for (int i = 0; i < 2; ++i) {
        f.far[i] = w.far ? reinterpret_cast<uint8_t *>(p) : nullptr;
        if (w.far) p += align256((size_t)f.nflag);
    }
    f.bits = reinterpret_cast<uint32_t *>(p);
    p += align256((size_t)f.nflag / 8);
    f.cand_cap = cand_capacity(g.n);
    for (int i = 0; i < 2; ++i) {
        f.cand[i] = reinterpret_cast<int32_t *>(p);
        p += align256(sizeof(int32_t) * (size_t)f.cand_cap);
    }
    f.ccount = reinterpret_cast<unsigned long long *>(p);
    p += align256(sizeof(unsigned long long) * 3 * kCandRegions);
    f.rstat = reinterpret_cast<unsigned long long *>(p);
    p += align256(sizeof(unsigned long long) * kStatWords);
    f.bound = w.bound ? reinterpret_cast<uint32_t *>(p) : nullptr;
    if (w.bound) p += align256(sizeof(uint32_t) * (size_t)std::max(g.n, 1));
    for (int k = 0; k < kMaxParts; ++k) {
        f.qse[k] = nullptr;
        f.qs[k] = nullptr;
    }
    for (int k = 0; k < g.np; ++k) {
        const size_t c = (size_t)(g.cap[k] > 0 ? g.cap[k] : 1);
        f.qse[k] = reinterpret_cast<uint2 *>(p);
        p += align256(c * 8);
        f.qs[k] = reinterpret_cast<int32_t *>(p);
        p += align256(c * 4);
    }
    f.ctl = reinterpret_cast<unsigned long long *>(p);
}

}  // namespace gr
