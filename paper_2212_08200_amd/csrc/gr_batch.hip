// Batched multi-source SSSP on gfx950: up to 64 independent queries on one
// graph advance together, one source per lane of a wave64.
//
// Distances are kept vertex-major, D[v * 64 + s] for source slot s, so the 64
// distances of a vertex fill one 256-byte row.  Relaxing an arc u -> v for
// every source active at u is then one coalesced row read of D[v] (plus the
// row of D[u]) instead of one random 4-byte access per source, and the arc
// itself is read once for all sources.  Each source follows the paper's
// relaxation rule independently (Listing 4): for source s active at u,
// new = D[u][s] (+) w, atomic min into D[v][s], and s becomes active at v iff
// new is smaller than the value read.  Per-vertex 64-bit masks record which
// sources are active; a vertex is in the shared frontier when its mask is
// non-zero, and the single-source filter compacts that frontier.
//
// Every source's distances are the unique shortest-path vector of its own
// query (the result does not depend on how relaxations interleave), so row s
// of the output is bit-identical to a single-source query from srcs[s].
#include "gr_device.h"

#include <hip/hip_runtime.h>

namespace gr {

// ---------------------------------------------------------------------------
// init: D = INF, masks and flags cleared, counters cleared.
__global__ __launch_bounds__(kBlk) void k_batch_fill(uint32_t *__restrict__ D, int64_t nrow, uint32_t inf,
                                                     uint64_t *m0, uint64_t *m1, int64_t nmask, uint8_t *f0,
                                                     uint8_t *f1, int64_t nflag, unsigned long long *ctl) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const uint4 q = make_uint4(inf, inf, inf, inf);
    for (int64_t i = tid; i < nrow * (kBatchLanes / 4); i += stride) reinterpret_cast<uint4 *>(D)[i] = q;
    for (int64_t i = tid; i < nmask; i += stride) {
        m0[i] = 0ull;
        m1[i] = 0ull;
    }
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = tid; i < nflag / 16; i += stride) {
        reinterpret_cast<uint4 *>(f0)[i] = z;
        reinterpret_cast<uint4 *>(f1)[i] = z;
    }
    for (int64_t i = tid; i < kCtlWords; i += stride) ctl[i] = 0ull;
}

// Sources: slot s starts at srcs[s] with distance 0 and is active there.
// One thread per slot; the mask bits of duplicate sources are merged with an
// atomic or.
__global__ void k_batch_sources(uint32_t *__restrict__ D, uint64_t *__restrict__ m0, uint8_t *__restrict__ f0,
                                const int32_t *__restrict__ srcs, int32_t k) {
    const int s = threadIdx.x;
    if (s < k) {
        const int64_t v = srcs[s];
        D[v * kBatchLanes + s] = 0u;
        atomicOr(reinterpret_cast<unsigned long long *>(m0 + v), 1ull << s);
        f0[v] = 1;
    }
}

// ---------------------------------------------------------------------------
// batched push.  Like the single-source push, block j relaxes arc ranks
// [j*per, min(E, (j+1)*per)) of the frontier (entries (first arc, u) with
// exclusive arc-count prefix sums), staging windows of entries in LDS.  Within
// a window each wave takes a contiguous run of ranks, kBatchArcs at a time;
// every lane is one source.
// 4 arcs at a time (58 VGPRs, 8 waves per SIMD): a 64-source R-MAT 22 launch
// takes 95 ms, against 103 ms with 2, 125 ms with 8 and 167 ms with 16
constexpr int kBatchArcs = 4;

struct BatchPushArgs {
    const uint2 *adj;
    uint32_t *D;
    const uint64_t *mcur;
    uint64_t *mnext;
    uint8_t *nflags;
    const uint2 *qse;
    const int32_t *qs;
    int32_t F, E, per;
};

template <int WT>
__global__ __launch_bounds__(kBlk) void k_batch_push(BatchPushArgs a) {
    __shared__ int32_t sS[kWin + 1];
    __shared__ uint32_t sRow[kWin];
    __shared__ uint32_t sU[kWin];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t beg64 = (int64_t)blockIdx.x * a.per;
    if (a.F <= 0 || beg64 >= a.E) return;
    const int32_t beg = (int32_t)beg64;
    const int32_t end = (int32_t)min<int64_t>(beg64 + a.per, a.E);
    const uint64_t lanebit = 1ull << lane;

    int32_t i0 = find_entry(a.qs, a.F, beg);
    int32_t e = beg;
    while (e < end) {
        const int32_t cnt = min(kWin, a.F - i0);
        for (int t = threadIdx.x; t < cnt; t += kBlk) {
            const uint2 q = a.qse[i0 + t];
            sS[t] = a.qs[i0 + t];
            sRow[t] = q.x;
            sU[t] = q.y;
        }
        for (int t = cnt + threadIdx.x; t <= kWin; t += kBlk)
            sS[t] = (t == cnt) ? ((i0 + cnt < a.F) ? a.qs[i0 + cnt] : a.E) : INT32_MAX;
        __syncthreads();
        const int32_t wend = min(end, sS[cnt]);
        // this wave's contiguous share of the window's ranks
        const int32_t span = wend - e;
        const int32_t share = (span + (kBlk / 64) - 1) / (kBlk / 64);
        const int32_t r0 = e + wid * share;
        const int32_t r1 = min(wend, r0 + share);
        for (int32_t x0 = r0; x0 < r1; x0 += kBatchArcs) {
            int32_t pos[kBatchArcs];
            uint2 arc[kBatchArcs];
            uint64_t msk[kBatchArcs];
            uint32_t du[kBatchArcs], dv[kBatchArcs];
#pragma unroll
            for (int it = 0; it < kBatchArcs; ++it) {
                const int32_t x = min(x0 + it, r1 - 1);  // clamped ranks repeat the last arc
                int32_t p = 0;
#pragma unroll
                for (int b = kWin / 2; b >= 1; b >>= 1) p = (sS[p + b] <= x) ? p + b : p;
                pos[it] = p;
            }
#pragma unroll
            for (int it = 0; it < kBatchArcs; ++it) {
                const int32_t x = min(x0 + it, r1 - 1);
                arc[it] = load_arc(a.adj + sRow[pos[it]] + (uint32_t)(x - sS[pos[it]]));
                msk[it] = a.mcur[sU[pos[it]]];
            }
#pragma unroll
            for (int it = 0; it < kBatchArcs; ++it) {
                const bool act = (msk[it] & lanebit) != 0ull;
                du[it] = act ? a.D[(int64_t)sU[pos[it]] * kBatchLanes + lane] : 0u;
                dv[it] = act ? a.D[(int64_t)arc[it].x * kBatchLanes + lane] : 0u;
            }
#pragma unroll
            for (int it = 0; it < kBatchArcs; ++it) {
                const bool act = (x0 + it < r1) && ((msk[it] & lanebit) != 0ull);
                const uint32_t nd = plus<WT>(du[it], arc[it].y);
                const bool better = act && nd < dv[it];
                if (better)
                    __hip_atomic_fetch_min(a.D + (int64_t)arc[it].x * kBatchLanes + lane, nd, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t won = __ballot(better);
                if (won && lane == 0) {
                    __hip_atomic_fetch_or(reinterpret_cast<unsigned long long *>(a.mnext + arc[it].x), won,
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    a.nflags[arc[it].x] = 1;
                }
            }
        }
        i0 += cnt;
        e = wend;
        __syncthreads();  // window reuse
    }
}

// ---------------------------------------------------------------------------
// output: D (n x 64, vertex-major) -> out[s][v] for s < k, through an LDS
// tile of 64 vertices x 64 slots so that both sides are coalesced.
__global__ __launch_bounds__(kBlk) void k_batch_output(const uint32_t *__restrict__ D, int32_t n, int32_t k,
                                                       uint32_t *const *__restrict__ out) {
    __shared__ uint32_t tile[64][65];
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    for (int i = threadIdx.x; i < 64 * 64; i += kBlk) {
        const int r = i >> 6, c = i & 63;
        tile[r][c] = (v0 + r < n) ? D[(v0 + r) * kBatchLanes + c] : 0u;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * 64; i += kBlk) {
        const int s = i >> 6, r = i & 63;
        if (s < k && v0 + r < n) out[s][v0 + r] = tile[r][s];
    }
}

// ---------------------------------------------------------------------------
// launch wrappers and workspace

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t batch_bytes(const DevGraph &g) {
    const int64_t ng = groups_for(g.n);
    const int64_t nv = ng * kGroupVerts;
    size_t b = 0;
    b += align256((size_t)g.n * kBatchLanes * 4);   // D
    b += 2 * align256((size_t)nv * 8);              // masks
    b += 2 * align256((size_t)nv);                  // flags
    b += align256((size_t)(g.cap[0] > 0 ? g.cap[0] : 1) * 8) + align256((size_t)(g.cap[0] > 0 ? g.cap[0] : 1) * 4);
    b += align256(kCtlWords * 8);
    b += align256(kBatchLanes * sizeof(void *)) + align256(kBatchLanes * 4);
    return b;
}

void batch_carve(BatchWs &w, void *base, const DevGraph &g) {
    const int64_t ng = groups_for(g.n);
    const int64_t nv = ng * kGroupVerts;
    char *p = static_cast<char *>(base);
    w.D = reinterpret_cast<uint32_t *>(p);
    p += align256((size_t)g.n * kBatchLanes * 4);
    for (int i = 0; i < 2; ++i) {
        w.mask[i] = reinterpret_cast<uint64_t *>(p);
        p += align256((size_t)nv * 8);
    }
    Frontier &f = w.f;
    f.ngroups = (int32_t)ng;
    f.nflag = nv;
    f.np = 1;
    f.cand_cap = 0;
    f.ccount = nullptr;
    f.rstat = nullptr;
    f.bound = nullptr;
    for (int i = 0; i < 2; ++i) {
        f.flags[i] = reinterpret_cast<uint8_t *>(p);
        p += align256((size_t)nv);
        f.far[i] = nullptr;  // no near-far split for batched queries
        f.cand[i] = nullptr;  // no small rounds either
    }
    for (int k = 0; k < kMaxParts; ++k) {
        f.qse[k] = nullptr;
        f.qs[k] = nullptr;
    }
    const size_t c = (size_t)(g.cap[0] > 0 ? g.cap[0] : 1);
    f.qse[0] = reinterpret_cast<uint2 *>(p);
    p += align256(c * 8);
    f.qs[0] = reinterpret_cast<int32_t *>(p);
    p += align256(c * 4);
    f.ctl = reinterpret_cast<unsigned long long *>(p);
    p += align256(kCtlWords * 8);
    w.out_ptrs = reinterpret_cast<uint32_t **>(p);
    p += align256(kBatchLanes * sizeof(void *));
    w.srcs = reinterpret_cast<int32_t *>(p);
}

hipError_t launch_batch_init(const DevGraph &g, const BatchWs &w, int32_t k, hipStream_t st) {
    const uint32_t inf = g.wt == 1 ? kInfF32 : kInfU32;
    const int64_t nv = (int64_t)w.f.ngroups * kGroupVerts;
    int64_t grid = ((int64_t)g.n * (kBatchLanes / 4) + kBlk * 4 - 1) / (kBlk * 4);
    if (grid > 16384) grid = 16384;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_batch_fill, dim3((unsigned)grid), dim3(kBlk), 0, st, w.D, (int64_t)g.n, inf, w.mask[0],
                       w.mask[1], nv, w.f.flags[0], w.f.flags[1], w.f.nflag, w.f.ctl);
    hipLaunchKernelGGL(k_batch_sources, dim3(1), dim3(kBatchLanes), 0, st, w.D, w.mask[0], w.f.flags[0], w.srcs, k);
    return hipGetLastError();
}

hipError_t launch_batch_push(const DevGraph &g, const BatchWs &w, int64_t iter, int32_t F, int32_t E, int num_cu,
                             hipStream_t st) {
    if (F <= 0 || E <= 0) return hipSuccess;
    // many small blocks balance the uneven per-arc work (active sources per
    // vertex vary): 64 sources on R-MAT 22 take 84.6 ms with 128 blocks per
    // CU, 85.7 with 64, 87.5 with 32, 94.3 with 8
    int64_t per = ((int64_t)E + (int64_t)num_cu * 128 - 1) / ((int64_t)num_cu * 128);
    if (per < 512) per = 512;
    const int grid = (int)(((int64_t)E + per - 1) / per);
    BatchPushArgs a;
    a.adj = g.adj;
    a.D = w.D;
    a.mcur = w.mask[iter & 1];
    a.mnext = w.mask[(iter + 1) & 1];
    a.nflags = w.f.flags[(iter + 1) & 1];
    a.qse = w.f.qse[0];
    a.qs = w.f.qs[0];
    a.F = F;
    a.E = E;
    a.per = (int32_t)per;
    if (g.wt == 1) hipLaunchKernelGGL(k_batch_push<1>, dim3(grid), dim3(kBlk), 0, st, a);
    else hipLaunchKernelGGL(k_batch_push<0>, dim3(grid), dim3(kBlk), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_batch_output(const DevGraph &g, const BatchWs &w, int32_t k, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_output, dim3((unsigned)((g.n + 63) / 64)), dim3(kBlk), 0, st, w.D, g.n, k,
                       w.out_ptrs);
    return hipGetLastError();
}

}  // namespace gr
