// Single-workgroup loop for small graphs (Section III-A's loop, Listing 4's
// advance, with the whole query in one workgroup's LDS).
//
// Graphs of a few thousand vertices, such as small meshes, take one round per
// hop of their diameter, and each round of the other loops costs a kernel
// launch or a grid-wide barrier plus round trips to the L2.  Here one
// workgroup of 1024 threads copies the distances and arcs into LDS (arcs
// packed as a 16-bit head and a 16-bit weight, either padded to a power-of-two
// number of slots per vertex or behind row offsets), keeps the frontier as a
// list of vertex ids in LDS, and runs the bulk-synchronous rounds with
// workgroup barriers and LDS atomics: a round is well under a microsecond.
// A batch of queries runs one such workgroup per query in one launch.
//
// Round r: every vertex u of list r is expanded by a group of lanes: for each
// arc (u, v, w), new = dist[u] + w, offered to v with an LDS atomic min.
// Each vertex's LDS word holds its distance shifted left by one and a free
// bit (set: not on the next list).  Expanding u sets u's free bit with an
// atomic or, whose result is the distance the group uses; an offer writes
// new << 1 (free bit clear), and the offer that took v's word from free to
// queued appends v to list r + 1.  One word per vertex: an improvement that
// lands after u's atomic or finds u free and queues it again, and one that
// lands before is read by it.  dist[u] is thus read when u is expanded, so
// an improvement found earlier in the same round is used (as the other
// loops read dist[u] when staging their frontier).  One workgroup barrier
// ends each round (with row offsets, a second one precedes the hubs' arcs);
// the loop ends when a round appends nothing, at the same fixed point.  Distances take 31 bits, which every graph that fits
// allows (gr_lds.h).

#include "gr_lds.h"

#include "gr_device.h"

namespace gr {

namespace {

constexpr int kLdsThreads = 1024;
constexpr int kCopy = 8;  // loads in flight per thread while copying the graph
// Row-offset layout: a vertex of more than kHubDeg arcs (a hub) is not walked
// by its group; the group's first lane lists it with its distance, and after
// a workgroup barrier all 1024 threads relax the listed hubs' arcs together
// (R-MAT of 2-4 K vertices: 6-11% less time; with 64 as the threshold the
// many mid-size hubs made it slower).  A graph that fits holds fewer than
// kLdsWords / kHubDeg hubs, so the list cannot overflow.
constexpr int32_t kHubDeg = 256;
constexpr int32_t kHubCap = 256;
static_assert(kLdsWords / (kHubDeg + 1) < kHubCap, "every hub of a graph that fits is listed");

struct LdsArgs {
    int64_t max_rounds;
    unsigned long long *stat;    // k x kLdsStatWords
    LdsJob job[kLdsMaxBatch];    // workgroup b runs job[b]
};

// WT: 0 uint32 weights, 2 unit steps; LG: log2 of the lanes per vertex;
// ELL: the arcs come padded to 2^LG slots per vertex (no row offsets).
template <int WT, int LG, bool ELL>
__global__ __launch_bounds__(kLdsThreads) void k_lds(LdsArgs a) {
    __shared__ uint32_t sMem[kLdsWords];
    __shared__ int32_t sCnt[3];
    __shared__ unsigned long long sArcs, sExp;
    __shared__ uint2 sHub[ELL ? 1 : kHubCap];  // (hub, its distance)
    __shared__ int32_t sHubCnt[2];             // by round parity
    const int t = threadIdx.x;
    const LdsJob &job = a.job[blockIdx.x];
    const int32_t n = job.n, m = job.m, src = job.src;
    const int32_t *const ro = job.ro;
    const uint2 *const adj = job.adj;
    uint32_t *const dist = job.dist;
    unsigned long long *const stat = a.stat + (size_t)blockIdx.x * kLdsStatWords;
    uint32_t *sW = sMem;  // dist << 1 | free bit
    int32_t *sRo = reinterpret_cast<int32_t *>(sMem + n);  // row offsets (CSR layout only)
    uint32_t *sArc = ELL ? sMem + n : sMem + 2 * n + 1;
    const int32_t arc_words = ELL ? (n << LG) : m;
    // the two lists, as one array indexed from list 0 (an offset, not a
    // pointer chosen at run time, keeps the accesses LDS instructions)
    uint16_t *sL = reinterpret_cast<uint16_t *>(sArc + arc_words);
    for (int32_t v = t; v < n; v += kLdsThreads) sW[v] = kInfU32;  // unreached and free
    // the copies issue kCopy loads before the first LDS store (indexes past
    // the end read the last element again)
    if constexpr (ELL) {
        const uint32_t *const ell = job.ell;
        for (int32_t e0 = t; e0 < arc_words; e0 += kLdsThreads * kCopy) {
            uint32_t x[kCopy];
#pragma unroll
            for (int k = 0; k < kCopy; ++k) x[k] = ell[min(e0 + k * kLdsThreads, arc_words - 1)];
#pragma unroll
            for (int k = 0; k < kCopy; ++k)
                if (e0 + k * kLdsThreads < arc_words) sArc[e0 + k * kLdsThreads] = x[k];
        }
    } else {
        for (int32_t v0 = t; v0 <= n; v0 += kLdsThreads * kCopy) {
            int32_t x[kCopy];
#pragma unroll
            for (int k = 0; k < kCopy; ++k) x[k] = ro[min(v0 + k * kLdsThreads, n)];
#pragma unroll
            for (int k = 0; k < kCopy; ++k)
                if (v0 + k * kLdsThreads <= n) sRo[v0 + k * kLdsThreads] = x[k];
        }
        for (int32_t e0 = t; e0 < m; e0 += kLdsThreads * kCopy) {
            uint2 x[kCopy];
#pragma unroll
            for (int k = 0; k < kCopy; ++k) x[k] = adj[min(e0 + k * kLdsThreads, m - 1)];
#pragma unroll
            for (int k = 0; k < kCopy; ++k)
                if (e0 + k * kLdsThreads < m) sArc[e0 + k * kLdsThreads] = WT == 2 ? x[k].x : (x[k].x << 16) | x[k].y;
        }
    }
    if (t == 0) {
        sCnt[0] = 1;
        sCnt[1] = 0;
        sCnt[2] = 0;
        sArcs = 0ull;
        sExp = 0ull;
        sHubCnt[0] = 0;
        sHubCnt[1] = 0;
    }
    __syncthreads();
    if (t == 0) {
        sW[src] = 0u;  // distance 0, queued
        sL[0] = (uint16_t)src;
    }
    __syncthreads();
    uint32_t arcs = 0, expanded = 0;
    constexpr int32_t lg = LG;
    const int slot = t & ((1 << lg) - 1), lead = (t & 63) - slot;
    int64_t r = 0;
    // one arc of the row-offset layout relaxed with its tail's distance du
    const auto relax_csr = [&](int32_t e, uint32_t du, int32_t ln, int kn) {
        const uint32_t x = sArc[e];
        const uint32_t v = WT == 2 ? x : x >> 16;
        const uint32_t nw = (du + (WT == 2 ? 1u : (x & 0xFFFFu))) << 1;  // queued
        const uint32_t old = __hip_atomic_fetch_min(&sW[v], nw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        // the atomic took v from free to queued: v goes on list r + 1
        if (nw < old && (old & 1u)) sL[ln + atomicAdd(&sCnt[kn], 1)] = (uint16_t)v;
    };
    // List r's length is sCnt[kr] (kr = r mod 3), list r + 1 is counted in
    // sCnt[kn], and sCnt[kz] (last read in round r - 1) is cleared for round
    // r + 1's appends: one barrier per round.
    int kr = 0, kn = 1, kz = 2;
    for (; r < a.max_rounds; ++r) {
        const int32_t lc = (int32_t)(r & 1) * n, ln = n - lc;  // list r, list r + 1
        const int32_t cnt = sCnt[kr];
        // the thread's first list entry is read beside the count (entries
        // past the count are stale ids, or uninitialised, and go unused)
        uint32_t u_first = sL[lc + min(t >> lg, n - 1)];
        asm volatile("" : "+v"(u_first));  // keeps the read ahead of the test below
        if (cnt == 0) break;  // uniform: read after a barrier
        const int hb = (int)(r & 1);  // this round's hub count
        if (t == 0) {
            sCnt[kz] = 0;
            if constexpr (!ELL) sHubCnt[hb ^ 1] = 0;  // last read in round r - 1
        }
        // G = 2^lg lanes of one wave expand a vertex together: the group's
        // first lane frees u and reads dist[u] in one atomic, the distance is
        // broadcast across the group, and lane s of the group takes the arcs
        // e0 + s, e0 + s + G, ...
        for (int32_t i = t; i < (cnt << lg); i += kLdsThreads) {
            const uint32_t u = i == t ? u_first : sL[lc + (i >> lg)];
            // CSR: the row's bounds; padded: the lane's slot
            int32_t e0 = 0, e1 = 0;
            uint32_t xe = kLdsNoArc;
            if constexpr (ELL) xe = sArc[(u << lg) + slot];
            else {
                e0 = sRo[u];
                e1 = sRo[u + 1];
            }
            uint32_t du = 0u;
            if (slot == 0) du = __hip_atomic_fetch_or(&sW[u], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> 1;
            // broadcast from the group's first lane (a DPP move within quads
            // measured no faster than this permute for groups of 2 and 4)
            if constexpr (LG > 0) du = (uint32_t)__builtin_amdgcn_ds_bpermute(lead << 2, (int)du);
            if constexpr (ELL) {
                // slots fill from the first: slot 0 holds an arc iff u has one
                expanded += slot == 0 && xe != kLdsNoArc ? 1u : 0u;
                if (xe != kLdsNoArc) {
                    ++arcs;
                    const uint32_t v = xe >> 16;
                    const uint32_t nw = (du + (WT == 2 ? 1u : (xe & 0xFFFFu))) << 1;  // queued
                    const uint32_t old =
                        __hip_atomic_fetch_min(&sW[v], nw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (nw < old && (old & 1u)) sL[ln + atomicAdd(&sCnt[kn], 1)] = (uint16_t)v;
                }
            } else if (e1 - e0 > kHubDeg) {
                if (slot == 0) {
                    expanded += 1u;
                    sHub[atomicAdd(&sHubCnt[hb], 1)] = make_uint2(u, du);
                }
            } else {
                expanded += slot == 0 && e1 > e0 ? 1u : 0u;
                for (int32_t e = e0 + slot; e < e1; e += 1 << lg) {
                    ++arcs;
                    relax_csr(e, du, ln, kn);
                }
            }
        }
        if constexpr (!ELL) {
            __syncthreads();  // uniform: every thread reaches it
            const int32_t nh = sHubCnt[hb];
            for (int32_t h = 0; h < nh; ++h) {
                const uint2 hu = sHub[h];
                const int32_t e0 = sRo[hu.x], e1 = sRo[hu.x + 1];
                for (int32_t e = e0 + t; e < e1; e += kLdsThreads) {
                    ++arcs;
                    relax_csr(e, hu.y, ln, kn);
                }
            }
        }
        __syncthreads();
        const int k = kr;
        kr = kn;
        kn = kz;
        kz = k;
    }
    for (int32_t v = t; v < n; v += kLdsThreads) {
        const uint32_t d = sW[v] >> 1;
        dist[v] = d == (kInfU32 >> 1) ? kInfU32 : d;
    }
    if (arcs) atomicAdd(&sArcs, (unsigned long long)arcs);
    if (expanded) atomicAdd(&sExp, (unsigned long long)expanded);
    __syncthreads();
    if (t == 0) {  // system scope: stat may be host memory
        __hip_atomic_store(stat + 0, (unsigned long long)r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(stat + 1, sCnt[kr] == 0 ? 1ull : 2ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(stat + 2, sArcs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(stat + 3, sExp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

template <int WT, bool ELL>
void launch_lg(int lg, dim3 grid, dim3 block, hipStream_t st, const LdsArgs &a) {
    switch (lg) {
        case 0: hipLaunchKernelGGL((k_lds<WT, 0, ELL>), grid, block, 0, st, a); break;
        case 1: hipLaunchKernelGGL((k_lds<WT, 1, ELL>), grid, block, 0, st, a); break;
        case 2: hipLaunchKernelGGL((k_lds<WT, 2, ELL>), grid, block, 0, st, a); break;
        case 3: hipLaunchKernelGGL((k_lds<WT, 3, ELL>), grid, block, 0, st, a); break;
        default: hipLaunchKernelGGL((k_lds<WT, 4, ELL>), grid, block, 0, st, a); break;
    }
}

}  // namespace

int64_t lds_words(int32_t n, int32_t m) {
    return 2 * (int64_t)n + 1 + m + (n + 1) / 2 * 2;
}

hipError_t launch_lds(const LdsJob *jobs, int32_t k, int wt, int64_t max_rounds, unsigned long long *stat,
                      hipStream_t st) {
    if (wt == 1 || !jobs || k < 1 || k > kLdsMaxBatch) return hipErrorInvalidValue;
    LdsArgs a{max_rounds, stat, {}};
    // lanes per expanded vertex: the average degree rounded up to a power of
    // two, at most 16 (the largest over the jobs: more lanes than a vertex
    // has arcs only idle)
    int32_t lg = 0;
    for (int32_t b = 0; b < k; ++b) {
        const LdsJob &j = jobs[b];
        const bool fits = lds_fits(j.n, j.m) || (j.ell && lds_ell_fits(j.n, j.ell_lg));
        if (!fits || j.src < 0 || j.src >= j.n || !j.ro || !j.dist || (j.m > 0 && !j.adj)) return hipErrorInvalidValue;
        a.job[b] = j;
        while (lg < 4 && ((int64_t)j.n << lg) < j.m) ++lg;
    }
    // the padded layout when every job has it with the same slot count
    bool ell = true;
    for (int32_t b = 0; b < k && ell; ++b)
        ell = jobs[b].ell && jobs[b].ell_lg == jobs[0].ell_lg && lds_ell_fits(jobs[b].n, jobs[b].ell_lg);
    // the row-offset layout needs every graph to fit it
    for (int32_t b = 0; b < k && !ell; ++b)
        if (!lds_fits(jobs[b].n, jobs[b].m)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)k), block(kLdsThreads);
    if (ell) {
        if (wt == 2) launch_lg<2, true>(jobs[0].ell_lg, grid, block, st, a);
        else launch_lg<0, true>(jobs[0].ell_lg, grid, block, st, a);
    } else {
        if (wt == 2) launch_lg<2, false>(lg, grid, block, st, a);
        else launch_lg<0, false>(lg, grid, block, st, a);
    }
    return hipGetLastError();
}

}  // namespace gr
