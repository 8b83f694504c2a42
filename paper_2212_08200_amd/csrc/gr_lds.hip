// Single-workgroup loop for small graphs (Section III-A's loop, Listing 4's
// advance, with the whole query in one workgroup's LDS).
//
// Graphs of a few thousand vertices, such as small meshes, take one round per
// hop of their diameter, and each round of the other loops costs a kernel
// launch or a grid-wide barrier plus round trips to the L2.  Here one
// workgroup of 1024 threads copies the distances, row offsets and arcs into
// LDS (arcs packed as a 16-bit head and a 16-bit weight), keeps the frontier
// as a list of vertex ids in LDS, and runs the bulk-synchronous rounds with
// workgroup barriers and LDS atomics: a round is a few hundred cycles.
//
// Round r: every vertex u of list r is expanded by one thread: for each arc
// (u, v, w), new = dist[u] (+) w; if new beats dist[v], an LDS atomic min;
// when it lowered dist[v] and v is not yet in list r + 1 (a membership bit,
// claimed with an atomic or), v is appended.  After a barrier, list r + 1's
// membership bits are cleared.  dist[u] is read when u is expanded, so an
// improvement found earlier in the same round is used (as the other loops
// read dist[u] when staging their frontier).  The loop ends when a round
// appends nothing; the fixed point is the same.

#include "gr_lds.h"

#include "gr_device.h"

namespace gr {

namespace {

constexpr int kLdsThreads = 1024;

struct LdsArgs {
    int32_t n, m, src;
    int64_t max_rounds;
    const int32_t *ro;
    const uint2 *adj;
    uint32_t *dist;
    unsigned long long *stat;
};

template <int WT>
__global__ __launch_bounds__(kLdsThreads) void k_lds(LdsArgs a) {
    __shared__ uint32_t sMem[kLdsWords];
    __shared__ int32_t sCnt[2];
    __shared__ unsigned long long sArcs, sExp;
    const int t = threadIdx.x;
    const int32_t n = a.n, m = a.m;
    const int32_t nw = (n + 31) / 32;
    uint32_t *sD = sMem;
    int32_t *sRo = reinterpret_cast<int32_t *>(sMem + n);
    uint32_t *sArc = sMem + 2 * n + 1;
    uint32_t *sIn = sArc + m;
    uint16_t *sL[2] = {reinterpret_cast<uint16_t *>(sIn + nw), reinterpret_cast<uint16_t *>(sIn + nw) + n};
    const uint32_t inf = WT == 1 ? kInfF32 : kInfU32;
    for (int32_t v = t; v < n; v += kLdsThreads) sD[v] = inf;
    for (int32_t v = t; v <= n; v += kLdsThreads) sRo[v] = a.ro[v];
    for (int32_t e = t; e < m; e += kLdsThreads) {
        const uint2 x = a.adj[e];
        sArc[e] = WT == 2 ? x.x : (x.x << 16) | x.y;
    }
    for (int32_t w = t; w < nw; w += kLdsThreads) sIn[w] = 0u;
    if (t == 0) {
        sD[a.src] = 0u;
        sL[0][0] = (uint16_t)a.src;
        sCnt[0] = 1;
        sCnt[1] = 0;
        sArcs = 0ull;
        sExp = 0ull;
    }
    __syncthreads();
    uint32_t arcs = 0, expanded = 0;
    int64_t r = 0;
    for (; r < a.max_rounds; ++r) {
        const int c = (int)(r & 1);
        const int32_t cnt = sCnt[c];
        if (cnt == 0) break;  // uniform: read after a barrier
        for (int32_t i = t; i < cnt; i += kLdsThreads) {
            const uint32_t u = sL[c][i];
            const uint32_t du = sD[u];
            const int32_t e0 = sRo[u], e1 = sRo[u + 1];
            arcs += (uint32_t)(e1 - e0);
            expanded += e1 > e0 ? 1u : 0u;
            for (int32_t e = e0; e < e1; ++e) {
                const uint32_t x = sArc[e];
                const uint32_t v = WT == 2 ? x : x >> 16;
                const uint32_t nd = plus<WT>(du, WT == 2 ? 1u : (x & 0xFFFFu));
                if (nd < sD[v]) {
                    const uint32_t old = atomicMin(&sD[v], nd);
                    if (nd < old) {
                        const uint32_t bit = 1u << (v & 31u);
                        if (!(atomicOr(&sIn[v >> 5], bit) & bit)) sL[c ^ 1][atomicAdd(&sCnt[c ^ 1], 1)] = (uint16_t)v;
                    }
                }
            }
        }
        __syncthreads();
        // list r + 1 is complete: clear its membership bits and list r's count
        const int32_t nc = sCnt[c ^ 1];
        for (int32_t i = t; i < nc; i += kLdsThreads) {
            const uint32_t v = sL[c ^ 1][i];
            atomicAnd(&sIn[v >> 5], ~(1u << (v & 31u)));
        }
        if (t == 0) sCnt[c] = 0;
        __syncthreads();
    }
    for (int32_t v = t; v < n; v += kLdsThreads) a.dist[v] = sD[v];
    if (arcs) atomicAdd(&sArcs, (unsigned long long)arcs);
    if (expanded) atomicAdd(&sExp, (unsigned long long)expanded);
    __syncthreads();
    if (t == 0) {  // system scope: stat may be host memory
        __hip_atomic_store(a.stat + 0, (unsigned long long)r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(a.stat + 1, sCnt[r & 1] == 0 ? 1ull : 2ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(a.stat + 2, sArcs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(a.stat + 3, sExp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace

int64_t lds_words(int32_t n, int32_t m) {
    return 2 * (int64_t)n + 1 + m + (n + 31) / 32 + (n + 1) / 2 * 2;
}

hipError_t launch_lds(int32_t n, int32_t m, int wt, const int32_t *ro, const uint2 *adj, int32_t src,
                      uint32_t *dist_out, int64_t max_rounds, unsigned long long *stat, hipStream_t st) {
    if (!lds_fits(n, m) || src < 0 || src >= n || wt == 1) return hipErrorInvalidValue;
    LdsArgs a{n, m, src, max_rounds, ro, adj, dist_out, stat};
    if (wt == 2) hipLaunchKernelGGL(k_lds<2>, dim3(1), dim3(kLdsThreads), 0, st, a);
    else hipLaunchKernelGGL(k_lds<0>, dim3(1), dim3(kLdsThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace gr
