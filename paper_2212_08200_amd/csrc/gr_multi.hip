// Multi-query engine kernels (see gr_multi.h): independent single-source
// queries on one or several graphs share every launch of a round.
//
// The union queue of a round holds entries (first arc, u) of every live
// query, each tagged with its slot, in any order, with the exclusive prefix
// sum of their arc counts.  The push spreads the round's arcs evenly over the
// blocks (the load-balanced search of the single-source push), so a hub of a
// large graph and the short frontier of a small one are expanded by the same
// launch, and each relaxation applies Listing 4's rule in its own slot's
// distance array: new = dist[u] (+) w; atomic min into dist[v]; v joins the
// slot's next frontier iff new was below the value read (the marked set is the
// set of improved vertices, as in the single-source push).
#include "gr_device.h"
#include "gr_multi.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace gr {

// Global-memory pointers.  Pointers read from LDS or from the control block
// are otherwise generic, and generic (flat) loads and atomics share the wait
// counter of LDS reads: every LDS read of a push loop would then wait for all
// memory operations in flight.
template <class T>
using gptr = T __attribute__((address_space(1))) *;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ gptr<T> to_global(T *p) {
    return (gptr<T>)p;
}

__device__ __forceinline__ uint2 load_arc(gptr<const uint2> p) {
    const unsigned long long x = __builtin_nontemporal_load(reinterpret_cast<gptr<const unsigned long long>>(p));
    return make_uint2((uint32_t)x, (uint32_t)(x >> 32));
}

constexpr int kMqItems = 8;                    // arcs in flight per lane
constexpr int32_t kMqChunk = kBlk * kMqItems;  // smallest arc range of a block

__device__ __forceinline__ uint32_t plus_wt(int wt, uint32_t d, uint32_t w) {
    return wt == 1 ? plus<1>(d, w) : (wt == 2 ? plus<2>(d, w) : plus<0>(d, w));
}

__device__ __forceinline__ unsigned long long ld_relaxed(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlk) void k_mq_reset(MqCtl *ctl) {
    unsigned long long *w = reinterpret_cast<unsigned long long *>(ctl);
    const int64_t words = (int64_t)sizeof(MqCtl) / 8;
    for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < words; i += (int64_t)gridDim.x * kBlk) w[i] = 0ull;
}

// Admissions: slot entries, distances (INF, 0 at the source), cleared marks,
// the source appended to the queue of the round the next push runs.  Then the
// live set.  Blocks stride over the admitted slots' vertices.
__global__ __launch_bounds__(kBlk) void k_mq_update(MqBufs b, MqUpdate u) {
    MqCtl *ctl = b.ctl;
    const int64_t tid = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlk;
    for (int i = 0; i < u.nadmit; ++i) {
        const MqSlot &s = u.admit[i];
        const uint32_t inf = s.wt == 1 ? kInfF32 : kInfU32;
        const int32_t src = u.admit_src[i];
        for (int64_t v = tid; v < s.n; v += stride) s.dist[v] = v == src ? 0u : inf;
        for (int64_t w = tid; w < (int64_t)s.nflag * 2 / 16; w += stride)
            reinterpret_cast<uint4 *>(s.flags)[w] = make_uint4(0u, 0u, 0u, 0u);
        for (int64_t w = tid; w < (int64_t)s.ngroups * 2; w += stride) s.dirty[w] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const unsigned long long r = ctl->st_round[0];
        for (int i = 0; i < u.nadmit; ++i) {
            const int sl = u.admit_slot[i];
            const MqSlot &s = u.admit[i];
            ctl->slot[sl] = s;
            ctl->slot_rounds[sl] = 0ull;
            const int32_t src = u.admit_src[i];
            const int32_t first = s.ro[src];
            const int32_t deg = s.ro[src + 1] - first;
            if (deg > 0) {
                const unsigned long long c =
                    atomicAdd(&ctl->cnt[r % 3][0], 1ull | ((unsigned long long)(uint32_t)deg << 32));
                const int64_t pos = (int64_t)(c & 0xFFFFFFFFull);
                b.qse[r & 1][pos] = make_uint2((uint32_t)first, (uint32_t)src);
                b.qs[r & 1][pos] = (int32_t)(c >> 32);
                b.qslot[r & 1][pos] = (uint8_t)sl;
                ctl->slot_cnt[r % 3][sl] += 1ull;
            }
        }
        if (u.nlive >= 0) {
            ctl->nlive = u.nlive;
            for (int i = 0; i < kMqSlots; ++i) ctl->live[i] = u.live[i];
            for (int i = 0; i <= kMqSlots; ++i) ctl->gpre[i] = u.gpre[i];
        }
    }
}

// ---------------------------------------------------------------------------
// Local-hop list of a push block: (slot, vertex, candidate) entries, with a
// direct-mapped table from (slot, vertex) to its entry, so that a vertex
// improved again before its hop keeps one entry with the smaller candidate.
// A table miss (another key in the way, or an entry still being written by
// another wave) only adds a second entry, which is harmless: each entry is
// one expansion.
constexpr int kMqTag = 2048;

__device__ __forceinline__ bool local_keep(uint32_t v, uint32_t nd, int sl, uint32_t *lv, uint32_t *ld, uint8_t *ls,
                                           int32_t *ln, int32_t *tag) {
    const uint32_t h = (v * 2654435761u + (uint32_t)sl * 40503u) >> 21;  // 11 bits
    // the entry's fields are written before its tag is published (release),
    // and read after the tag (acquire), so a hit sees a complete entry
    const int32_t q = __hip_atomic_load(&tag[h], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (q >= 0 && q < kMqLocalCap && lv[q] == v && ls[q] == (uint8_t)sl) {
        atomicMin(&ld[q], nd);
        return true;
    }
    const int32_t p = atomicAdd(ln, 1);
    if (p >= kMqLocalCap) return false;
    lv[p] = v;
    ld[p] = nd;
    ls[p] = (uint8_t)sl;
    __hip_atomic_store(&tag[h], p, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    return true;
}

// ---------------------------------------------------------------------------
// push of the round in st_round[0]

__global__ __launch_bounds__(kBlk) void k_mq_push(MqBufs b) {
    __shared__ int32_t sS[kWin + 1];
    __shared__ gptr<const uint2> sArc[kWin];
    __shared__ uint32_t sDu[kWin];
    __shared__ uint8_t sSl[kWin];
    __shared__ gptr<uint32_t> tDist[kMqSlots];
    __shared__ gptr<uint8_t> tFl[kMqSlots];
    __shared__ gptr<uint8_t> tDirty[kMqSlots];
    __shared__ gptr<const uint2> tAdj[kMqSlots];
    __shared__ gptr<const int32_t> tRo[kMqSlots];
    __shared__ int32_t tWt[kMqSlots];
    __shared__ int32_t tLight[kMqSlots];
    __shared__ uint32_t lV[2][kMqLocalCap], lD[2][kMqLocalCap];
    __shared__ uint8_t lS[2][kMqLocalCap];
    __shared__ int32_t lN[2];
    __shared__ int32_t lTag[kMqTag];
    MqCtl *ctl = b.ctl;
    const int hops = b.local_hops > 1 ? b.local_hops : 1;
    const unsigned long long r = ctl->st_round[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->st_round[1] = r;
    const unsigned long long c = ld_relaxed(&ctl->cnt[r % 3][0]);
    const int32_t F = (int32_t)(c & 0xFFFFFFFFull), E = (int32_t)(c >> 32);
    if (F <= 0) return;  // idle round (uniform)
    const int cur = (int)(r & 1), nxt = cur ^ 1;
    if (blockIdx.x == 0) {
        // counters of the next round's queue (last used two rounds ago)
        if (threadIdx.x == 0) {
            ctl->cnt[(r + 1) % 3][0] = 0ull;
            ctl->rounds += 1ull;
            ctl->edges += (unsigned long long)E;
            ctl->frontier += (unsigned long long)F;
        }
        if (threadIdx.x < kMqSlots) {
            const int s = threadIdx.x;
            ctl->slot_cnt[(r + 1) % 3][s] = 0ull;
            if (ctl->slot_cnt[r % 3][s] > 0ull) ctl->slot_rounds[s] += 1ull;
        }
    }
    if (threadIdx.x < kMqSlots) {
        const MqSlot &s = ctl->slot[threadIdx.x];
        tDist[threadIdx.x] = to_global(s.dist);
        tFl[threadIdx.x] = to_global(s.flags + (size_t)nxt * s.nflag);
        tDirty[threadIdx.x] = to_global(s.dirty + (size_t)nxt * s.ngroups);
        tAdj[threadIdx.x] = to_global(s.adj);
        tRo[threadIdx.x] = to_global(s.ro);
        tWt[threadIdx.x] = s.wt;
        tLight[threadIdx.x] = s.light;
    }
    if (threadIdx.x == 0) lN[0] = 0;
    for (int t = threadIdx.x; t < kMqTag; t += kBlk) lTag[t] = -1;
    __syncthreads();
    const uint2 *__restrict__ qse = b.qse[cur];
    const int32_t *__restrict__ qs = b.qs[cur];
    const uint8_t *__restrict__ qsl = b.qslot[cur];
    const int32_t per = (int32_t)max<int64_t>(kMqChunk, ((int64_t)E + gridDim.x - 1) / gridDim.x);
    const int32_t chunks = (int32_t)(((int64_t)E + per - 1) / per);
    for (int32_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
        const int32_t beg = ch * per;
        const int32_t end = (int32_t)min<int64_t>((int64_t)beg + per, E);
        int32_t i0 = find_entry(qs, F, beg);
        int32_t e = beg;
        while (e < end) {
            const int32_t cnt = min(kWin, F - i0);
            for (int t = threadIdx.x; t < cnt; t += kBlk) {
                const uint2 q = qse[i0 + t];
                const int sl = qsl[i0 + t];
                sS[t] = qs[i0 + t];
                sArc[t] = tAdj[sl] + q.x;
                sDu[t] = tDist[sl][q.y];  // read now: a value lowered earlier in the round saves work
                sSl[t] = (uint8_t)sl;
            }
            for (int t = cnt + threadIdx.x; t <= kWin; t += kBlk)
                sS[t] = (t == cnt) ? ((i0 + cnt < F) ? qs[i0 + cnt] : E) : INT32_MAX;
            __syncthreads();
            const int32_t wend = min(end, sS[cnt]);
            for (int32_t x0 = e + (int32_t)threadIdx.x; x0 < wend; x0 += kBlk * kMqItems) {
                int32_t xr[kMqItems], pos[kMqItems];
#pragma unroll
                for (int it = 0; it < kMqItems; ++it) {
                    xr[it] = min(x0 + it * kBlk, wend - 1);
                    pos[it] = 0;
                }
#pragma unroll
                for (int bb = kWin / 2; bb >= 1; bb >>= 1) {
#pragma unroll
                    for (int it = 0; it < kMqItems; ++it) {
                        const int32_t p = pos[it] + bb;
                        pos[it] = (sS[p] <= xr[it]) ? p : pos[it];
                    }
                }
                uint2 arc[kMqItems];
                int sl[kMqItems];
#pragma unroll
                for (int it = 0; it < kMqItems; ++it) {
                    arc[it] = load_arc(sArc[pos[it]] + (xr[it] - sS[pos[it]]));
                    sl[it] = sSl[pos[it]];
                }
                uint32_t nd[kMqItems], cv[kMqItems];
#pragma unroll
                for (int it = 0; it < kMqItems; ++it) {
                    nd[it] = plus_wt(tWt[sl[it]], sDu[pos[it]], arc[it].y);
                    cv[it] = tDist[sl[it]][arc[it].x];
                }
#pragma unroll
                for (int it = 0; it < kMqItems; ++it) {
                    if (x0 + it * kBlk < wend && nd[it] < cv[it]) {
                        const uint32_t v = arc[it].x;
                        __hip_atomic_fetch_min(tDist[sl[it]] + v, nd[it], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const bool kept =
                            hops > 1 && tLight[sl[it]] && local_keep(v, nd[it], sl[it], lV[0], lD[0], lS[0], &lN[0], lTag);
                        if (!kept) {
                            tFl[sl[it]][v] = 1;
                            tDirty[sl[it]][v >> kGroupShift] = 1;
                        }
                    }
                }
            }
            i0 += cnt;
            e = wend;
            __syncthreads();  // window reuse
        }
    }
    // local hops over the light-graph vertices this block improved
    uint32_t st_v = 0, st_e = 0;
    for (int h = 1; h < hops; ++h) {
        const int sp = (h - 1) & 1, dp = h & 1;
        __syncthreads();
        const int32_t nloc = min(lN[sp], kMqLocalCap);
        if (nloc == 0) break;  // uniform: LDS read after a barrier
        __syncthreads();       // every thread has read lN[sp] before lN[dp] is reset
        if (threadIdx.x == 0) lN[dp] = 0;
        for (int t = threadIdx.x; t < kMqTag; t += kBlk) lTag[t] = -1;
        __syncthreads();
        const bool last = h == hops - 1;
        for (int32_t i = threadIdx.x; i < nloc; i += kBlk) {
            const uint32_t v = lV[sp][i], c = lD[sp][i];
            const int sl = lS[sp][i];
            const int32_t st = tRo[sl][v];
            const int32_t deg = min(tRo[sl][v + 1] - st, kMqLight);
            uint2 arc[kMqLight];
            uint32_t cur[kMqLight], nd[kMqLight];
#pragma unroll
            for (int it = 0; it < kMqLight; ++it) arc[it] = it < deg ? load_arc(tAdj[sl] + st + it) : make_uint2(0u, 0u);
#pragma unroll
            for (int it = 0; it < kMqLight; ++it) {
                nd[it] = plus_wt(tWt[sl], c, arc[it].y);
                // unguarded: an item past the degree reads vertex 0 (its arc is
                // (0, 0)); a guarded load with a default value made each item
                // wait for the previous one
                cur[it] = tDist[sl][arc[it].x];
            }
            st_v += deg > 0 ? 1u : 0u;
            st_e += (uint32_t)deg;
#pragma unroll
            for (int it = 0; it < kMqLight; ++it) {
                if (it < deg && nd[it] < cur[it]) {
                    const uint32_t w = arc[it].x;
                    __hip_atomic_fetch_min(tDist[sl] + w, nd[it], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const bool kept = !last && local_keep(w, nd[it], sl, lV[dp], lD[dp], lS[dp], &lN[dp], lTag);
                    if (!kept) {
                        tFl[sl][w] = 1;
                        tDirty[sl][w >> kGroupShift] = 1;
                    }
                }
            }
        }
    }
    if (hops > 1) {
        int32_t x[2] = {(int32_t)st_v, (int32_t)st_e}, tot[2];
        block_scan<2>(x, tot);
        if (threadIdx.x == 0 && tot[0] > 0) {
            atomicAdd(&ctl->frontier, (unsigned long long)tot[0]);
            atomicAdd(&ctl->edges, (unsigned long long)tot[1]);
        }
    }
}

// ---------------------------------------------------------------------------
// filter of the round in st_round[1]: compacts the marks of every dirty group
// of every live slot into the next union queue.

__global__ __launch_bounds__(kBlk) void k_mq_filter(MqBufs b) {
    __shared__ int32_t sGpre[kMqSlots + 1];
    __shared__ int32_t sLive[kMqSlots];
    __shared__ int32_t sList[kBlk];
    __shared__ int32_t sCount;
    __shared__ unsigned long long sBase;
    MqCtl *ctl = b.ctl;
    const unsigned long long r = ctl->st_round[1];
    const unsigned long long c = ld_relaxed(&ctl->cnt[r % 3][0]);
    const int32_t F = (int32_t)(c & 0xFFFFFFFFull);
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->st_round[0] = F > 0 ? r + 1 : r;
    if (F <= 0) return;
    const int cur = (int)(r & 1), nxt = cur ^ 1;
    if (b.mask[0]) {
        // batched same-graph queries: the active-source masks of this round
        // were read by the push that just ended; they are cleared whole, with
        // streaming stores (cheaper than a random store per frontier vertex)
        uint4 *mc = reinterpret_cast<uint4 *>(b.mask[cur]);
        const int64_t words = (int64_t)ctl->slot[0].n / 2;  // two masks per 16-byte word
        for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < words; i += (int64_t)gridDim.x * kBlk)
            mc[i] = make_uint4(0u, 0u, 0u, 0u);
        if ((ctl->slot[0].n & 1) && blockIdx.x == 0 && threadIdx.x == 0) b.mask[cur][ctl->slot[0].n - 1] = 0ull;
    }
    const int32_t nlive = ctl->nlive;
    for (int t = threadIdx.x; t <= kMqSlots; t += kBlk) {
        if (t < kMqSlots) sLive[t] = ctl->live[t];
        sGpre[t] = t <= nlive ? ctl->gpre[t] : INT32_MAX;
    }
    __syncthreads();
    const int32_t GT = sGpre[nlive];
    unsigned long long *ncnt = &ctl->cnt[(r + 1) % 3][0];
    // block b owns groups b, b + G, b + 2G, ... (G = grid size): its threads
    // test the dirty bytes of up to 256 of them at once, then the whole block
    // compacts each dirty one
    const int64_t G = gridDim.x;
    const int64_t mine = GT > (int64_t)blockIdx.x ? (GT - 1 - (int64_t)blockIdx.x) / G + 1 : 0;
    for (int64_t j0 = 0; j0 < mine; j0 += kBlk) {
        if (threadIdx.x == 0) sCount = 0;
        __syncthreads();
        const int64_t jj = j0 + threadIdx.x;
        if (jj < mine) {
            const int64_t x = (int64_t)blockIdx.x + jj * G;
            int j = 0;  // live index of group x: largest j with gpre[j] <= x
#pragma unroll
            for (int bb = kMqSlots / 2; bb >= 1; bb >>= 1) j = (j + bb < nlive && sGpre[j + bb] <= x) ? j + bb : j;
            const MqSlot &s = ctl->slot[sLive[j]];
            const int32_t g = (int32_t)(x - sGpre[j]);
            if (to_global(s.dirty)[(size_t)nxt * s.ngroups + g]) sList[atomicAdd(&sCount, 1)] = (int32_t)x;
        }
        __syncthreads();
        const int nd = sCount;
        for (int q = 0; q < nd; ++q) {
            const int32_t xg = sList[q];
            int j = 0;
#pragma unroll
            for (int bb = kMqSlots / 2; bb >= 1; bb >>= 1) j = (j + bb < nlive && sGpre[j + bb] <= xg) ? j + bb : j;
            const int sl = sLive[j];
            const MqSlot &s = ctl->slot[sl];
            const int64_t g = xg - sGpre[j];
            gptr<uint8_t> fl = to_global(s.flags + (size_t)nxt * s.nflag);
            gptr<const int32_t> ro = to_global(s.ro);
            const int64_t base = g * kGroupVerts + threadIdx.x * 16;
            const u32x4 w = reinterpret_cast<gptr<const u32x4>>(fl)[base >> 4];
            uint32_t m = 0;
#pragma unroll
            for (int bt = 0; bt < 16; ++bt) {
                const uint32_t word = bt < 4 ? w.x : bt < 8 ? w.y : bt < 12 ? w.z : w.w;
                m |= (((word >> ((bt & 3) * 8)) & 0xFFu) != 0u ? 1u : 0u) << bt;
            }
            if (m) reinterpret_cast<gptr<u32x4>>(fl)[base >> 4] = u32x4{0u, 0u, 0u, 0u};
            int32_t xx[2] = {0, 0}, tot[2];
            for (uint32_t mm = m; mm; mm &= mm - 1) {
                const int64_t u = base + __builtin_ctz(mm);
                const int32_t d = ro[u + 1] - ro[u];
                xx[0] += d > 0 ? 1 : 0;
                xx[1] += d;
            }
            block_scan<2>(xx, tot);
            if (threadIdx.x == 0) {
                to_global(s.dirty)[(size_t)nxt * s.ngroups + g] = 0;
                sBase = tot[0] ? atomicAdd(ncnt, (unsigned long long)tot[0] | ((unsigned long long)tot[1] << 32)) : 0ull;
                if (tot[0]) atomicAdd(&ctl->slot_cnt[(r + 1) % 3][sl], (unsigned long long)tot[0]);
            }
            __syncthreads();
            int32_t pos = (int32_t)(sBase & 0xFFFFFFFFull) + xx[0];
            int32_t spos = (int32_t)(sBase >> 32) + xx[1];
            for (uint32_t mm = m; mm; mm &= mm - 1) {
                const int64_t u = base + __builtin_ctz(mm);
                const int32_t f = ro[u];
                const int32_t d = ro[u + 1] - f;
                if (d > 0) {
                    b.qse[nxt][pos] = make_uint2((uint32_t)f, (uint32_t)u);
                    b.qs[nxt][pos] = spos;
                    b.qslot[nxt][pos] = (uint8_t)sl;
                    ++pos;
                    spos += d;
                }
            }
            __syncthreads();  // sBase reuse
        }
    }
}

// ---------------------------------------------------------------------------
// Batched same-graph queries: up to 64 sources, one per lane of a wave.  Each
// arc of a queued vertex u is read once for every source active at u; lane s
// relaxes it for source s (Listing 4's rule in row s of the vertex-major
// distance matrix), and a wave ballot of the lanes that improved v sets v's
// next mask with one atomic or.

__global__ __launch_bounds__(kBlk) void k_mq_batch_init(MqBufs b, MqSlot s, uint32_t *__restrict__ D, uint32_t inf) {
    const int64_t tid = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlk;
    const uint4 q = make_uint4(inf, inf, inf, inf);
    for (int64_t i = tid; i < (int64_t)s.n * (kBatchLanes / 4); i += stride) reinterpret_cast<uint4 *>(D)[i] = q;
    for (int64_t i = tid; i < s.n; i += stride) {
        b.mask[0][i] = 0ull;
        b.mask[1][i] = 0ull;
    }
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t w = tid; w < (int64_t)s.nflag * 2 / 16; w += stride) reinterpret_cast<uint4 *>(s.flags)[w] = z;
    for (int64_t w = tid; w < (int64_t)s.ngroups * 2; w += stride) s.dirty[w] = 0;
}

// One block of 64 threads: lane j starts source j at distance 0, active at
// its vertex; then each distinct source vertex with arcs becomes one entry of
// round 0's queue, and slot 0 becomes the only live slot.
__global__ void k_mq_batch_sources(MqBufs b, MqSlot s, uint32_t *__restrict__ D, MqBatchSrc src) {
    MqCtl *ctl = b.ctl;
    const int j = threadIdx.x;
    if (j < src.k) {
        const int64_t v = src.src[j];
        D[v * kBatchLanes + j] = 0u;
        atomicOr(reinterpret_cast<unsigned long long *>(b.mask[0] + v), 1ull << j);
    }
    __syncthreads();
    if (j == 0) {
        ctl->slot[0] = s;
        ctl->nlive = 1;
        ctl->live[0] = 0;
        ctl->gpre[0] = 0;
        for (int i = 1; i <= kMqSlots; ++i) ctl->gpre[i] = s.ngroups;
        for (int i = 0; i < src.k; ++i) {
            bool first = true;
            for (int t = 0; t < i; ++t) first = first && src.src[t] != src.src[i];
            const int32_t v = src.src[i];
            const int32_t f = s.ro[v], d = s.ro[v + 1] - f;
            if (!first || d <= 0) continue;
            const unsigned long long c = ctl->cnt[0][0];
            const int64_t pos = (int64_t)(c & 0xFFFFFFFFull);
            b.qse[0][pos] = make_uint2((uint32_t)f, (uint32_t)v);
            b.qs[0][pos] = (int32_t)(c >> 32);
            b.qslot[0][pos] = 0;
            ctl->cnt[0][0] = c + (1ull | ((unsigned long long)(uint32_t)d << 32));
            ctl->slot_cnt[0][0] += 1ull;
        }
    }
}

// 4 arcs per wave iteration and many small blocks (each takes at least 512
// arcs): the uneven per-arc work (active sources vary by vertex) balances
// over the grid.
constexpr int kBatchArcs = 4;
constexpr int32_t kBatchMinPer = 512;

template <int WT>
__global__ __launch_bounds__(kBlk) void k_mq_batch_push(MqBufs b, uint32_t *__restrict__ D) {
    __shared__ int32_t sS[kWin + 1];
    __shared__ uint32_t sRow[kWin];
    __shared__ uint32_t sU[kWin];
    MqCtl *ctl = b.ctl;
    const unsigned long long r = ctl->st_round[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->st_round[1] = r;
    const unsigned long long c = ld_relaxed(&ctl->cnt[r % 3][0]);
    const int32_t F = (int32_t)(c & 0xFFFFFFFFull), E = (int32_t)(c >> 32);
    if (F <= 0) return;
    const int cur = (int)(r & 1), nxt = cur ^ 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->cnt[(r + 1) % 3][0] = 0ull;
        ctl->slot_cnt[(r + 1) % 3][0] = 0ull;
        ctl->rounds += 1ull;
        ctl->edges += (unsigned long long)E;
        ctl->frontier += (unsigned long long)F;
        ctl->slot_rounds[0] += 1ull;
    }
    const int32_t per = (int32_t)max<int64_t>(kBatchMinPer, ((int64_t)E + gridDim.x - 1) / gridDim.x);
    const int64_t beg64 = (int64_t)blockIdx.x * per;
    if (beg64 >= E) return;  // uniform per block
    const int32_t beg = (int32_t)beg64;
    const int32_t end = (int32_t)min<int64_t>(beg64 + per, E);
    const MqSlot &sl = ctl->slot[0];
    const uint2 *__restrict__ adj = sl.adj;
    uint8_t *nfl = sl.flags + (size_t)nxt * sl.nflag;
    uint8_t *ndirty = sl.dirty + (size_t)nxt * sl.ngroups;
    const uint64_t *__restrict__ mcur = b.mask[cur];
    uint64_t *mnext = b.mask[nxt];
    const uint2 *__restrict__ qse = b.qse[cur];
    const int32_t *__restrict__ qs = b.qs[cur];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t lanebit = 1ull << lane;
    uint32_t pairs = 0;

    int32_t i0 = find_entry(qs, F, beg);
    int32_t e = beg;
    while (e < end) {
        const int32_t cnt = min(kWin, F - i0);
        for (int t = threadIdx.x; t < cnt; t += kBlk) {
            const uint2 q = qse[i0 + t];
            sS[t] = qs[i0 + t];
            sRow[t] = q.x;
            sU[t] = q.y;
        }
        for (int t = cnt + threadIdx.x; t <= kWin; t += kBlk)
            sS[t] = (t == cnt) ? ((i0 + cnt < F) ? qs[i0 + cnt] : E) : INT32_MAX;
        __syncthreads();
        const int32_t wend = min(end, sS[cnt]);
        // this wave's contiguous share of the window's ranks
        const int32_t span = wend - e;
        const int32_t share = (span + (kBlk / 64) - 1) / (kBlk / 64);
        const int32_t r0 = e + wid * share;
        const int32_t r1 = min(wend, r0 + share);
        // 64 ranks at a time: lane l finds the entry of rank x0 + l and loads
        // that arc and its tail's mask (one search, one arc load and one mask
        // load per 64 arcs); the wave then walks the 64 arcs, taking each
        // one's fields from the lane that staged it (register broadcasts, no
        // per-arc search or uniform loads).
        for (int32_t x0 = r0; x0 < r1; x0 += 64) {
            const int32_t cntj = min(64, r1 - x0);
            const int32_t xl = min(x0 + lane, r1 - 1);
            int32_t p = 0;
#pragma unroll
            for (int bb = kWin / 2; bb >= 1; bb >>= 1) p = (sS[p + bb] <= xl) ? p + bb : p;
            const uint32_t ul = sU[p];
            const uint2 al = load_arc(adj + sRow[p] + (uint32_t)(xl - sS[p]));
            const uint64_t ml = mcur[ul];
            const uint32_t mlo = (uint32_t)ml, mhi = (uint32_t)(ml >> 32);
            for (int32_t j = 0; j < cntj; j += kBatchArcs) {
                uint32_t uu[kBatchArcs], vv[kBatchArcs], ww[kBatchArcs], du[kBatchArcs], dv[kBatchArcs];
                bool act[kBatchArcs];
#pragma unroll
                for (int it = 0; it < kBatchArcs; ++it) {
                    const int jj = min(j + it, cntj - 1);  // clamped: repeats the last arc, masked below
                    uu[it] = (uint32_t)__builtin_amdgcn_readlane((int)ul, jj);
                    vv[it] = (uint32_t)__builtin_amdgcn_readlane((int)al.x, jj);
                    ww[it] = (uint32_t)__builtin_amdgcn_readlane((int)al.y, jj);
                    const uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)mhi, jj) << 32) |
                                       (uint32_t)__builtin_amdgcn_readlane((int)mlo, jj);
                    act[it] = (j + it < cntj) && ((m >> lane) & 1ull) != 0ull;
                }
                // Every lane loads: an inactive lane reads its entry of u's row
                // (read for du anyway) instead of v's, so no line of v's row that
                // no active lane needs is fetched, and the loads stay
                // unpredicated (a predicated load with a default value costs a
                // wait for every load in flight on the path that writes it).
#pragma unroll
                for (int it = 0; it < kBatchArcs; ++it) {
                    uint32_t w = act[it] ? vv[it] : uu[it];
                    asm volatile("" : "+v"(w));  // keeps the select: no load-or-copy branch
                    du[it] = D[(int64_t)uu[it] * kBatchLanes + lane];
                    dv[it] = D[(int64_t)w * kBatchLanes + lane];
                }
#pragma unroll
                for (int it = 0; it < kBatchArcs; ++it) {
                    pairs += act[it] ? 1u : 0u;
                    const uint32_t nd = plus<WT>(du[it], ww[it]);
                    const bool better = act[it] && nd < dv[it];
                    if (better)
                        __hip_atomic_fetch_min(D + (int64_t)vv[it] * kBatchLanes + lane, nd, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    const uint64_t won = __ballot(better);
                    if (won && lane == 0) {
                        const uint32_t v = vv[it];
                        __hip_atomic_fetch_or(reinterpret_cast<unsigned long long *>(mnext + v), won,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        nfl[v] = 1;
                        ndirty[v >> kGroupShift] = 1;
                    }
                }
            }
        }
        i0 += cnt;
        e = wend;
        __syncthreads();  // window reuse
    }
    int32_t x[1] = {(int32_t)pairs}, tot[1];
    block_scan<1>(x, tot);
    if (threadIdx.x == 0 && tot[0]) atomicAdd(&ctl->pairs, (unsigned long long)tot[0]);
}

// D (n x 64, vertex-major) -> rows[j][v] for j < k, through an LDS tile of 64
// vertices x 64 sources so that both sides are coalesced.
__global__ __launch_bounds__(kBlk) void k_mq_batch_output(const uint32_t *__restrict__ D, int32_t n, int32_t k,
                                                          MqOutRows rows) {
    __shared__ uint32_t tile[64][65];
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    for (int i = threadIdx.x; i < 64 * 64; i += kBlk) {
        const int r = i >> 6, cc = i & 63;
        tile[r][cc] = (v0 + r < n) ? D[(v0 + r) * kBatchLanes + cc] : 0u;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * 64; i += kBlk) {
        const int j = i >> 6, r = i & 63;
        if (j < k && v0 + r < n) rows.row[j][v0 + r] = tile[r][j];
    }
}

// ---------------------------------------------------------------------------

size_t mq_ctl_bytes() { return (sizeof(MqCtl) + 255) & ~size_t(255); }

hipError_t mq_reset(const MqBufs &b, hipStream_t st) {
    hipLaunchKernelGGL(k_mq_reset, dim3(4), dim3(kBlk), 0, st, b.ctl);
    return hipGetLastError();
}

hipError_t mq_update(const MqBufs &b, const MqUpdate &u, hipStream_t st) {
    int64_t work = 1;
    for (int i = 0; i < u.nadmit; ++i) work = std::max<int64_t>(work, u.admit[i].n);
    int grid = (int)std::min<int64_t>(2048, (work + kBlk * 4 - 1) / (kBlk * 4));
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_mq_update, dim3(grid), dim3(kBlk), 0, st, b, u);
    return hipGetLastError();
}

hipError_t mq_batch_init(const MqBufs &b, const MqSlot &s, uint32_t *D, const MqBatchSrc &src, hipStream_t st) {
    const uint32_t inf = s.wt == 1 ? kInfF32 : kInfU32;
    int64_t grid = ((int64_t)s.n * (kBatchLanes / 4) + kBlk * 4 - 1) / (kBlk * 4);
    grid = std::min<int64_t>(std::max<int64_t>(grid, 1), 16384);
    hipLaunchKernelGGL(k_mq_batch_init, dim3((unsigned)grid), dim3(kBlk), 0, st, b, s, D, inf);
    hipLaunchKernelGGL(k_mq_batch_sources, dim3(1), dim3(kBatchLanes), 0, st, b, s, D, src);
    return hipGetLastError();
}

hipError_t mq_batch_round(const MqBufs &b, uint32_t *D, int wt, int push_grid, int filter_grid, hipStream_t st) {
    if (wt == 1) hipLaunchKernelGGL(k_mq_batch_push<1>, dim3(push_grid), dim3(kBlk), 0, st, b, D);
    else hipLaunchKernelGGL(k_mq_batch_push<0>, dim3(push_grid), dim3(kBlk), 0, st, b, D);
    hipLaunchKernelGGL(k_mq_filter, dim3(filter_grid), dim3(kBlk), 0, st, b);
    return hipGetLastError();
}

hipError_t mq_batch_output(const uint32_t *D, int32_t n, int32_t k, const MqOutRows &rows, hipStream_t st) {
    hipLaunchKernelGGL(k_mq_batch_output, dim3((unsigned)((n + 63) / 64)), dim3(kBlk), 0, st, D, n, k, rows);
    return hipGetLastError();
}

hipError_t mq_round(const MqBufs &b, int push_grid, int filter_grid, hipStream_t st) {
    hipLaunchKernelGGL(k_mq_push, dim3(push_grid), dim3(kBlk), 0, st, b);
    hipLaunchKernelGGL(k_mq_filter, dim3(filter_grid), dim3(kBlk), 0, st, b);
    return hipGetLastError();
}

}  // namespace gr
