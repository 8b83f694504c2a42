// HIP kernels for frontier-driven SSSP on gfx950 (MI355X).
//
// Operators (Osama et al., Section IV-C) on a CSR graph (Section IV-A) and a
// frontier kept both as a dense bitmap and a sparse queue (Section IV-B):
//   k_init    dist = INF, dist[src] = 0, frontier = {src} (Listing 4 set-up)
//   k_push    advance, push direction (Listing 3 / Listing 4 condition):
//             every out-edge of the sparse frontier is relaxed with an
//             atomic min; the destination joins the next bitmap iff the new
//             value is strictly smaller than the old one.  Edges are spread
//             evenly over blocks by a load-balanced search over the prefix
//             sum of frontier out-degrees, so one hub's edges are shared by
//             many blocks and every lane reads consecutive edges.
//   k_pull    advance, pull direction over the transposed graph
//             (Section III-C): each vertex takes the min over its in-arcs
//             from active vertices; one owner per vertex, no global atomics.
//   k_filter  deduplicated, compacted next frontier from the bitmap: vertex
//             ids (sorted within a block), their out-degree prefix sums and
//             the totals (F, E) that the convergence test reads.
//
// Distances are 32-bit patterns; binary32 values are non-negative, so their
// bit patterns order like the values and one uint32 atomic min serves both
// weight types.
#include "gr_internal.h"

#include <hip/hip_runtime.h>

namespace gr {

constexpr int kBlk = 256;  // threads per block (4 wave64)

// ---------------------------------------------------------------------------
// (+): uint32 add saturating at INF, or binary32 add (round to nearest even)
// clamped at FLT_MAX.  A clamped value equals INF and never wins a min.
template <int WT>
__device__ __forceinline__ uint32_t plus(uint32_t d, uint32_t w) {
    if constexpr (WT == 0) {
        uint32_t s = d + w;
        return s < d ? kInfU32 : s;
    } else {
        float s = __uint_as_float(d) + __uint_as_float(w);
        uint32_t b = __float_as_uint(s);
        return b > kInfF32 ? kInfF32 : b;
    }
}

// Arcs are streamed once per advance: non-temporal loads keep them from
// evicting the distance array and bitmaps from the caches.
__device__ __forceinline__ uint2 load_arc(const uint2 *p) {
    const unsigned long long x = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long *>(p));
    return make_uint2((uint32_t)x, (uint32_t)(x >> 32));
}

// Marks v in a frontier bitmap and its group summary.  The plain read first
// skips the atomic when the bit is already visible as set; bits are only set
// during an advance, so a stale read can only miss a set bit, never invent one.
__device__ __forceinline__ void mark(uint64_t *bits, uint64_t *sum, uint32_t v) {
    const uint64_t bit = 1ull << (v & 63);
    uint64_t *w = bits + (v >> 6);
    if (*reinterpret_cast<volatile uint64_t *>(w) & bit) return;
    uint64_t old = atomicOr(reinterpret_cast<unsigned long long *>(w), (unsigned long long)bit);
    if (old == 0) {
        const uint32_t g = v >> kGroupShift;
        atomicOr(reinterpret_cast<unsigned long long *>(sum + (g >> 6)), 1ull << (g & 63));
    }
}

// Relaxation of one edge (Listing 4): new = du (+) w, atomic min, strict <.
// The plain pre-read of dist[v] may be stale (older, hence larger or equal),
// so skipping when new >= pre-read never drops a needed update.
template <int WT>
__device__ __forceinline__ void relax(uint32_t *dist, uint64_t *nbits, uint64_t *nsum, uint32_t du, uint2 a) {
    const uint32_t v = a.x;
    const uint32_t nd = plus<WT>(du, a.y);
    const uint32_t cur = __builtin_nontemporal_load(dist + v);
    if (nd < cur) {
        const uint32_t old = atomicMin(dist + v, nd);
        if (nd < old) mark(nbits, nsum, v);
    }
}

// ---------------------------------------------------------------------------
// init
__global__ __launch_bounds__(kBlk) void k_init(uint32_t *__restrict__ dist, int32_t n, uint32_t inf, int32_t src,
                                               const int32_t *__restrict__ ro, uint64_t *b0, uint64_t *b1,
                                               int64_t nwords, uint64_t *s0, uint64_t *s1, int64_t nsumw,
                                               int32_t *q0, int32_t *s0q, unsigned long long *ctl) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v < n; v += stride) dist[v] = (v == src) ? 0u : inf;
    const int64_t sw = src >> 6;
    for (int64_t w = tid; w < nwords; w += stride) {
        b0[w] = (w == sw) ? (1ull << (src & 63)) : 0ull;
        b1[w] = 0ull;
    }
    const int64_t sg = src >> kGroupShift;
    for (int64_t w = tid; w < nsumw; w += stride) {
        s0[w] = (w == (sg >> 6)) ? (1ull << (sg & 63)) : 0ull;
        s1[w] = 0ull;
    }
    if (tid == 0) {
        const int32_t deg = ro[src + 1] - ro[src];
        q0[0] = src;
        s0q[0] = 0;
        ctl[0] = deg > 0 ? (1ull | ((unsigned long long)deg << 32)) : 0ull;
        for (int i = 1; i < kCtlWords; ++i) ctl[i] = 0ull;
    }
}

// ---------------------------------------------------------------------------
// push advance with load-balanced search.
//
// The sparse frontier q[0..F) has exclusive out-degree prefix sums s[0..F)
// (strictly increasing: the filter drops vertices without out-edges) and
// E = total.  Block b relaxes edge ranks [b*per_block, min(E, (b+1)*per_block)).
// It finds the frontier entry holding its first rank with a 256-way search,
// then walks windows of up to kWin consecutive entries staged in LDS; each
// lane maps its rank to an entry by binary search in LDS and reads the arc at
// ro[u] + (rank - s[entry]).  Consecutive lanes read consecutive arcs.
constexpr int kWin = 256;
constexpr int kPushItems = 4;

__device__ __forceinline__ int32_t find_entry(const int32_t *__restrict__ s, int32_t F, int32_t rank) {
    // Largest i in [0, F) with s[i] <= rank (s[0] = 0 <= rank); block-wide.
    int32_t lo = 0, hi = F;  // s[lo] <= rank < s[hi] (s[F] = E)
    while (hi - lo > 1) {
        const int64_t span = hi - lo;
        const int32_t p = lo + (int32_t)((span * threadIdx.x) / kBlk);
        const int ok = s[p] <= rank;
        const int c = __syncthreads_count(ok);  // samples are monotone: a prefix is <= rank
        const int32_t nlo = lo + (int32_t)((span * (c - 1)) / kBlk);
        const int32_t nhi = (c < kBlk) ? lo + (int32_t)((span * c) / kBlk) : hi;
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

template <int WT>
__global__ __launch_bounds__(kBlk) void k_push(const int32_t *__restrict__ ro, const uint2 *__restrict__ adj,
                                               uint32_t *__restrict__ dist, const int32_t *__restrict__ q,
                                               const int32_t *__restrict__ s, int32_t F, int32_t E,
                                               int32_t per_block, uint64_t *__restrict__ nbits,
                                               uint64_t *__restrict__ nsum) {
    __shared__ int32_t sS[kWin + 1];
    __shared__ int32_t sRow[kWin];
    __shared__ uint32_t sDu[kWin];

    const int64_t beg64 = (int64_t)blockIdx.x * per_block;
    if (beg64 >= E) return;
    const int32_t beg = (int32_t)beg64;
    const int32_t end = (int32_t)min<int64_t>(beg64 + per_block, E);

    int32_t i0 = find_entry(s, F, beg);
    int32_t e = beg;
    while (e < end) {
        const int32_t cnt = min(kWin, F - i0);
        for (int t = threadIdx.x; t < cnt; t += kBlk) {
            const int32_t u = q[i0 + t];
            sS[t] = s[i0 + t];
            sRow[t] = ro[u];
            sDu[t] = __builtin_nontemporal_load(dist + u);
        }
        if (threadIdx.x == 0) sS[cnt] = (i0 + cnt < F) ? s[i0 + cnt] : E;
        __syncthreads();
        const int32_t wend = min(end, sS[cnt]);
        for (int32_t x0 = e + threadIdx.x; x0 < wend; x0 += kBlk * kPushItems) {
            int32_t j[kPushItems];
            uint2 a[kPushItems];
#pragma unroll
            for (int k = 0; k < kPushItems; ++k) {
                const int32_t x = x0 + k * kBlk;
                int lo = 0, hi = cnt - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (sS[mid] <= x) lo = mid;
                    else hi = mid - 1;
                }
                j[k] = lo;
            }
#pragma unroll
            for (int k = 0; k < kPushItems; ++k) {
                const int32_t x = x0 + k * kBlk;
                if (x < wend) a[k] = load_arc(adj + sRow[j[k]] + (x - sS[j[k]]));
            }
#pragma unroll
            for (int k = 0; k < kPushItems; ++k) {
                const int32_t x = x0 + k * kBlk;
                if (x < wend) relax<WT>(dist, nbits, nsum, sDu[j[k]], a[k]);
            }
        }
        i0 += cnt;
        e = wend;
        __syncthreads();  // window reuse
    }
}

// ---------------------------------------------------------------------------
// pull advance: block owns vertices [v0, v0 + kBlk); its in-arcs are the
// contiguous CSC range [ro_in[v0], ro_in[v0 + kBlk]).  Lanes stride over that
// range, map each arc to its owner by binary search in LDS, and fold
// candidates dist[u] (+) w of active u into an LDS min per owner.  Then each
// owner compares with dist[v], stores the improvement (it is the only writer
// of dist[v] in this launch) and the wave writes its 64-bit bitmap word.
template <int WT>
__global__ __launch_bounds__(kBlk) void k_pull(int32_t n, const int32_t *__restrict__ ro_in,
                                               const uint2 *__restrict__ adj_in, uint32_t *__restrict__ dist,
                                               const uint64_t *__restrict__ cbits, uint64_t *__restrict__ nbits,
                                               uint64_t *__restrict__ nsum) {
    __shared__ int32_t sOff[kBlk + 1];
    __shared__ uint32_t sMin[kBlk];
    const int32_t v0 = blockIdx.x * kBlk;
    const int32_t nv = min(kBlk, n - v0);
    for (int t = threadIdx.x; t <= nv; t += kBlk) sOff[t] = ro_in[v0 + t];
    sMin[threadIdx.x] = kInfU32;
    __syncthreads();
    const int32_t a0 = sOff[0], a1 = sOff[nv];
    for (int32_t x = a0 + threadIdx.x; x < a1; x += kBlk) {
        const uint2 a = load_arc(adj_in + x);
        const uint32_t u = a.x;
        if ((cbits[u >> 6] >> (u & 63)) & 1ull) {
            int lo = 0, hi = nv - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (sOff[mid] <= x) lo = mid;
                else hi = mid - 1;
            }
            const uint32_t du = __builtin_nontemporal_load(dist + u);
            if (du != (WT == 0 ? kInfU32 : kInfF32)) atomicMin(&sMin[lo], plus<WT>(du, a.y));
        }
    }
    __syncthreads();
    const int32_t v = v0 + threadIdx.x;
    bool improved = false;
    if (threadIdx.x < nv) {
        const uint32_t cand = sMin[threadIdx.x];
        const uint32_t cur = dist[v];
        if (cand < cur) {
            dist[v] = cand;
            improved = true;
        }
    }
    const uint64_t word = __ballot(improved);
    if ((threadIdx.x & 63) == 0 && word) {
        nbits[v >> 6] = word;  // block is 64-aligned: this wave owns the word
        const uint32_t g = (uint32_t)v >> kGroupShift;
        atomicOr(reinterpret_cast<unsigned long long *>(nsum + (g >> 6)), 1ull << (g & 63));
    }
}

// ---------------------------------------------------------------------------
// filter: one block per 4096-vertex group; thread t owns vertices
// [base + 16 t, base + 16 t + 16), so the block's output is in vertex order.
// Reserves its slice of the next queue and of the degree prefix sum with one
// 64-bit atomic add of (count | degree_sum << 32).  Also clears the current
// frontier's bitmap (guided by its summary) so it can hold the frontier after
// next, and the last block to finish clears the current summary and counter.
constexpr int kVpt = kGroupVerts / kBlk;  // 16

__device__ __forceinline__ void block_scan2(int32_t &a, int32_t &b, int32_t &tot_a, int32_t &tot_b) {
    // exclusive scan of (a, b) over the block; returns totals.
    __shared__ int32_t wa[kBlk / 64], wb[kBlk / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t ia = a, ib = b;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t ta = __shfl_up(ia, o, 64), tb = __shfl_up(ib, o, 64);
        if (lane >= o) {
            ia += ta;
            ib += tb;
        }
    }
    if (lane == 63) {
        wa[wid] = ia;
        wb[wid] = ib;
    }
    __syncthreads();
    int32_t pa = 0, pb = 0;
    tot_a = 0;
    tot_b = 0;
#pragma unroll
    for (int w = 0; w < kBlk / 64; ++w) {
        if (w < wid) {
            pa += wa[w];
            pb += wb[w];
        }
        tot_a += wa[w];
        tot_b += wb[w];
    }
    a = pa + ia - a;
    b = pb + ib - b;
    __syncthreads();
}

__global__ __launch_bounds__(kBlk) void k_filter(int32_t n, const int32_t *__restrict__ ro,
                                                 const uint64_t *__restrict__ nbits,
                                                 const uint64_t *__restrict__ nsum, uint64_t *__restrict__ cbits,
                                                 uint64_t *__restrict__ csum, int64_t nsumw,
                                                 int32_t *__restrict__ q, int32_t *__restrict__ s,
                                                 unsigned long long *__restrict__ ctl_next,
                                                 unsigned long long *__restrict__ ctl_cur,
                                                 unsigned long long *__restrict__ done) {
    __shared__ unsigned long long sh_base;
    const int32_t g = blockIdx.x;
    const bool cur_has = (csum[g >> 6] >> (g & 63)) & 1ull;
    const bool nxt_has = (nsum[g >> 6] >> (g & 63)) & 1ull;
    if (cur_has && threadIdx.x < kGroupWords) cbits[(int64_t)g * kGroupWords + threadIdx.x] = 0ull;
    if (nxt_has) {
        const int64_t base = (int64_t)g * kGroupVerts + threadIdx.x * kVpt;
        const uint64_t word = nbits[base >> 6];
        const uint32_t mask16 = (uint32_t)(word >> (base & 63)) & 0xFFFFu;
        uint32_t keep = 0;
        int32_t cnt = 0, dsum = 0;
        for (int k = 0; k < kVpt; ++k) {
            if ((mask16 >> k) & 1u) {
                const int64_t v = base + k;
                const int32_t d = ro[v + 1] - ro[v];
                if (d > 0) {
                    keep |= 1u << k;
                    ++cnt;
                    dsum += d;
                }
            }
        }
        int32_t tc, td;
        block_scan2(cnt, dsum, tc, td);
        if (threadIdx.x == 0) {
            sh_base = tc ? atomicAdd(ctl_next, (unsigned long long)tc | ((unsigned long long)td << 32)) : 0ull;
        }
        __syncthreads();
        int32_t qpos = (int32_t)(sh_base & 0xFFFFFFFFull) + cnt;
        int32_t spos = (int32_t)(sh_base >> 32) + dsum;
        for (int k = 0; k < kVpt; ++k) {
            if ((keep >> k) & 1u) {
                const int64_t v = base + k;
                q[qpos] = (int32_t)v;
                s[qpos] = spos;
                ++qpos;
                spos += ro[v + 1] - ro[v];
            }
        }
    }
    // Last block out clears the current summary and counter slot.
    __shared__ bool last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(done, 1ull) == gridDim.x - 1;
    }
    __syncthreads();
    if (last) {
        for (int64_t w = threadIdx.x; w < nsumw; w += kBlk) csum[w] = 0ull;
        if (threadIdx.x == 0) {
            *ctl_cur = 0ull;
            *done = 0ull;
        }
    }
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
            if ((b & 0x80000000u) && b != 0x80000000u) e |= 4u;  // negative (but -0 is allowed)
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
    int32_t dummy = 0, tot, td;
    int32_t ex = t;
    block_scan2(ex, dummy, tot, td);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < len) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0 && bsum) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_add(int32_t *__restrict__ out, int64_t len, const int32_t *__restrict__ boff) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) out[i] += boff[i / kScanChunk];
}

__global__ void k_scatter_in(int32_t n, const int32_t *__restrict__ ro, const uint2 *__restrict__ adj,
                             const int32_t *__restrict__ ro_in, int32_t *__restrict__ fill,
                             uint2 *__restrict__ adj_in) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        for (int32_t e = ro[u]; e < ro[u + 1]; ++e) {
            const uint2 a = adj[e];
            const int32_t p = atomicAdd(fill + a.x, 1);
            adj_in[ro_in[a.x] + p] = make_uint2((uint32_t)u, a.y);
        }
    }
}

// Symmetric iff every row is strictly increasing and each arc u -> v of
// weight w has a reverse arc v -> u of the same weight bits.
__global__ void k_symmetry(int32_t n, const int32_t *__restrict__ ro, const uint2 *__restrict__ adj,
                           unsigned int *not_sym) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n && !bad; u += stride) {
        for (int32_t e = ro[u]; e < ro[u + 1] && !bad; ++e) {
            const uint2 a = adj[e];
            if (e + 1 < ro[u + 1] && adj[e + 1].x <= a.x) {
                bad = true;
                break;
            }
            int32_t lo = ro[a.x], hi = ro[a.x + 1];
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if ((int64_t)adj[mid].x < u) lo = mid + 1;
                else hi = mid;
            }
            if (lo >= ro[a.x + 1] || (int64_t)adj[lo].x != u || adj[lo].y != a.y) bad = true;
        }
    }
    if (bad) atomicOr(not_sym, 1u);
}

// ---------------------------------------------------------------------------
// launch wrappers

static inline int grid_for(int64_t items, int per_block, int cap) {
    int64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

hipError_t launch_init(const DevGraph &g, uint32_t *dist, int32_t src, const Frontier &f, hipStream_t st) {
    const uint32_t inf = g.wt == 1 ? kInfF32 : kInfU32;
    const int grid = grid_for(g.n, kBlk * 4, 8192);
    hipLaunchKernelGGL(k_init, dim3(grid), dim3(kBlk), 0, st, dist, g.n, inf, src, g.ro, f.bits[0], f.bits[1],
                       f.nwords, f.sum[0], f.sum[1], f.nsumw, f.q[0], f.s[0], f.ctl);
    return hipGetLastError();
}

hipError_t launch_push(const DevGraph &g, uint32_t *dist, const Frontier &f, int parity, int32_t F, int32_t E,
                       int num_cu, hipStream_t st) {
    if (F <= 0 || E <= 0) return hipSuccess;
    int64_t per = ((int64_t)E + (int64_t)num_cu * 8 - 1) / ((int64_t)num_cu * 8);
    if (per < 2048) per = 2048;
    per = (per + 255) & ~int64_t(255);
    const int grid = (int)(((int64_t)E + per - 1) / per);
    const int p = parity & 1, np = p ^ 1;
    if (g.wt == 1)
        hipLaunchKernelGGL(k_push<1>, dim3(grid), dim3(kBlk), 0, st, g.ro, g.adj, dist, f.q[p], f.s[p], F, E,
                           (int32_t)per, f.bits[np], f.sum[np]);
    else
        hipLaunchKernelGGL(k_push<0>, dim3(grid), dim3(kBlk), 0, st, g.ro, g.adj, dist, f.q[p], f.s[p], F, E,
                           (int32_t)per, f.bits[np], f.sum[np]);
    return hipGetLastError();
}

hipError_t launch_pull(const DevGraph &g, uint32_t *dist, const Frontier &f, int parity, hipStream_t st) {
    const int grid = (g.n + kBlk - 1) / kBlk;
    const int p = parity & 1, np = p ^ 1;
    if (g.wt == 1)
        hipLaunchKernelGGL(k_pull<1>, dim3(grid), dim3(kBlk), 0, st, g.n, g.ro_in, g.adj_in, dist, f.bits[p],
                           f.bits[np], f.sum[np]);
    else
        hipLaunchKernelGGL(k_pull<0>, dim3(grid), dim3(kBlk), 0, st, g.n, g.ro_in, g.adj_in, dist, f.bits[p],
                           f.bits[np], f.sum[np]);
    return hipGetLastError();
}

hipError_t launch_filter(const DevGraph &g, const Frontier &f, int parity, hipStream_t st) {
    const int p = parity & 1, np = p ^ 1;
    hipLaunchKernelGGL(k_filter, dim3(f.ngroups), dim3(kBlk), 0, st, g.n, g.ro, f.bits[np], f.sum[np], f.bits[p],
                       f.sum[p], f.nsumw, f.q[np], f.s[np], f.ctl + np, f.ctl + p, f.ctl + 2);
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
    // out[0..len) = exclusive scan of in; tmp needs >= 2 * ceil(len / 1024) + 2048 ints.
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
        hipLaunchKernelGGL(k_scatter_in, dim3(grid_for(n, kBlk, 16384)), dim3(kBlk), 0, st, n, ro, adj, ro_in, fill,
                           adj_in);
    return hipGetLastError();
}

hipError_t launch_symmetry_check(int32_t n, const int32_t *ro, const uint2 *adj, unsigned int *not_sym,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_symmetry, dim3(grid_for(n, kBlk, 16384)), dim3(kBlk), 0, st, n, ro, adj, not_sym);
    return hipGetLastError();
}

hipError_t launch_canon_negzero(uint2 *adj, int32_t m, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_canon_negzero, dim3(grid_for(m, kBlk * 8, 16384)), dim3(kBlk), 0, st, adj, m);
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

// ---------------------------------------------------------------------------
// frontier workspace layout

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t frontier_bytes(int64_t n) {
    const int64_t ng = groups_for(n);
    const int64_t nw = ng * kGroupWords;
    const int64_t ns = (ng + 63) / 64;
    size_t b = 0;
    b += 2 * align256(nw * 8);
    b += 2 * align256(ns * 8);
    b += 4 * align256((size_t)(n > 0 ? n : 1) * 4);
    b += align256(kCtlWords * 8);
    return b;
}

void frontier_carve(Frontier &f, void *base, int64_t n) {
    const int64_t ng = groups_for(n);
    f.ngroups = (int32_t)ng;
    f.nwords = ng * kGroupWords;
    f.nsumw = (ng + 63) / 64;
    char *p = static_cast<char *>(base);
    for (int i = 0; i < 2; ++i) {
        f.bits[i] = reinterpret_cast<uint64_t *>(p);
        p += align256(f.nwords * 8);
    }
    for (int i = 0; i < 2; ++i) {
        f.sum[i] = reinterpret_cast<uint64_t *>(p);
        p += align256(f.nsumw * 8);
    }
    for (int i = 0; i < 2; ++i) {
        f.q[i] = reinterpret_cast<int32_t *>(p);
        p += align256((size_t)(n > 0 ? n : 1) * 4);
        f.s[i] = reinterpret_cast<int32_t *>(p);
        p += align256((size_t)(n > 0 ? n : 1) * 4);
    }
    f.ctl = reinterpret_cast<unsigned long long *>(p);
}

}  // namespace gr
