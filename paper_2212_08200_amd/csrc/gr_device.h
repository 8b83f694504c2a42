// Device helpers shared by the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "gr_internal.h"

namespace gr {

constexpr int kBlk = 256;  // threads per block (4 wave64)
constexpr int kWin = 256;  // frontier entries staged in LDS per window

// ---------------------------------------------------------------------------
// (+): uint32 add saturating at INF, or binary32 add (round to nearest even)
// clamped at FLT_MAX, or (WT = 2) one hop.  A clamped value equals INF and
// never wins a min.
template <int WT>
__device__ __forceinline__ uint32_t plus(uint32_t d, uint32_t w) {
    if constexpr (WT == 2) {  // unit weights (breadth-first search): the arc weight is not used
        (void)w;
        return d == kInfU32 ? kInfU32 : d + 1u;
    } else if constexpr (WT == 0) {
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

// Element idx of base.  With O32 the address is formed as a uniform base plus
// a 32-bit byte offset, so each lane holds one offset register instead of a
// 64-bit address (a large share of the registers of the gather-heavy loops);
// the caller guarantees idx * sizeof(T) < 2^32.
template <bool O32, typename T>
__device__ __forceinline__ T *elem(T *base, uint32_t idx) {
    if constexpr (O32) {
        using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
        return reinterpret_cast<T *>(reinterpret_cast<C *>(base) + (uint32_t)(idx * (uint32_t)sizeof(T)));
    } else {
        return base + idx;
    }
}

// Exclusive block-wide scan of V values per thread; tot receives the totals.
template <int V>
__device__ __forceinline__ void block_scan(int32_t (&x)[V], int32_t (&tot)[V]) {
    __shared__ int32_t wtot[kBlk / 64][V];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t inc[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
        inc[i] = x[i];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t t = __shfl_up(inc[i], o, 64);
            if (lane >= o) inc[i] += t;
        }
        if (lane == 63) wtot[wid][i] = inc[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < V; ++i) {
        int32_t pre = 0, t = 0;
#pragma unroll
        for (int w = 0; w < kBlk / 64; ++w) {
            if (w < wid) pre += wtot[w][i];
            t += wtot[w][i];
        }
        tot[i] = t;
        x[i] = pre + inc[i] - x[i];
    }
    __syncthreads();
}

// Largest i in [0, F) with s[i] <= rank, for a strictly increasing s with
// s[0] = 0 <= rank, found by the whole block: each round samples 256 evenly
// spaced positions and keeps the segment where the samples cross rank.
__device__ __forceinline__ int32_t find_entry(const int32_t *__restrict__ s, int32_t F, int32_t rank) {
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

}  // namespace gr
