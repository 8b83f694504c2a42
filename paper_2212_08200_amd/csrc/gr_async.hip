// Asynchronous convergence loop (Section III-A: an execution policy without
// the barrier at the end of each advance; Section III-B: the frontier as an
// asynchronous queue whose elements are passed as messages).
//
// One persistent kernel drains a device worklist of vertex ids.  A block
// reserves a run of list positions, takes the ids that have arrived there,
// expands them (thread-mapped for short adjacency lists, load-balanced over
// the block for long ones) and appends the vertices it improved.  There are
// no rounds and no grid barrier: a vertex improved while others are still
// expanding is queued and expanded as soon as a block reaches it.
//
// Shared state and its protocol (every cross-block access is an atomic that
// executes at the device's coherence point; a dependent access is issued
// only after the earlier one has returned):
//   dist[v]   lowered by a returning atomic min; a vertex is queued only when
//             the min returns a larger old value (a strict decrease, as the
//             paper's relax operator)
//   inq[v]    one byte per vertex, accessed as 32-bit words: set when v is
//             appended, cleared by the block that takes v from the list,
//             before that block reads dist[v].  A decrease that finds the
//             flag set is seen by that later read, so every decrease is
//             followed by an expansion with the decreased value or a smaller
//             one -- the condition for the unique fixed point.  At most one
//             entry per vertex is outstanding.
//   list      linear worklist of cap entries, initialised to kEmpty; a
//             producer reserves positions with one atomic add on `tail` per
//             block and writes them with atomic exchanges; a consumer
//             reserves positions with an atomic add on `head` and takes each
//             one with an exchange back to kEmpty, waiting until it has been
//             written.  Positions at or past cap are not written: their
//             vertices are spilled (a byte per vertex) and listed again by
//             the host for the next phase.
//   done      entries fully processed (their appends already reserved) plus
//             spilled entries.  done == tail means no entry is in flight and
//             none can be created: every block leaves.
// Every wait is bounded by the caller's spin limit (status 3 ends the query).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gr_device.h"

namespace gr {

namespace {

constexpr int32_t kEmpty = -1;
constexpr int kAsyncLight = 8;   // adjacency lists up to this long are expanded by one thread
constexpr int kAsyncItems = 8;   // arcs in flight per thread in the block-mapped expansion

struct AsyncArgs {
    int32_t n;
    const int32_t *ro;
    const uint2 *adj;
    uint32_t *dist;
    uint32_t *inq;   // in-queue bytes, as words
    uint8_t *spill;  // spilled vertices (next phase)
    int32_t *list;
    int64_t cap;
    unsigned long long *ctl;  // kAsync* words
    uint64_t spin_ticks;
    uint32_t inf;
    int32_t src;
    int64_t nflag;  // bytes per flag array (multiple of 16)
};

__device__ __forceinline__ unsigned long long ld(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long ld_acq(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Relaxes N arcs (valid[i] set) with source distances du[i]; take[i] tells
// whether arc i's destination must be appended (it decreased and was not
// queued).  The three steps are batched over the N arcs so that their memory
// operations overlap: plain pre-read (a stale value is larger, never wrong),
// returning atomic min, then the in-queue flag.
template <int WT, bool O32, int N>
__device__ __forceinline__ void relax_async(const AsyncArgs &a, const uint2 (&arc)[N], const uint32_t (&du)[N],
                                            const bool (&valid)[N], bool (&take)[N]) {
    // No default values on the loads and atomics below: a guarded load or
    // atomic whose result gets a default on the other path made each item
    // wait for the one before.  Invalid items read vertex 0 (arc (0, 0) or a
    // valid clamped arc), and old / was are read only where they were set.
    uint32_t nd[N], cur[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        nd[i] = plus<WT>(du[i], arc[i].y);
        cur[i] = *elem<O32>(a.dist, arc[i].x);
    }
    uint32_t old[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        take[i] = valid[i] && nd[i] < cur[i];
        if (take[i])
            old[i] = __hip_atomic_fetch_min(elem<O32>(a.dist, arc[i].x), nd[i], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t was[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        take[i] = take[i] && nd[i] < old[i];
        const uint32_t v = arc[i].x;
        if (take[i])
            was[i] = __hip_atomic_fetch_or(elem<O32>(a.inq, v >> 2), 1u << ((v & 3u) * 8u), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) take[i] = take[i] && ((was[i] >> ((arc[i].x & 3u) * 8u)) & 0xFFu) == 0u;
}

// All threads of the block call this.  Appends arc[i].x for take[i] set: one
// atomic add on the tail per block; positions past cap spill.  Thread 0
// accumulates the block's spilled count in *spilled.
template <int N>
__device__ __forceinline__ void append_async(const AsyncArgs &a, const uint2 (&arc)[N], const bool (&take)[N],
                                             int32_t *spilled) {
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
    if (threadIdx.x == 0 && total > 0) {
        const unsigned long long b = atomicAdd(a.ctl + kAsyncTail, (unsigned long long)total);
        sBase = b;
        const long long room = a.cap - (long long)b;
        *spilled += room >= total ? 0 : (room <= 0 ? total : total - (int32_t)room);
    }
    __syncthreads();
    if (total == 0) return;
    int64_t pos = (int64_t)sBase + before + (inc - c);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if (take[i]) {
            if (pos < a.cap)
                (void)__hip_atomic_exchange(a.list + pos, (int32_t)arc[i].x, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
            else
                a.spill[arc[i].x] = 1;  // read by the next launch only
            ++pos;
        }
    }
    __syncthreads();  // sBase / sWave reuse
}

enum : int { kCmdWork = 0, kCmdWait = 1, kCmdExit = 2 };

template <int WT, bool O32>
__global__ __launch_bounds__(kBlk) void k_async(AsyncArgs a) {
    __shared__ int sCmd;
    __shared__ unsigned long long sHead;
    __shared__ int32_t sTake;
    __shared__ int32_t sSpill;
    __shared__ int32_t hCount;
    __shared__ int32_t hStart[kBlk];
    __shared__ int32_t hS[kBlk + 1];
    __shared__ uint32_t hDu[kBlk];
    unsigned long long *ctl = a.ctl;
    int64_t mine = -1;  // list position this thread has reserved and not yet taken
    uint64_t t_last = wall_clock64();
    unsigned long long n_items = 0, n_arcs = 0;
    for (;;) {
        // 1. reserve new positions once the block holds none
        const int holding = __syncthreads_count(mine >= 0);
        if (threadIdx.x == 0) {
            sCmd = kCmdWork;
            sTake = 0;
            sSpill = 0;
            hCount = 0;
            if (holding == 0) {
                if (ld(ctl + kAsyncStatus) != 0ull) {
                    sCmd = kCmdExit;
                } else {
                    const unsigned long long d = ld_acq(ctl + kAsyncDone);
                    const unsigned long long t = ld(ctl + kAsyncTail);
                    const unsigned long long h = ld(ctl + kAsyncHead);
                    if (d == t) {
                        sCmd = kCmdExit;
                    } else if (h < t) {
                        const unsigned long long k = min((unsigned long long)kBlk, t - h);
                        sHead = atomicAdd(ctl + kAsyncHead, k);
                        sTake = (int32_t)k;
                    }
                }
            }
        }
        __syncthreads();
        if (sCmd == kCmdExit) break;
        if ((int)threadIdx.x < sTake) {
            mine = (int64_t)sHead + threadIdx.x;
            if (mine >= a.cap) mine = -1;  // never written: that vertex spilled
        }
        // 2. take the reserved positions that have been written
        int32_t v = -1;
        if (mine >= 0) {
            const int32_t x = __hip_atomic_exchange(a.list + mine, kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (x != kEmpty) {
                v = x;
                mine = -1;
            }
        }
        int32_t st = 0, deg = 0;
        uint32_t du = 0;
        if (v >= 0) {
            const uint32_t sh = ((uint32_t)v & 3u) * 8u;
            const uint32_t was = __hip_atomic_fetch_and(elem<O32>(a.inq, (uint32_t)v >> 2), ~(0xFFu << sh),
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((was >> sh) & 0xFFu) {  // always: an entry carries its vertex's flag
                du = __hip_atomic_load(elem<O32>(a.dist, (uint32_t)v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                st = a.ro[v];
                deg = a.ro[v + 1] - st;
            }
        }
        const int got = __syncthreads_count(v >= 0);
        if (got == 0) {
            // nothing arrived: the query may be over, failed, or still running
            if (threadIdx.x == 0) {
                int cmd = kCmdWait;
                if (ld(ctl + kAsyncStatus) != 0ull) {
                    cmd = kCmdExit;
                } else {
                    const unsigned long long d = ld_acq(ctl + kAsyncDone);
                    if (d == ld(ctl + kAsyncTail)) {
                        cmd = kCmdExit;
                    } else if (wall_clock64() - t_last > a.spin_ticks) {
                        __hip_atomic_store(ctl + kAsyncStatus, 3ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        cmd = kCmdExit;
                    }
                }
                sCmd = cmd;
            }
            __syncthreads();
            if (sCmd == kCmdExit) break;
            __builtin_amdgcn_s_sleep(4);
            continue;
        }
        t_last = wall_clock64();
        if (v >= 0) {
            n_items += 1;
            n_arcs += (unsigned long long)deg;
        }
        // 3. thread-mapped expansion of the short lists
        const bool light = v >= 0 && deg <= kAsyncLight;
        if (v >= 0 && !light) {
            const int h = atomicAdd(&hCount, 1);
            hStart[h] = st;
            hS[h] = deg;
            hDu[h] = du;
        }
        {
            uint2 arc[kAsyncLight];
            uint32_t dv[kAsyncLight];
            bool valid[kAsyncLight], take[kAsyncLight];
#pragma unroll
            for (int i = 0; i < kAsyncLight; ++i) {
                valid[i] = light && i < deg;
                arc[i] = valid[i] ? load_arc(elem<O32>(a.adj, (uint32_t)(st + i))) : make_uint2(0u, 0u);
                dv[i] = du;
            }
            relax_async<WT, O32, kAsyncLight>(a, arc, dv, valid, take);
            append_async<kAsyncLight>(a, arc, take, &sSpill);
        }
        // 4. block-mapped expansion of the long lists (searched by arc rank)
        const int hc = hCount;
        if (hc > 0) {
            int32_t x[1] = {(int)threadIdx.x < hc ? hS[threadIdx.x] : 0}, tot[1];
            block_scan<1>(x, tot);
            if ((int)threadIdx.x < hc) hS[threadIdx.x] = x[0];
            for (int t = hc + threadIdx.x; t <= kBlk; t += kBlk) hS[t] = (t == hc) ? tot[0] : INT32_MAX;
            __syncthreads();
            const int32_t H = tot[0];
            for (int32_t x0 = 0; x0 < H; x0 += kBlk * kAsyncItems) {
                int32_t xr[kAsyncItems], pos[kAsyncItems];
#pragma unroll
                for (int i = 0; i < kAsyncItems; ++i) {
                    xr[i] = min(x0 + (int32_t)threadIdx.x + i * kBlk, H - 1);
                    pos[i] = 0;
                }
#pragma unroll
                for (int b = kBlk / 2; b >= 1; b >>= 1) {
#pragma unroll
                    for (int i = 0; i < kAsyncItems; ++i) {
                        const int32_t p = pos[i] + b;
                        pos[i] = (hS[p] <= xr[i]) ? p : pos[i];
                    }
                }
                uint2 arc[kAsyncItems];
                uint32_t dv[kAsyncItems];
                bool valid[kAsyncItems], take[kAsyncItems];
#pragma unroll
                for (int i = 0; i < kAsyncItems; ++i) {
                    valid[i] = x0 + (int32_t)threadIdx.x + i * kBlk < H;
                    arc[i] = load_arc(elem<O32>(a.adj, (uint32_t)(hStart[pos[i]] + (xr[i] - hS[pos[i]]))));
                    dv[i] = hDu[pos[i]];
                }
                relax_async<WT, O32, kAsyncItems>(a, arc, dv, valid, take);
                append_async<kAsyncItems>(a, arc, take, &sSpill);
            }
        }
        // 5. the taken entries are done (their appends are reserved), and so
        // are the appends that spilled
        __syncthreads();
        if (threadIdx.x == 0)
            atomicAdd(ctl + kAsyncDone, (unsigned long long)got + (unsigned long long)sSpill);
    }
    // statistics
    __shared__ unsigned long long sStat[2];
    if (threadIdx.x == 0) sStat[0] = sStat[1] = 0ull;
    __syncthreads();
    if (n_items) {
        atomicAdd(&sStat[0], n_items);
        atomicAdd(&sStat[1], n_arcs);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (sStat[0]) atomicAdd(ctl + kAsyncStatItems, sStat[0]);
        if (sStat[1]) atomicAdd(ctl + kAsyncStatArcs, sStat[1]);
    }
}

// dist, in-queue and spill bytes, the list and the counters of a query whose
// worklist starts as {src}.
__global__ __launch_bounds__(kBlk) void k_async_init(AsyncArgs a) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v < a.n; v += stride) a.dist[v] = (v == a.src) ? 0u : a.inf;
    const int64_t sw = a.src >> 2;
    for (int64_t w = tid; w < a.nflag / 4; w += stride) {
        a.inq[w] = (w == sw) ? (1u << ((a.src & 3) * 8)) : 0u;
        reinterpret_cast<uint32_t *>(a.spill)[w] = 0u;
    }
    for (int64_t i = tid; i < a.cap; i += stride) a.list[i] = (i == 0) ? a.src : kEmpty;
    if (tid < kAsyncCtlWords) a.ctl[tid] = (tid == kAsyncTail) ? 1ull : 0ull;
}

// Next phase: positions and counters restart from zero (statistics and the
// status are kept); the list is all kEmpty again since every written
// position was taken.
__global__ void k_async_reset(unsigned long long *ctl) {
    if (threadIdx.x == 0) {
        ctl[kAsyncHead] = 0ull;
        ctl[kAsyncTail] = 0ull;
        ctl[kAsyncDone] = 0ull;
    }
}

// Lists the spilled vertices (their in-queue flags stay set) and clears
// their spill bytes; those past the list's capacity stay spilled.
__global__ __launch_bounds__(kBlk) void k_async_relist(AsyncArgs a) {
    __shared__ int32_t sWave[kBlk / 64];
    __shared__ unsigned long long sBase;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int64_t b = (int64_t)blockIdx.x * kBlk; b < a.n; b += (int64_t)gridDim.x * kBlk) {
        const int64_t v = b + threadIdx.x;
        const bool take = v < a.n && a.spill[v] != 0;
        const unsigned long long bal = __ballot(take);
        const int32_t inw = __popcll(bal);
        if (lane == 0) sWave[wid] = inw;
        __syncthreads();
        int32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kBlk / 64; ++w) {
            before += w < wid ? sWave[w] : 0;
            total += sWave[w];
        }
        if (threadIdx.x == 0 && total > 0) sBase = atomicAdd(a.ctl + kAsyncTail, (unsigned long long)total);
        __syncthreads();
        if (take) {
            const int64_t pos = (int64_t)sBase + before + __popcll(bal & ((1ull << lane) - 1ull));
            if (pos < a.cap) {  // the others stay spilled for a later phase
                a.list[pos] = (int32_t)v;
                a.spill[v] = 0;
            }
        }
        __syncthreads();
    }
}

// After a relist: the vertices that did not fit are counted as done (they
// are spilled again), so that the phase ends once the listed ones are.
__global__ void k_async_carry(unsigned long long *ctl, int64_t cap) {
    if (threadIdx.x == 0) {
        const unsigned long long t = ctl[kAsyncTail];
        ctl[kAsyncDone] = t > (unsigned long long)cap ? t - (unsigned long long)cap : 0ull;
    }
}

template <int WT, bool O32>
int async_occupancy() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_async<WT, O32>, kBlk, 0) != hipSuccess) return 0;
    return nb;
}

}  // namespace

int64_t async_capacity(int32_t n) { return 4 * (int64_t)std::max(n, 1) + 1024; }

static size_t list_bytes(int64_t cap) { return ((size_t)cap * sizeof(int32_t) + 255) & ~(size_t)255; }

size_t async_bytes(int64_t cap) { return list_bytes(cap) + sizeof(unsigned long long) * kAsyncCtlWords; }

unsigned long long *async_ctl(int64_t cap, void *ws) {
    return reinterpret_cast<unsigned long long *>(static_cast<char *>(ws) + list_bytes(cap));
}

static AsyncArgs async_args(const DevGraph &g, uint32_t *dist, int32_t src, const Frontier &f, void *ws, int64_t cap,
                            uint64_t spin_ticks) {
    AsyncArgs a;
    a.n = g.n;
    a.ro = g.ro;
    a.adj = g.adj;
    a.dist = dist;
    a.inq = reinterpret_cast<uint32_t *>(f.flags[0]);
    a.spill = f.flags[1];
    a.cap = cap;
    a.list = static_cast<int32_t *>(ws);
    a.ctl = async_ctl(cap, ws);
    a.spin_ticks = spin_ticks;
    a.inf = g.wt == 1 ? kInfF32 : kInfU32;
    a.src = src;
    a.nflag = f.nflag;
    return a;
}

hipError_t launch_async_init(const DevGraph &g, uint32_t *dist, int32_t src, const Frontier &f, void *ws, int64_t cap,
                             hipStream_t st) {
    const AsyncArgs a = async_args(g, dist, src, f, ws, cap, 0);
    const int64_t items = std::max<int64_t>(std::max<int64_t>(g.n, cap), a.nflag / 4);
    const int64_t b = (items + kBlk * 4 - 1) / (kBlk * 4);
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(b, 1), 8192);
    hipLaunchKernelGGL(k_async_init, dim3(grid), dim3(kBlk), 0, st, a);
    return hipGetLastError();
}

int async_blocks(const DevGraph &g, int num_cu) {
    // one block per 64K arcs, between 64 and two per CU: measured best (R-MAT
    // 22: 512 blocks, 8.5 ms, against 11.7 ms with 1024; road-like 2048^2:
    // 256, 13.6 against 21.4 ms; grid 64^2: 128 or fewer, 1.2 against 4.3 ms)
    // -- more blocks than the worklist keeps busy only add counter traffic
    const int64_t b = std::min<int64_t>(std::max<int64_t>((int64_t)g.m >> 16, 64), 2 * (int64_t)std::max(num_cu, 1));
    return (int)b;
}

hipError_t launch_async(const DevGraph &g, uint32_t *dist, const Frontier &f, void *ws, int64_t cap, int blocks,
                        uint64_t spin_ticks, hipStream_t st) {
    const AsyncArgs a = async_args(g, dist, 0, f, ws, cap, spin_ticks);
    const bool o32 = (uint64_t)g.m * 8ull < (1ull << 32) && (uint64_t)g.n * 4ull < (1ull << 32);
    int occ = 0;
    switch (g.wt) {
        case 1: occ = o32 ? async_occupancy<1, true>() : async_occupancy<1, false>(); break;
        case 2: occ = o32 ? async_occupancy<2, true>() : async_occupancy<2, false>(); break;
        default: occ = o32 ? async_occupancy<0, true>() : async_occupancy<0, false>(); break;
    }
    // blocks need not be co-resident (no block waits for one that has not
    // started); at most the resident count
    if (occ < 1) return hipErrorInvalidConfiguration;
    const int grid = std::max(1, blocks);
#define GR_ASYNC_LAUNCH(W, O) hipLaunchKernelGGL((k_async<W, O>), dim3(grid), dim3(kBlk), 0, st, a)
    switch (g.wt) {
        case 1:
            if (o32) GR_ASYNC_LAUNCH(1, true); else GR_ASYNC_LAUNCH(1, false);
            break;
        case 2:
            if (o32) GR_ASYNC_LAUNCH(2, true); else GR_ASYNC_LAUNCH(2, false);
            break;
        default:
            if (o32) GR_ASYNC_LAUNCH(0, true); else GR_ASYNC_LAUNCH(0, false);
            break;
    }
#undef GR_ASYNC_LAUNCH
    return hipGetLastError();
}

hipError_t launch_async_relist(const DevGraph &g, const Frontier &f, void *ws, int64_t cap, hipStream_t st) {
    const AsyncArgs a = async_args(g, nullptr, 0, f, ws, cap, 0);
    hipLaunchKernelGGL(k_async_reset, dim3(1), dim3(64), 0, st, a.ctl);
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(((int64_t)g.n + kBlk - 1) / kBlk, 1), 4096);
    hipLaunchKernelGGL(k_async_relist, dim3(grid), dim3(kBlk), 0, st, a);
    hipLaunchKernelGGL(k_async_carry, dim3(1), dim3(64), 0, st, a.ctl, cap);
    return hipGetLastError();
}

}  // namespace gr
