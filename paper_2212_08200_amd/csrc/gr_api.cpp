// Host runtime of the C ABI declared in include/gr.h: graph store, loop
// drivers (host-driven and device-driven), batched queries and the server.
#include "gr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <thread>
#include <unordered_map>
#include <cstdarg>
#include <cstddef>
#include <cmath>
#include <cfloat>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "gr_internal.h"
#include "gr_lds.h"
#include "gr_multi.h"
#include "gr_noalloc.h"
#include "gr_sched.h"

using namespace gr;

// ---------------------------------------------------------------------------
// errors

static thread_local std::string t_last_error;

static gr_status fail(gr_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
static gr_status fail(gr_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_last_error = buf;
    return s;
}

static gr_status hip_fail(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory) return fail(GR_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e));
    return fail(GR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call)                                  \
    do {                                               \
        hipError_t _e = (call);                        \
        if (_e != hipSuccess) return hip_fail(_e, #call); \
    } while (0)

extern "C" const char *gr_status_string(gr_status s) {
    switch (s) {
        case GR_OK: return "GR_OK";
        case GR_ERR_INVALID_ARG: return "GR_ERR_INVALID_ARG";
        case GR_ERR_SOURCE_RANGE: return "GR_ERR_SOURCE_RANGE";
        case GR_ERR_OUT_OF_MEMORY: return "GR_ERR_OUT_OF_MEMORY";
        case GR_ERR_NO_CAPACITY: return "GR_ERR_NO_CAPACITY";
        case GR_ERR_NOT_READY: return "GR_ERR_NOT_READY";
        case GR_ERR_ITER_LIMIT: return "GR_ERR_ITER_LIMIT";
        case GR_ERR_HIP: return "GR_ERR_HIP";
        case GR_ERR_UNKNOWN_TICKET: return "GR_ERR_UNKNOWN_TICKET";
    }
    return "GR_ERR_UNKNOWN";
}

extern "C" const char *gr_last_error(void) { return t_last_error.c_str(); }

extern "C" const char *gr_version(void) { return "gr 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// device properties and the stream-ordered pool

struct DeviceInfo {
    int num_cu = 0;
    bool coop = false;
    int wall_khz = 0;  // rate of the device's constant-rate clock
};

static std::mutex g_dev_mu;
static std::vector<DeviceInfo> g_devs;

static gr_status device_info(int dev, DeviceInfo *out) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if ((int)g_devs.size() <= dev) g_devs.resize(dev + 1);
    DeviceInfo &d = g_devs[dev];
    if (d.num_cu == 0) {
        int cu = 0, coop = 0;
        HIP_TRY(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev));
        HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
        d.wall_khz = khz;
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;  // keep freed workspaces cached in the pool
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
        d.num_cu = cu;
        d.coop = coop != 0;
    }
    *out = d;
    return GR_OK;
}

// Small pinned host buffer per thread for per-iteration counters.
static unsigned long long *pinned_slot() {
    static thread_local unsigned long long *p = nullptr;
    if (!p) {
        void *q = nullptr;
        if (hipHostMalloc(&q, 8192, hipHostMallocDefault) != hipSuccess) return nullptr;
        p = static_cast<unsigned long long *>(q);
    }
    return p;
}

// ---------------------------------------------------------------------------
// graph

// Partitioned push layout is built by default when the graph is large enough
// for the distance array to outgrow one XCD's L2 and most arcs join distant
// vertex ids (so that the plain layout would scatter dist accesses).
static constexpr int32_t kPartitionMinN = 1 << 17;
// An arc is "near" when |u - v| < n / 64: true for nearly all arcs of grids and
// meshes, and for about 3% of the arcs of a graph with random vertex ids.
static inline int32_t locality_span(int32_t n) { return std::max(n / 64, 64); }
// Small rounds of the queued loop apply to graphs of at most this degree.
static constexpr int32_t kSmallMaxDegree = 64;
// Pull -> push when the frontier holds fewer than n / beta vertices (Beamer et
// al.'s default).
static constexpr int32_t kDefaultBeta = 24;
// Small rounds expand the vertices a block improved for this many hops
// before the next round takes the rest (measured on the 2048^2 road-like
// graph: 5.6 ms with 2, 5.35 with 4, 5.4 with 6, 5.6 with 8, 6.1 with 12;
// plain grid 2048^2: 69 / 51 / 42 / 48 / 53 ms).
static constexpr int32_t kDefaultLocalHops = 6;
static constexpr int32_t kAsyncDefaultMaxN = 1 << 16;  // see graph_build

struct gr_graph {
    int device = 0;
    DevGraph plain{};  // np = 1: push over the CSR as given
    DevGraph part{};   // np = 8: partitioned push layout (when built)
    bool has_part = false;
    int32_t *d_ro = nullptr;
    uint2 *d_adj = nullptr;
    int32_t *d_ro_in = nullptr;  // == d_ro when symmetric
    uint2 *d_adj_in = nullptr;   // == d_adj when symmetric
    int32_t *d_pro = nullptr;
    uint2 *d_padj = nullptr;
    int32_t *d_mem_u[2] = {nullptr, nullptr};  // membership lists: plain, partitioned
    uint2 *d_mem_sd[2] = {nullptr, nullptr};
    bool pull = false;
    bool csc_separate = false;
    size_t dev_bytes = 0;
    std::vector<int32_t> h_ro;
    int32_t max_degree = 0;
    // AUTO schedule: defaults, replaced by gr_graph_tune
    int32_t auto_layout = GR_LAYOUT_PLAIN;
    int32_t auto_loop = GR_LOOP_QUEUED;
    int32_t auto_dense_ratio = kDenseRatio;
    int32_t auto_alpha_x16 = 0;
    uint32_t auto_delta = 0;  // near-far split width (0: off)
    bool auto_small = false;  // queued loop: small rounds
    int32_t auto_relax = GR_RELAX_DIST;  // push's relaxation filter
    int32_t auto_async_blocks = 0;       // asynchronous loop's block count (0: async_blocks())
    int32_t auto_local_hops = kDefaultLocalHops;  // small rounds' local hops
    // single-workgroup loop: the graph fits one workgroup's LDS (lds_fit), and
    // every weight is below 2^16 (lds_w16: weighted queries can pack arcs)
    bool lds_fit = false;
    bool lds_w16 = false;
    // the arcs padded to 2^ell_lg per vertex (lds_ell_words), for the
    // single-workgroup loop's padded layout; nullptr when it does not fit
    uint32_t *d_ell = nullptr;
    int32_t ell_lg = 0;
    // iterations of the last completed queued-loop query (first chunk size)
    mutable std::atomic<int32_t> last_iters{0};
    double locality = 1.0;  // fraction of arcs with |u - v| < locality_span(n)
};

static gr_status validate_host(int32_t n, int32_t m, const int32_t *ro, const int32_t *col, const uint32_t *w,
                               gr_weight_type wt) {
    if (ro[0] != 0) return fail(GR_ERR_INVALID_ARG, "row_offsets[0] = %d, expected 0", ro[0]);
    if (ro[n] != m) return fail(GR_ERR_INVALID_ARG, "row_offsets[n] = %d, expected m = %d", ro[n], m);
    for (int32_t v = 0; v < n; ++v)
        if (ro[v + 1] < ro[v]) return fail(GR_ERR_INVALID_ARG, "row_offsets decrease at row %d", v);
    for (int32_t e = 0; e < m; ++e)
        if (col[e] < 0 || col[e] >= n)
            return fail(GR_ERR_INVALID_ARG, "col_indices[%d] = %d outside [0, %d)", e, col[e], n);
    if (wt == GR_W_F32) {
        for (int32_t e = 0; e < m; ++e) {
            const uint32_t b = w[e];
            if ((b & 0x7F800000u) == 0x7F800000u)
                return fail(GR_ERR_INVALID_ARG, "weight %d is not finite (bits 0x%08x)", e, b);
            if ((b & 0x80000000u) && b != 0x80000000u)
                return fail(GR_ERR_INVALID_ARG, "weight %d is negative (bits 0x%08x)", e, b);
        }
    }
    return GR_OK;
}

static void graph_free(gr_graph *g) {
    if (!g) return;
    if (g->d_ro_in && g->d_ro_in != g->d_ro) (void)hipFree(g->d_ro_in);
    if (g->d_adj_in && g->d_adj_in != g->d_adj) (void)hipFree(g->d_adj_in);
    if (g->d_ro) (void)hipFree(g->d_ro);
    if (g->d_adj) (void)hipFree(g->d_adj);
    if (g->d_ell) (void)hipFree(g->d_ell);
    if (g->d_pro) (void)hipFree(g->d_pro);
    if (g->d_padj) (void)hipFree(g->d_padj);
    for (int i = 0; i < 2; ++i) {
        if (g->d_mem_u[i]) (void)hipFree(g->d_mem_u[i]);
        if (g->d_mem_sd[i]) (void)hipFree(g->d_mem_sd[i]);
    }
    delete g;
}

// Device scratch freed on every exit path of graph_build.
struct Scratch {
    std::vector<void *> ptrs;
    ~Scratch() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <class T>
    hipError_t alloc(T **p, size_t bytes) {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, bytes ? bytes : 1);
        if (e == hipSuccess) ptrs.push_back(q);
        *p = static_cast<T *>(q);
        return e;
    }
};

#define BUILD_TRY(call, what)                      \
    do {                                           \
        hipError_t _e = (call);                    \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

// Membership lists of a push layout (which vertices have arcs into each partition).
static gr_status build_members(gr_graph *g, DevGraph &d, int which, hipStream_t st, Scratch &sc) {
    const int32_t n = d.n, np = d.np;
    const int64_t len = (int64_t)np * (n + 1) + 1;
    int64_t total = 0;
    for (int k = 0; k < np; ++k) total += d.cap[k];
    int32_t *cnt = nullptr, *pos = nullptr, *tmp = nullptr;
    long long *off = nullptr;
    BUILD_TRY(sc.alloc(&cnt, sizeof(int32_t) * (size_t)len), "hipMalloc(member counts)");
    BUILD_TRY(sc.alloc(&pos, sizeof(int32_t) * (size_t)len), "hipMalloc(member offsets)");
    BUILD_TRY(sc.alloc(&tmp, sizeof(int32_t) * scan_tmp_ints(len)), "hipMalloc(scan)");
    BUILD_TRY(sc.alloc(&off, sizeof(long long) * (kMaxParts + 1)), "hipMalloc(member offsets)");
    BUILD_TRY(hipMalloc(&g->d_mem_u[which], sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1)),
              "hipMalloc(members)");
    BUILD_TRY(hipMalloc(&g->d_mem_sd[which], sizeof(uint2) * (size_t)std::max<int64_t>(total, 1)),
              "hipMalloc(members)");
    BUILD_TRY(launch_members(n, np, d.pro, cnt, pos, tmp, g->d_mem_u[which], g->d_mem_sd[which], off, st),
              "membership lists");
    long long hoff[kMaxParts + 1] = {0};
    BUILD_TRY(hipMemcpyAsync(hoff, off, sizeof(long long) * (np + 1), hipMemcpyDeviceToHost, st), "copy offsets");
    BUILD_TRY(hipStreamSynchronize(st), "membership lists");
    if (hoff[np] != total) return fail(GR_ERR_HIP, "membership lists hold %lld entries, expected %lld", hoff[np],
                                       (long long)total);
    d.mem_u = g->d_mem_u[which];
    d.mem_sd = g->d_mem_sd[which];
    for (int k = 0; k <= kMaxParts; ++k) d.mem_off[k] = k <= np ? hoff[k] : hoff[np];
    g->dev_bytes += (size_t)total * 12;
    return GR_OK;
}

static gr_status build_partition(gr_graph *g, int32_t n, int32_t m, hipStream_t st, Scratch &sc) {
    const int np = kMaxParts;
    int32_t psize = (int32_t)((n + np - 1) / np);
    if (n >= 64 * np) psize = (psize + 63) & ~63;  // partitions start on bitmap words
    const int64_t len = (int64_t)np * (n + 1) + 1;
    int32_t *cnt = nullptr, *pm = nullptr, *tmp = nullptr;
    unsigned long long *caps = nullptr;
    BUILD_TRY(hipMalloc(&g->d_pro, sizeof(int32_t) * (size_t)len), "hipMalloc(partition offsets)");
    BUILD_TRY(hipMalloc(&g->d_padj, sizeof(uint2) * (size_t)std::max(m, 1)), "hipMalloc(partition arcs)");
    BUILD_TRY(sc.alloc(&cnt, sizeof(int32_t) * (size_t)len), "hipMalloc(partition counts)");
    BUILD_TRY(sc.alloc(&pm, sizeof(int32_t) * (size_t)len), "hipMalloc(partition offsets)");
    BUILD_TRY(sc.alloc(&tmp, sizeof(int32_t) * scan_tmp_ints(len)), "hipMalloc(scan)");
    BUILD_TRY(sc.alloc(&caps, sizeof(unsigned long long) * kMaxParts), "hipMalloc(caps)");
    BUILD_TRY(hipMemsetAsync(caps, 0, sizeof(unsigned long long) * kMaxParts, st), "memset caps");
    BUILD_TRY(launch_partition_build(n, m, g->d_ro, g->d_adj, np, psize, g->d_pro, g->d_padj, cnt, pm, tmp, caps, st),
              "partition build");
    unsigned long long hc[kMaxParts];
    BUILD_TRY(hipMemcpyAsync(hc, caps, sizeof hc, hipMemcpyDeviceToHost, st), "copy caps");
    BUILD_TRY(hipStreamSynchronize(st), "partition build");
    DevGraph &d = g->part;
    d = g->plain;
    d.np = np;
    d.psize = psize;
    d.pro = g->d_pro;
    d.padj = g->d_padj;
    for (int k = 0; k < kMaxParts; ++k) d.cap[k] = (int32_t)hc[k];
    g->has_part = true;
    g->dev_bytes += sizeof(int32_t) * (size_t)len + sizeof(uint2) * (size_t)std::max(m, 1);
    return build_members(g, d, 1, st, sc);
}

static gr_status graph_build(gr_graph *g, int32_t n, int32_t m, const int32_t *ro, const int32_t *col,
                             const void *weights, gr_weight_type wt, uint32_t flags, hipStream_t st) {
    const bool dev_in = flags & GR_INPUT_DEVICE;
    Scratch sc;
    BUILD_TRY(hipGetDevice(&g->device), "hipGetDevice");
    BUILD_TRY(hipMalloc(&g->d_ro, sizeof(int32_t) * ((size_t)n + 1)), "hipMalloc(row_offsets)");
    BUILD_TRY(hipMalloc(&g->d_adj, sizeof(uint2) * (size_t)std::max(m, 1)), "hipMalloc(arcs)");
    g->dev_bytes = sizeof(int32_t) * ((size_t)n + 1) + sizeof(uint2) * (size_t)std::max(m, 1);
    int32_t *tcol = nullptr;
    uint32_t *tw = nullptr;
    unsigned int *flag = nullptr;
    unsigned long long *near = nullptr;
    const hipMemcpyKind kind = dev_in ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    BUILD_TRY(sc.alloc(&flag, 64), "hipMalloc(flag)");
    BUILD_TRY(sc.alloc(&near, 64), "hipMalloc(flag)");
    BUILD_TRY(sc.alloc(&tcol, sizeof(int32_t) * (size_t)std::max(m, 1)), "hipMalloc(staging)");
    BUILD_TRY(sc.alloc(&tw, sizeof(uint32_t) * (size_t)std::max(m, 1)), "hipMalloc(staging)");
    BUILD_TRY(hipMemcpyAsync(g->d_ro, ro, sizeof(int32_t) * ((size_t)n + 1), kind, st), "upload row_offsets");
    if (m > 0) {
        BUILD_TRY(hipMemcpyAsync(tcol, col, sizeof(int32_t) * (size_t)m, kind, st), "upload col_indices");
        BUILD_TRY(hipMemcpyAsync(tw, weights, sizeof(uint32_t) * (size_t)m, kind, st), "upload weights");
    }
    BUILD_TRY(hipMemsetAsync(flag, 0, 64, st), "memset");
    BUILD_TRY(hipMemsetAsync(near, 0, 64, st), "memset");
    if (dev_in) {
        unsigned int err = 0;
        BUILD_TRY(launch_validate(n, m, g->d_ro, tcol, tw, (int)wt, flag, st), "validate");
        BUILD_TRY(hipMemcpyAsync(&err, flag, sizeof err, hipMemcpyDeviceToHost, st), "validate");
        BUILD_TRY(hipStreamSynchronize(st), "validate");
        if (err)
            return fail(GR_ERR_INVALID_ARG, "device CSR is malformed (%s%s%s)", (err & 1) ? "row_offsets " : "",
                        (err & 2) ? "col_indices " : "", (err & 4) ? "weights" : "");
        g->h_ro.resize((size_t)n + 1);
        BUILD_TRY(hipMemcpy(g->h_ro.data(), g->d_ro, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost),
                  "copy row_offsets");
    } else {
        g->h_ro.assign(ro, ro + (size_t)n + 1);
    }
    BUILD_TRY(launch_pack_arcs(tcol, tw, m, g->d_adj, st), "pack arcs");
    if (wt == GR_W_F32) BUILD_TRY(launch_canon_negzero(g->d_adj, m, st), "canonicalise -0");
    int32_t nonempty = 0;
    for (int32_t v = 0; v < n; ++v) {
        const int32_t d = g->h_ro[v + 1] - g->h_ro[v];
        g->max_degree = std::max(g->max_degree, d);
        nonempty += d > 0;
    }
    // Small rounds by default where they apply (bounded degree): measured
    // faster on grids and road-like graphs, whose many rounds are small.
    g->auto_small = g->max_degree <= kSmallMaxDegree;
    // The bound array pays where many arcs reach the same vertices within a
    // round (skewed degrees: measured faster on R-MAT, slower on road-like
    // graphs, whose relaxations are mostly first improvements).
    g->auto_relax = g->max_degree > kSmallMaxDegree ? GR_RELAX_BOUND : GR_RELAX_DIST;
    // Small bounded-degree graphs (meshes up to 256^2) run many rounds of a
    // few vertices each: the asynchronous loop needs no launch per round
    // (grid 64^2: 0.9 ms against 2.0 ms queued; 128^2: 1.9 against 4.8 ms;
    // 256^2 even; larger grids and every R-MAT graph favour the queued loop).
    if (g->max_degree <= kSmallMaxDegree && n <= kAsyncDefaultMaxN) g->auto_loop = GR_LOOP_ASYNC;
    // Graphs that fit one workgroup's LDS: the single-workgroup loop (a round
    // is a workgroup barrier: grid 64^2 0.09 ms against 0.85 asynchronous).
    g->lds_fit = lds_fits(n, m);
    int32_t ell_lg = 0;
    while (ell_lg < kLdsEllMaxLg && (1 << ell_lg) < g->max_degree) ++ell_lg;
    const bool ell_shape = (1 << ell_lg) >= g->max_degree && lds_ell_fits(n, ell_lg);
    if ((g->lds_fit || ell_shape) && wt == GR_W_U32) {
        std::vector<uint2> h((size_t)std::max(m, 1));
        BUILD_TRY(hipMemcpyAsync(h.data(), g->d_adj, sizeof(uint2) * (size_t)m, hipMemcpyDeviceToHost, st),
                  "copy arcs");
        BUILD_TRY(hipStreamSynchronize(st), "copy arcs");
        uint32_t wmax = 0;
        for (int32_t e = 0; e < m; ++e) wmax = std::max(wmax, h[(size_t)e].y);
        g->lds_w16 = wmax < 65536u;
        // padded layout: every vertex's arcs in 2^lg slots (lg from the
        // maximum degree), so a lane finds its arc without the row offsets;
        // it also fits meshes a little larger than the row-offset layout
        // does (no offsets: a 81 x 81 grid against 75 x 75)
        const int32_t lg = ell_lg;
        if (g->lds_w16 && ell_shape) {
            std::vector<uint32_t> ell((size_t)n << lg, kLdsNoArc);
            for (int32_t v = 0; v < n; ++v)
                for (int32_t e = g->h_ro[v]; e < g->h_ro[v + 1]; ++e)
                    ell[((size_t)v << lg) + (size_t)(e - g->h_ro[v])] = (h[(size_t)e].x << 16) | h[(size_t)e].y;
            BUILD_TRY(hipMalloc(&g->d_ell, sizeof(uint32_t) * ell.size()), "hipMalloc(padded arcs)");
            BUILD_TRY(hipMemcpy(g->d_ell, ell.data(), sizeof(uint32_t) * ell.size(), hipMemcpyHostToDevice),
                      "copy padded arcs");
            g->ell_lg = lg;
            g->dev_bytes += sizeof(uint32_t) * ell.size();
        }
    }
    // Also on skewed ones: a hub's arcs take many passes of one group of
    // lanes, but R-MAT graphs of 1-4 K vertices still run 2.3-3.2x faster
    // than with the queued loop (scale 10 to 12: 0.08-0.14 ms against 0.26-0.32).
    if ((g->lds_fit || g->d_ell) && g->lds_w16) g->auto_loop = GR_LOOP_LDS;
    // Large skewed graphs: few, heavy rounds, where the host-driven loop's
    // push grid of 16 blocks per CU beats the step kernel (R-MAT 22: 3.48 ms
    // against 3.63); smaller ones keep the queued loop (no host round trip
    // per round).
    if (g->max_degree > kSmallMaxDegree && m >= (1 << 26)) g->auto_loop = GR_LOOP_HOST;
    BUILD_TRY(launch_locality(n, g->d_ro, g->d_adj, locality_span(n), near, st), "locality");
    unsigned long long hnear = 0;
    BUILD_TRY(hipMemcpyAsync(&hnear, near, sizeof hnear, hipMemcpyDeviceToHost, st), "locality");

    g->d_ro_in = g->d_ro;
    g->d_adj_in = g->d_adj;
    if (!(flags & GR_NO_PULL)) {
        unsigned int not_sym = 0;
        BUILD_TRY(hipMemsetAsync(flag, 0, 64, st), "memset");
        BUILD_TRY(launch_symmetry_check(n, g->d_ro, g->d_adj, flag, st), "symmetry check");
        BUILD_TRY(hipMemcpyAsync(&not_sym, flag, sizeof not_sym, hipMemcpyDeviceToHost, st), "symmetry check");
        BUILD_TRY(hipStreamSynchronize(st), "symmetry check");
        if (not_sym) {
            int32_t *scratch = nullptr;
            const size_t nsc = (2 * (size_t)n + 1) + scan_tmp_ints((int64_t)n + 1);
            g->d_ro_in = nullptr;
            g->d_adj_in = nullptr;
            BUILD_TRY(hipMalloc(&g->d_ro_in, sizeof(int32_t) * ((size_t)n + 1)), "hipMalloc(csc)");
            BUILD_TRY(hipMalloc(&g->d_adj_in, sizeof(uint2) * (size_t)std::max(m, 1)), "hipMalloc(csc)");
            BUILD_TRY(sc.alloc(&scratch, sizeof(int32_t) * nsc), "hipMalloc(csc scratch)");
            BUILD_TRY(launch_csc_build(n, m, g->d_ro, g->d_adj, g->d_ro_in, g->d_adj_in, scratch, st), "csc build");
            g->csc_separate = true;
            g->dev_bytes += sizeof(int32_t) * ((size_t)n + 1) + sizeof(uint2) * (size_t)std::max(m, 1);
        }
        g->pull = true;
    }
    BUILD_TRY(hipStreamSynchronize(st), "graph upload");
    g->locality = m > 0 ? (double)hnear / (double)m : 1.0;

    DevGraph &d = g->plain;
    d.n = n;
    d.m = m;
    d.wt = (int32_t)wt;
    d.ro = g->d_ro;
    d.adj = g->d_adj;
    d.ro_in = g->d_ro_in;
    d.adj_in = g->d_adj_in;
    d.np = 1;
    d.psize = n;
    d.pro = g->d_ro;
    d.padj = g->d_adj;
    for (int k = 0; k < kMaxParts; ++k) d.cap[k] = 0;
    d.cap[0] = nonempty;
    {
        gr_status s = build_members(g, d, 0, st, sc);
        if (s != GR_OK) return s;
    }

    const bool want_part = !(flags & GR_NO_PARTITION) &&
                           ((flags & GR_FORCE_PARTITION) || (n >= kPartitionMinN && g->locality < 0.5));
    if (want_part) {
        gr_status s = build_partition(g, n, m, st, sc);
        if (s != GR_OK) return s;
        g->auto_layout = GR_LAYOUT_PARTITIONED;
    }
    return GR_OK;
}

extern "C" gr_status gr_graph_create_csr(gr_graph **out, int32_t n, int32_t m, const int32_t *row_offsets,
                                         const int32_t *col_indices, const void *weights, gr_weight_type wt,
                                         uint32_t flags, void *stream) {
    if (!out) return fail(GR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1) return fail(GR_ERR_INVALID_ARG, "n = %d, expected >= 1", n);
    if (m < 0 || m == INT32_MAX) return fail(GR_ERR_INVALID_ARG, "m = %d outside [0, 2^31 - 1)", m);
    if (wt != GR_W_U32 && wt != GR_W_F32) return fail(GR_ERR_INVALID_ARG, "unknown weight type %d", (int)wt);
    const uint32_t known = GR_INPUT_DEVICE | GR_NO_PULL | GR_NO_PARTITION | GR_FORCE_PARTITION;
    if (flags & ~known) return fail(GR_ERR_INVALID_ARG, "unknown flags 0x%x", flags & ~known);
    if ((flags & GR_NO_PARTITION) && (flags & GR_FORCE_PARTITION))
        return fail(GR_ERR_INVALID_ARG, "GR_NO_PARTITION and GR_FORCE_PARTITION are exclusive");
    if (!row_offsets || (m > 0 && (!col_indices || !weights)))
        return fail(GR_ERR_INVALID_ARG, "NULL array for n = %d, m = %d", n, m);
    if (!(flags & GR_INPUT_DEVICE)) {
        gr_status s = validate_host(n, m, row_offsets, col_indices, static_cast<const uint32_t *>(weights), wt);
        if (s != GR_OK) return s;
    }
    gr_graph *g = new (std::nothrow) gr_graph();
    if (!g) return fail(GR_ERR_OUT_OF_MEMORY, "host allocation");
    gr_status s = graph_build(g, n, m, row_offsets, col_indices, weights, wt, flags,
                              static_cast<hipStream_t>(stream));
    if (s != GR_OK) {
        graph_free(g);
        return s;
    }
    *out = g;
    return GR_OK;
}

extern "C" gr_status gr_graph_destroy(gr_graph *g) {
    if (!g) return fail(GR_ERR_INVALID_ARG, "graph is NULL");
    graph_free(g);
    return GR_OK;
}

extern "C" gr_status gr_graph_info(const gr_graph *g, int32_t *n, int32_t *m, gr_weight_type *wt,
                                   size_t *dev_bytes) {
    if (!g) return fail(GR_ERR_INVALID_ARG, "graph is NULL");
    if (n) *n = g->plain.n;
    if (m) *m = g->plain.m;
    if (wt) *wt = static_cast<gr_weight_type>(g->plain.wt);
    if (dev_bytes) *dev_bytes = g->dev_bytes;
    return GR_OK;
}

extern "C" gr_status gr_graph_layout(const gr_graph *g, int32_t *has_csc, int32_t *pull_enabled,
                                     int32_t *partitions) {
    if (!g) return fail(GR_ERR_INVALID_ARG, "graph is NULL");
    if (has_csc) *has_csc = g->csc_separate ? 1 : 0;
    if (pull_enabled) *pull_enabled = g->pull ? 1 : 0;
    if (partitions) *partitions = g->has_part ? kMaxParts : 1;
    return GR_OK;
}

// ---------------------------------------------------------------------------
// single-source loop drivers

// AUTO direction: pull when frontier out-edges * alpha_x16 >= 16 * m; the
// untuned default (alpha 0) never pulls: on the measured graphs push is faster
// in every round.

struct RunCfg {
    int loop;
    int direction;
    int32_t alpha_x16;
    int32_t beta;  // pull -> push when |frontier| * beta < n
    int64_t max_iters;
    bool max_iters_given;  // set by the caller (else the default cap)
    bool timing;
    int layout;
    int filter;
    int32_t dense_ratio;
    bool small;      // queued loop: small rounds from candidate lists
    int32_t local_hops;  // small rounds: hops a block expands before appending
    bool bound;      // push filters relaxations with the upper-bound array
    uint32_t delta;  // near-far split width (weight-type bits); 0 = off
    int64_t barrier_timeout_us;
    const DevGraph *dg;
};

static gr_status check_opts(const gr_graph *g, const gr_sssp_opts *o, RunCfg *rc) {
    rc->loop = o ? o->loop : GR_LOOP_AUTO;
    rc->direction = o ? o->direction : GR_DIR_AUTO;
    rc->alpha_x16 = (o && o->alpha_x16 > 0) ? o->alpha_x16 : g->auto_alpha_x16;
    rc->beta = (o && o->beta > 0) ? o->beta : kDefaultBeta;
    if (o && o->beta < 0) return fail(GR_ERR_INVALID_ARG, "beta = %d is negative", o->beta);
    rc->max_iters = (o && o->max_iters > 0) ? o->max_iters : (int64_t)g->plain.n + 1;
    rc->max_iters_given = o && o->max_iters > 0;
    const int layout = o ? o->layout : GR_LAYOUT_AUTO;
    if (!g->pull) rc->alpha_x16 = 0;  // the device-side AUTO rule must never pick pull then
    if (rc->loop < GR_LOOP_AUTO || rc->loop > GR_LOOP_LDS)
        return fail(GR_ERR_INVALID_ARG, "unknown loop mode %d", rc->loop);
    if (rc->direction < GR_DIR_AUTO || rc->direction > GR_DIR_ALTERNATE)
        return fail(GR_ERR_INVALID_ARG, "unknown direction %d", rc->direction);
    if ((rc->direction == GR_DIR_PULL || rc->direction == GR_DIR_ALTERNATE) && !g->pull)
        return fail(GR_ERR_INVALID_ARG, "pull traversal requested but the graph was built with GR_NO_PULL");
    if (layout < GR_LAYOUT_AUTO || layout > GR_LAYOUT_PARTITIONED)
        return fail(GR_ERR_INVALID_ARG, "unknown layout %d", layout);
    if (layout == GR_LAYOUT_PARTITIONED && !g->has_part)
        return fail(GR_ERR_INVALID_ARG, "partitioned layout requested but the graph has none");
    const int lay = layout == GR_LAYOUT_AUTO ? g->auto_layout : layout;
    rc->dg = (lay == GR_LAYOUT_PLAIN || !g->has_part) ? &g->plain : &g->part;
    rc->layout = rc->dg->np > 1 ? GR_LAYOUT_PARTITIONED : GR_LAYOUT_PLAIN;
    rc->timing = o && o->timing;
    rc->filter = o ? o->filter : 0;
    rc->dense_ratio = g->auto_dense_ratio;
    rc->barrier_timeout_us = (o && o->barrier_timeout_us > 0) ? o->barrier_timeout_us : 20000000;
    if (rc->filter < 0 || rc->filter > 3) return fail(GR_ERR_INVALID_ARG, "unknown filter mode %d", rc->filter);
    rc->small = rc->filter == 3 || (rc->filter == 0 && g->auto_small);
    rc->local_hops = (o && o->local_hops > 0) ? o->local_hops : g->auto_local_hops;
    if (o && (o->local_hops < 0 || o->local_hops > 64))
        return fail(GR_ERR_INVALID_ARG, "local_hops = %d outside [0, 64]", o->local_hops);
    if (rc->filter == 3) rc->filter = 0;
    const int32_t relax = (o && o->relax_filter) ? o->relax_filter : g->auto_relax;
    if (relax != GR_RELAX_DIST && relax != GR_RELAX_BOUND)
        return fail(GR_ERR_INVALID_ARG, "unknown relax_filter %d", relax);
    rc->bound = relax == GR_RELAX_BOUND;
    uint32_t d = (o && o->delta) ? o->delta : g->auto_delta;
    if (d == GR_DELTA_OFF) d = 0;
    if (d && g->plain.wt == GR_W_F32) {
        float x;
        std::memcpy(&x, &d, 4);
        if (!(x > 0.f && x <= FLT_MAX)) return fail(GR_ERR_INVALID_ARG, "delta must be a positive finite binary32");
    }
    if (rc->loop == GR_LOOP_LDS) {
        if (!g->lds_fit && !g->d_ell)
            return fail(GR_ERR_INVALID_ARG, "the single-workgroup loop needs a graph that fits one workgroup's LDS "
                                            "(n = %d, m = %d do not)", g->plain.n, g->plain.m);
        if (rc->direction == GR_DIR_PULL || rc->direction == GR_DIR_ALTERNATE)
            return fail(GR_ERR_INVALID_ARG, "the single-workgroup loop runs push only");
        if (o && o->delta && o->delta != GR_DELTA_OFF)
            return fail(GR_ERR_INVALID_ARG, "the single-workgroup loop has no near-far split");
        d = 0;
    }
    if (rc->loop == GR_LOOP_ASYNC) {
        if (rc->direction == GR_DIR_PULL || rc->direction == GR_DIR_ALTERNATE)
            return fail(GR_ERR_INVALID_ARG, "the asynchronous loop runs push only");
        if (o && o->delta && o->delta != GR_DELTA_OFF)
            return fail(GR_ERR_INVALID_ARG, "the asynchronous loop has no near-far split");
        d = 0;
    }
    rc->delta = d;
    if (d) {
        if (rc->direction == GR_DIR_PULL || rc->direction == GR_DIR_ALTERNATE)
            return fail(GR_ERR_INVALID_ARG, "the near-far split runs push only");
        rc->alpha_x16 = 0;
        // each raise of the threshold settles at least one vertex for good
        if (!(o && o->max_iters > 0)) rc->max_iters = std::min<int64_t>(8 * ((int64_t)g->plain.n + 1), INT32_MAX);
    }
    return GR_OK;
}

// AUTO: push -> pull when the frontier's out-arcs reach m / alpha; pull ->
// push when the frontier holds fewer than n / beta vertices (Beamer et al.'s
// two rules, with hysteresis on the previous round's direction).
static bool choose_pull(const gr_graph *g, const RunCfg &rc, int64_t iter, int64_t E, int64_t F, bool prev) {
    if (!g->pull) return false;
    switch (rc.direction) {
        case GR_DIR_PUSH: return false;
        case GR_DIR_PULL: return true;
        case GR_DIR_ALTERNATE: return (iter & 1) != 0;
        default:
            if (rc.alpha_x16 <= 0) return false;
            if (prev) return F * rc.beta >= (int64_t)g->plain.n;
            return E * rc.alpha_x16 >= (int64_t)16 * g->plain.m;
    }
}


static gr_status run_host_loop(const gr_graph *g, int32_t src, uint32_t *dist, hipStream_t st, const RunCfg &rc,
                               gr_sssp_stats *stats) {
    DeviceInfo di;
    gr_status s = device_info(g->device, &di);
    if (s != GR_OK) return s;
    unsigned long long *hp = pinned_slot();
    if (!hp) return fail(GR_ERR_OUT_OF_MEMORY, "pinned host buffer");
    const DevGraph &dg = *rc.dg;
    void *ws = nullptr;
    const WsParts parts{rc.delta != 0, rc.bound};
    HIP_TRY(hipMallocAsync(&ws, frontier_bytes(dg, parts), st));
    Frontier f;
    frontier_carve(f, ws, dg, parts);
    gr_sssp_stats local{};
    local.loop = GR_LOOP_HOST;
    local.layout = rc.layout;
    local.relax_filter = rc.bound ? GR_RELAX_BOUND : GR_RELAX_DIST;
    gr_status status = GR_OK;
    // Optional per-launch timing: events around the advance and the filter.
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (rc.timing)
        for (auto &x : ev)
            if (hipEventCreate(&x) != hipSuccess) x = nullptr;
    const bool timed = rc.timing && ev[0] && ev[1] && ev[2];
    const bool split = rc.delta != 0;
    uint32_t T = split ? next_threshold(0u, rc.delta, dg.wt) : kInfU32;
    hipError_t e = launch_init(dg, dist, src, f, T, split, st);
    // Frontier 0 = {src}: its counts are known on the host for one partition.
    FrontierCounts c{};
    if (dg.np == 1) {
        const int32_t d = g->h_ro[src + 1] - g->h_ro[src];
        c.F[0] = d > 0 ? 1 : 0;
        c.E[0] = d;
    } else {
        if (e == hipSuccess)
            e = hipMemcpyAsync(hp, f.ctl, sizeof(unsigned long long) * kSlotWords, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        read_counts(hp, &c);
    }
    int64_t iter = 0;
    bool prev_pull = false;
    while (e == hipSuccess) {
        // An empty frontier ends the query unless the near-far split holds
        // vertices back: then the round only raises the threshold and filters.
        const bool idle = c.Fsum() == 0;
        if (idle && (!split || c.far_count == 0)) break;
        if (iter >= rc.max_iters) {
            status = fail(GR_ERR_ITER_LIMIT, "iteration cap %lld reached", (long long)rc.max_iters);
            break;
        }
        if (idle) T = next_threshold(c.far_min, rc.delta, dg.wt);
        const int64_t E = c.Esum();
        const bool pull = !idle && choose_pull(g, rc, iter, E, c.Fsum(), prev_pull);
        prev_pull = pull;
        if (timed) (void)hipEventRecord(ev[0], st);
        if (idle) {
        } else if (pull) {
            // breadth-first search: every round of this loop is one level, so
            // the frontier's vertices all have depth iter
            e = launch_pull(dg, dist, f, iter, st, dg.wt == 2 ? (uint32_t)iter : kInfU32);
            local.pull_iterations++;
            local.arcs_pulled += dg.m;
        } else {
            e = launch_push(dg, dist, f, iter, c, di.num_cu, st);
            local.edges_pushed += E;
            local.push_frontier_sum += c.Fsum();
            local.push_launches++;
        }
        local.launches += 2;
        local.frontier_sum += c.Fsum();
        local.frontier_max = std::max<int64_t>(local.frontier_max, c.Fsum());
        if (timed) (void)hipEventRecord(ev[1], st);
        // the streaming filter pays off once the next frontier is likely large
        const bool dense = rc.filter == 2 || (rc.filter == 0 && c.Fsum() * rc.dense_ratio >= (int64_t)dg.n);
        if (e == hipSuccess) e = launch_filter(dg, f, iter, nullptr, dense, dist, split, T, st);
        if (timed) (void)hipEventRecord(ev[2], st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hp, counters_after(f, iter), sizeof(unsigned long long) * kSlotWords,
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        if (timed) {
            float a = 0.f, b = 0.f;
            (void)hipEventElapsedTime(&a, ev[0], ev[1]);
            (void)hipEventElapsedTime(&b, ev[1], ev[2]);
            (pull ? local.pull_us : local.push_us) += 1e3 * a;
            local.filter_us += 1e3 * b;
        }
        read_counts(hp, &c);
        ++iter;
    }
    local.iterations = (int32_t)iter;
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    hipError_t e2 = hipFreeAsync(ws, st);
    if (e != hipSuccess) return hip_fail(e, "sssp host loop");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    if (stats) *stats = local;
    return status;
}

static gr_status run_persistent(const gr_graph *g, int32_t src, uint32_t *dist, hipStream_t st, const RunCfg &rc,
                                gr_sssp_stats *stats) {
    DeviceInfo di;
    gr_status s = device_info(g->device, &di);
    if (s != GR_OK) return s;
    if (!di.coop) return fail(GR_ERR_HIP, "device does not support cooperative launches");
    const DevGraph &dg = *rc.dg;
    PersistentCfg cfg;
    cfg.grid = persistent_grid(dg, di.num_cu);
    if (cfg.grid < kMaxParts) return fail(GR_ERR_HIP, "no co-resident grid for the device-driven loop");
    cfg.max_iters = (int32_t)std::min<int64_t>(rc.max_iters, INT32_MAX);
    cfg.alpha_x16 = rc.alpha_x16;
    cfg.beta = rc.beta;
    cfg.direction = rc.direction;
    cfg.filter = rc.filter;
    cfg.dense_ratio = rc.dense_ratio;
    cfg.delta = rc.delta;
    cfg.small = 0;
    cfg.local_hops = 1;
    cfg.spin_ticks = (uint64_t)rc.barrier_timeout_us * (uint64_t)di.wall_khz / 1000ull;
    unsigned long long *hp = pinned_slot();
    if (!hp) return fail(GR_ERR_OUT_OF_MEMORY, "pinned host buffer");
    void *ws = nullptr;
    const WsParts parts{rc.delta != 0, rc.bound};
    HIP_TRY(hipMallocAsync(&ws, frontier_bytes(dg, parts), st));
    Frontier f;
    frontier_carve(f, ws, dg, parts);
    hipEvent_t ev[2] = {nullptr, nullptr};
    const bool timed = rc.timing && hipEventCreate(&ev[0]) == hipSuccess && hipEventCreate(&ev[1]) == hipSuccess;
    hipError_t e = launch_init(dg, dist, src, f, rc.delta ? next_threshold(0u, rc.delta, dg.wt) : kInfU32,
                               rc.delta != 0, st);
    if (e == hipSuccess && timed) e = hipEventRecord(ev[0], st);
    if (e == hipSuccess) e = launch_persistent(dg, dist, f, cfg, st);
    if (e == hipSuccess && timed) e = hipEventRecord(ev[1], st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hp, f.ctl + kLoopStateWord, sizeof(LoopState), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    LoopState ls{};
    if (e == hipSuccess) std::memcpy(&ls, hp, sizeof ls);
    gr_sssp_stats local{};
    local.loop = GR_LOOP_PERSISTENT;
    local.layout = rc.layout;
    local.relax_filter = rc.bound ? GR_RELAX_BOUND : GR_RELAX_DIST;
    local.iterations = (int32_t)ls.iter;
    local.pull_iterations = (int32_t)ls.pull_iters;
    local.edges_pushed = (int64_t)ls.edges_pushed;
    local.arcs_pulled = (int64_t)ls.arcs_pulled;
    local.frontier_sum = (int64_t)ls.frontier_sum;
    local.push_frontier_sum = (int64_t)ls.push_frontier_sum;
    local.frontier_max = (int32_t)ls.frontier_max;
    local.push_launches = 1;
    local.launches = 1;
    if (timed) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
        local.push_us = 1e3 * ms;  // the whole loop is one launch
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    hipError_t e2 = hipFreeAsync(ws, st);
    if (e != hipSuccess) return hip_fail(e, "device-driven loop");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    if (stats) *stats = local;
    if (ls.status == 2) return fail(GR_ERR_ITER_LIMIT, "iteration cap %lld reached", (long long)rc.max_iters);
    if (ls.status == 3) return fail(GR_ERR_HIP, "device-driven loop: a grid-barrier wait exceeded %lld us",
                                    (long long)rc.barrier_timeout_us);
    if (ls.status != 1) return fail(GR_ERR_HIP, "device-driven loop ended in state %llu", ls.status);
    return GR_OK;
}

// Queued loop: launches of the step kernel are enqueued in chunks without
// waiting; the host reads the loop state once per chunk, one chunk behind, so
// the device always has the next chunk queued.  The first chunk covers the
// launch count of the previous query on this graph; later chunks grow from 4
// to 64.  Launches queued past the end return at once; the call waits for the
// last chunk so that its state copy has landed before the pinned slot is
// reused.
static constexpr int64_t kPhaseLogCap = 1 << 16;

static gr_status run_queued(const gr_graph *g, int32_t src, uint32_t *dist, hipStream_t st, const RunCfg &rc,
                            gr_sssp_stats *stats) {
    DeviceInfo di;
    gr_status s = device_info(g->device, &di);
    if (s != GR_OK) return s;
    unsigned long long *hp = pinned_slot();
    if (!hp) return fail(GR_ERR_OUT_OF_MEMORY, "pinned host buffer");
    static_assert(2 * sizeof(LoopState) <= 8192, "pinned slot holds two loop states");
    const DevGraph &dg = *rc.dg;
    PersistentCfg cfg;
    cfg.grid = di.num_cu * 8;
    cfg.max_iters = (int32_t)std::min<int64_t>(rc.max_iters, INT32_MAX);
    cfg.alpha_x16 = rc.alpha_x16;
    cfg.beta = rc.beta;
    cfg.direction = rc.direction;
    cfg.filter = rc.filter;
    cfg.dense_ratio = rc.dense_ratio;
    cfg.delta = rc.delta;
    cfg.spin_ticks = 0;
    cfg.local_hops = rc.local_hops;
    // Small rounds (filter 3, or the tuned default) need push-only rounds
    // (they consume the flags), no near-far split, and a bounded degree (a
    // block expands its heavier vertices alone).
    cfg.small = rc.small && rc.delta == 0 && g->max_degree <= kSmallMaxDegree &&
                (rc.direction == GR_DIR_PUSH || (rc.direction == GR_DIR_AUTO && rc.alpha_x16 == 0));
    void *ws = nullptr;
    const WsParts parts{rc.delta != 0, rc.bound};
    HIP_TRY(hipMallocAsync(&ws, frontier_bytes(dg, parts), st));
    Frontier f;
    frontier_carve(f, ws, dg, parts);
    int8_t *plog = nullptr;
    hipEvent_t evc[2] = {nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (auto &x : evc)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
    if (e == hipSuccess && rc.timing) {
        e = hipMallocAsync(reinterpret_cast<void **>(&plog), (size_t)kPhaseLogCap, st);
        if (e == hipSuccess) e = hipMemsetAsync(plog, 0, (size_t)kPhaseLogCap, st);
    }
    std::vector<hipEvent_t> tev;  // with timing: begin/end of each launch
    if (e == hipSuccess)
        e = launch_init(dg, dist, src, f, rc.delta ? next_threshold(0u, rc.delta, dg.wt) : kInfU32, rc.delta != 0,
                        st);
    int64_t issued = 0;
    int c = 0;
    int64_t K = std::clamp<int64_t>(g->last_iters.load(std::memory_order_relaxed) + 1, 4, 512);
    LoopState fin{};
    bool done = false;
    const int grid_full = cfg.grid;
    bool small_seen = false;  // the last state read back was in small rounds
    while (e == hipSuccess && !done) {
        // Small rounds touch few vertices: a chunk that is expected to run
        // them launches a quarter of the grid (every phase is correct at any
        // grid size), which shortens the launch of the mostly idle blocks.
        cfg.grid = small_seen ? std::max(kMaxParts, grid_full / 4) : grid_full;
        for (int64_t i = 0; i < K && e == hipSuccess; ++i) {
            hipEvent_t b = nullptr, en = nullptr;
            if (rc.timing && issued + i < kPhaseLogCap) {
                if (hipEventCreate(&b) == hipSuccess) tev.push_back(b); else b = nullptr;
                if (hipEventCreate(&en) == hipSuccess) tev.push_back(en); else en = nullptr;
                if (!b || !en) b = en = nullptr;
            }
            e = launch_step(dg, dist, f, cfg, issued + i, plog, plog ? kPhaseLogCap : 0, b, en, st);
        }
        issued += K;
        unsigned long long *slot = hp + (c & 1) * (sizeof(LoopState) / 8);
        if (e == hipSuccess)
            e = hipMemcpyAsync(slot, f.ctl + kLoopStateWord, sizeof(LoopState), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(evc[c & 1], st);
        if (e == hipSuccess && c >= 1) {
            e = hipEventSynchronize(evc[(c - 1) & 1]);
            LoopState ls;
            std::memcpy(&ls, hp + ((c - 1) & 1) * (sizeof(LoopState) / 8), sizeof ls);
            if (e == hipSuccess && ls.status != 0) {
                fin = ls;
                done = true;
            }
            small_seen = cfg.small && ls.st_phase[0] == 2 && ls.st_phase[1] == 2;
        }
        ++c;
        K = std::min<int64_t>(64, 4ll << std::min(c - 1, 4));
    }
    if (e == hipSuccess) e = hipEventSynchronize(evc[(c - 1) & 1]);  // the last chunk's copy
    if (e == hipSuccess && done) std::memcpy(&fin, hp + ((c - 1) & 1) * (sizeof(LoopState) / 8), sizeof fin);
    gr_sssp_stats local{};
    local.loop = GR_LOOP_QUEUED;
    local.layout = rc.layout;
    local.relax_filter = rc.bound ? GR_RELAX_BOUND : GR_RELAX_DIST;
    local.iterations = (int32_t)fin.iter;
    local.pull_iterations = (int32_t)fin.pull_iters;
    local.edges_pushed = (int64_t)fin.edges_pushed;
    local.arcs_pulled = (int64_t)fin.arcs_pulled;
    local.frontier_sum = (int64_t)fin.frontier_sum;
    local.push_frontier_sum = (int64_t)fin.push_frontier_sum;
    local.frontier_max = (int32_t)fin.frontier_max;
    local.small_rounds = (int32_t)fin.small_rounds;
    local.push_launches = (int32_t)(fin.iter - fin.pull_iters);
    local.launches = (int32_t)std::min<int64_t>(issued, INT32_MAX);
    if (e == hipSuccess && plog) {
        // launch times by what each launch ran: advances and small rounds
        // count as push (pull rounds are not split out here), filters as filter
        std::vector<int8_t> h((size_t)std::min<int64_t>(issued, kPhaseLogCap));
        e = hipMemcpyAsync(h.data(), plog, h.size(), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        for (size_t i = 0; e == hipSuccess && 2 * i + 1 < tev.size() && i < h.size(); ++i) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, tev[2 * i], tev[2 * i + 1]);
            // launches that returned at once (query over) count with the filters
            (h[i] == 1 || h[i] == 3 ? local.push_us : local.filter_us) += 1e3 * ms;
        }
        if (fin.pull_iters > 0 && fin.pull_iters == fin.iter) {
            local.pull_us = local.push_us;
            local.push_us = 0;
        }
    }
    for (auto &x : tev) (void)hipEventDestroy(x);
    for (auto &x : evc)
        if (x) (void)hipEventDestroy(x);
    if (plog) (void)hipFreeAsync(plog, st);
    hipError_t e2 = hipFreeAsync(ws, st);
    if (e != hipSuccess) return hip_fail(e, "queued loop");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    // launches this query needed: about 2 per round, 1 per small round
    if (fin.status == 1)
        g->last_iters.store((int32_t)std::min<int64_t>(2 * (int64_t)fin.iter - (int64_t)fin.small_rounds + 1, INT32_MAX),
                            std::memory_order_relaxed);
    if (stats) *stats = local;
    if (fin.status == 2) return fail(GR_ERR_ITER_LIMIT, "iteration cap %lld reached", (long long)rc.max_iters);
    return GR_OK;
}

// Asynchronous loop: one persistent kernel drains a device worklist (see
// gr_async.hip) per phase; a phase ends early only when the list overflowed,
// and the next one starts from the spilled vertices.  The host waits for
// each phase (phases beyond the first are rare: the list holds 4 n entries).
// Single-workgroup loop (gr_lds.hip): one launch runs the whole query in one
// workgroup's LDS (k queries: k workgroups); the host reads each workgroup's
// four statistics words.
static gr_status lds_launch_wait(const LdsJob *jobs, int32_t k, hipStream_t st, int wt, int64_t max_rounds,
                                 bool timing, unsigned long long **stat_out, float *us_out) {
    // the kernel writes its statistics straight into the thread's pinned
    // buffer (mapped host memory): no workspace, no copy
    unsigned long long *hp = pinned_slot();
    if (!hp) return fail(GR_ERR_OUT_OF_MEMORY, "pinned host buffer");
    for (int i = 0; i < k * kLdsStatWords; ++i) hp[i] = 0ull;
    hipEvent_t ev[2] = {nullptr, nullptr};
    const bool timed = timing && hipEventCreate(&ev[0]) == hipSuccess && hipEventCreate(&ev[1]) == hipSuccess;
    if (timed) (void)hipEventRecord(ev[0], st);
    hipError_t e = launch_lds(jobs, k, wt, max_rounds, hp, st);
    if (timed) (void)hipEventRecord(ev[1], st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    float us = 0.f;
    if (timed && e == hipSuccess) (void)hipEventElapsedTime(&us, ev[0], ev[1]);
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(e, "single-workgroup loop");
    for (int32_t b = 0; b < k; ++b) {
        const unsigned long long code = hp[b * kLdsStatWords + 1];
        if (code == 0ull) return fail(GR_ERR_HIP, "single-workgroup loop wrote no result");
        if (code == 2ull) return fail(GR_ERR_ITER_LIMIT, "iteration cap %lld reached", (long long)max_rounds);
    }
    *stat_out = hp;
    *us_out = us;
    return GR_OK;
}

static gr_status run_lds(const gr_graph *g, int32_t src, uint32_t *dist, hipStream_t st, const RunCfg &rc,
                         gr_sssp_stats *stats) {
    const DevGraph &dg = g->plain;
    const int wt = rc.dg->wt == 2 ? 2 : dg.wt;
    if (!g->lds_fit && !g->d_ell) return fail(GR_ERR_INVALID_ARG, "the graph does not fit the single-workgroup loop");
    if (wt != 2 && !(dg.wt == GR_W_U32 && g->lds_w16))
        return fail(GR_ERR_INVALID_ARG, "the single-workgroup loop packs weights in 16 bits: uint32 weights "
                                        "below 65,536 only");
    unsigned long long *hp = nullptr;
    float us = 0.f;
    const LdsJob job{dg.ro, dg.adj, g->d_ell, dist, dg.n, dg.m, src, g->ell_lg};
    gr_status s = lds_launch_wait(&job, 1, st, wt, rc.max_iters, rc.timing, &hp, &us);
    if (s != GR_OK) return s;
    if (stats) {
        gr_sssp_stats local{};
        local.loop = GR_LOOP_LDS;
        local.layout = GR_LAYOUT_PLAIN;
        local.relax_filter = GR_RELAX_DIST;
        local.iterations = (int32_t)std::min<unsigned long long>(hp[0], INT32_MAX);
        local.edges_pushed = (int64_t)hp[2];
        local.push_frontier_sum = local.frontier_sum = (int64_t)hp[3];
        local.push_launches = local.launches = 1;
        local.push_us = 1e3 * us;
        *stats = local;
    }
    return GR_OK;
}

// Batched queries on graphs whose default is the single-workgroup loop: one
// workgroup per query, all in one launch (no shared work between queries:
// each workgroup holds its own copy of its graph in its compute unit's LDS).
// rows[i] receives query i's distances; iterations (optional) its rounds.
static_assert(kLdsMaxBatch >= kBatchLanes, "a batch fits one launch of the single-workgroup loop");
static gr_status run_lds_batch(const gr_graph *const *graphs, const int32_t *srcs, int32_t k, uint32_t *const *rows,
                               hipStream_t st, gr_multi_stats *stats, int32_t *iterations) {
    LdsJob jobs[kLdsMaxBatch];
    int64_t max_rounds = 1;
    for (int32_t i = 0; i < k; ++i) {
        const DevGraph &dg = graphs[i]->plain;
        jobs[i] = LdsJob{dg.ro, dg.adj, graphs[i]->d_ell, rows[i], dg.n, dg.m, srcs[i], graphs[i]->ell_lg};
        max_rounds = std::max<int64_t>(max_rounds, (int64_t)dg.n + 1);
    }
    unsigned long long *hp = nullptr;
    float us = 0.f;
    gr_status s = lds_launch_wait(jobs, k, st, GR_W_U32, max_rounds, false, &hp, &us);
    if (s != GR_OK) return s;
    if (stats) {
        gr_multi_stats local{};
        for (int32_t b = 0; b < k; ++b) {
            const unsigned long long *x = hp + b * kLdsStatWords;
            local.rounds = std::max(local.rounds, (int32_t)std::min<unsigned long long>(x[0], INT32_MAX));
            local.edges_pushed += (int64_t)x[2];
            local.frontier_sum += (int64_t)x[3];
        }
        local.replays = 0;  // no captured chunk: one launch, one wait
        local.source_relaxations = local.edges_pushed;
        *stats = local;
    }
    if (iterations)
        for (int32_t b = 0; b < k; ++b)
            iterations[b] = (int32_t)std::min<unsigned long long>(hp[b * kLdsStatWords], INT32_MAX);
    return GR_OK;
}

static gr_status run_async(const gr_graph *g, int32_t src, uint32_t *dist, hipStream_t st, const RunCfg &rc,
                           gr_sssp_stats *stats) {
    DeviceInfo di;
    gr_status s = device_info(g->device, &di);
    if (s != GR_OK) return s;
    const DevGraph &dg = *rc.dg;
    const uint64_t spin = (uint64_t)rc.barrier_timeout_us * (uint64_t)di.wall_khz / 1000ull;
    unsigned long long *hp = pinned_slot();
    if (!hp) return fail(GR_ERR_OUT_OF_MEMORY, "pinned host buffer");
    void *ws = nullptr, *aws = nullptr;
    // the asynchronous loop uses the flag arrays only (in-queue bytes, spill marks)
    const WsParts parts{false, false};
    HIP_TRY(hipMallocAsync(&ws, frontier_bytes(dg, parts), st));
    // GR_ASYNC_LIST_CAP (entries, >= 1) lowers the list's capacity: a test
    // hook for the overflow path
    int64_t cap = async_capacity(dg.n);
    if (const char *ev = getenv("GR_ASYNC_LIST_CAP")) {
        const long long c = atoll(ev);
        if (c >= 1) cap = std::min<int64_t>(cap, c);
    }
    hipError_t e = hipMallocAsync(&aws, async_bytes(cap), st);
    if (e != hipSuccess) {
        (void)hipFreeAsync(ws, st);
        return hip_fail(e, "hipMallocAsync");
    }
    Frontier f;
    frontier_carve(f, ws, dg, parts);
    unsigned long long *ctl = async_ctl(cap, aws);
    const int blocks = g->auto_async_blocks > 0 ? g->auto_async_blocks : async_blocks(dg, di.num_cu);
    hipEvent_t ev[2] = {nullptr, nullptr};
    const bool timed = rc.timing && hipEventCreate(&ev[0]) == hipSuccess && hipEventCreate(&ev[1]) == hipSuccess;
    gr_status status = GR_OK;
    int64_t phases = 0;
    double us = 0;
    e = launch_async_init(dg, dist, src, f, aws, cap, st);
    while (e == hipSuccess) {
        if (timed) e = hipEventRecord(ev[0], st);
        if (e == hipSuccess) e = launch_async(dg, dist, f, aws, cap, blocks, spin, st);
        if (e == hipSuccess && timed) e = hipEventRecord(ev[1], st);
        if (e == hipSuccess) e = hipMemcpyAsync(hp, ctl, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hp + 3, ctl + kAsyncTail, sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        ++phases;
        if (timed) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
            us += 1e3 * ms;
        }
        if (hp[0] == 3ull) {
            status = fail(GR_ERR_HIP, "asynchronous loop: a worklist wait exceeded %lld us",
                          (long long)rc.barrier_timeout_us);
            break;
        }
        if (hp[3] <= (unsigned long long)cap) break;  // drained without spilling: done
        // each phase expands at least one vertex, so phases end without a cap
        // unless the caller set one
        if (rc.max_iters_given && phases >= rc.max_iters) {
            status = fail(GR_ERR_ITER_LIMIT, "phase cap %lld reached", (long long)rc.max_iters);
            break;
        }
        e = launch_async_relist(dg, f, aws, cap, st);
    }
    gr_sssp_stats local{};
    local.loop = GR_LOOP_ASYNC;
    local.layout = GR_LAYOUT_PLAIN;
    local.relax_filter = GR_RELAX_DIST;
    local.iterations = (int32_t)phases;
    local.edges_pushed = (int64_t)hp[2];
    local.frontier_sum = (int64_t)hp[1];
    local.push_frontier_sum = (int64_t)hp[1];
    local.push_launches = (int32_t)phases;
    local.launches = (int32_t)(2 * phases);  // init, then one phase (+ a relist before each later one)
    local.push_us = us;
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    hipError_t e2 = hipFreeAsync(aws, st);
    hipError_t e3 = hipFreeAsync(ws, st);
    if (e != hipSuccess) return hip_fail(e, "asynchronous loop");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    if (e3 != hipSuccess) return hip_fail(e3, "hipFreeAsync");
    if (status != GR_OK) return status;
    if (stats) *stats = local;
    return GR_OK;
}

extern "C" gr_status gr_sssp_ex(const gr_graph *g, int32_t src, void *dist_out, void *stream,
                                const gr_sssp_opts *opts, gr_sssp_stats *stats) {
    if (!g) return fail(GR_ERR_INVALID_ARG, "graph is NULL");
    if (!dist_out) return fail(GR_ERR_INVALID_ARG, "dist_out is NULL");
    if (src < 0 || src >= g->plain.n) return fail(GR_ERR_SOURCE_RANGE, "src = %d outside [0, %d)", src, g->plain.n);
    RunCfg rc;
    gr_status s = check_opts(g, opts, &rc);
    if (s != GR_OK) return s;
    int loop = rc.loop;
    if (loop == GR_LOOP_AUTO) {
        loop = g->auto_loop;
        // the asynchronous and single-workgroup loops are push-only and have
        // no near-far split
        if ((loop == GR_LOOP_ASYNC || loop == GR_LOOP_LDS) &&
            (rc.direction == GR_DIR_PULL || rc.direction == GR_DIR_ALTERNATE || rc.delta))
            loop = GR_LOOP_QUEUED;
    }
    if (loop == GR_LOOP_LDS)
        return run_lds(g, src, static_cast<uint32_t *>(dist_out), static_cast<hipStream_t>(stream), rc, stats);
    if (loop == GR_LOOP_ASYNC)
        return run_async(g, src, static_cast<uint32_t *>(dist_out), static_cast<hipStream_t>(stream), rc, stats);
    if (loop == GR_LOOP_QUEUED)
        return run_queued(g, src, static_cast<uint32_t *>(dist_out), static_cast<hipStream_t>(stream), rc, stats);
    if (loop == GR_LOOP_PERSISTENT)
        return run_persistent(g, src, static_cast<uint32_t *>(dist_out), static_cast<hipStream_t>(stream), rc, stats);
    return run_host_loop(g, src, static_cast<uint32_t *>(dist_out), static_cast<hipStream_t>(stream), rc, stats);
}

extern "C" gr_status gr_sssp(const gr_graph *g, int32_t src, void *dist_out, void *stream) {
    return gr_sssp_ex(g, src, dist_out, stream, nullptr, nullptr);
}

// Allocation-free variant of the queued loop: the frontier workspace is the
// device's fixed scratch array, the loop state is read into host stack memory
// (one synchronising copy per chunk of launches), and no event, pool block or
// pinned buffer is created.
static gr_status run_queued_fixed(const gr_graph *g, int32_t src, uint32_t *dist, hipStream_t st, const RunCfg &rc,
                                  void *ws) {
    DeviceInfo di;
    gr_status s = device_info(g->device, &di);
    if (s != GR_OK) return s;
    const DevGraph &dg = *rc.dg;
    PersistentCfg cfg;
    cfg.grid = di.num_cu * 8;
    cfg.max_iters = (int32_t)std::min<int64_t>(rc.max_iters, INT32_MAX);
    cfg.alpha_x16 = rc.alpha_x16;
    cfg.beta = rc.beta;
    cfg.direction = rc.direction;
    cfg.filter = rc.filter;
    cfg.dense_ratio = rc.dense_ratio;
    cfg.delta = 0;
    cfg.spin_ticks = 0;
    cfg.local_hops = rc.local_hops;
    cfg.small = rc.small && g->max_degree <= kSmallMaxDegree &&
                (rc.direction == GR_DIR_PUSH || (rc.direction == GR_DIR_AUTO && rc.alpha_x16 == 0));
    Frontier f;
    frontier_carve(f, ws, dg, WsParts{false, rc.bound});
    // k_init clears every flag, counter and control word the loop reads
    hipError_t e = launch_init(dg, dist, src, f, kInfU32, false, st);
    int64_t issued = 0;
    int64_t K = std::clamp<int64_t>(g->last_iters.load(std::memory_order_relaxed) + 1, 4, 512);
    LoopState ls{};
    while (e == hipSuccess) {
        for (int64_t i = 0; i < K && e == hipSuccess; ++i)
            e = launch_step(dg, dist, f, cfg, issued + i, nullptr, 0, nullptr, nullptr, st);
        issued += K;
        if (e == hipSuccess) e = hipMemcpyAsync(&ls, f.ctl + kLoopStateWord, sizeof ls, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess || ls.status != 0) break;
        K = std::min<int64_t>(64, 2 * K);
    }
    if (e != hipSuccess) return hip_fail(e, "allocation-free queued loop");
    if (ls.status == 1)
        g->last_iters.store((int32_t)std::min<int64_t>(2 * (int64_t)ls.iter - (int64_t)ls.small_rounds + 1, INT32_MAX),
                            std::memory_order_relaxed);
    if (ls.status == 2) return fail(GR_ERR_ITER_LIMIT, "iteration cap %lld reached", (long long)rc.max_iters);
    if (ls.status != 1) return fail(GR_ERR_HIP, "allocation-free loop ended in state %llu", ls.status);
    return GR_OK;
}

extern "C" gr_status gr_sssp_noalloc(const gr_graph *g, int32_t src, void *dist_out, void *stream) {
    if (!g) return fail(GR_ERR_INVALID_ARG, "graph is NULL");
    if (!dist_out) return fail(GR_ERR_INVALID_ARG, "dist_out is NULL");
    if (src < 0 || src >= g->plain.n) return fail(GR_ERR_SOURCE_RANGE, "src = %d outside [0, %d)", src, g->plain.n);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != g->device)
        return fail(GR_ERR_INVALID_ARG, "current device %d is not the graph's device %d", dev, g->device);
    RunCfg rc;
    gr_status s = check_opts(g, nullptr, &rc);
    if (s != GR_OK) return s;
    // plain layout (one queue), no near-far split: the smallest workspace
    rc.dg = &g->plain;
    rc.layout = GR_LAYOUT_PLAIN;
    rc.delta = 0;
    const size_t need = frontier_bytes(g->plain, WsParts{false, rc.bound});
    if (need > kNoAllocScratchBytes)
        return fail(GR_ERR_NO_CAPACITY, "the query needs %zu bytes of workspace, the fixed scratch holds %zu", need,
                    kNoAllocScratchBytes);
    void *ws = nullptr;
    HIP_TRY(noalloc_scratch(&ws));
    return run_queued_fixed(g, src, static_cast<uint32_t *>(dist_out), static_cast<hipStream_t>(stream), rc, ws);
}

// Breadth-first search: the same operators and loops over a unit-weight view
// of the graph (weight mode 2: every arc adds one hop, its stored weight is
// not read).  The default direction rule pulls when the frontier's out-edges
// reach m / 14 (the ratio of Beamer et al.), where the pull scans only the
// in-arcs of vertices without a depth yet.
static constexpr int32_t kBfsAlphaX16 = 16 * 14;

extern "C" gr_status gr_bfs_ex(const gr_graph *g, int32_t src, void *depth_out, void *stream,
                               const gr_sssp_opts *opts, gr_sssp_stats *stats) {
    if (!g) return fail(GR_ERR_INVALID_ARG, "graph is NULL");
    if (!depth_out) return fail(GR_ERR_INVALID_ARG, "depth_out is NULL");
    if (src < 0 || src >= g->plain.n) return fail(GR_ERR_SOURCE_RANGE, "src = %d outside [0, %d)", src, g->plain.n);
    if (opts && opts->delta && opts->delta != GR_DELTA_OFF)
        return fail(GR_ERR_INVALID_ARG, "the near-far split does not apply to breadth-first search");
    gr_sssp_opts o = opts ? *opts : gr_sssp_opts{};
    o.delta = GR_DELTA_OFF;
    RunCfg rc;
    gr_status s = check_opts(g, &o, &rc);
    if (s != GR_OK) return s;
    // default: direction-optimising on skewed graphs; bounded-degree graphs
    // (grids, meshes) never build frontiers large enough to pull and run
    // push-only, which lets the queued loop use small rounds
    if (!(opts && opts->alpha_x16 > 0))
        rc.alpha_x16 = (g->pull && g->max_degree > kSmallMaxDegree) ? kBfsAlphaX16 : 0;
    // hop counts leave few redundant relaxations: dist unless asked otherwise
    if (!(opts && opts->relax_filter)) rc.bound = false;
    // AUTO: the single-workgroup loop on graphs that fit one workgroup's LDS
    // (push only: not when pull or alternation is asked for, nor with a
    // near-far split); else the host-driven loop on skewed graphs (few
    // rounds, direction-optimising: R-MAT 22 1.23 ms against 1.34 queued),
    // the queued loop on bounded-degree ones (thousands of rounds: grid
    // 2048^2 39 ms against 172)
    int loop = rc.loop;
    if (loop == GR_LOOP_AUTO) {
        const bool push_only = !(rc.direction == GR_DIR_PULL || rc.direction == GR_DIR_ALTERNATE || rc.delta);
        loop = (g->lds_fit || g->d_ell) && push_only ? GR_LOOP_LDS
               : g->max_degree > kSmallMaxDegree ? GR_LOOP_HOST
                                                 : GR_LOOP_QUEUED;
    }
    if (loop == GR_LOOP_PERSISTENT)
        return fail(GR_ERR_INVALID_ARG, "the device-driven persistent loop runs weighted queries only");
    DevGraph unit = *rc.dg;
    unit.wt = 2;
    rc.dg = &unit;
    uint32_t *d = static_cast<uint32_t *>(depth_out);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (loop == GR_LOOP_ASYNC) return run_async(g, src, d, st, rc, stats);
    if (loop == GR_LOOP_LDS) return run_lds(g, src, d, st, rc, stats);
    return loop == GR_LOOP_QUEUED ? run_queued(g, src, d, st, rc, stats) : run_host_loop(g, src, d, st, rc, stats);
}

extern "C" gr_status gr_bfs(const gr_graph *g, int32_t src, void *depth_out, void *stream) {
    return gr_bfs_ex(g, src, depth_out, stream, nullptr, nullptr);
}

// ---------------------------------------------------------------------------
// batched multi-source queries

// One query with the graph's AUTO schedule (a batch of one source).
static gr_status run_single_auto(const gr_graph *g, int32_t src, uint32_t *dist, hipStream_t st,
                                 gr_multi_stats *stats) {
    RunCfg rc;
    gr_status s = check_opts(g, nullptr, &rc);
    if (s != GR_OK) return s;
    const int loop = g->auto_loop;
    gr_sssp_stats one{};
    if (loop == GR_LOOP_ASYNC) s = run_async(g, src, dist, st, rc, &one);
    else if (loop == GR_LOOP_LDS) s = run_lds(g, src, dist, st, rc, &one);
    else if (loop == GR_LOOP_QUEUED) s = run_queued(g, src, dist, st, rc, &one);
    else if (loop == GR_LOOP_PERSISTENT) s = run_persistent(g, src, dist, st, rc, &one);
    else s = run_host_loop(g, src, dist, st, rc, &one);
    if (s == GR_OK && stats) {
        stats->rounds = one.iterations;
        stats->replays = 0;
        stats->edges_pushed = one.edges_pushed;
        stats->frontier_sum = one.frontier_sum;
        stats->source_relaxations = one.edges_pushed;
    }
    return s;
}

// ---------------------------------------------------------------------------
// multi-query sessions (gr_multi.h): one-shot gr_sssp_multi calls and the
// query server's executors

static inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Multi-query rounds whose queue holds fewer than kMqNarrowArcs arcs replay a
// capture on kMqNarrowGrid blocks per launch.
static constexpr int kMqNarrowGrid = 256;
static constexpr int64_t kMqNarrowArcs = 256 * 2048;

// Bytes of the session's control block readback: everything before the slot
// table (counters, round state, statistics, per-slot round counts).
static constexpr size_t kMqReadBytes = offsetof(MqCtl, nlive);
static_assert(kMqReadBytes % 8 == 0, "readback is whole words");

struct MqSession {
    int device = 0;
    int grid = 0;   // push launch
    int fgrid = 0;  // filter launch
    int rounds_per_replay = 0;
    int64_t qcap = 0;
    hipStream_t st = nullptr;  // the stream the memory was taken on (and is returned on)
    void *mem = nullptr;
    MqBufs b{};
    hipStream_t cap = nullptr;
    // captured rounds: [0] on the full grids, [1] on narrow grids for rounds
    // whose queue holds few arcs (the multi-query engine; a launch of many
    // idle blocks costs more than the work of a short round)
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int nexec = 0;
    unsigned char *h = nullptr;  // pinned: two readback buffers
    bool own_h = false;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int64_t replays = 0;
};

static void mq_destroy(MqSession *s) {
    for (int i = 0; i < 2; ++i) {
        if (s->exec[i]) (void)hipGraphExecDestroy(s->exec[i]);
        if (s->graph[i]) (void)hipGraphDestroy(s->graph[i]);
    }
    if (s->cap) (void)hipStreamDestroy(s->cap);
    for (auto &e : s->ev)
        if (e) (void)hipEventDestroy(e);
    if (s->h && s->own_h) (void)hipHostFree(s->h);
    if (s->mem) (void)hipFreeAsync(s->mem, s->st);
    *s = MqSession{};
}

// Queue memory per entry: (first arc, vertex) 8 + prefix 4 + slot 1, two queues.
static size_t mq_queue_bytes(int64_t qcap) {
    const size_t c = (size_t)std::max<int64_t>(qcap, 1);
    return 2 * (al256(c * 8) + al256(c * 4) + al256(c));
}

// What one captured round launches: the multi-query push and filter, or the
// batched same-graph push (vertex-major distances D, weight type wt) and filter.
struct MqMode {
    uint32_t *D = nullptr;  // non-NULL: batched same-graph queries
    uint64_t *mask[2] = {nullptr, nullptr};
    int wt = 0;
    int local_hops = 1;     // multi-query push: local hops on light graphs
};

// Allocates a session for queues of qcap entries (stream-ordered on st),
// captures `rounds` rounds as one HIP graph, and clears the control block on
// st.  own_pinned: a pinned readback buffer of its own (long-lived sessions);
// otherwise the calling thread's.
static gr_status mq_create(MqSession *s, int64_t qcap, int rounds, hipStream_t st, const MqMode &mode,
                           bool own_pinned) {
    static_assert(2 * ((kMqReadBytes + 255) & ~size_t(255)) <= 8192, "readbacks fit the thread's pinned buffer");
    *s = MqSession{};
    HIP_TRY(hipGetDevice(&s->device));
    DeviceInfo di;
    gr_status gs = device_info(s->device, &di);
    if (gs != GR_OK) return gs;
    // batched push: many small blocks balance the uneven per-arc work (64
    // sources on R-MAT 22: 84.6 ms with 128 blocks per CU, 94.3 with 8)
    s->grid = mode.D ? di.num_cu * 128 : di.num_cu * 8;
    s->fgrid = di.num_cu * 4;
    s->rounds_per_replay = rounds;
    s->qcap = std::max<int64_t>(qcap, 1);
    s->st = st;
    const size_t cb = mq_ctl_bytes();
    hipError_t e = hipMallocAsync(&s->mem, cb + mq_queue_bytes(s->qcap), st);
    if (e != hipSuccess) {
        s->mem = nullptr;
        return fail(GR_ERR_OUT_OF_MEMORY, "multi-query session of %lld queue entries: %s", (long long)s->qcap,
                    hipGetErrorString(e));
    }
    char *p = static_cast<char *>(s->mem);
    s->b.ctl = reinterpret_cast<MqCtl *>(p);
    p += cb;
    const size_t c = (size_t)s->qcap;
    for (int i = 0; i < 2; ++i) {
        s->b.qse[i] = reinterpret_cast<uint2 *>(p);
        p += al256(c * 8);
        s->b.qs[i] = reinterpret_cast<int32_t *>(p);
        p += al256(c * 4);
        s->b.qslot[i] = reinterpret_cast<uint8_t *>(p);
        p += al256(c);
    }
    s->b.qcap = s->qcap;
    s->b.mask[0] = mode.mask[0];
    s->b.mask[1] = mode.mask[1];
    s->b.local_hops = mode.D ? 1 : std::max(1, mode.local_hops);
    if (own_pinned) {
        e = hipHostMalloc(reinterpret_cast<void **>(&s->h), 2 * al256(kMqReadBytes), hipHostMallocDefault);
        s->own_h = e == hipSuccess;
    } else {
        s->h = reinterpret_cast<unsigned char *>(pinned_slot());
        if (!s->h) e = hipErrorOutOfMemory;
    }
    if (e != hipSuccess) {
        s->h = nullptr;
        mq_destroy(s);
        return fail(GR_ERR_OUT_OF_MEMORY, "pinned readback buffer");
    }
    for (auto &x : s->ev)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking);
    // every launch reads its round from the control block, so one capture
    // serves every replay of the session
    s->nexec = mode.D ? 1 : 2;
    for (int x = 0; x < s->nexec && e == hipSuccess; ++x) {
        const int pg = x == 0 ? s->grid : kMqNarrowGrid, fg = x == 0 ? s->fgrid : kMqNarrowGrid;
        e = hipStreamBeginCapture(s->cap, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
            hipError_t e1 = hipSuccess;
            for (int i = 0; i < rounds && e1 == hipSuccess; ++i)
                e1 = mode.D ? mq_batch_round(s->b, mode.D, mode.wt, pg, fg, s->cap) : mq_round(s->b, pg, fg, s->cap);
            e = hipStreamEndCapture(s->cap, &s->graph[x]);
            if (e == hipSuccess) e = e1;
        }
        if (e == hipSuccess) e = hipGraphInstantiateWithFlags(&s->exec[x], s->graph[x], 0);
    }
    if (e == hipSuccess) e = mq_reset(s->b, st);
    if (e != hipSuccess) {
        mq_destroy(s);
        return hip_fail(e, "multi-query session set-up");
    }
    return GR_OK;
}

// Per-query workspace: next-frontier marks (2 x nflag) and dirty-group bytes (2 x ngroups).
static size_t mq_slot_bytes(int32_t n) {
    const int64_t ng = groups_for(n);
    return al256((size_t)ng * kGroupVerts * 2) + al256((size_t)ng * 2);
}

static MqSlot mq_slot(const gr_graph *g, uint32_t *dist, void *ws, int wt) {
    MqSlot s{};
    s.ro = g->plain.ro;
    s.adj = g->plain.adj;
    s.dist = dist;
    s.n = g->plain.n;
    s.wt = wt;
    s.ngroups = (int32_t)groups_for(s.n);
    s.nflag = s.ngroups * kGroupVerts;
    s.flags = static_cast<uint8_t *>(ws);
    s.dirty = static_cast<uint8_t *>(ws) + al256((size_t)s.nflag * 2);
    s.light = g->max_degree <= kMqLight ? 1 : 0;
    s.pad = 0;
    return s;
}

// Live set of an update: slot ids and the prefix sum of their group counts.
static void mq_live(MqUpdate &u, const std::vector<int> &live, const std::vector<int32_t> &ngroups_of_slot) {
    u.nlive = (int32_t)live.size();
    std::memset(u.live, 0, sizeof u.live);
    int32_t acc = 0;
    for (size_t i = 0; i < live.size(); ++i) {
        u.live[i] = (uint8_t)live[i];
        u.gpre[i] = acc;
        acc += ngroups_of_slot[live[i]];
    }
    for (size_t i = live.size(); i <= (size_t)kMqSlots; ++i) u.gpre[i] = acc;
}

struct MqRead {
    unsigned long long round;  // round the next push runs
    int32_t F, E;              // its queue
    unsigned long long slot_cnt[kMqSlots];
    unsigned long long slot_rounds[kMqSlots];
    unsigned long long rounds, edges, frontier;
};

static MqRead mq_parse(const unsigned char *h) {
    MqCtl c;
    std::memcpy(static_cast<void *>(&c), h, kMqReadBytes);
    MqRead r{};
    r.round = c.st_round[0];
    r.F = (int32_t)(c.cnt[r.round % 3][0] & 0xFFFFFFFFull);
    r.E = (int32_t)(c.cnt[r.round % 3][0] >> 32);
    for (int s = 0; s < kMqSlots; ++s) {
        r.slot_cnt[s] = c.slot_cnt[r.round % 3][s];
        r.slot_rounds[s] = c.slot_rounds[s];
    }
    r.rounds = c.rounds;
    r.edges = c.edges;
    r.frontier = c.frontier;
    return r;
}

// Enqueues one replay of the captured rounds and the readback into buffer i;
// last_E: arcs of the latest queue read back (-1: unknown), which picks the
// narrow grids when it is small.
static hipError_t mq_replay(MqSession *s, int i, hipStream_t st, int64_t last_E = -1) {
    const int x = (s->nexec > 1 && last_E >= 0 && last_E < kMqNarrowArcs) ? 1 : 0;
    hipError_t e = hipGraphLaunch(s->exec[x], st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->h + i * al256(kMqReadBytes), s->b.ctl, kMqReadBytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(s->ev[i], st);
    if (e == hipSuccess) ++s->replays;
    return e;
}

static gr_status check_same_device(const gr_graph *g) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != g->device) return fail(GR_ERR_INVALID_ARG, "current device %d is not the graph's device %d", dev,
                                      g->device);
    return GR_OK;
}

static constexpr int kMqRoundsPerReplay = 8;

extern "C" gr_status gr_sssp_multi(const gr_graph *const *graphs, const int32_t *srcs, int32_t k,
                                   void *const *dist_out, void *stream, gr_multi_stats *stats,
                                   int32_t *iterations) {
    if (!graphs || !srcs || !dist_out) return fail(GR_ERR_INVALID_ARG, "NULL graphs, srcs or dist_out");
    if (k < 1 || k > kMqSlots) return fail(GR_ERR_INVALID_ARG, "k = %d outside [1, %d]", k, kMqSlots);
    int64_t sum_n = 0, sum_m = 0;
    for (int32_t i = 0; i < k; ++i) {
        const gr_graph *g = graphs[i];
        if (!g) return fail(GR_ERR_INVALID_ARG, "graphs[%d] is NULL", i);
        if (!dist_out[i]) return fail(GR_ERR_INVALID_ARG, "dist_out[%d] is NULL", i);
        if (srcs[i] < 0 || srcs[i] >= g->plain.n)
            return fail(GR_ERR_SOURCE_RANGE, "srcs[%d] = %d outside [0, %d)", i, srcs[i], g->plain.n);
        gr_status s = check_same_device(g);
        if (s != GR_OK) return s;
        sum_n += g->plain.n;
        sum_m += g->plain.m;
    }
    if (sum_m > INT32_MAX)
        return fail(GR_ERR_INVALID_ARG, "the queries' graphs hold %lld arcs together, more than 2^31 - 1",
                    (long long)sum_m);
    hipStream_t st = static_cast<hipStream_t>(stream);
    // every graph's default is the single-workgroup loop: one workgroup per query
    bool all_lds = k <= kLdsMaxBatch;
    // (one launch takes one arc layout: every graph fits the row-offset one,
    // or all have the padded one with the same slot count)
    bool all_csr = true, all_ell = true;
    for (int32_t i = 0; i < k && all_lds; ++i) {
        all_lds = graphs[i]->auto_loop == GR_LOOP_LDS;
        all_csr = all_csr && graphs[i]->lds_fit;
        all_ell = all_ell && graphs[i]->d_ell && graphs[i]->ell_lg == graphs[0]->ell_lg;
    }
    all_lds = all_lds && (all_csr || all_ell);
    if (all_lds) {
        std::vector<uint32_t *> rows((size_t)k);
        for (int32_t i = 0; i < k; ++i) rows[i] = static_cast<uint32_t *>(dist_out[i]);
        return run_lds_batch(graphs, srcs, k, rows.data(), st, stats, iterations);
    }
    MqSession ses;
    MqMode mode;
    for (int32_t i = 0; i < k; ++i) mode.local_hops = std::max(mode.local_hops, graphs[i]->auto_local_hops);
    gr_status gs = mq_create(&ses, sum_n, kMqRoundsPerReplay, st, mode, false);
    if (gs != GR_OK) return gs;
    std::vector<size_t> off((size_t)k + 1, 0);
    for (int32_t i = 0; i < k; ++i) off[i + 1] = off[i] + mq_slot_bytes(graphs[i]->plain.n);
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, off[k], st);
    if (e != hipSuccess) {
        mq_destroy(&ses);
        return hip_fail(e, "hipMallocAsync");
    }
    std::vector<int> live;
    std::vector<int32_t> ngr(kMqSlots, 0);
    for (int32_t i = 0; i < k; ++i) {
        live.push_back(i);
        ngr[i] = (int32_t)groups_for(graphs[i]->plain.n);
    }
    for (int32_t i0 = 0; i0 < k && e == hipSuccess; i0 += 16) {
        MqUpdate u{};
        u.nadmit = std::min<int32_t>(16, k - i0);
        for (int32_t j = 0; j < u.nadmit; ++j) {
            const int32_t i = i0 + j;
            u.admit_slot[j] = i;
            u.admit_src[j] = srcs[i];
            u.admit[j] = mq_slot(graphs[i], static_cast<uint32_t *>(dist_out[i]), static_cast<char *>(ws) + off[i],
                                 graphs[i]->plain.wt);
        }
        if (i0 + 16 >= k) mq_live(u, live, ngr);
        else u.nlive = -1;
        e = mq_update(ses.b, u, st);
    }
    gr_status status = GR_OK;
    MqRead rd{};
    int64_t last_E = -1;
    while (e == hipSuccess) {
        e = mq_replay(&ses, 0, st, last_E);
        if (e == hipSuccess) e = hipEventSynchronize(ses.ev[0]);
        if (e != hipSuccess) break;
        rd = mq_parse(ses.h);
        last_E = rd.E;
        if (rd.F == 0) break;
        bool over = false;
        for (int32_t i = 0; i < k; ++i)
            over = over || rd.slot_rounds[i] > (unsigned long long)graphs[i]->plain.n + 1;
        if (over) {
            status = fail(GR_ERR_ITER_LIMIT, "a query ran past n + 1 rounds");
            break;
        }
    }
    if (e == hipSuccess) e = hipFreeAsync(ws, st);
    else (void)hipFreeAsync(ws, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && stats) {
        stats->rounds = (int32_t)rd.rounds;
        stats->replays = (int32_t)ses.replays;
        stats->edges_pushed = (int64_t)rd.edges;
        stats->frontier_sum = (int64_t)rd.frontier;
        stats->source_relaxations = (int64_t)rd.edges;
    }
    if (e == hipSuccess && iterations)
        for (int32_t i = 0; i < k; ++i) iterations[i] = (int32_t)rd.slot_rounds[i];
    mq_destroy(&ses);
    if (e != hipSuccess) return hip_fail(e, "multi-query loop");
    return status;
}

// Batched same-graph queries (gr_sssp_batch, k >= 2): vertex-major distances,
// one wave lane per source, the round loop on the device, replayed from one
// captured HIP graph; the host reads the control block once per replay.
static gr_status run_batch_dev(const gr_graph *g, const int32_t *srcs, int32_t k, uint32_t *const *out_rows,
                               hipStream_t st, gr_multi_stats *stats) {
    const DevGraph &dg = g->plain;
    const int64_t n = dg.n;
    const size_t dbytes = al256((size_t)n * kBatchLanes * 4), mbytes = al256((size_t)n * 8);
    void *ws = nullptr;
    HIP_TRY(hipMallocAsync(&ws, dbytes + 2 * mbytes + mq_slot_bytes(dg.n), st));
    char *p = static_cast<char *>(ws);
    MqMode mode;
    mode.D = reinterpret_cast<uint32_t *>(p);
    mode.mask[0] = reinterpret_cast<uint64_t *>(p + dbytes);
    mode.mask[1] = reinterpret_cast<uint64_t *>(p + dbytes + mbytes);
    mode.wt = dg.wt;
    MqSession ses;
    gr_status gs = mq_create(&ses, n, kMqRoundsPerReplay, st, mode, false);
    if (gs != GR_OK) {
        (void)hipFreeAsync(ws, st);
        return gs;
    }
    const MqSlot slot = mq_slot(g, nullptr, p + dbytes + 2 * mbytes, dg.wt);
    MqBatchSrc bs{};
    bs.k = k;
    for (int32_t i = 0; i < k; ++i) bs.src[i] = srcs[i];
    hipError_t e = mq_batch_init(ses.b, slot, mode.D, bs, st);
    gr_status status = GR_OK;
    MqRead rd{};
    while (e == hipSuccess) {
        e = mq_replay(&ses, 0, st);
        if (e == hipSuccess) e = hipEventSynchronize(ses.ev[0]);
        if (e != hipSuccess) break;
        rd = mq_parse(ses.h);
        if (rd.F == 0) break;
        if (rd.rounds > (unsigned long long)n + 1) {
            status = fail(GR_ERR_ITER_LIMIT, "iteration cap %lld reached", (long long)n + 1);
            break;
        }
    }
    unsigned long long pairs = 0;
    if (e == hipSuccess && status == GR_OK) {
        MqOutRows rows{};
        for (int32_t i = 0; i < k; ++i) rows.row[i] = out_rows[i];
        e = mq_batch_output(mode.D, dg.n, k, rows, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ses.h, &ses.b.ctl->pairs, sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess) std::memcpy(&pairs, ses.h, sizeof pairs);
    }
    (void)hipFreeAsync(ws, st);
    const int64_t replays = ses.replays;
    mq_destroy(&ses);
    if (e != hipSuccess) return hip_fail(e, "batched queries");
    if (stats) {
        stats->rounds = (int32_t)rd.rounds;
        stats->replays = (int32_t)replays;
        stats->edges_pushed = (int64_t)rd.edges;
        stats->frontier_sum = (int64_t)rd.frontier;
        stats->source_relaxations = (int64_t)pairs;
    }
    return status;
}

extern "C" gr_status gr_sssp_batch_ex(const gr_graph *g, const int32_t *srcs, int32_t k, void *dist_out,
                                      void *stream, gr_multi_stats *stats) {
    if (!g) return fail(GR_ERR_INVALID_ARG, "graph is NULL");
    if (!srcs || !dist_out) return fail(GR_ERR_INVALID_ARG, "NULL srcs or dist_out");
    if (k < 1 || k > kBatchLanes) return fail(GR_ERR_INVALID_ARG, "k = %d outside [1, %d]", k, kBatchLanes);
    for (int32_t i = 0; i < k; ++i)
        if (srcs[i] < 0 || srcs[i] >= g->plain.n)
            return fail(GR_ERR_SOURCE_RANGE, "srcs[%d] = %d outside [0, %d)", i, srcs[i], g->plain.n);
    gr_status s = check_same_device(g);
    if (s != GR_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (k == 1) return run_single_auto(g, srcs[0], static_cast<uint32_t *>(dist_out), st, stats);
    std::vector<uint32_t *> rows((size_t)k);
    for (int32_t i = 0; i < k; ++i) rows[i] = static_cast<uint32_t *>(dist_out) + (size_t)i * g->plain.n;
    if (g->auto_loop == GR_LOOP_LDS) {
        std::vector<const gr_graph *> gs((size_t)k, g);
        return run_lds_batch(gs.data(), srcs, k, rows.data(), st, stats, nullptr);
    }
    return run_batch_dev(g, srcs, k, rows.data(), st, stats);
}

extern "C" gr_status gr_sssp_batch(const gr_graph *g, const int32_t *srcs, int32_t k, void *dist_out,
                                   void *stream) {
    return gr_sssp_batch_ex(g, srcs, k, dist_out, stream, nullptr);
}

// ---------------------------------------------------------------------------
// query server: continuous batching over multi-query sessions

static int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum TicketState { kQueued = 0, kRunning = 1, kDone = 2 };

struct Ticket {
    TicketState state = kQueued;
    gr_query_result res{};
};

struct gr_server {
    int device = 0;
    size_t budget = 0;
    gr_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv;
    std::vector<const gr_graph *> graphs;
    std::unique_ptr<SlotPolicy> policy;
    std::unordered_map<uint64_t, Ticket> tickets;
    uint64_t next_ticket = 1;
    size_t in_flight = 0;
    bool stopping = false;
    std::vector<std::thread> workers;
};

static QuerySize query_size(const gr_graph *g) {
    // its marks and dirty bytes, and its share of the session's two queues
    return QuerySize{mq_slot_bytes(g->plain.n) + (size_t)g->plain.n * 26, g->plain.n, g->plain.m};
}

// One executor: a session of up to max_batch slots on its own stream.  Each
// pass admits what fits into free slots (an update launch), enqueues a replay
// of the captured rounds, and then processes the readback of the previous
// replay, so the device always has the next chunk of rounds queued.  A query
// is complete when a readback taken after its admission shows no entry of its
// slot in the next round's queue; its distances are then final (they are the
// caller's buffer, updated in place).
struct LiveQuery {
    SchedQuery q;
    QuerySize z;
    void *ws = nullptr;
    int64_t admit_replay = 0;  // first replay enqueued after its admission
    int32_t batch = 0;
};

static void server_worker(gr_server *s, int exec_id) {
    (void)hipSetDevice(s->device);
    hipStream_t st = nullptr, st_direct = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
    // queries on graphs whose default is the single-workgroup loop run outside
    // the session: one workgroup per query, one launch per batch, on a stream
    // of their own, created when the first such query waits (streams beyond
    // the hardware queues share them; without it they join the session)
    bool direct_tried = false;
    const int nslots = s->cfg.max_batch;
    MqSession ses;
    bool have_ses = false;
    int64_t qcap = 0;
    std::vector<LiveQuery> slot((size_t)kMqSlots);
    std::vector<bool> used((size_t)kMqSlots, false);
    std::vector<int32_t> ngr((size_t)kMqSlots, 0);
    std::vector<int32_t> qrounds((size_t)kMqSlots, 0);
    int nused = 0;
    int64_t used_n = 0, used_m = 0;
    bool live_changed = false;
    int64_t outstanding = -1;  // replay whose readback is pending
    int64_t last_E = -1;       // arcs of the queue in the latest readback
    gr_status broken = GR_OK;   // a HIP failure ends every query of this executor with it
    if (!st) broken = fail(GR_ERR_HIP, "query server: no stream for an executor");
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // 0. direct queries: taken from anywhere in the FIFO, run and completed
        // here (the session's replays already queued keep the device busy)
        if (broken == GR_OK && !direct_tried && s->policy->has_direct()) {
            direct_tried = true;
            lk.unlock();
            if (hipStreamCreateWithFlags(&st_direct, hipStreamNonBlocking) != hipSuccess) st_direct = nullptr;
            lk.lock();
        }
        if (broken == GR_OK && st_direct) {
            const std::vector<SchedQuery> dq = s->policy->take_direct(kLdsMaxBatch);
            if (!dq.empty()) {
                const int64_t t_start = now_ns();
                for (const SchedQuery &q : dq) {
                    Ticket &t = s->tickets[q.ticket];
                    t.state = kRunning;
                    t.res.t_start_ns = t_start;
                }
                lk.unlock();
                LdsJob jobs[kLdsMaxBatch];
                int64_t max_rounds = 1;
                for (size_t b = 0; b < dq.size(); ++b) {
                    const gr_graph *g = s->graphs[dq[b].graph];
                    const DevGraph &dg = g->plain;
                    jobs[b] = LdsJob{dg.ro,  dg.adj, g->d_ell, static_cast<uint32_t *>(dq[b].dst),
                                     dg.n,   dg.m,   dq[b].src, g->ell_lg};
                    max_rounds = std::max<int64_t>(max_rounds, (int64_t)dg.n + 1);
                }
                unsigned long long *hp = nullptr;
                float us = 0.f;
                const gr_status ds =
                    lds_launch_wait(jobs, (int32_t)dq.size(), st_direct, GR_W_U32, max_rounds, false, &hp, &us);
                const int64_t t_done = now_ns();
                lk.lock();
                for (size_t b = 0; b < dq.size(); ++b) {
                    Ticket &t = s->tickets[dq[b].ticket];
                    t.state = kDone;
                    t.res.status = ds;
                    t.res.t_done_ns = t_done;
                    t.res.batch_size = (int32_t)dq.size();
                    t.res.iterations =
                        ds == GR_OK ? (int32_t)std::min<unsigned long long>(hp[b * kLdsStatWords], INT32_MAX) : 0;
                }
                s->cv.notify_all();
            }
        }
        // 1. admissions
        std::vector<SchedQuery> adm;
        if (broken == GR_OK && st) {
            const SchedQuery *h = s->policy->head();
            if (h && nused == 0) {
                // the session's queue holds max_batch queries of the largest registered graph
                int64_t need = 1;
                for (const gr_graph *g : s->graphs) need = std::max<int64_t>(need, g->plain.n);
                need *= nslots;
                if (!have_ses || need > qcap) {
                    lk.unlock();
                    if (have_ses) {
                        (void)hipStreamSynchronize(st);
                        mq_destroy(&ses);
                        have_ses = false;
                        outstanding = -1;  // nothing live: its readback is not needed
                        last_E = -1;
                    }
                    MqMode mode;
                    mode.local_hops = s->cfg.local_hops;
                    gr_status gs = mq_create(&ses, need, kMqRoundsPerReplay, st, mode, true);
                    lk.lock();
                    if (gs != GR_OK) broken = gs;
                    else {
                        have_ses = true;
                        qcap = need;
                    }
                }
            }
            if (have_ses)
                adm = s->policy->admit(SessionRoom{nslots - nused, qcap - used_n, (int64_t)INT32_MAX - used_m},
                                       &s->in_flight);
        }
        if (broken != GR_OK) {
            // fail everything this executor holds and every query still queued
            for (int i = 0; i < kMqSlots; ++i)
                if (used[i]) {
                    Ticket &t = s->tickets[slot[i].q.ticket];
                    t.state = kDone;
                    t.res.status = broken;
                    t.res.t_done_ns = now_ns();
                    s->in_flight -= slot[i].z.bytes;
                    used[i] = false;
                }
            nused = 0;
            for (const SchedQuery &q : s->policy->take_all()) {
                Ticket &t = s->tickets[q.ticket];
                t.state = kDone;
                t.res.status = broken;
                t.res.t_done_ns = now_ns();
            }
            s->cv.notify_all();
            if (s->stopping) break;
            s->cv.wait(lk);
            continue;
        }
        const int64_t t_adm = now_ns();
        std::vector<std::pair<int, const gr_graph *>> newq;
        for (const SchedQuery &q : adm) {
            int i = 0;
            while (used[i]) ++i;
            used[i] = true;
            ++nused;
            LiveQuery &L = slot[i];
            L = LiveQuery{};
            L.q = q;
            L.z = query_size(s->graphs[q.graph]);
            used_n += L.z.n;
            used_m += L.z.m;
            ngr[i] = (int32_t)groups_for(s->graphs[q.graph]->plain.n);
            newq.emplace_back(i, s->graphs[q.graph]);
            Ticket &t = s->tickets[q.ticket];
            t.state = kRunning;
            t.res.t_start_ns = t_adm;
        }
        for (auto &x : newq) slot[x.first].batch = nused;
        if (!adm.empty()) live_changed = true;
        const bool any_live = nused > 0;
        if (!any_live && outstanding < 0) {
            if (s->stopping && s->policy->pending() == 0) break;
            // direct queries that arrived while the lock was released above
            if (!((st_direct || !direct_tried) && s->policy->has_direct())) s->cv.wait(lk);
            continue;
        }
        lk.unlock();
        hipError_t e = hipSuccess;
        // 2. slot workspaces and the update launch (admissions + live set)
        for (auto &x : newq) {
            if (e == hipSuccess) e = hipMallocAsync(&slot[x.first].ws, mq_slot_bytes(x.second->plain.n), st);
        }
        if (e == hipSuccess && live_changed) {
            std::vector<int> live;
            for (int i = 0; i < kMqSlots; ++i)
                if (used[i]) live.push_back(i);
            size_t j = 0;
            do {
                MqUpdate u{};
                u.nadmit = 0;
                while (j < newq.size() && u.nadmit < 16) {
                    const int i = newq[j].first;
                    u.admit_slot[u.nadmit] = i;
                    u.admit_src[u.nadmit] = slot[i].q.src;
                    u.admit[u.nadmit] = mq_slot(newq[j].second, static_cast<uint32_t *>(slot[i].q.dst), slot[i].ws,
                                                newq[j].second->plain.wt);
                    ++u.nadmit;
                    ++j;
                }
                if (j >= newq.size()) mq_live(u, live, ngr);
                else u.nlive = -1;
                e = mq_update(ses.b, u, st);
            } while (e == hipSuccess && j < newq.size());
            live_changed = false;
        }
        for (auto &x : newq) slot[x.first].admit_replay = ses.replays;
        // 3. the next replay
        int64_t issued = -1;
        if (e == hipSuccess && any_live) {
            issued = ses.replays;
            e = mq_replay(&ses, (int)(issued & 1), st, last_E);
        }
        // 4. the previous replay's readback
        std::vector<int> done;
        if (e == hipSuccess && outstanding >= 0) {
            e = hipEventSynchronize(ses.ev[outstanding & 1]);
            if (e == hipSuccess) {
                const MqRead rd = mq_parse(ses.h + (outstanding & 1) * al256(kMqReadBytes));
                last_E = rd.E;
                for (int i = 0; i < kMqSlots; ++i)
                    if (used[i] && outstanding >= slot[i].admit_replay && rd.slot_cnt[i] == 0ull) {
                        done.push_back(i);
                        qrounds[i] = (int32_t)rd.slot_rounds[i];
                    }
            }
        }
        outstanding = issued;
        // finished queries' workspaces are freed after the replay just issued (stream order)
        for (int i : done)
            if (e == hipSuccess) e = hipFreeAsync(slot[i].ws, st);
        const int64_t t_done = now_ns();
        lk.lock();
        for (int i : done) {
            Ticket &t = s->tickets[slot[i].q.ticket];
            t.state = kDone;
            t.res.status = GR_OK;
            t.res.t_done_ns = t_done;
            t.res.batch_size = slot[i].batch;
            t.res.iterations = qrounds[i];
            s->in_flight -= slot[i].z.bytes;
            used[i] = false;
            --nused;
            used_n -= slot[i].z.n;
            used_m -= slot[i].z.m;
            ngr[i] = 0;
            live_changed = true;
        }
        if (!done.empty()) s->cv.notify_all();
        if (e != hipSuccess) {
            broken = hip_fail(e, "query server executor");
            outstanding = -1;
        }
    }
    lk.unlock();
    if (st) (void)hipStreamSynchronize(st);
    if (have_ses) mq_destroy(&ses);
    if (st) (void)hipStreamDestroy(st);
    if (st_direct) (void)hipStreamDestroy(st_direct);
    (void)exec_id;
}

extern "C" gr_status gr_server_create(gr_server **out, size_t hbm_budget_bytes, const gr_server_config *cfg) {
    if (!out) return fail(GR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    gr_server_config c{};
    if (cfg) c = *cfg;
    if (c.max_batch == 0) c.max_batch = kMqSlots;
    // three executors by default: their sessions' rounds are latency-bound, and
    // three in flight fill the device best (32 serving graphs: Q* 870, 1156,
    // 1287, 1178 queries/s with 1, 2, 3, 4 executors)
    if (c.num_streams == 0) c.num_streams = 3;
    if (c.max_batch < 1 || c.max_batch > kMqSlots)
        return fail(GR_ERR_INVALID_ARG, "max_batch = %d outside [1, %d]", c.max_batch, kMqSlots);
    if (c.num_streams < 1 || c.num_streams > 8)
        return fail(GR_ERR_INVALID_ARG, "num_streams = %d outside [1, 8]", c.num_streams);
    if (c.max_wait_us < 0) return fail(GR_ERR_INVALID_ARG, "max_wait_us = %d is negative", c.max_wait_us);
    if (c.local_hops == 0) c.local_hops = kDefaultLocalHops;
    if (c.local_hops < 1 || c.local_hops > 64)
        return fail(GR_ERR_INVALID_ARG, "local_hops = %d outside [1, 64]", c.local_hops);
    if (hbm_budget_bytes == 0) return fail(GR_ERR_INVALID_ARG, "zero memory budget");
    std::unique_ptr<gr_server> s(new (std::nothrow) gr_server());
    if (!s) return fail(GR_ERR_OUT_OF_MEMORY, "host allocation");
    HIP_TRY(hipGetDevice(&s->device));
    s->budget = hbm_budget_bytes;
    s->cfg = c;
    gr_server *raw = s.get();
    s->policy.reset(new SlotPolicy(hbm_budget_bytes, [raw](int32_t gid) { return query_size(raw->graphs[gid]); }));
    for (int i = 0; i < c.num_streams; ++i) s->workers.emplace_back(server_worker, raw, i);
    *out = s.release();
    return GR_OK;
}

extern "C" gr_status gr_server_add_graph(gr_server *s, const gr_graph *g, int32_t *graph_id) {
    if (!s || !g || !graph_id) return fail(GR_ERR_INVALID_ARG, "NULL argument");
    if (g->device != s->device)
        return fail(GR_ERR_INVALID_ARG, "graph on device %d, server on device %d", g->device, s->device);
    std::lock_guard<std::mutex> lk(s->mu);
    s->graphs.push_back(g);
    *graph_id = (int32_t)s->graphs.size() - 1;
    return GR_OK;
}

extern "C" gr_status gr_serve_submit(gr_server *s, int32_t graph_id, int32_t src, void *dist_out,
                                     uint64_t *ticket) {
    if (!s || !dist_out || !ticket) return fail(GR_ERR_INVALID_ARG, "NULL argument");
    const int64_t t = now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    if (graph_id < 0 || graph_id >= (int32_t)s->graphs.size())
        return fail(GR_ERR_INVALID_ARG, "unknown graph id %d", graph_id);
    const gr_graph *g = s->graphs[graph_id];
    if (src < 0 || src >= g->plain.n) return fail(GR_ERR_SOURCE_RANGE, "src = %d outside [0, %d)", src, g->plain.n);
    const size_t need = query_size(g).bytes;
    if (need > s->budget)
        return fail(GR_ERR_NO_CAPACITY, "a query on graph %d needs %zu bytes, budget is %zu", graph_id, need,
                    s->budget);
    const uint64_t id = s->next_ticket++;
    Ticket &tk = s->tickets[id];
    tk.res.status = GR_ERR_NOT_READY;
    tk.res.graph_id = graph_id;
    tk.res.src = src;
    tk.res.t_submit_ns = t;
    // queries on graphs that run the single-workgroup loop by default are
    // run outside the executors' sessions
    // (those whose graph fits the row-offset layout, which any mix of them shares)
    s->policy->push(SchedQuery{id, graph_id, src, dist_out, t, g->auto_loop == GR_LOOP_LDS && g->lds_fit});
    s->cv.notify_all();
    *ticket = id;
    return GR_OK;
}

extern "C" gr_status gr_serve_poll(gr_server *s, uint64_t ticket, gr_query_result *out) {
    if (!s) return fail(GR_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(GR_ERR_UNKNOWN_TICKET, "ticket %llu unknown", (unsigned long long)ticket);
    if (it->second.state != kDone) return GR_ERR_NOT_READY;
    if (out) *out = it->second.res;
    s->tickets.erase(it);
    return GR_OK;
}

extern "C" gr_status gr_server_destroy(gr_server *s) {
    if (!s) return fail(GR_ERR_INVALID_ARG, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv.notify_all();
    for (std::thread &t : s->workers) t.join();
    delete s;
    return GR_OK;
}

// ---------------------------------------------------------------------------
// autotuner

static std::string graph_signature(const gr_graph *g) {
    // n, m, weight type, degree statistics and a hash of the offsets
    uint64_t h = 1469598103934665603ull;
    const size_t step = std::max<size_t>(1, g->h_ro.size() / 4096);
    for (size_t i = 0; i < g->h_ro.size(); i += step) {
        h ^= (uint64_t)(uint32_t)g->h_ro[i];
        h *= 1099511628211ull;
    }
    char buf[256];
    snprintf(buf, sizeof buf, "n%d_m%d_w%d_dmax%d_loc%.3f_p%d_h%016llx", g->plain.n, g->plain.m, g->plain.wt,
             g->max_degree, g->locality, g->has_part ? 8 : 1, (unsigned long long)h);
    return buf;
}

static bool cache_lookup(const std::string &sig, gr_tune_result *r) {
    const char *path = getenv("GR_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char s[300];
        int lay, loop, dr, al;
        unsigned dl;
        int sm, rf, ab, lh;
        double ms;
        if (sscanf(line, "{\"sig\": \"%299[^\"]\", \"layout\": %d, \"loop\": %d, \"dense_ratio\": %d, \"alpha_x16\": %d, "
                         "\"delta\": %u, \"small\": %d, \"relax_filter\": %d, \"async_blocks\": %d, "
                         "\"local_hops\": %d, \"best_ms\": %lf}",
                   s, &lay, &loop, &dr, &al, &dl, &sm, &rf, &ab, &lh, &ms) == 11 &&
            sig == s) {
            r->layout = lay;
            r->loop = loop;
            r->dense_ratio = dr;
            r->alpha_x16 = al;
            r->delta = dl;
            r->small = sm;
            r->relax_filter = rf;
            r->async_blocks = ab;
            r->local_hops = lh;
            r->best_ms = ms;
            found = true;  // the last matching line wins
        }
    }
    fclose(f);
    return found;
}

static void cache_store(const std::string &sig, const gr_tune_result &r) {
    const char *path = getenv("GR_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "{\"sig\": \"%s\", \"layout\": %d, \"loop\": %d, \"dense_ratio\": %d, \"alpha_x16\": %d, "
               "\"delta\": %u, \"small\": %d, \"relax_filter\": %d, \"async_blocks\": %d, \"local_hops\": %d, "
               "\"best_ms\": %.6f}\n",
            sig.c_str(), r.layout, r.loop, r.dense_ratio, r.alpha_x16, r.delta, r.small, r.relax_filter, r.async_blocks,
            r.local_hops, r.best_ms);
    fclose(f);
}

struct TuneCfg {
    int32_t layout, loop, dense_ratio, alpha_x16;
    uint32_t delta;
    int32_t small;
    int32_t relax;
    int32_t async_blocks;  // 0: the default
    int32_t local_hops;
};

static void apply_auto(gr_graph *g, const TuneCfg &c) {
    g->auto_layout = c.layout;
    g->auto_loop = c.loop;
    g->auto_dense_ratio = c.dense_ratio;
    g->auto_alpha_x16 = c.alpha_x16;
    g->auto_delta = c.delta;
    g->auto_small = c.small != 0;
    g->auto_relax = c.relax;
    g->auto_async_blocks = c.async_blocks;
    g->auto_local_hops = c.local_hops;
}

// Near-far split widths to try: multiples of the mean weight of a sample of
// arcs (weight-type bits).
static std::vector<uint32_t> delta_candidates(const gr_graph *g, hipStream_t st) {
    std::vector<uint32_t> out;
    const int32_t m = g->plain.m;
    if (m <= 0) return out;
    const int32_t ns = std::min<int32_t>(m, 4096);
    std::vector<uint2> h((size_t)ns);
    if (hipMemcpyAsync(h.data(), g->plain.adj, sizeof(uint2) * (size_t)ns, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return out;
    double mean = 0;
    for (const uint2 &a : h) {
        if (g->plain.wt == GR_W_F32) {
            float x;
            std::memcpy(&x, &a.y, 4);
            mean += x;
        } else {
            mean += a.y;
        }
    }
    mean /= ns;
    for (double f : {0.25, 1.0, 4.0, 16.0}) {
        const double d = mean * f;
        uint32_t bits;
        if (g->plain.wt == GR_W_F32) {
            const float x = (float)std::max(d, 1e-30);
            std::memcpy(&bits, &x, 4);
        } else {
            bits = (uint32_t)std::min(std::max(d, 1.0), 4.0e9);
        }
        out.push_back(bits);
    }
    return out;
}

extern "C" gr_status gr_graph_tune(gr_graph *g, const int32_t *srcs, int32_t nsrcs, int32_t reps, void *stream,
                                   gr_tune_result *out) {
    if (!g) return fail(GR_ERR_INVALID_ARG, "graph is NULL");
    if (!srcs || nsrcs < 1) return fail(GR_ERR_INVALID_ARG, "no sources to tune with");
    if (reps < 1) reps = 1;
    for (int32_t i = 0; i < nsrcs; ++i)
        if (srcs[i] < 0 || srcs[i] >= g->plain.n)
            return fail(GR_ERR_SOURCE_RANGE, "srcs[%d] = %d outside [0, %d)", i, srcs[i], g->plain.n);
    gr_tune_result r{};
    const std::string sig = graph_signature(g);
    if (cache_lookup(sig, &r)) {
        if (r.layout == GR_LAYOUT_PARTITIONED && !g->has_part) r.layout = GR_LAYOUT_PLAIN;
        if (r.alpha_x16 > 0 && !g->pull) r.alpha_x16 = 0;
        if (r.delta) r.alpha_x16 = 0;
        if (r.relax_filter != GR_RELAX_BOUND) r.relax_filter = GR_RELAX_DIST;
        if (r.async_blocks < 0 || r.async_blocks > 65536) r.async_blocks = 0;
        if (r.local_hops < 1 || r.local_hops > 64) r.local_hops = kDefaultLocalHops;
        apply_auto(g, TuneCfg{r.layout, r.loop, r.dense_ratio, r.alpha_x16, r.delta, r.small, r.relax_filter,
                              r.async_blocks, r.local_hops});
        r.from_cache = 1;
        if (out) *out = r;
        return GR_OK;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    void *dist = nullptr;
    HIP_TRY(hipMallocAsync(&dist, sizeof(uint32_t) * (size_t)g->plain.n, st));
    gr_status status = GR_OK;
    int trials = 0;
    auto measure = [&](const TuneCfg &c, double *ms) -> gr_status {
        gr_sssp_opts o{};
        o.loop = c.loop;
        o.layout = c.layout;
        o.alpha_x16 = c.alpha_x16 > 0 ? c.alpha_x16 : 0;
        o.direction = c.alpha_x16 > 0 ? GR_DIR_AUTO : GR_DIR_PUSH;
        o.delta = (c.delta && c.loop != GR_LOOP_ASYNC && c.loop != GR_LOOP_LDS) ? c.delta : GR_DELTA_OFF;
        if (c.loop == GR_LOOP_ASYNC || c.loop == GR_LOOP_LDS) o.direction = GR_DIR_PUSH;
        o.filter = c.small ? 3 : 0;
        o.relax_filter = c.relax;
        o.local_hops = c.local_hops;
        const int32_t saved = g->auto_dense_ratio, saved_ab = g->auto_async_blocks;
        g->auto_dense_ratio = c.dense_ratio;
        g->auto_async_blocks = c.async_blocks;
        std::vector<double> t;
        gr_status s = GR_OK;
        for (int32_t rep = 0; rep <= reps && s == GR_OK; ++rep) {
            for (int32_t i = 0; i < nsrcs && s == GR_OK; ++i) {
                const auto t0 = std::chrono::steady_clock::now();
                s = gr_sssp_ex(g, srcs[i], dist, st, &o, nullptr);
                if (s == GR_OK && hipStreamSynchronize(st) != hipSuccess) s = fail(GR_ERR_HIP, "tuning query");
                const double d = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                                     .count();
                if (rep > 0) t.push_back(d);  // rep 0 warms up
            }
        }
        g->auto_dense_ratio = saved;
        g->auto_async_blocks = saved_ab;
        ++trials;
        if (s != GR_OK) return s;
        std::sort(t.begin(), t.end());
        *ms = t[t.size() / 2];
        return GR_OK;
    };
    TuneCfg best{g->auto_layout, g->auto_loop, g->auto_dense_ratio, g->auto_alpha_x16, g->auto_delta,
                 g->auto_small ? 1 : 0, g->auto_relax, g->auto_async_blocks, g->auto_local_hops};
    double best_ms = 0;
    status = measure(best, &best_ms);
    const double default_ms = best_ms;
    // greedy: one knob at a time, the others at their best so far
    std::vector<std::pair<int, std::vector<int32_t>>> knobs;
    knobs.push_back({0, g->has_part ? std::vector<int32_t>{GR_LAYOUT_PLAIN, GR_LAYOUT_PARTITIONED}
                                    : std::vector<int32_t>{GR_LAYOUT_PLAIN}});
    {
        DeviceInfo di;
        const bool coop = device_info(g->device, &di) == GR_OK && di.coop &&
                          persistent_grid(g->plain, di.num_cu) >= kMaxParts;
        std::vector<int32_t> loops = coop ? std::vector<int32_t>{GR_LOOP_HOST, GR_LOOP_QUEUED, GR_LOOP_PERSISTENT,
                                                                 GR_LOOP_ASYNC}
                                          : std::vector<int32_t>{GR_LOOP_HOST, GR_LOOP_QUEUED, GR_LOOP_ASYNC};
        if ((g->lds_fit || g->d_ell) && g->lds_w16) loops.push_back(GR_LOOP_LDS);
        knobs.push_back({1, loops});
    }
    knobs.push_back({2, {8, 64, 512}});
    if (g->pull) knobs.push_back({3, {0, 8, 32}});
    {
        std::vector<int32_t> ds{0};
        for (uint32_t d : delta_candidates(g, st)) ds.push_back((int32_t)d);
        knobs.push_back({4, ds});
    }
    if (g->max_degree <= kSmallMaxDegree) knobs.push_back({5, {0, 1}});
    knobs.push_back({6, {GR_RELAX_DIST, GR_RELAX_BOUND}});
    knobs.push_back({7, {64, 128, 256, 512, 1024}});  // asynchronous loop only
    if (g->max_degree <= kSmallMaxDegree) knobs.push_back({8, {1, 2, 4, 6, 8, 16}});  // small rounds only
    for (const auto &kv : knobs) {
        for (int32_t v : kv.second) {
            if (status != GR_OK) break;
            TuneCfg c = best;
            if (c.loop == GR_LOOP_ASYNC && kv.first != 1 && kv.first != 7) continue;  // the others do not apply
            if (c.loop == GR_LOOP_LDS && kv.first != 1) continue;
            if (kv.first == 7 && c.loop != GR_LOOP_ASYNC) continue;
            if (kv.first == 4) {
                if (c.delta == (uint32_t)v) continue;
                c.delta = (uint32_t)v;
                if (c.delta) c.alpha_x16 = 0;  // the split runs push only
            } else if (kv.first == 5) {
                if (c.small == v || c.loop != GR_LOOP_QUEUED || c.delta) continue;
                c.small = v;
            } else if (kv.first == 7) {
                if (c.async_blocks == v) continue;
                c.async_blocks = v;
            } else if (kv.first == 8) {
                if (c.local_hops == v || !c.small || c.loop != GR_LOOP_QUEUED || c.delta) continue;
                c.local_hops = v;
            } else if (kv.first == 6) {
                if (c.relax == v) continue;
                c.relax = v;
            } else if (kv.first == 3 && c.delta) {
                continue;
            } else {
                int32_t *field = kv.first == 0 ? &c.layout : kv.first == 1 ? &c.loop : kv.first == 2 ? &c.dense_ratio
                                                                                                   : &c.alpha_x16;
                if (*field == v) continue;
                *field = v;
            }
            double ms = 0;
            status = measure(c, &ms);
            if (status == GR_OK && ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
    }
    (void)hipFreeAsync(dist, st);
    (void)hipStreamSynchronize(st);
    if (status != GR_OK) return status;
    apply_auto(g, best);
    r.layout = best.layout;
    r.loop = best.loop;
    r.dense_ratio = best.dense_ratio;
    r.alpha_x16 = best.alpha_x16;
    r.delta = best.delta;
    r.small = best.small;
    r.relax_filter = best.relax;
    r.async_blocks = best.async_blocks;
    r.local_hops = best.local_hops;
    r.best_ms = best_ms;
    r.default_ms = default_ms;
    r.trials = trials;
    cache_store(sig, r);
    if (out) *out = r;
    return GR_OK;
}
