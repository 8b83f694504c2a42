// Host runtime of the C ABI declared in include/gr.h: graph store, loop
// drivers (host-driven and device-driven), batched queries and the server.
#include "gr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gr_internal.h"

namespace gr {
hipError_t launch_canon_negzero(uint2 *adj, int32_t m, hipStream_t st);
size_t scan_tmp_ints(int64_t len);
}  // namespace gr

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
        if (hipHostMalloc(&q, 256, hipHostMallocDefault) != hipSuccess) return nullptr;
        p = static_cast<unsigned long long *>(q);
    }
    return p;
}

// ---------------------------------------------------------------------------
// graph

struct gr_graph {
    int device = 0;
    DevGraph dg{};
    int32_t *d_ro = nullptr;
    uint2 *d_adj = nullptr;
    int32_t *d_ro_in = nullptr;  // == d_ro when symmetric
    uint2 *d_adj_in = nullptr;   // == d_adj when symmetric
    bool pull = false;
    bool csc_separate = false;
    size_t dev_bytes = 0;
    std::vector<int32_t> h_ro;
    int32_t max_degree = 0;
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
    delete g;
}

static gr_status graph_build(gr_graph *g, int32_t n, int32_t m, const int32_t *ro, const int32_t *col,
                             const void *weights, gr_weight_type wt, uint32_t flags, hipStream_t st) {
    const bool dev_in = flags & GR_INPUT_DEVICE;
    HIP_TRY(hipGetDevice(&g->device));
    HIP_TRY(hipMalloc(&g->d_ro, sizeof(int32_t) * ((size_t)n + 1)));
    HIP_TRY(hipMalloc(&g->d_adj, sizeof(uint2) * (size_t)std::max(m, 1)));
    g->dev_bytes = sizeof(int32_t) * ((size_t)n + 1) + sizeof(uint2) * (size_t)std::max(m, 1);
    int32_t *tcol = nullptr;
    uint32_t *tw = nullptr;
    unsigned int *flag = nullptr;
    auto cleanup = [&]() {
        if (tcol) (void)hipFree(tcol);
        if (tw) (void)hipFree(tw);
        if (flag) (void)hipFree(flag);
    };
    hipError_t e;
    const hipMemcpyKind kind = dev_in ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if ((e = hipMalloc(&flag, 64)) != hipSuccess) { cleanup(); return hip_fail(e, "hipMalloc(flag)"); }
    if ((e = hipMalloc(&tcol, sizeof(int32_t) * (size_t)std::max(m, 1))) != hipSuccess ||
        (e = hipMalloc(&tw, sizeof(uint32_t) * (size_t)std::max(m, 1))) != hipSuccess) {
        cleanup();
        return hip_fail(e, "hipMalloc(staging)");
    }
    if ((e = hipMemcpyAsync(g->d_ro, ro, sizeof(int32_t) * ((size_t)n + 1), kind, st)) != hipSuccess ||
        (m > 0 && (e = hipMemcpyAsync(tcol, col, sizeof(int32_t) * (size_t)m, kind, st)) != hipSuccess) ||
        (m > 0 && (e = hipMemcpyAsync(tw, weights, sizeof(uint32_t) * (size_t)m, kind, st)) != hipSuccess) ||
        (e = hipMemsetAsync(flag, 0, 64, st)) != hipSuccess) {
        cleanup();
        return hip_fail(e, "upload");
    }
    if (dev_in) {
        unsigned int err = 0;
        if ((e = launch_validate(n, m, g->d_ro, tcol, tw, (int)wt, flag, st)) != hipSuccess ||
            (e = hipMemcpyAsync(&err, flag, sizeof err, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess) {
            cleanup();
            return hip_fail(e, "validate");
        }
        if (err) {
            cleanup();
            return fail(GR_ERR_INVALID_ARG, "device CSR is malformed (%s%s%s)", (err & 1) ? "row_offsets " : "",
                        (err & 2) ? "col_indices " : "", (err & 4) ? "weights" : "");
        }
        g->h_ro.resize((size_t)n + 1);
        if ((e = hipMemcpy(g->h_ro.data(), g->d_ro, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost)) !=
            hipSuccess) {
            cleanup();
            return hip_fail(e, "copy row_offsets");
        }
    } else {
        g->h_ro.assign(ro, ro + (size_t)n + 1);
    }
    if ((e = launch_pack_arcs(tcol, tw, m, g->d_adj, st)) != hipSuccess ||
        (wt == GR_W_F32 && (e = launch_canon_negzero(g->d_adj, m, st)) != hipSuccess)) {
        cleanup();
        return hip_fail(e, "pack arcs");
    }
    for (int32_t v = 0; v < n; ++v) g->max_degree = std::max(g->max_degree, g->h_ro[v + 1] - g->h_ro[v]);

    g->d_ro_in = g->d_ro;
    g->d_adj_in = g->d_adj;
    if (!(flags & GR_NO_PULL)) {
        unsigned int not_sym = 0;
        if ((e = hipMemsetAsync(flag, 0, 64, st)) != hipSuccess ||
            (e = launch_symmetry_check(n, g->d_ro, g->d_adj, flag, st)) != hipSuccess ||
            (e = hipMemcpyAsync(&not_sym, flag, sizeof not_sym, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess) {
            cleanup();
            return hip_fail(e, "symmetry check");
        }
        if (not_sym) {
            int32_t *scratch = nullptr;
            const size_t sc = (2 * (size_t)n + 1) + scan_tmp_ints((int64_t)n + 1);
            if ((e = hipMalloc(&g->d_ro_in, sizeof(int32_t) * ((size_t)n + 1))) != hipSuccess ||
                (e = hipMalloc(&g->d_adj_in, sizeof(uint2) * (size_t)std::max(m, 1))) != hipSuccess ||
                (e = hipMalloc(&scratch, sizeof(int32_t) * sc)) != hipSuccess) {
                if (scratch) (void)hipFree(scratch);
                cleanup();
                return hip_fail(e, "hipMalloc(csc)");
            }
            e = launch_csc_build(n, m, g->d_ro, g->d_adj, g->d_ro_in, g->d_adj_in, scratch, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            (void)hipFree(scratch);
            if (e != hipSuccess) {
                cleanup();
                return hip_fail(e, "csc build");
            }
            g->csc_separate = true;
            g->dev_bytes += sizeof(int32_t) * ((size_t)n + 1) + sizeof(uint2) * (size_t)std::max(m, 1);
        }
        g->pull = true;
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) {
        cleanup();
        return hip_fail(e, "graph upload");
    }
    cleanup();
    g->dg.n = n;
    g->dg.m = m;
    g->dg.wt = (int32_t)wt;
    g->dg.ro = g->d_ro;
    g->dg.adj = g->d_adj;
    g->dg.ro_in = g->d_ro_in;
    g->dg.adj_in = g->d_adj_in;
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
    if (flags & ~(GR_INPUT_DEVICE | GR_NO_PULL)) return fail(GR_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
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

extern "C" gr_status gr_graph_info(const gr_graph *g, int32_t *n, int32_t *m, int32_t *wt, size_t *dev_bytes,
                                   int32_t *has_csc, int32_t *pull_enabled) {
    if (!g) return fail(GR_ERR_INVALID_ARG, "graph is NULL");
    if (n) *n = g->dg.n;
    if (m) *m = g->dg.m;
    if (wt) *wt = g->dg.wt;
    if (dev_bytes) *dev_bytes = g->dev_bytes;
    if (has_csc) *has_csc = g->csc_separate ? 1 : 0;
    if (pull_enabled) *pull_enabled = g->pull ? 1 : 0;
    return GR_OK;
}

// ---------------------------------------------------------------------------
// single-source loop drivers

static constexpr int32_t kDefaultAlphaX16 = 32;  // pull when E >= m / 2

struct RunCfg {
    int loop;
    int direction;
    int32_t alpha_x16;
    int64_t max_iters;
};

static gr_status check_opts(const gr_graph *g, const gr_sssp_opts *o, RunCfg *rc) {
    rc->loop = o ? o->loop : GR_LOOP_AUTO;
    rc->direction = o ? o->direction : GR_DIR_AUTO;
    rc->alpha_x16 = (o && o->alpha_x16 > 0) ? o->alpha_x16 : kDefaultAlphaX16;
    rc->max_iters = (o && o->max_iters > 0) ? o->max_iters : (int64_t)g->dg.n + 1;
    if (rc->loop < GR_LOOP_AUTO || rc->loop > GR_LOOP_PERSISTENT)
        return fail(GR_ERR_INVALID_ARG, "unknown loop mode %d", rc->loop);
    if (rc->direction < GR_DIR_AUTO || rc->direction > GR_DIR_ALTERNATE)
        return fail(GR_ERR_INVALID_ARG, "unknown direction %d", rc->direction);
    if ((rc->direction == GR_DIR_PULL || rc->direction == GR_DIR_ALTERNATE) && !g->pull)
        return fail(GR_ERR_INVALID_ARG, "pull traversal requested but the graph was built with GR_NO_PULL");
    return GR_OK;
}

static bool choose_pull(const gr_graph *g, const RunCfg &rc, int64_t iter, int32_t F, int32_t E) {
    (void)F;
    if (!g->pull) return false;
    switch (rc.direction) {
        case GR_DIR_PUSH: return false;
        case GR_DIR_PULL: return true;
        case GR_DIR_ALTERNATE: return (iter & 1) != 0;
        default: return (int64_t)E * rc.alpha_x16 >= (int64_t)16 * g->dg.m;
    }
}

static gr_status run_host_loop(const gr_graph *g, int32_t src, uint32_t *dist, hipStream_t st, const RunCfg &rc,
                               gr_sssp_stats *stats) {
    DeviceInfo di;
    gr_status s = device_info(g->device, &di);
    if (s != GR_OK) return s;
    unsigned long long *hp = pinned_slot();
    if (!hp) return fail(GR_ERR_OUT_OF_MEMORY, "pinned host buffer");
    const int64_t n = g->dg.n;
    void *ws = nullptr;
    HIP_TRY(hipMallocAsync(&ws, frontier_bytes(n), st));
    Frontier f;
    frontier_carve(f, ws, n);
    gr_sssp_stats local{};
    local.loop = GR_LOOP_HOST;
    gr_status status = GR_OK;
    hipError_t e = launch_init(g->dg, dist, src, f, st);
    const int32_t dsrc = g->h_ro[src + 1] - g->h_ro[src];
    int32_t F = dsrc > 0 ? 1 : 0, E = dsrc;
    int parity = 0;
    int64_t iter = 0;
    while (e == hipSuccess && F > 0) {
        if (iter >= rc.max_iters) {
            status = fail(GR_ERR_ITER_LIMIT, "iteration cap %lld reached", (long long)rc.max_iters);
            break;
        }
        const bool pull = choose_pull(g, rc, iter, F, E);
        local.frontier_sum += F;
        local.frontier_max = std::max(local.frontier_max, F);
        if (pull) {
            e = launch_pull(g->dg, dist, f, parity, st);
            local.pull_iterations++;
            local.arcs_pulled += g->dg.m;
        } else {
            e = launch_push(g->dg, dist, f, parity, F, E, di.num_cu, st);
            local.edges_pushed += E;
        }
        if (e == hipSuccess) e = launch_filter(g->dg, f, parity, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hp, f.ctl + (parity ^ 1), 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        const unsigned long long c = *hp;
        F = (int32_t)(c & 0xFFFFFFFFull);
        E = (int32_t)(c >> 32);
        parity ^= 1;
        ++iter;
    }
    local.iterations = (int32_t)iter;
    hipError_t e2 = hipFreeAsync(ws, st);
    if (e != hipSuccess) return hip_fail(e, "sssp host loop");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    if (stats) *stats = local;
    return status;
}

extern "C" gr_status gr_sssp_ex(const gr_graph *g, int32_t src, void *dist_out, void *stream,
                                const gr_sssp_opts *opts, gr_sssp_stats *stats) {
    if (!g) return fail(GR_ERR_INVALID_ARG, "graph is NULL");
    if (!dist_out) return fail(GR_ERR_INVALID_ARG, "dist_out is NULL");
    if (src < 0 || src >= g->dg.n) return fail(GR_ERR_SOURCE_RANGE, "src = %d outside [0, %d)", src, g->dg.n);
    RunCfg rc;
    gr_status s = check_opts(g, opts, &rc);
    if (s != GR_OK) return s;
    return run_host_loop(g, src, static_cast<uint32_t *>(dist_out), static_cast<hipStream_t>(stream), rc, stats);
}

extern "C" gr_status gr_sssp(const gr_graph *g, int32_t src, void *dist_out, void *stream) {
    return gr_sssp_ex(g, src, dist_out, stream, nullptr, nullptr);
}
