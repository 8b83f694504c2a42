/*
 * CPU ORACLE FOR SINGLE-SOURCE SHORTEST PATHS -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the correctness reference for the GPU path.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or constant generator with the GPU library.
 *
 * What is computed (the definition the paper's SSSP reaches, Section IV-D,
 * Listing 4): for a directed graph in CSR form (Listing 1), weights w >= 0 of
 * type T (uint32 or IEEE binary32) and a source s,
 *     dist[v] = min over paths s = v0 -> v1 -> ... -> vk = v of
 *               ((0 (+) w1) (+) w2) ... (+) wk
 * with dist[s] = 0 and dist[v] = INF when no path exists.  (+) is uint32
 * addition saturating at INF_U32 = 0xFFFFFFFF, or binary32 addition rounded
 * to nearest-even; binary32 INF is FLT_MAX, the initial value of Listing 4.
 * A fold that reaches or passes INF is reported as INF.
 *
 * Functions:
 *   oracle_dijkstra  -- textbook binary-heap Dijkstra with lazy deletion
 *                       (Cormen et al., cited by Listing 3's caption).
 *   oracle_bsp       -- the paper's bulk-synchronous push loop, run
 *                       sequentially in the order of Listings 3 and 4:
 *                       frontier {s}; each round expands every active vertex,
 *                       relaxes each out-edge with a min that returns the old
 *                       value, and appends the destination when the new value
 *                       is strictly smaller; stops when the frontier is empty.
 *                       Also counts rounds, relaxations and frontier sizes.
 *   oracle_certify   -- O(n + m) certificate that a distance vector equals the
 *                       definition above (see its comment).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared oracle.c -o liboracle.so
 * (no -ffast-math: binary32 additions must round to nearest-even).
 */
#include <float.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define INF_U32 0xFFFFFFFFu

/* ---- the (+) operation, one place per type ---------------------------- */

static inline uint32_t add_u32(uint32_t d, uint32_t w) {
    uint64_t s = (uint64_t)d + (uint64_t)w;
    return s >= (uint64_t)INF_U32 ? INF_U32 : (uint32_t)s;
}

static inline float add_f32(float d, float w) {
    float s = d + w; /* binary32 add (SSE addss), round-to-nearest-even */
    return s >= FLT_MAX ? FLT_MAX : s;
}

static inline float bits_to_f(uint32_t b) {
    float f;
    memcpy(&f, &b, 4);
    return f;
}

static inline uint32_t f_to_bits(float f) {
    uint32_t b;
    memcpy(&b, &f, 4);
    return b;
}

/* ---- binary min-heap of (key, vertex), lexicographic ------------------ */

typedef struct {
    double key; /* holds a uint32 or a binary32 value exactly */
    int32_t v;
} item;

typedef struct {
    item *a;
    int64_t size, cap;
} heap;

static int heap_less(const item *x, const item *y) {
    return x->key < y->key || (x->key == y->key && x->v < y->v);
}

static int heap_push(heap *h, double key, int32_t v) {
    if (h->size == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        item *na = (item *)realloc(h->a, (size_t)nc * sizeof(item));
        if (!na) return -1;
        h->a = na;
        h->cap = nc;
    }
    int64_t i = h->size++;
    h->a[i].key = key;
    h->a[i].v = v;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!heap_less(&h->a[i], &h->a[p])) break;
        item t = h->a[i]; h->a[i] = h->a[p]; h->a[p] = t;
        i = p;
    }
    return 0;
}

static item heap_pop(heap *h) {
    item top = h->a[0];
    h->a[0] = h->a[--h->size];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < h->size && heap_less(&h->a[l], &h->a[s])) s = l;
        if (r < h->size && heap_less(&h->a[r], &h->a[s])) s = r;
        if (s == i) break;
        item t = h->a[i]; h->a[i] = h->a[s]; h->a[s] = t;
        i = s;
    }
    return top;
}

/*
 * Dijkstra.  wtype 0: uint32 weights and distances; 1: binary32 (bits in w
 * and dist_out).  Returns 0, or -1 on allocation failure / bad source.
 */
int oracle_dijkstra(int32_t n, const int32_t *ro, const int32_t *col, const uint32_t *w, int wtype,
                    int32_t src, uint32_t *dist_out) {
    if (src < 0 || src >= n) return -1;
    heap h = {0, 0, 0};
    if (wtype == 0) {
        for (int32_t v = 0; v < n; ++v) dist_out[v] = INF_U32;
        dist_out[src] = 0;
        if (heap_push(&h, 0.0, src)) return -1;
        while (h.size > 0) {
            item it = heap_pop(&h);
            uint32_t d = (uint32_t)it.key;
            int32_t u = it.v;
            if (d > dist_out[u]) continue; /* stale entry */
            for (int32_t e = ro[u]; e < ro[u + 1]; ++e) {
                int32_t v = col[e];
                uint32_t nd = add_u32(d, w[e]);
                if (nd < dist_out[v]) {
                    dist_out[v] = nd;
                    if (heap_push(&h, (double)nd, v)) { free(h.a); return -1; }
                }
            }
        }
    } else {
        float *dist = (float *)malloc((size_t)n * sizeof(float));
        if (!dist) return -1;
        for (int32_t v = 0; v < n; ++v) dist[v] = FLT_MAX;
        dist[src] = 0.0f;
        if (heap_push(&h, 0.0, src)) { free(dist); return -1; }
        while (h.size > 0) {
            item it = heap_pop(&h);
            float d = (float)it.key;
            int32_t u = it.v;
            if (d > dist[u]) continue;
            for (int32_t e = ro[u]; e < ro[u + 1]; ++e) {
                int32_t v = col[e];
                float nd = add_f32(d, bits_to_f(w[e]));
                if (nd < dist[v]) {
                    dist[v] = nd;
                    if (heap_push(&h, (double)nd, v)) { free(h.a); free(dist); return -1; }
                }
            }
        }
        for (int32_t v = 0; v < n; ++v) dist_out[v] = f_to_bits(dist[v]);
        free(dist);
    }
    free(h.a);
    return 0;
}

/*
 * The paper's BSP push loop, executed sequentially.  stats (may be NULL)
 * receives {rounds, relaxations, sum of frontier sizes, max frontier size}.
 * Duplicates are kept in the output frontier, as Listing 3 appends under a
 * mutex without deduplication.  Returns 0, -1 on failure, -2 if the round
 * count exceeds max_rounds.
 */
int oracle_bsp(int32_t n, const int32_t *ro, const int32_t *col, const uint32_t *w, int wtype, int32_t src,
               int64_t max_rounds, uint32_t *dist_out, int64_t *stats) {
    if (src < 0 || src >= n) return -1;
    int64_t fcap = 1024, fn = 0, gcap = 1024, gn = 0;
    int32_t *f = (int32_t *)malloc((size_t)fcap * sizeof(int32_t));
    int32_t *g = (int32_t *)malloc((size_t)gcap * sizeof(int32_t));
    float *df = NULL;
    if (!f || !g) { free(f); free(g); return -1; }
    if (wtype == 0) {
        for (int32_t v = 0; v < n; ++v) dist_out[v] = INF_U32;
        dist_out[src] = 0;
    } else {
        df = (float *)malloc((size_t)n * sizeof(float));
        if (!df) { free(f); free(g); return -1; }
        for (int32_t v = 0; v < n; ++v) df[v] = FLT_MAX;
        df[src] = 0.0f;
    }
    f[fn++] = src;
    int64_t rounds = 0, relax = 0, fsum = 0, fmax = 0;
    int rc = 0;
    while (fn != 0) {
        if (rounds >= max_rounds) { rc = -2; break; }
        ++rounds;
        fsum += fn;
        if (fn > fmax) fmax = fn;
        gn = 0;
        for (int64_t i = 0; i < fn; ++i) {
            int32_t u = f[i];
            for (int32_t e = ro[u]; e < ro[u + 1]; ++e) {
                int32_t v = col[e];
                int better;
                ++relax;
                if (wtype == 0) {
                    uint32_t nd = add_u32(dist_out[u], w[e]);
                    uint32_t old = dist_out[v];
                    if (nd < old) dist_out[v] = nd; /* atomic::min, returns old */
                    better = nd < old;
                } else {
                    float nd = add_f32(df[u], bits_to_f(w[e]));
                    float old = df[v];
                    if (nd < old) df[v] = nd;
                    better = nd < old;
                }
                if (better) {
                    if (gn == gcap) {
                        int32_t *ng = (int32_t *)realloc(g, (size_t)(2 * gcap) * sizeof(int32_t));
                        if (!ng) { rc = -1; goto done; }
                        g = ng;
                        gcap *= 2;
                    }
                    g[gn++] = v;
                }
            }
        }
        { int32_t *t = f; f = g; g = t; int64_t tc = fcap; fcap = gcap; gcap = tc; fn = gn; }
    }
done:
    if (wtype != 0) {
        for (int32_t v = 0; v < n; ++v) dist_out[v] = f_to_bits(df[v]);
        free(df);
    }
    if (stats) {
        stats[0] = rounds;
        stats[1] = relax;
        stats[2] = fsum;
        stats[3] = fmax;
    }
    free(f);
    free(g);
    return rc;
}

/*
 * Certificate.  dist equals the definition iff
 *   (0) every value is INF or a valid distance (binary32: finite, >= +0,
 *       not -0; uint32: any value),
 *   (1) dist[s] = 0,
 *   (2) for every arc u -> v with dist[u] != INF: dist[v] <= dist[u] (+) w,
 *   (3) every v with dist[v] != INF is reached from s along "tight" arcs
 *       (dist[u] != INF and dist[u] (+) w == dist[v]).
 * (3) makes each finite dist[v] the fold of a real path; (2) bounds it by the
 * fold of every path (induction along the path, (+) being monotone in its
 * left operand).  Returns 0 when valid, else the number of the first failed
 * condition (10 for (0)), and writes an offending vertex to *bad (if not NULL).
 */
int oracle_certify(int32_t n, const int32_t *ro, const int32_t *col, const uint32_t *w, int wtype, int32_t src,
                   const uint32_t *dist, int32_t *bad) {
    const uint32_t INF = wtype == 0 ? INF_U32 : f_to_bits(FLT_MAX);
    if (bad) *bad = -1;
    if (src < 0 || src >= n) return 1;
    if (wtype != 0) {
        for (int32_t v = 0; v < n; ++v) {
            float x = bits_to_f(dist[v]);
            if (dist[v] & 0x80000000u || !(x <= FLT_MAX)) { if (bad) *bad = v; return 10; }
        }
    }
    if (dist[src] != 0) { if (bad) *bad = src; return 1; }
    for (int32_t u = 0; u < n; ++u) {
        if (dist[u] == INF) continue;
        for (int32_t e = ro[u]; e < ro[u + 1]; ++e) {
            int32_t v = col[e];
            int ok;
            if (wtype == 0) ok = dist[v] <= add_u32(dist[u], w[e]);
            else ok = bits_to_f(dist[v]) <= add_f32(bits_to_f(dist[u]), bits_to_f(w[e]));
            if (!ok) { if (bad) *bad = v; return 2; }
        }
    }
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    int32_t *q = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!seen || !q) { free(seen); free(q); return -1; }
    int64_t qh = 0, qt = 0;
    seen[src] = 1;
    q[qt++] = src;
    while (qh < qt) {
        int32_t u = q[qh++];
        for (int32_t e = ro[u]; e < ro[u + 1]; ++e) {
            int32_t v = col[e];
            if (seen[v] || dist[v] == INF) continue;
            int tight;
            if (wtype == 0) tight = add_u32(dist[u], w[e]) == dist[v];
            else tight = add_f32(bits_to_f(dist[u]), bits_to_f(w[e])) == bits_to_f(dist[v]);
            if (tight) {
                seen[v] = 1;
                q[qt++] = v;
            }
        }
    }
    int rc = 0;
    for (int32_t v = 0; v < n; ++v)
        if (dist[v] != INF && !seen[v]) { if (bad) *bad = v; rc = 3; break; }
    free(seen);
    free(q);
    return rc;
}

/* Breadth-first search from src (Section III-C names BFS as the other vertex
 * program on the same operators): depth[v] = fewest arcs on a path src -> v,
 * 0xFFFFFFFF when v is unreachable.  Textbook FIFO-queue BFS; arc weights are
 * not read.  Returns 0, or -1 on allocation failure. */
int oracle_bfs(int32_t n, const int32_t *ro, const int32_t *col, int32_t src, uint32_t *depth) {
    for (int32_t v = 0; v < n; ++v) depth[v] = INF_U32;
    if (n == 0) return 0;
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!q) return -1;
    int32_t head = 0, tail = 0;
    depth[src] = 0;
    q[tail++] = src;
    while (head < tail) {
        const int32_t u = q[head++];
        for (int32_t e = ro[u]; e < ro[u + 1]; ++e) {
            const int32_t v = col[e];
            if (depth[v] == INF_U32) {
                depth[v] = depth[u] + 1u;
                q[tail++] = v;
            }
        }
    }
    free(q);
    return 0;
}
