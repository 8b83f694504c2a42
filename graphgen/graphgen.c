/*
 * Seeded synthetic graph generators.  Shared by the CPU oracle's tests and by
 * the GPU path's tests and benchmark: this file holds no shortest-path
 * arithmetic, only input construction.
 *
 * Random numbers come from a counter-based generator built on the SplitMix64
 * output function (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014):
 *     sm64(x): z = x + 0x9E3779B97F4A7C15;
 *              z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9;
 *              z = (z ^ (z >> 27)) * 0x94D049BB133111EB;
 *              return z ^ (z >> 31);
 *     h(seed, a, b) = sm64(sm64(sm64(seed) ^ a) ^ b)
 * Every draw is a pure function of (seed, key), so the output does not depend
 * on thread count or scheduling.
 *
 * Bounded integers use Lemire's multiply-shift range reduction
 * ("Fast random integer generation in an interval", TOMACS 2019) on the high
 * 32 bits of a hash.  fp32 weights in (0,1] are ((h >> 40) + 1) * 2^-24,
 * which is exact in binary32 and never subnormal.
 *
 * CSR convention (the paper's csr_t, Listing 1): int32 row_offsets[n+1],
 * int32 column_indices[m], 32-bit weight bits[m] (uint32 value or IEEE
 * binary32 bits).  Rows are sorted by destination, without duplicates or
 * self-loops.
 *
 * Built with: gcc -O2 -fopenmp -fPIC -shared graphgen.c -o libgraphgen.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint64_t sm64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t gg_hash(uint64_t seed, uint64_t a, uint64_t b) {
    return sm64(sm64(sm64(seed) ^ a) ^ b);
}

/* uniform integer in [lo, hi] from the high 32 bits of h (Lemire). */
static inline uint32_t bounded_u32(uint64_t h, uint32_t lo, uint32_t hi) {
    uint64_t span = (uint64_t)hi - (uint64_t)lo + 1ull; /* 1 .. 2^32 */
    uint64_t x = h >> 32;
    return lo + (uint32_t)((x * span) >> 32);
}

static inline uint32_t f32_bits_unit(uint64_t h) {
    /* ((h >> 40) + 1) * 2^-24, in (0, 1], exact. */
    uint32_t k = (uint32_t)(h >> 40) + 1u; /* 1 .. 2^24 */
    float f = (float)k * (1.0f / 16777216.0f);
    uint32_t bits;
    memcpy(&bits, &f, 4);
    return bits;
}

/* wtype: 0 = uint32 in [wlo, whi]; 1 = fp32 in (0, 1]. */
uint32_t gg_weight(uint64_t wseed, uint64_t a, uint64_t b, int wtype, uint32_t wlo, uint32_t whi) {
    uint64_t h = gg_hash(wseed, a, b);
    return wtype == 1 ? f32_bits_unit(h) : bounded_u32(h, wlo, whi);
}

typedef struct {
    int32_t n;
    int64_t m;
    int32_t *ro;
    int32_t *col;
    uint32_t *w;
} gg_csr;

void gg_free(gg_csr *g) {
    if (!g) return;
    free(g->ro);
    free(g->col);
    free(g->w);
    g->ro = NULL;
    g->col = NULL;
    g->w = NULL;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Builds a CSR from a list of arcs (src[i] -> dst[i]), dropping self-loops and
 * duplicates, sorting each row.  If symmetric != 0 every arc is also inserted
 * reversed.  Weights: symmetric graphs draw one weight per unordered pair
 * h(wseed, min, max); directed graphs one per arc h(wseed, u, v).
 */
static int build_csr(int32_t n, int64_t na, const int32_t *src, const int32_t *dst, int symmetric,
                     uint64_t wseed, int wtype, uint32_t wlo, uint32_t whi, gg_csr *out) {
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < na; ++i) {
        int32_t u = src[i], v = dst[i];
        if (u == v) continue;
        __atomic_fetch_add(&cnt[u + 1], 1, __ATOMIC_RELAXED);
        if (symmetric) __atomic_fetch_add(&cnt[v + 1], 1, __ATOMIC_RELAXED);
    }
    for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int64_t tot = cnt[n];
    int32_t *tmp = (int32_t *)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(int32_t));
    int64_t *pos = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    if (!tmp || !pos) {
        free(cnt); free(tmp); free(pos);
        return -1;
    }
    memcpy(pos, cnt, (size_t)(n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < na; ++i) {
        int32_t u = src[i], v = dst[i];
        if (u == v) continue;
        int64_t p = __atomic_fetch_add(&pos[u], 1, __ATOMIC_RELAXED);
        tmp[p] = v;
        if (symmetric) {
            int64_t q = __atomic_fetch_add(&pos[v], 1, __ATOMIC_RELAXED);
            tmp[q] = u;
        }
    }
    free(pos);
    /* sort + dedupe each row in place; record the new length */
    int32_t *len = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!len) {
        free(cnt); free(tmp);
        return -1;
    }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t u = 0; u < n; ++u) {
        int32_t *r = tmp + cnt[u];
        int64_t d = cnt[u + 1] - cnt[u];
        if (d > 1) qsort(r, (size_t)d, sizeof(int32_t), cmp_i32);
        int64_t k = 0;
        for (int64_t j = 0; j < d; ++j)
            if (k == 0 || r[j] != r[k - 1]) r[k++] = r[j];
        len[u] = (int32_t)k;
    }
    int64_t m = 0;
    for (int32_t u = 0; u < n; ++u) m += len[u];
    if (m >= 2147483647ll) {
        free(cnt); free(tmp); free(len);
        return -2;
    }
    out->n = n;
    out->m = m;
    out->ro = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
    out->col = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    out->w = (uint32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint32_t));
    if (!out->ro || !out->col || !out->w) {
        gg_free(out);
        free(cnt); free(tmp); free(len);
        return -1;
    }
    out->ro[0] = 0;
    for (int32_t u = 0; u < n; ++u) out->ro[u + 1] = out->ro[u] + len[u];
#pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t u = 0; u < n; ++u) {
        const int32_t *r = tmp + cnt[u];
        int32_t base = out->ro[u];
        for (int32_t j = 0; j < len[u]; ++j) {
            int32_t v = r[j];
            out->col[base + j] = v;
            uint64_t a = (uint64_t)(uint32_t)u, b = (uint64_t)(uint32_t)v;
            if (symmetric && b < a) { uint64_t t = a; a = b; b = t; }
            out->w[base + j] = gg_weight(wseed, a, b, wtype, wlo, whi);
        }
    }
    free(cnt);
    free(tmp);
    free(len);
    return 0;
}

/*
 * side x side 4-neighbour grid (vertex id = r*side + c), one weight per
 * directed arc, plus `shortcuts` undirected long-range edges with endpoints
 * uniform over all vertices drawn from sseed (road-like variant).
 */
int gg_grid(int32_t side, uint64_t wseed, int wtype, uint32_t wlo, uint32_t whi,
            int64_t shortcuts, uint64_t sseed, gg_csr *out) {
    memset(out, 0, sizeof(*out));
    if (side <= 0 || (int64_t)side * side >= 2147483647ll) return -3;
    int32_t n = side * side;
    int64_t na = 2ll * ((int64_t)side * (side - 1)) * 2 + 2 * shortcuts;
    int32_t *src = (int32_t *)malloc((size_t)(na > 0 ? na : 1) * sizeof(int32_t));
    int32_t *dst = (int32_t *)malloc((size_t)(na > 0 ? na : 1) * sizeof(int32_t));
    if (!src || !dst) {
        free(src); free(dst);
        return -1;
    }
    int64_t k = 0;
    for (int32_t r = 0; r < side; ++r)
        for (int32_t c = 0; c < side; ++c) {
            int32_t u = r * side + c;
            if (r > 0) { src[k] = u; dst[k] = u - side; ++k; }
            if (c > 0) { src[k] = u; dst[k] = u - 1; ++k; }
            if (c + 1 < side) { src[k] = u; dst[k] = u + 1; ++k; }
            if (r + 1 < side) { src[k] = u; dst[k] = u + side; ++k; }
        }
    for (int64_t i = 0; i < shortcuts; ++i) {
        uint64_t h = gg_hash(sseed, (uint64_t)i, 0);
        uint64_t g = gg_hash(sseed, (uint64_t)i, 1);
        int32_t a = (int32_t)bounded_u32(h, 0, (uint32_t)(n - 1));
        int32_t b = (int32_t)bounded_u32(g, 0, (uint32_t)(n - 1));
        src[k] = a; dst[k] = b; ++k;
        src[k] = b; dst[k] = a; ++k;
    }
    int rc = build_csr(n, k, src, dst, 0, wseed, wtype, wlo, whi, out);
    free(src);
    free(dst);
    return rc;
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): edge_factor * 2^scale
 * tuples, each choosing one of four quadrants per level with probabilities
 * (a, b, c, 1-a-b-c) from 32-bit draws; vertex ids relabelled by a seeded
 * Fisher-Yates permutation; symmetrised, self-loops and duplicates dropped;
 * one weight per unordered pair.
 */
int gg_rmat(int scale, int edge_factor, double a, double b, double c, uint64_t gseed, uint64_t pseed,
            uint64_t wseed, int wtype, uint32_t wlo, uint32_t whi, gg_csr *out) {
    memset(out, 0, sizeof(*out));
    if (scale < 1 || scale > 30 || edge_factor < 1) return -3;
    int32_t n = (int32_t)1 << scale;
    int64_t ne = (int64_t)edge_factor * n;
    const double two32 = 4294967296.0;
    uint64_t ta = (uint64_t)(a * two32), tab = (uint64_t)((a + b) * two32),
             tabc = (uint64_t)((a + b + c) * two32);
    int32_t *src = (int32_t *)malloc((size_t)ne * sizeof(int32_t));
    int32_t *dst = (int32_t *)malloc((size_t)ne * sizeof(int32_t));
    int32_t *perm = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!src || !dst || !perm) {
        free(src); free(dst); free(perm);
        return -1;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ne; ++i) {
        uint32_t u = 0, v = 0;
        uint64_t h = 0;
        for (int l = 0; l < scale; ++l) {
            if ((l & 1) == 0) h = gg_hash(gseed, (uint64_t)i, (uint64_t)(l >> 1));
            uint64_t q = (l & 1) ? (h >> 32) : (h & 0xFFFFFFFFull);
            uint32_t bu, bv;
            if (q < ta) { bu = 0; bv = 0; }
            else if (q < tab) { bu = 0; bv = 1; }
            else if (q < tabc) { bu = 1; bv = 0; }
            else { bu = 1; bv = 1; }
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        src[i] = (int32_t)u;
        dst[i] = (int32_t)v;
    }
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    for (int32_t i = n - 1; i > 0; --i) {
        uint32_t j = bounded_u32(gg_hash(pseed, (uint64_t)i, 0), 0, (uint32_t)i);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ne; ++i) {
        src[i] = perm[src[i]];
        dst[i] = perm[dst[i]];
    }
    free(perm);
    int rc = build_csr(n, ne, src, dst, 1, wseed, wtype, wlo, whi, out);
    free(src);
    free(dst);
    return rc;
}

/* Directed random graph: na arcs with uniform endpoints (tests only). */
int gg_uniform(int32_t n, int64_t na, uint64_t gseed, uint64_t wseed, int wtype, uint32_t wlo, uint32_t whi,
               int symmetric, gg_csr *out) {
    memset(out, 0, sizeof(*out));
    if (n <= 0 || na < 0) return -3;
    int32_t *src = (int32_t *)malloc((size_t)(na > 0 ? na : 1) * sizeof(int32_t));
    int32_t *dst = (int32_t *)malloc((size_t)(na > 0 ? na : 1) * sizeof(int32_t));
    if (!src || !dst) {
        free(src); free(dst);
        return -1;
    }
    for (int64_t i = 0; i < na; ++i) {
        src[i] = (int32_t)bounded_u32(gg_hash(gseed, (uint64_t)i, 0), 0, (uint32_t)(n - 1));
        dst[i] = (int32_t)bounded_u32(gg_hash(gseed, (uint64_t)i, 1), 0, (uint32_t)(n - 1));
    }
    int rc = build_csr(n, na, src, dst, symmetric, wseed, wtype, wlo, whi, out);
    free(src);
    free(dst);
    return rc;
}

/* k seeded sources, uniform over vertices with out-degree > 0 (rejection). */
int gg_pick_sources(int32_t n, const int32_t *ro, uint64_t seed, int32_t k, int32_t *out) {
    int64_t nz = 0;
    for (int32_t v = 0; v < n; ++v) nz += ro[v + 1] > ro[v];
    if (nz == 0) return -4;
    uint64_t ctr = 0;
    for (int32_t i = 0; i < k; ++i) {
        for (;;) {
            uint32_t v = bounded_u32(gg_hash(seed, ctr++, 0), 0, (uint32_t)(n - 1));
            if (ro[v + 1] > ro[v]) { out[i] = (int32_t)v; break; }
        }
    }
    return 0;
}

int gg_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
