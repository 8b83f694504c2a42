/*
 * gr.h -- C ABI of a frontier-driven single-source shortest path (SSSP)
 * library for AMD Instinct MI355X (gfx950).
 *
 * The operation is the paper's parallel native-graph SSSP (Osama, Porumbescu,
 * Owens, "Essentials of Parallel Graph Analytics", Section IV-D, Listing 4):
 * starting from dist = INF, dist[src] = 0 and the frontier {src}, repeat
 *   advance  -- relax every out-edge (u -> v, w) of the active frontier:
 *               new = dist[u] (+) w; old = atomic-min(dist[v], new);
 *               v joins the next frontier iff new < old (Listing 3/4),
 *   filter   -- deduplicate and compact the next frontier,
 *   converge -- stop when the frontier is empty (Section III, item 4),
 * over a graph stored as a CSR matrix (Section IV-A, Listing 1), with a
 * transposed (CSC) copy for pull traversal (Section III-C).
 *
 * The result is unique and independent of schedule: for every vertex v,
 *   dist[v] = min over paths src = v0 -> ... -> vk = v of the left fold
 *             ((0 (+) w1) (+) w2) ... (+) wk,
 * dist[src] = 0, and INF when no path exists (or when every fold reaches INF).
 * (+) is uint32 addition saturating at GR_DIST_INF_U32, or IEEE-754 binary32
 * addition rounded to nearest-even.  Distances are therefore bit-exact for
 * both weight types whatever the traversal order.
 *
 * Conventions shared by every call
 *  - Every call returns gr_status; argument errors are detected on the host
 *    before anything is enqueued, and the text of the last error of the
 *    calling thread is available from gr_last_error().
 *  - "stream" is a hipStream_t (NULL = the null stream), passed as void* so
 *    that this header needs no HIP headers.
 *  - Graph ids, vertex ids, offsets and edge counts are int32: n < 2^31 and
 *    m < 2^31 (the paper's csr_t uses int).
 *  - Distances are 32-bit: uint32 values, or binary32 bit patterns.  INF is
 *    GR_DIST_INF_U32, or FLT_MAX (GR_DIST_INF_F32_BITS), the initial value of
 *    Listing 4.
 */
#ifndef GR_H_
#define GR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GR_OK = 0,
    GR_ERR_INVALID_ARG = 1,   /* malformed CSR, bad weight, bad pointer/size/flag */
    GR_ERR_SOURCE_RANGE = 2,  /* a source id outside [0, n) */
    GR_ERR_OUT_OF_MEMORY = 3, /* device or pinned host allocation failed */
    GR_ERR_NO_CAPACITY = 4,   /* a query can never fit the server's memory budget */
    GR_ERR_NOT_READY = 5,     /* a served query has not completed yet */
    GR_ERR_ITER_LIMIT = 6,    /* the iteration cap was reached (a bug for w >= 0) */
    GR_ERR_HIP = 7,           /* a HIP runtime call failed; see gr_last_error() */
    GR_ERR_UNKNOWN_TICKET = 8 /* poll of a ticket the server never issued */
} gr_status;

typedef enum { GR_W_U32 = 0, GR_W_F32 = 1 } gr_weight_type;

#define GR_DIST_INF_U32 0xFFFFFFFFu
#define GR_DIST_INF_F32_BITS 0x7F7FFFFFu

/* gr_graph_create_csr flags */
#define GR_INPUT_DEVICE 0x1u     /* the three arrays are device pointers */
#define GR_NO_PULL 0x2u          /* never build the transposed copy: push traversal only */
#define GR_NO_PARTITION 0x4u     /* never build the partitioned push layout */
#define GR_FORCE_PARTITION 0x8u  /* always build it (default: only for large graphs whose
                                    arcs mostly join distant vertex ids) */

typedef struct gr_graph gr_graph;
typedef struct gr_server gr_server;

/*
 * Builds a device-resident graph from a CSR matrix (Section IV-A, Listing 1:
 * row_offsets, column_indices, values; rows = cols = n).
 *   n            number of vertices, 1 <= n < 2^31
 *   m            number of arcs, 0 <= m < 2^31
 *   row_offsets  int32[n+1], row_offsets[0] = 0, non-decreasing, [n] = m
 *   col_indices  int32[m], each in [0, n); arc u -> col_indices[e] for
 *                e in [row_offsets[u], row_offsets[u+1])
 *   weights      m values of type wt: uint32 (any value), or binary32 that
 *                must be finite and >= 0 (-0.0 is stored as +0.0)
 *   flags        GR_INPUT_DEVICE, GR_NO_PULL, GR_NO_PARTITION, GR_FORCE_PARTITION
 *   stream       stream for the upload and preprocessing
 * Self-loops and parallel arcs are accepted.  The arrays are copied; the
 * caller keeps ownership.  Host arrays are validated on the host; device
 * arrays (GR_INPUT_DEVICE) are validated by a device pass.  Unless
 * GR_NO_PULL is given, a transposed copy (CSC) is built for pull traversal,
 * and dropped again when the arcs and weights turn out to be symmetric (the
 * CSR then serves both directions).  Returns GR_ERR_INVALID_ARG for a
 * malformed matrix.  A second, partitioned copy of the arcs may be built for
 * push traversal: arcs grouped by destination into 8 vertex ranges, so that
 * the blocks working on one range touch one eighth of the distance array
 * (see GR_NO_PARTITION / GR_FORCE_PARTITION).  The call returns after the
 * graph is ready.
 */
gr_status gr_graph_create_csr(gr_graph **out, int32_t n, int32_t m, const int32_t *row_offsets,
                              const int32_t *col_indices, const void *weights, gr_weight_type wt,
                              uint32_t flags, void *stream);

/* Frees the graph's device memory.  No query on it may still be running. */
gr_status gr_graph_destroy(gr_graph *g);

/* Size, weight type and device footprint of a graph (the dimensions of the
 * csr_t of Section IV-A, Listing 1).  Any output pointer may be NULL.
 * dev_bytes counts every device allocation the graph holds (CSR, transposed
 * copy, partitioned push layout, membership lists). */
gr_status gr_graph_info(const gr_graph *g, int32_t *n, int32_t *m, gr_weight_type *wt, size_t *dev_bytes);

/* Which traversal structures were built (see gr_graph_create_csr).  Any output
 * pointer may be NULL.  has_csc: 1 when a separate transposed copy is stored,
 * 0 when the CSR serves pull too (symmetric) or pull is off.  pull_enabled:
 * 1 unless the graph was built with GR_NO_PULL.  partitions: 8 when the
 * partitioned push layout exists, else 1. */
gr_status gr_graph_layout(const gr_graph *g, int32_t *has_csc, int32_t *pull_enabled, int32_t *partitions);

/*
 * Single-source shortest paths from src (Section IV-D, Listing 4).
 *   dist_out  device memory for n 32-bit values of the graph's weight type;
 *             it is used as the working distance array, so it must not alias
 *             anything else in use.  Contents on return: the unique result.
 * Work is ordered on `stream`.  Depending on the loop schedule the call may
 * wait for the stream while it runs (host-driven loop) or return after
 * enqueueing (device-driven loop); the result is complete once the stream
 * has been synchronised.  Concurrent calls on the same graph are allowed on
 * different streams.  GR_ERR_SOURCE_RANGE if src is outside [0, n).
 */
gr_status gr_sssp(const gr_graph *g, int32_t src, void *dist_out, void *stream);

/*
 * gr_sssp for callers that cannot allocate memory: code that is being
 * captured into a HIP graph, tight serving loops, and harnesses that forbid
 * hipMalloc.  Same arguments and result as gr_sssp; it calls no hipMalloc,
 * hipFree, pool allocation or pinned-memory allocation, and creates no event.
 *   - Workspace: a fixed array of 96 MiB (GR_NOALLOC_SCRATCH_BYTES) that the
 *     library holds on every GPU it runs on until the process ends.  A query
 *     needs about 14 bytes per vertex (18 when the graph's default uses the
 *     bound relaxation filter) plus 2 MiB (the plain CSR layout, one
 *     frontier queue); a graph whose workspace exceeds the array returns
 *     GR_ERR_NO_CAPACITY before anything is enqueued.  Graphs of up to about
 *     five to seven million vertices fit.
 *   - Schedule: the queued (device-driven) loop over the plain CSR layout,
 *     without a near-far split; the direction, filter and relaxation-filter
 *     defaults are the graph's.  The call waits for `stream` once per chunk
 *     of launches and returns when the query has finished.
 *   - The current device must be the graph's device (GR_ERR_INVALID_ARG).
 *   - Every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents (each call clears what it reads first).  Calls that
 *     overlap on one GPU -- from other threads or on other streams -- race
 *     and give wrong results; serialise them.
 */
#define GR_NOALLOC_SCRATCH_BYTES (96u << 20)
gr_status gr_sssp_noalloc(const gr_graph *g, int32_t src, void *dist_out, void *stream);

/* Loop schedule of gr_sssp_ex (Section III-A: execution policies). */
typedef enum {
    GR_LOOP_AUTO = 0,       /* the library's choice: gr_graph_tune's if run, else the
                               single-workgroup loop for graphs of maximum out-degree <= 64
                               that fit it (GR_LOOP_LDS), the asynchronous loop for other
                               graphs of maximum out-degree <= 64 and n <= 65,536 (the
                               queued loop when the request needs pull or a near-far
                               split), the host-driven loop for graphs of maximum
                               out-degree > 64 and m >= 2^26, the queued loop otherwise */
    GR_LOOP_HOST = 1,       /* one launch per operator, host reads the frontier size */
    GR_LOOP_PERSISTENT = 2, /* one cooperative launch, device-side grid barrier */
    GR_LOOP_QUEUED = 3,     /* launches enqueued ahead in chunks; each reads the frontier
                               size from device memory; the host checks once per chunk */
    GR_LOOP_ASYNC = 4,      /* asynchronous (Section III-A without the per-advance barrier,
                               III-B frontier as a message queue): one persistent kernel
                               drains a device worklist of improved vertices; no rounds.
                               Push only over the plain CSR (direction PULL / ALTERNATE and
                               an explicit delta are GR_ERR_INVALID_ARG; layout, filter and
                               relax_filter are ignored).  Extra workspace: 16 n bytes.
                               stats: iterations = worklist phases (1 unless the list of
                               4 n entries overflowed), frontier_sum = vertex expansions.
                               The call waits for the stream after each phase.  The
                               environment variable GR_ASYNC_LIST_CAP (entries, >= 1)
                               lowers the list capacity, to test the overflow path. */
    GR_LOOP_LDS = 5         /* single workgroup (Section III-A's loop with a workgroup
                               barrier per round): one launch of one 1024-thread workgroup
                               copies the distances, row offsets and arcs (a 16-bit head and
                               a 16-bit weight each) into LDS and runs every round there.
                               Graphs with 3 n + m <= 39,900 or so (about 156 KiB of LDS;
                               a 75 x 75 grid fits), or, with uint32 weights below 65,536
                               and maximum out-degree D <= 16, (2 + P) n <= 39,900 or so,
                               P the power of two >= D (arcs padded to P slots per vertex:
                               an 81 x 81 grid fits); and, for SSSP, uint32 weights below
                               65,536; else GR_ERR_INVALID_ARG.  Push only (direction
                               PULL / ALTERNATE and an explicit delta are
                               GR_ERR_INVALID_ARG; layout, filter and relax_filter are
                               ignored).  AUTO picks it for every graph that fits
                               (for SSSP, with such weights).  stats: iterations = rounds,
                               frontier_sum = vertex expansions, launches = 1. */
} gr_loop_mode;

/* Traversal direction policy (Section III-C: push vs pull). */
typedef enum {
    GR_DIR_AUTO = 0,      /* switch on frontier size (alpha and beta rules below) */
    GR_DIR_PUSH = 1,      /* push every iteration */
    GR_DIR_PULL = 2,      /* pull every iteration (needs pull enabled) */
    GR_DIR_ALTERNATE = 3  /* push and pull alternately (a test of switching) */
} gr_direction;

/* Arc layout used by push (see gr_graph_create_csr). */
typedef enum {
    GR_LAYOUT_AUTO = 0,        /* partitioned when the graph has it */
    GR_LAYOUT_PLAIN = 1,       /* the CSR as given */
    GR_LAYOUT_PARTITIONED = 2  /* needs the partitioned layout */
} gr_layout;

typedef struct {
    int32_t loop;       /* gr_loop_mode */
    int32_t direction;  /* gr_direction */
    int32_t alpha_x16;  /* GR_DIR_AUTO, after a push round: pull when frontier out-edges *
                           alpha_x16 >= 16 * m; 0 = the graph's default (never, unless
                           gr_graph_tune chose a value) */
    int32_t max_iters;  /* iteration cap; 0 = n + 1 (never reached for w >= 0) */
    int32_t layout;     /* gr_layout */
    int32_t timing;     /* 1: time every operator launch with HIP events (stats *_us fields) */
    int32_t filter;     /* 0 auto, 1 always the per-group flag scan, 2 always the
                           per-partition member-list scan, 3 auto plus small rounds: in
                           the queued loop, a round that improved at most 2^18 vertices
                           hands the next round a list of them instead of a filter pass
                           (graphs of degree <= 64, push only, no near-far split) */
    int32_t barrier_timeout_us; /* device-driven loop: bound on one grid-barrier wait;
                                   0 = 20 s.  Exceeding it ends the query with GR_ERR_HIP. */
    uint32_t delta;     /* near-far split width, in the weight type (a uint32 value, or the
                           bits of a positive finite binary32): improved vertices whose
                           distance is not below the threshold are held back until the
                           frontier runs empty, then the threshold rises to the smallest
                           held-back distance (+) delta.  0 = the graph's default (off
                           unless gr_graph_tune chose one); GR_DELTA_OFF = off.  Needs
                           push: GR_DIR_PULL / GR_DIR_ALTERNATE are GR_ERR_INVALID_ARG. */
    int32_t relax_filter; /* what push compares a candidate distance with before its atomic
                             min: GR_RELAX_* below.  0 = the graph's default (the bound
                             array on graphs of maximum out-degree > 64, unless
                             gr_graph_tune chose otherwise; breadth-first search: dist). */
    int32_t beta;         /* GR_DIR_AUTO, after a pull round: keep pulling while the frontier
                             holds at least n / beta vertices, else push (0 = 24).  Pull ->
                             push and push -> pull (alpha_x16) are Beamer et al.'s rules. */
    int32_t local_hops;   /* small rounds (filter 3 or the graph's default): a block expands
                             the vertices it improved again, with the distance that improved
                             them, for up to local_hops - 1 further hops before handing the
                             rest to the next round (1 = every improvement waits for the next
                             round).  0 = the graph's default (6, unless gr_graph_tune chose
                             another); at most 64. */
} gr_sssp_opts;

/* Relaxation filters of push (gr_sssp_opts.relax_filter).  Either way the
 * result is the same; only the number of atomic operations differs. */
#define GR_RELAX_DIST 1  /* read dist[v]; the atomic min's result is not used */
#define GR_RELAX_BOUND 2 /* read a per-vertex upper bound on dist[v] that push keeps with
                            plain stores of the candidates it sends to the atomic min.
                            The bound stays current in the cache of the die that relaxes
                            v, and the pre-reads stay off the lines that the atomics are
                            updating; faster on skewed graphs, slower on road-like ones.
                            Costs 4 bytes per vertex of query workspace. */

#define GR_DELTA_OFF 0xFFFFFFFFu

typedef struct {
    int32_t iterations;        /* advance/filter rounds executed */
    int32_t pull_iterations;   /* of which pull */
    int64_t edges_pushed;      /* out-edges expanded by push (relaxations) */
    int64_t arcs_pulled;       /* in-arcs scanned by pull */
    int64_t frontier_sum;      /* sum of frontier sizes over the rounds */
    int64_t push_frontier_sum; /* of which in push rounds */
    int32_t frontier_max;
    int32_t loop;              /* the gr_loop_mode that ran */
    int32_t push_launches;
    int32_t layout;            /* the gr_layout that ran */
    double push_us;            /* with opts.timing: summed push / pull / filter launch times */
    double pull_us;
    double filter_us;
    int32_t small_rounds;      /* queued loop: rounds expanded from a candidate list */
    int32_t launches;          /* kernel launches of the loop (queued: including the ones
                                  enqueued past the end, which return at once) */
    int32_t relax_filter;      /* the GR_RELAX_* push ran with */
} gr_sssp_stats;

/* gr_sssp with an explicit schedule; opts and stats may be NULL.  stats are
 * filled when the call returns for the host-driven loop, and after the stream
 * has been synchronised for the device-driven loop. */
gr_status gr_sssp_ex(const gr_graph *g, int32_t src, void *dist_out, void *stream, const gr_sssp_opts *opts,
                     gr_sssp_stats *stats);

/* Schedule chosen by gr_graph_tune (also what GR_*_AUTO resolve to). */
typedef struct {
    int32_t layout;       /* gr_layout that won (PLAIN or PARTITIONED) */
    int32_t loop;         /* gr_loop_mode that won (HOST or PERSISTENT) */
    int32_t dense_ratio;  /* streaming filter when frontier size * dense_ratio >= n */
    int32_t alpha_x16;    /* pull threshold (0 = never pull) */
    double best_ms;       /* median time of one query with that schedule */
    double default_ms;    /* the same before tuning */
    int32_t trials;       /* timed configurations */
    int32_t from_cache;   /* 1 when read from the tuning cache file */
    uint32_t delta;       /* chosen near-far split width (weight-type bits; 0 = off) */
    int32_t small;        /* 1: small rounds (filter 3) in the queued loop */
    int32_t relax_filter; /* GR_RELAX_DIST or GR_RELAX_BOUND */
    int32_t async_blocks; /* blocks of the asynchronous loop (0: the library's default) */
    int32_t local_hops;   /* small rounds' local hops (see gr_sssp_opts) */
} gr_tune_result;

/*
 * Autotuner: times candidate schedules -- push layout, loop driver, filter
 * threshold, pull threshold, near-far split width, small rounds and their local
 * hops, relaxation filter, the asynchronous loop's block count -- with a greedy search (one knob at a time, each
 * candidate timed as the median of `reps` queries from srcs[0..nsrcs)), and
 * keeps the fastest as the graph's AUTO configuration.  Every candidate
 * computes the same distances.  When the environment variable GR_TUNE_CACHE
 * names a file, results are read from / appended to it, keyed by a signature
 * of the graph (n, m, weight type, degree statistics).  out may be NULL.
 * The graph must not be queried concurrently while it is being tuned.
 */
gr_status gr_graph_tune(gr_graph *g, const int32_t *srcs, int32_t nsrcs, int32_t reps, void *stream,
                        gr_tune_result *out);

/*
 * Breadth-first search from src (Section III-C: the same advance / filter
 * operators and convergence loop as SSSP, with every arc counting one hop).
 *   depth_out  device memory for n uint32: the fewest arcs on a path from src,
 *              GR_DIST_INF_U32 for unreachable vertices, 0 at src.  The stored
 *              weights are not read (any weight type).
 * The default direction policy switches to pull when the frontier's out-edges
 * reach m / 14; pull then scans only the in-arcs of vertices without a depth.
 * opts as for gr_sssp_ex, except: delta must be 0 / GR_DELTA_OFF, the
 * persistent loop is GR_ERR_INVALID_ARG, and AUTO runs the single-workgroup
 * loop (push only) on graphs that fit one workgroup's LDS unless pull or
 * alternation is asked for, else the host-driven loop on graphs of maximum
 * out-degree > 64 and the queued loop otherwise.
 */
gr_status gr_bfs(const gr_graph *g, int32_t src, void *depth_out, void *stream);
gr_status gr_bfs_ex(const gr_graph *g, int32_t src, void *depth_out, void *stream, const gr_sssp_opts *opts,
                    gr_sssp_stats *stats);

/* Statistics of gr_sssp_batch_ex and gr_sssp_multi. */
typedef struct {
    int32_t rounds;             /* rounds in which some query's frontier was not empty */
    int32_t replays;            /* replays of the captured chunk of rounds (one host wait each); 0 when
                                   none runs (k = 1, or the single-workgroup loop) */
    int64_t edges_pushed;       /* arcs expanded (a batched arc serves every source active at its tail) */
    int64_t frontier_sum;       /* frontier entries expanded */
    int64_t source_relaxations; /* (arc, query) relaxations: for gr_sssp_batch_ex the (arc, active source)
                                   pairs, for gr_sssp_multi equal to edges_pushed */
} gr_multi_stats;

/*
 * k independent SSSP queries on one graph in one batched computation
 * (Section IV-D, Listing 4 for each source).
 *   srcs      host int32[k], each in [0, n); duplicates allowed
 *   k         1 <= k <= 64
 *   dist_out  device memory, k x n row-major: row i holds the result of srcs[i]
 * Row i is bit-identical to gr_sssp(g, srcs[i], ...).  For k >= 2 the
 * distances are kept vertex-major (the 64 distances of a vertex in one
 * 256-byte row) and every arc of a frontier vertex is read once for all the
 * sources active there, one source per wave lane.  The round loop runs on the
 * device: every launch reads its round from device memory, so 8 rounds
 * (push, filter) are captured once as a HIP graph and replayed; the host waits
 * for the stream once per replay to see whether the frontier is empty, and
 * the call returns when the result is complete.  Workspace, stream-ordered
 * from the device pool and returned before the call ends: 256 bytes per
 * vertex (distances) + 16 (masks) + about 28 (frontier marks and two queues).
 * k = 1 runs gr_sssp's schedule.  A graph whose AUTO loop is the single-
 * workgroup loop (GR_LOOP_LDS) runs that loop for every source instead, one
 * workgroup per source in one launch, with no workspace.  The current device
 * must be the graph's.
 */
gr_status gr_sssp_batch(const gr_graph *g, const int32_t *srcs, int32_t k, void *dist_out, void *stream);
/* gr_sssp_batch with statistics (stats may be NULL). */
gr_status gr_sssp_batch_ex(const gr_graph *g, const int32_t *srcs, int32_t k, void *dist_out, void *stream,
                           gr_multi_stats *stats);

/*
 * k independent single-source queries, each on its own graph -- graphs may
 * repeat and may differ in size and weight type -- advanced together: every
 * round is one push launch and one filter launch over the union of the k
 * frontiers, spread evenly over the blocks by the frontier's arc counts
 * (Section IV-D, Listing 4 for each query, in its own distance array).
 *   graphs      host array of k graph handles, all on the current device
 *   srcs        host int32[k], srcs[i] in [0, n of graphs[i])
 *   k           1 <= k <= 64
 *   dist_out    host array of k device pointers; dist_out[i] receives the n
 *               values (of graphs[i]'s weight type) of query i and is its
 *               working array (the k buffers must not overlap)
 *   stats       optional
 *   iterations  optional host int32[k]: rounds in which query i's frontier
 *               was not empty
 * dist_out[i] is bit-identical to gr_sssp(graphs[i], srcs[i], ...).  The
 * arcs of the k graphs must total less than 2^31 (GR_ERR_INVALID_ARG).  The
 * round loop runs on the device from one captured HIP graph of 8 rounds; the
 * call waits for the stream once per replay and returns when every query is
 * done.  Workspace: 26 bytes per vertex summed over the queries (two union
 * queues) + 2 bytes per vertex of each query (frontier marks), stream-ordered
 * from the device pool and returned before the call ends.  When every
 * graph's AUTO loop is the single-workgroup loop (GR_LOOP_LDS), and all fit
 * one arc layout (row offsets, or arcs padded to the same slot count), each
 * query runs that loop in a workgroup of its own, all in one launch, with no
 * workspace (stats->replays = 0).
 */
gr_status gr_sssp_multi(const gr_graph *const *graphs, const int32_t *srcs, int32_t k, void *const *dist_out,
                        void *stream, gr_multi_stats *stats, int32_t *iterations);

/* ---- serving ----------------------------------------------------------- */

typedef struct {
    int32_t max_batch;      /* queries one executor runs together, 1..64 (0 = 64) */
    int32_t num_streams;    /* executors, each with its own stream, 1..8 (0 = 3) */
    int32_t max_wait_us;    /* unused: queries join a running executor at its next chunk of
                               rounds, so none waits for company (must be >= 0) */
    int32_t local_hops;     /* push blocks expand the vertices they improved on graphs of degree
                               <= 8 for up to local_hops - 1 further hops within a round (as
                               gr_sssp_opts.local_hops; 1..64, 0 = 4) */
    int32_t reserved[4];
} gr_server_config;

typedef struct {
    int32_t status;      /* GR_OK, or the query's error */
    int32_t graph_id;
    int32_t src;
    int32_t batch_size;  /* queries live in its executor right after it was admitted */
    int64_t t_submit_ns; /* CLOCK_MONOTONIC times */
    int64_t t_start_ns;  /* admission into an executor */
    int64_t t_done_ns;
    int32_t iterations;  /* rounds in which the query's frontier was not empty */
    int32_t reserved;
} gr_query_result;

/* A query server with continuous batching.  Graphs stay resident; each
 * executor (a host thread with its own stream) keeps a multi-query session of
 * up to max_batch live queries whose rounds advance together (the engine of
 * gr_sssp_multi, one captured HIP graph of 8 rounds replayed per chunk).
 * Queries wait in one FIFO and join an executor between chunks, in arrival
 * order, as slots and memory free up: a query's footprint (2 bytes per vertex
 * of frontier marks + 26 bytes per vertex of the executor's union queues) must
 * fit hbm_budget_bytes next to every query already admitted.  A query is
 * complete when a chunk ends with its frontier empty; its distances are then
 * final in its dist_out.  Queries on graphs whose AUTO loop is the single-
 * workgroup loop (GR_LOOP_LDS) and that fit its row-offset layout take no slot: an executor takes up to 64 of
 * them from anywhere in the FIFO (they hold nothing the head waits for) and
 * runs them as one launch, one workgroup per query, on a stream of its own;
 * batch_size is then that launch's query count.  cfg may be NULL. */
gr_status gr_server_create(gr_server **out, size_t hbm_budget_bytes, const gr_server_config *cfg);
/* Registers a graph (not copied; it must outlive the server). */
gr_status gr_server_add_graph(gr_server *s, const gr_graph *g, int32_t *graph_id);
/* Queues one query; never blocks on the GPU.  dist_out: device memory for n
 * values, written when the ticket completes.  GR_ERR_NO_CAPACITY when the
 * query's footprint exceeds the whole budget. */
gr_status gr_serve_submit(gr_server *s, int32_t graph_id, int32_t src, void *dist_out, uint64_t *ticket);
/* GR_OK and *out filled once the query has completed (the ticket is then
 * retired), GR_ERR_NOT_READY before, GR_ERR_UNKNOWN_TICKET for a ticket never
 * issued or already retired. */
gr_status gr_serve_poll(gr_server *s, uint64_t ticket, gr_query_result *out);
/* Waits for every queued and running query, then frees the server. */
gr_status gr_server_destroy(gr_server *s);

/* ---- diagnostics ------------------------------------------------------- */

const char *gr_status_string(gr_status s);
/* Text of the calling thread's last error ("" if none). */
const char *gr_last_error(void);
/* Library version string. */
const char *gr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GR_H_ */
