#!/usr/bin/env python3
"""Single-GPU benchmark of frontier-driven SSSP through the gr C ABI.

One step = one complete single-source shortest-path query (init, then
advance / filter / convergence test until the frontier is empty) on the
R-MAT scale-22 graph (4,194,304 vertices, edge factor 16, a/b/c/d =
.57/.19/.19/.05, symmetrised, uint32 weights U[1,255]); steps cycle over the
64 seeded non-isolated sources of that workload.  The graph is generated from
seeds on the host and uploaded before timing; the timed region starts with
inputs resident in HBM.

Prints ONE JSON line on stdout:
  value       GTEPS = sum over steps of m_reached(src) / wall time, where
              m_reached = out-degree sum of the vertices the query reaches
  roofline    algorithmic bytes of the dominant kernel per launch -- 12 B
              per relaxed edge (arc 8 B + dist 4 B) + 20 B per frontier vertex
              (queue 4, offsets 8, dist 4, next-queue 4) -- divided by its
              launch time measured with HIP events on the query's stream (in
              a second pass over the same steps, outside the timed region),
              against the 8 TB/s HBM3E peak.  The kernel is k_step (every
              phase of a round) for the queued loop, k_push (the advance)
              for the host-driven loop.  traffic: HBM bytes per launch from
              the committed rocprofv3 counter summary when it matches the
              current kernel sources, else null; query_gbs / query_frac: the
              query's algorithmic bytes over the timed wall clock.
  cpu_baseline  the CPU oracle (binary-heap Dijkstra) on the host's cores, one
              thread per source, over a bounded sample of the same workload's
              sources (core count and CPU model stated)
  batched     64 sources in one gr_sssp_batch call against the same 64 run
              as looped single queries
  configs     the other configurations (grid 64^2, R-MAT 20 binary32,
              road-like 2048^2, plain grid 2048^2), single queries with the
              graph's AUTO schedule: ms, GTEPS, rounds, relaxation inflation
              and kernel roofline
  serving     32 resident graphs under open-loop Poisson arrivals
Progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "rmat22": "R-MAT scale 22 (edge factor 16, a=.57 b=.19 c=.19 d=.05, symmetrised, deduplicated), "
              "uint32 weights U[1,255], single-source SSSP, 64 seeded non-isolated sources cycled",
    "rmat20": "R-MAT scale 20 (edge factor 16, a=.57 b=.19 c=.19 d=.05, symmetrised, deduplicated), "
              "fp32 weights U(0,1], single-source SSSP from one seeded non-isolated source",
    "road2048": "2048x2048 4-neighbour grid + floor(0.001 n) random shortcuts, uint32 weights U[1,1000], "
                "single-source SSSP from vertex 0",
    "grid2048": "2048x2048 4-neighbour grid, uint32 weights U[1,1000], single-source SSSP from vertex 0",
    "grid64": "64x64 4-neighbour grid, uint32 weights U[1,100], single-source SSSP from vertex 0",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="rmat22", choices=sorted(WORKLOADS))
    ap.add_argument("--layout", type=int, default=0, help="gr_layout (0 auto, 1 plain, 2 partitioned)")
    ap.add_argument("--direction", type=int, default=0, help="gr_direction (0 auto, 1 push, 2 pull)")
    ap.add_argument("--loop", type=int, default=0,
                    help="gr_loop_mode (0 auto, 1 host, 2 persistent, 3 queued, 4 asynchronous)")
    ap.add_argument("--alpha", type=int, default=0,
                    help="direction switch: pull when frontier out-edges * alpha / 16 >= m (0: graph default)")
    ap.add_argument("--filter", type=int, default=0, help="filter (0 auto, 1 group, 2 streaming member lists)")
    ap.add_argument("--delta", type=float, default=0.0,
                    help="near-far split width in weight units (0: the graph's default)")
    ap.add_argument("--relax", type=int, default=0,
                    help="push relaxation filter (0 graph default, 1 pre-read dist, 2 upper-bound array)")
    ap.add_argument("--local-hops", type=int, default=0,
                    help="small rounds: hops a block expands before handing improvements to the next round "
                         "(0: the graph's default)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-source batched comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the single-query timings of the other configurations (grid 64^2, R-MAT 20 "
                         "binary32, road-like 2048^2, grid 2048^2)")
    ap.add_argument("--serve-queries", type=int, default=8000, help="open-loop queries per load level")
    ap.add_argument("--serve-fifo-queries", type=int, default=1000,
                    help="queries of each level's trace replayed through the one-at-a-time FIFO")
    ap.add_argument("--serve-executors", type=int, default=3,
                    help="server: executors (each a stream with its own multi-query session)")
    ap.add_argument("--serve-slots", type=int, default=64, help="server: live queries per executor")
    ap.add_argument("--serve-local-hops", type=int, default=0, help="server: local hops (0: the library's default)")
    ap.add_argument("--bfs", action="store_true",
                    help="time breadth-first search (gr_bfs_ex) instead of SSSP on the same workload")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip gr_graph_tune (the graph's untuned AUTO schedule is timed)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run one elementwise copy (b = a + 1) of this many MiB and exit: a kernel of "
                         "known traffic, for scaling the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (asked for --gpus %d, "
              "WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen as gg
    import paper_2212_08200_amd as gr

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    gr.lib()  # fails loudly when libgr.so is missing
    dev = torch.device("cuda:0")
    if args.copy_probe_mib > 0:
        nbytes = args.copy_probe_mib << 20
        a = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.add(a, 1, out=b)  # one elementwise kernel: reads nbytes, writes nbytes
        torch.cuda.synchronize()
        log("copy probe: %d bytes read, %d bytes written" % (nbytes, nbytes))
        return

    t0 = time.time()
    g, srcs = gg.workload(args.workload)
    log("generated %s: n=%d m=%d in %.1fs" % (args.workload, g.n, g.m, time.time() - t0))
    t0 = time.time()
    G = gr.Graph.from_csr(g)
    torch.cuda.synchronize()
    info = G.info()
    log("graph resident: %s (%.2fs)" % (info, time.time() - t0))
    inf = gr.GR_DIST_INF_F32_BITS if (g.wtype == gr.GR_W_F32 and not args.bfs) else gr.GR_DIST_INF_U32
    deg = np.diff(g.ro).astype(np.int64)
    srcs = [int(s) for s in srcs]
    dist = torch.empty(g.n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    opts = dict(loop=args.loop, direction=args.direction, layout=args.layout, filter=args.filter, alpha_x16=args.alpha,
                delta=gr.delta_bits(args.delta, g.wtype) if args.delta > 0 else 0, relax_filter=args.relax,
                local_hops=args.local_hops)

    tuned = None
    explicit = (args.loop or args.direction or args.layout or args.filter or args.alpha or args.delta or args.relax
                or args.local_hops)
    if not args.no_tune and not explicit and not args.bfs:
        # the autotuner picks the AUTO schedule from a few of the workload's sources
        t0 = time.time()
        tuned = G.tune(srcs[:4], reps=2, stream=torch.cuda.current_stream())
        log("tuned schedule: %s (%.1fs)" % (tuned, time.time() - t0))

    # m_reached per source (from the GPU result of its first run)
    reached = {}

    def run(i, timing=0):
        s = srcs[i % len(srcs)]
        if args.bfs:
            o = dict(opts)
            o.pop("delta")
            st = gr.gr_bfs_ex(G.handle, s, dist, stream=stream, timing=timing, **o)
        else:
            st = gr.gr_sssp_ex(G.handle, s, dist, stream=stream, timing=timing, **opts)
        return s, st

    for i in range(max(args.warmup, 1)):
        s, st = run(i)
    torch.cuda.synchronize()
    for s in sorted(set(srcs[(args.warmup + i) % len(srcs)] for i in range(args.steps))):
        if s not in reached:
            gr.gr_sssp_ex(G.handle, s, dist, stream=stream, **opts)
            d = dist.cpu().numpy().view(np.uint32)
            reached[s] = int(deg[d != inf].sum())
    log("warm-up done; timing %d steps" % args.steps)

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    edges = 0
    iters = 0
    q_bytes = 0
    relax = 0
    stats_last = None
    for i in range(args.steps):
        s, st = run(args.warmup + i)
        edges += reached[s]
        iters += st["iterations"]
        q_bytes += 12 * st["edges_pushed"] + 20 * st["push_frontier_sum"]
        relax += st["edges_pushed"]
        stats_last = st
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = 1e3 * t_total / args.steps
    gteps = edges / t_total / 1e9
    log("timed: %.3f ms/step, %.2f GTEPS, %d iterations/step, %.0f M relaxations/step" % (
        ms_per_step, gteps, iters // args.steps, q_bytes / 12e6 / args.steps))

    # Kernel roofline: the same steps again, now with HIP events around every
    # advance launch on the query's stream (outside the timed region: the
    # events add gaps between launches).
    # The queued loop runs every phase (advance, filter, small round) in one
    # kernel, k_step: its launches are timed together (all of them, including
    # the few queued past the end of a query) against the round's bytes.
    push_us = 0.0
    alg_bytes = 0
    launches = 0
    for i in range(args.steps):
        s, st = run(args.warmup + i, timing=1)
        alg_bytes += 12 * st["edges_pushed"] + 20 * st["push_frontier_sum"]
        if st["loop"] == 3:
            push_us += st["push_us"] + st["filter_us"]
            launches += st["launches"]
        else:
            push_us += st["push_us"]
            launches += st["push_launches"]
    torch.cuda.synchronize()
    roof = None
    if launches and push_us > 0:
        achieved = alg_bytes / (push_us * 1e-6) / 1e9
        kern = {2: "k_persistent", 3: "k_step", 4: "k_async", 5: "k_lds"}.get(stats_last["loop"], "k_push")
        loop_name = {1: "host", 2: "persistent", 3: "queued", 4: "async", 5: "lds"}.get(stats_last["loop"], "?")
        layout_name = {1: "plain", 2: "partitioned"}.get(stats_last["layout"], "?")
        relax_name = {1: "dist", 2: "bound"}.get(stats_last["relax_filter"], "?")
        traffic = counter_traffic(kern, args.workload, loop_name, layout_name, relax_name)
        roof = {"kernel": kern, "bound": "hbm",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_launch": int(alg_bytes / launches), "avg_launch_us": round(push_us / launches, 2),
                "launches": launches,
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                # whole query: algorithmic bytes of all rounds over the timed wall clock
                "query_gbs": round(q_bytes / t_total / 1e9, 1),
                "query_frac": round(q_bytes / t_total / 1e9 / HBM_PEAK_GBS, 4)}
        if kern == "k_lds":
            roof["limiter"] = "LDS latency (one workgroup, one round per barrier)"

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(g, srcs, deg, inf, args.cpu_seconds)
        log("cpu oracle: %s" % cpu)

    batched = None
    if not args.no_batched and args.workload == "rmat22" and not args.bfs:
        for s in srcs:  # every batched source needs its reached-arc count
            if s not in reached:
                gr.gr_sssp_ex(G.handle, s, dist, stream=stream, **opts)
                d = dist.cpu().numpy().view(np.uint32)
                reached[s] = int(deg[d != inf].sum())
        batched = measure_batched(G, g, srcs, reached, ms_per_step, torch, np, gr, dev, opts)
        log("batched: %s" % batched)
    G.close()
    del dist
    torch.cuda.empty_cache()

    configs = None
    if not args.no_configs and args.workload == "rmat22" and not args.bfs:
        configs = {}
        for name, steps in (("grid64", 100), ("rmat20", 20), ("road2048", 10), ("grid2048", 3)):
            configs[name] = measure_config(name, steps, torch, np, gr, gg, dev)
            log("config %s: %s" % (name, configs[name]))

    serving = None
    if not args.no_serving:
        serving = measure_serving(args, torch, np, gr, gg, dev)
        log("serving: %s" % serving)

    out = {
        "metric": ("BFS GTEPS (measurement of the second vertex program; not the headline)" if args.bfs else
                   "SSSP GTEPS + HBM GB/s (single vs batched); p50/p99 query latency at fixed QPS"),
        "value": round(gteps, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if g.wtype == gr.GR_W_F32 else "u32",
        "data": "synthetic (seeded generator)",
        "config": {"workload": WORKLOADS[args.workload], "n": g.n, "m": g.m,
                   "layout": {1: "plain", 2: "partitioned"}.get(stats_last["layout"], "?") if stats_last else None,
                   "loop": {1: "host", 2: "persistent", 3: "queued", 4: "async", 5: "lds"}.get(stats_last["loop"], "?")
                   if stats_last else None,
                   "delta": args.delta or None,
                   "relax_filter": {1: "dist", 2: "bound"}.get(stats_last["relax_filter"]) if stats_last else None,
                   "iterations_per_query": iters / max(args.steps, 1),
                   # relaxations performed per query, and per reached arc (work inflation)
                   "relaxations_per_query": round(relax / max(args.steps, 1)),
                   "relaxation_inflation": round(relax / max(edges, 1), 3),
                   "tuned": ({k: tuned[k] for k in ("layout", "loop", "dense_ratio", "alpha_x16", "delta", "small",
                                                   "relax_filter", "async_blocks", "local_hops", "best_ms",
                                                   "default_ms", "trials")}
                             if tuned else None)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "batched": batched,
        "configs": configs,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


def host_cpu():
    """Threads the CPU legs may use on this host (the process's affinity set, and
    no more than OMP_NUM_THREADS when that is set) and the host's CPU model."""
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        cores = min(cores, int(omp))
    model = "?"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return max(cores, 1), model


def cpu_baseline(g, srcs, deg, inf, seconds):
    """The CPU oracle (binary-heap Dijkstra, oracle.dijkstra) on the host cores:
    one thread per source (the oracle is C called through ctypes, which releases
    the GIL), as many sources as there are threads per wave, waves until about
    `seconds` of wall time have passed; value = reached arcs / wall time.  A
    single-thread figure on the first source is reported beside it."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    cores, model = host_cpu()
    t1 = time.perf_counter()
    d = oracle.dijkstra(g, srcs[0])
    one_s = time.perf_counter() - t1
    one_edges = int(deg[d != inf].sum())

    def job(s):
        dd = oracle.dijkstra(g, s)
        return int(deg[dd != inf].sum())

    done, edges = 0, 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        while done < len(srcs):
            wave = srcs[done:done + cores]
            edges += sum(ex.map(job, wave))
            done += len(wave)
            if time.perf_counter() - t0 >= seconds:
                break
    wall = time.perf_counter() - t0
    return {"value": round(edges / wall / 1e9, 5), "unit": "GTEPS", "cores": cores, "kind": "oracle",
            "sample": "%d of the %d sources on the full graph, one thread per source on %d threads, %.1f s wall "
                      "(binary-heap Dijkstra)" % (done, len(srcs), cores, wall),
            "cpu_model": model, "nproc": os.cpu_count(),
            "single_thread_gteps": round(one_edges / one_s / 1e9, 5)}


def kernel_roofline(stats_list, wall_s, q_bytes):
    """Kernel roofline from per-query statistics gathered with timing on: the
    algorithmic bytes of the advance rounds (12 B per relaxed edge + 20 B per
    frontier vertex) over the summed launch times of the dominant kernel."""
    push_us, alg, launches, last = 0.0, 0, 0, None
    for st in stats_list:
        alg += 12 * st["edges_pushed"] + 20 * st["push_frontier_sum"]
        if st["loop"] == 3:
            push_us += st["push_us"] + st["filter_us"]
            launches += st["launches"]
        else:
            push_us += st["push_us"]
            launches += st["push_launches"]
        last = st
    if not launches or push_us <= 0:
        return None
    achieved = alg / (push_us * 1e-6) / 1e9
    kern = {2: "k_persistent", 3: "k_step", 4: "k_async", 5: "k_lds"}.get(last["loop"], "k_push")
    roof = {"kernel": kern, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_launch": int(alg / launches),
            "avg_launch_us": round(push_us / launches, 2), "launches": launches,
            "query_gbs": round(q_bytes / wall_s / 1e9, 1),
            "query_frac": round(q_bytes / wall_s / 1e9 / HBM_PEAK_GBS, 4)}
    if kern == "k_lds":
        # the whole query runs in one workgroup's LDS: its limit is the chain of
        # dependent LDS accesses per round, not HBM; the HBM figure is context
        roof["limiter"] = "LDS latency (one workgroup, one round per barrier)"
    return roof


def measure_config(name, steps, torch, np, gr, gg, dev):
    """One other configuration, single-source queries with the graph's AUTO
    schedule: time per query (wall clock around `steps` queries), GTEPS,
    rounds, relaxation inflation, and the dominant kernel's roofline."""
    t0 = time.time()
    g, srcs = gg.workload(name)
    G = gr.Graph.from_csr(g)
    gen_s = time.time() - t0
    s = int(srcs[0])
    inf = gr.GR_DIST_INF_F32_BITS if g.wtype == gr.GR_W_F32 else gr.GR_DIST_INF_U32
    dist = torch.empty(g.n, dtype=torch.int32, device=dev)
    st = gr.gr_sssp_ex(G.handle, s, dist)
    d = dist.cpu().numpy().view(np.uint32)
    reached = int(np.diff(g.ro).astype(np.int64)[d != inf].sum())
    for _ in range(2):
        gr.gr_sssp_ex(G.handle, s, dist)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = [gr.gr_sssp_ex(G.handle, s, dist) for _ in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    q_bytes = sum(12 * x["edges_pushed"] + 20 * x["push_frontier_sum"] for x in stats)
    timed = [gr.gr_sssp_ex(G.handle, s, dist, timing=1) for _ in range(min(steps, 5))]
    torch.cuda.synchronize()
    roof = kernel_roofline(timed, wall, q_bytes)
    last = stats[-1]
    batch = None
    if last["loop"] == 5:
        # graphs that fit one workgroup's LDS: 64 seeded sources (the
        # configuration's source first) in one gr_sssp_batch call, one
        # workgroup per source, against the same 64 as looped single queries
        bs = np.asarray([s] + [int(x) for x in gg.pick_sources(g, 7, 63)], np.int32)
        out = torch.empty((len(bs), g.n), dtype=torch.int32, device=dev)
        gr.gr_sssp_batch(G.handle, bs, out)
        torch.cuda.synchronize()
        reps = 20
        t1 = time.perf_counter()
        for _ in range(reps):
            gr.gr_sssp_batch(G.handle, bs, out)
        torch.cuda.synchronize()
        bms = 1e3 * (time.perf_counter() - t1) / reps
        t1 = time.perf_counter()
        for i, x in enumerate(bs):
            gr.gr_sssp_ex(G.handle, int(x), out[i])
        torch.cuda.synchronize()
        lms = 1e3 * (time.perf_counter() - t1)
        rows = out.cpu().numpy().view(np.uint32)
        deg = np.diff(g.ro).astype(np.int64)
        edges = sum(int(deg[r != inf].sum()) for r in rows)
        batch = {"k": len(bs), "ms_per_call": round(bms, 4), "gteps": round(edges / (bms * 1e-3) / 1e9, 3),
                 "looped_ms": round(lms, 3), "speedup_vs_looped": round(lms / bms, 2)}
    G.close()
    return {"workload": WORKLOADS[name], "n": g.n, "m": g.m, "src": s,
            "loop": {1: "host", 2: "persistent", 3: "queued", 4: "async", 5: "lds"}.get(last["loop"], "?"),
            "ms_per_query": round(1e3 * wall / steps, 4), "queries": steps,
            "gteps": round(reached * steps / wall / 1e9, 4),
            "rounds": last["iterations"], "relaxations": last["edges_pushed"],
            "relaxation_inflation": round(last["edges_pushed"] / max(reached, 1), 3),
            "roofline": roof, "batch64": batch, "setup_s": round(gen_s, 1)}


def counter_traffic(kernel, workload, loop, layout, relax):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when that summary is for another kernel / workload or the kernel
    sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_%s_counters.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, _, v = line.partition(":")
            fields[k.strip()] = v.strip()
    src = "".join(open(os.path.join(ROOT, "paper_2212_08200_amd", "csrc", f)).read()
                  for f in ("gr_kernels.hip", "gr_device.h", "gr_internal.h"))
    if fields.get("kernel_sources_sha256") != hashlib.sha256(src.encode()).hexdigest():
        return None
    if fields.get("loop") != loop or fields.get("layout") != layout or fields.get("relax_filter") != relax:
        return None
    try:
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def batch_traffic(workload):
    """HBM bytes of one whole 64-source gr_sssp_batch call (every kernel it
    launches) from the committed counter summary, or None when the summary is
    missing or the kernel sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_mq_batch_push_%s_counters.md" % workload)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, _, v = line.partition(":")
            fields[k.strip()] = v.strip()
    if fields.get("batch_sources_sha256") != batch_sources_sha256(ROOT):
        return None
    try:
        return int(fields["traffic_bytes_per_batch_call"])
    except (KeyError, ValueError):
        return None


def batch_sources_sha256(root=None):
    """sha256 of the sources of the batched call's kernels."""
    import hashlib
    root = root or ROOT
    src = "".join(open(os.path.join(root, "paper_2212_08200_amd", "csrc", f)).read()
                  for f in ("gr_multi.hip", "gr_multi.h", "gr_device.h", "gr_internal.h"))
    return hashlib.sha256(src.encode()).hexdigest()


def measure_batched(G, g, srcs, reached, single_ms, torch, np, gr, dev, opts):
    """64 sources in one gr_sssp_batch launch vs the same 64 as looped single queries."""
    k = len(srcs)
    out = torch.empty((k, g.n), dtype=torch.int32, device=dev)
    s_arr = np.asarray(srcs, np.int32)
    gr.gr_sssp_batch(G.handle, s_arr, out)  # warm-up
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        bst = gr.gr_sssp_batch_ex(G.handle, s_arr, out)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    edges = sum(reached[s] for s in srcs)
    # the same k sources as k single queries, one after the other, each into its own row
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, s in enumerate(srcs):
        gr.gr_sssp_ex(G.handle, s, out[i], **opts)
    torch.cuda.synchronize()
    looped_ms = 1e3 * (time.perf_counter() - t0)
    # algorithmic bytes of the batch: 8 B per arc expansion (the arc, read once for
    # every source active at its tail) + 4 B per (arc, active source) relaxation
    alg = 8 * bst["edges_pushed"] + 4 * bst["source_relaxations"]
    res = {"k": k, "ms_per_launch": round(ms, 3), "gteps": round(edges / (ms * 1e-3) / 1e9, 3),
           "rounds": bst["rounds"], "replays": bst["replays"], "arc_expansions": bst["edges_pushed"],
           "source_relaxations": bst["source_relaxations"], "algorithmic_bytes": alg,
           "algorithmic_gbs": round(alg / (ms * 1e-3) / 1e9, 1),
           "algorithmic_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "looped_ms": round(looped_ms, 3), "looped_gteps": round(edges / (looped_ms * 1e-3) / 1e9, 3),
           "speedup_vs_looped": round(looped_ms / ms, 3)}
    traffic = batch_traffic("rmat22") if k == 64 else None
    if traffic:
        # counted HBM bytes of one call (rocprofv3, copy-calibrated) over this run's call time
        res["hbm_bytes_per_launch"] = traffic
        res["hbm_gbs"] = round(traffic / (ms * 1e-3) / 1e9, 1)
        res["hbm_frac"] = round(traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return res


def measure_serving(args, torch, np, gr, gg, dev):
    """32 resident graphs served with continuous batching (gr_server_*):
    capacity Q* from a closed loop with 64 queries outstanding, then open-loop
    Poisson streams at 0.5 Q* and 0.8 Q*; latency = completion - scheduled
    arrival (no coordinated omission).  The first queries of the same trace,
    at the same arrival times, are replayed through a plain FIFO that runs one
    query at a time (max_batch 1, one executor): a queue alone."""
    t0 = time.time()
    graphs = gg.serving_graphs()
    Gs = [gr.Graph.from_csr(x) for x in graphs]
    deg = [np.diff(x.ro).astype(np.int64) for x in graphs]
    log("serving graphs: %d (%.1fs)" % (len(Gs), time.time() - t0))
    rng = np.random.default_rng(201)
    nq = max(args.serve_queries, 100)
    nfifo = min(nq, args.serve_fifo_queries)
    # query mix: graph uniform over 32, source uniform over non-isolated vertices
    nonzero = [np.flatnonzero(d > 0) for d in deg]
    mix = []
    for i in range(nq + 300):
        gi = int(rng.integers(0, len(graphs)))
        mix.append((gi, int(nonzero[gi][rng.integers(0, len(nonzero[gi]))])))
    # one output buffer per query of a run (no two queries in flight share one)
    outs = [torch.empty(graphs[gi].n, dtype=torch.int32, device=dev) for gi, _ in mix]
    inf = gr.GR_DIST_INF_U32
    edges_of = {}

    def serve(lo, hi, arrivals_ns, max_batch, executors):
        srv = gr.gr_server_create(64 << 30, max_batch=max_batch, num_streams=executors,
                                  local_hops=args.serve_local_hops)
        try:
            gids = [gr.gr_server_add_graph(srv, G.handle) for G in Gs]
            tickets = []
            start = time.monotonic_ns()
            for q, at in zip(range(lo, hi), arrivals_ns):
                gi, s = mix[q]
                due = start + int(at)
                while True:
                    now = time.monotonic_ns()
                    if now >= due:
                        break
                    if due - now > 200000:
                        time.sleep((due - now - 100000) / 1e9)
                tickets.append((gr.gr_serve_submit(srv, gids[gi], s, outs[q]), due))
                if len(tickets) % 1000 == 0:
                    log("  submitted %d of %d (max_batch %d)" % (len(tickets), hi - lo, max_batch))
            res = {}
            while len(res) < len(tickets):
                for t, due in tickets:
                    if t not in res:
                        r = gr.gr_serve_poll(srv, t)
                        if r is not None:
                            res[t] = r
                time.sleep(0.0005)
            lat, done_at = [], 0
            for t, due in tickets:
                r = res[t]
                assert r["status"] == gr.GR_OK
                lat.append(r["t_done_ns"] - due)
                done_at = max(done_at, r["t_done_ns"])
            return np.array(lat) / 1e6, (done_at - start) / 1e9, [res[t] for t, _ in tickets]
        finally:
            gr.gr_server_destroy(srv)

    def m_reached(gi, s):
        key = (gi, s)
        if key not in edges_of:
            d = torch.empty(graphs[gi].n, dtype=torch.int32, device=dev)
            gr.gr_sssp(Gs[gi].handle, s, d)
            dd = d.cpu().numpy().view(np.uint32)
            edges_of[key] = int(deg[gi][dd != inf].sum())
        return edges_of[key]

    def serve_closed(lo, hi, clients, max_batch):
        """Closed loop: `clients` queries outstanding; each completion submits the next."""
        srv = gr.gr_server_create(64 << 30, max_batch=max_batch, num_streams=args.serve_executors,
                                  local_hops=args.serve_local_hops)
        try:
            gids = [gr.gr_server_add_graph(srv, G.handle) for G in Gs]
            pending = {}
            nxt = [lo]
            start = time.monotonic_ns()
            done = 0

            def submit():
                q = nxt[0]
                if q >= hi:
                    return
                nxt[0] += 1
                gi, s = mix[q]
                pending[gr.gr_serve_submit(srv, gids[gi], s, outs[q])] = gi

            for _ in range(clients):
                submit()
            end_ns = start
            while pending:
                for t in list(pending):
                    r = gr.gr_serve_poll(srv, t)
                    if r is not None:
                        assert r["status"] == gr.GR_OK
                        del pending[t]
                        done += 1
                        end_ns = max(end_ns, r["t_done_ns"])
                        submit()
                        if done % 1000 == 0:
                            log("  closed loop: %d of %d done" % (done, hi - lo))
                time.sleep(0.0001)
            return done / ((end_ns - start) / 1e9)
        finally:
            gr.gr_server_destroy(srv)

    # capacity: closed loop with 64 queries outstanding (two per resident graph)
    serve_closed(0, 200, 64, args.serve_slots)
    qstar = serve_closed(300, 300 + nq, 64, args.serve_slots)
    log("serving capacity Q* = %.0f queries/s (closed loop, 64 outstanding)" % qstar)
    out = {"graphs": len(graphs), "executors": args.serve_executors, "slots": args.serve_slots,
           "capacity_qps": round(qstar, 1), "capacity_clients": 64, "queries_per_level": nq,
           "fifo_queries_per_level": nfifo, "levels": []}
    for frac in (0.5, 0.8):
        qps = frac * qstar
        gaps = rng.exponential(1.0 / qps, size=nq)
        arr = (np.cumsum(gaps) * 1e9).astype(np.int64)
        lat, span, res = serve(300, 300 + nq, arr, args.serve_slots, args.serve_executors)
        lat1, _, _ = serve(300, 300 + nfifo, arr[:nfifo], 1, 1)  # one query at a time, in arrival order
        edges = sum(m_reached(*mix[q]) for q in range(300, 300 + nq))
        sizes = np.array([r["batch_size"] for r in res])
        hist = {}
        for lo, hi in ((1, 1), (2, 4), (5, 8), (9, 16), (17, 32), (33, 64)):
            c = int(((sizes >= lo) & (sizes <= hi)).sum())
            if c:
                hist["%d" % lo if lo == hi else "%d-%d" % (lo, hi)] = c
        out["levels"].append({
            "offered_qps": round(qps, 1), "achieved_qps": round(nq / span, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "gteps": round(edges / span / 1e9, 3),
            "batch_size_hist": hist,
            "mean_rounds": round(float(np.mean([r["iterations"] for r in res])), 1),
            "fifo_unbatched_p50_ms": round(float(np.percentile(lat1, 50)), 3),
            "fifo_unbatched_p99_ms": round(float(np.percentile(lat1, 99)), 3)})
        log("serving level %.1f Q*: %s" % (frac, out["levels"][-1]))
    for G in Gs:
        G.close()
    return out


if __name__ == "__main__":
    main()
