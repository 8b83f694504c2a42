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
  roofline    algorithmic bytes of the push (advance) kernel per launch --
              12 B per relaxed edge (arc 8 B + dist 4 B) + 20 B per frontier
              vertex (queue 4, offsets 8, dist 4, next-queue 4) -- divided by
              its launch time measured with HIP events on the query's stream,
              against the 8 TB/s HBM3E peak
  cpu_baseline  the CPU oracle (binary-heap Dijkstra, one core) on a bounded
              sample of the same workload's sources
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
    ap.add_argument("--loop", type=int, default=0, help="gr_loop_mode (0 auto, 1 host, 2 persistent)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus %d, "
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

    t0 = time.time()
    g, srcs = gg.workload(args.workload)
    log("generated %s: n=%d m=%d in %.1fs" % (args.workload, g.n, g.m, time.time() - t0))
    t0 = time.time()
    G = gr.Graph.from_csr(g)
    torch.cuda.synchronize()
    info = G.info()
    log("graph resident: %s (%.2fs)" % (info, time.time() - t0))
    inf = gr.GR_DIST_INF_F32_BITS if g.wtype == gr.GR_W_F32 else gr.GR_DIST_INF_U32
    deg = np.diff(g.ro).astype(np.int64)
    srcs = [int(s) for s in srcs]
    dist = torch.empty(g.n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    opts = dict(loop=args.loop, direction=args.direction, layout=args.layout)

    # m_reached per source (from the GPU result of its first run)
    reached = {}

    def run(i, timing=0):
        s = srcs[i % len(srcs)]
        st = gr.gr_sssp_ex(G.handle, s, dist, stream=stream, timing=timing, **opts)
        return s, st

    for i in range(max(args.warmup, 1)):
        s, st = run(i)
    torch.cuda.synchronize()
    for s in sorted(set(srcs[i % len(srcs)] for i in range(args.steps))):
        if s not in reached:
            gr.gr_sssp_ex(G.handle, s, dist, stream=stream, **opts)
            d = dist.cpu().numpy().view(np.uint32)
            reached[s] = int(deg[d != inf].sum())
    log("warm-up done; timing %d steps" % args.steps)

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    edges = 0
    push_us = 0.0
    alg_bytes = 0
    launches = 0
    iters = 0
    stats_last = None
    for i in range(args.steps):
        s, st = run(args.warmup + i, timing=1)
        edges += reached[s]
        push_us += st["push_us"]
        alg_bytes += 12 * st["edges_pushed"] + 20 * st["push_frontier_sum"]
        launches += st["push_launches"]
        iters += st["iterations"]
        stats_last = st
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = 1e3 * t_total / args.steps
    gteps = edges / t_total / 1e9
    log("timed: %.3f ms/step, %.2f GTEPS, %d iterations/step" % (ms_per_step, gteps, iters // args.steps))

    roof = None
    if launches and push_us > 0:
        achieved = alg_bytes / (push_us * 1e-6) / 1e9
        roof = {"kernel": "k_push", "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "bytes_per_launch": int(alg_bytes / launches), "avg_launch_us": round(push_us / launches, 2),
                "launches": launches}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t_cpu = 0.0
        e_cpu = 0
        done = 0
        while done < len(srcs) and (t_cpu < args.cpu_seconds or done == 0):
            s = srcs[done]
            t1 = time.perf_counter()
            d = oracle.dijkstra(g, s)
            t_cpu += time.perf_counter() - t1
            e_cpu += int(deg[d != inf].sum())
            done += 1
        cpu = {"value": round(e_cpu / t_cpu / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": "%d of %d sources on the full graph, %.1f s of single-thread binary-heap Dijkstra"
                         % (done, len(srcs), t_cpu)}
        log("cpu oracle: %s" % cpu)

    out = {
        "metric": "SSSP GTEPS + HBM GB/s (single vs batched); p50/p99 query latency at fixed QPS",
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
                   "loop": {1: "host", 2: "persistent"}.get(stats_last["loop"], "?") if stats_last else None,
                   "iterations_per_query": iters / max(args.steps, 1)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    G.close()


if __name__ == "__main__":
    main()
