"""GPU parity of the asynchronous loop (GR_LOOP_ASYNC): one persistent kernel
draining a device worklist, no rounds.  Distances are compared with the CPU
oracle element by element (tolerance 0: the fixed point is unique, whatever
order the vertices are expanded in), for SSSP with both weight types and for
BFS, on the configurations' shapes and on edge cases, including lists that
overflow and continue in later phases."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
gr = pytest.importorskip("paper_2212_08200_amd")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run(G, n, src, bfs=False, **kw):
    d = torch.full((n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    f = gr.gr_bfs_ex if bfs else gr.gr_sssp_ex
    kw.setdefault("barrier_timeout_us", 5_000_000)  # bounds any worklist wait (a query takes < 1 s)
    st = f(G.handle, int(src), d, loop=gr.GR_LOOP_ASYNC, **kw)
    torch.cuda.synchronize()
    return d.cpu().numpy().view(np.uint32), st


def check(g, srcs, tag, bfs=False, flags=0):
    G = gr.Graph.from_csr(g, flags=flags)
    try:
        for s in srcs:
            want = oracle.bfs(g, int(s)) if bfs else oracle.dijkstra(g, int(s))
            say("async %s %s src=%d n=%d m=%d" % ("bfs" if bfs else "sssp", tag, s, g.n, g.m))
            got, st = run(G, g.n, s, bfs=bfs)
            if not np.array_equal(got, want):
                v = int(np.flatnonzero(got != want)[0])
                raise AssertionError("%s src %d: vertex %d got 0x%08x want 0x%08x" % (tag, s, v, int(got[v]),
                                                                                     int(want[v])))
            assert st["loop"] == gr.GR_LOOP_ASYNC and st["iterations"] >= 1
            reached = int(np.count_nonzero(want != (gr.GR_DIST_INF_F32_BITS if (g.wtype == gg.W_F32 and not bfs)
                                                    else gr.GR_DIST_INF_U32)))
            assert st["frontier_sum"] >= reached  # every reached vertex was expanded at least once
    finally:
        G.close()


def test_async_small_configs():
    g, srcs = gg.workload("grid64")
    check(g, [int(srcs[0]), 4095, 2080], "grid64")
    for wtype in (gg.W_U32, gg.W_F32):
        g = gg.rmat(12, 16, gseed=61, pseed=62, wseed=63, wtype=wtype)
        check(g, gg.pick_sources(g, 64, 3), "rmat12_w%d" % wtype)


def test_async_directed_zero_weights_and_ragged():
    for seed in (1, 2):
        g = gg.uniform(5000, 30000, gseed=seed, wseed=seed + 10, wtype=gg.W_U32, wlo=0, whi=3)
        check(g, [0, 17, 4999], "uniform%d" % seed)
    for n in (4097, 257):
        g = gg.uniform(n, 6 * n, gseed=n, wseed=n + 1, wtype=gg.W_U32, wlo=1, whi=9)
        check(g, [0, n - 1], "ragged%d" % n)


def test_async_edge_cases():
    cases = [
        ("single_vertex", gg.from_arcs(1, []), 0),
        ("isolated_source", gg.from_arcs(4, [(1, 2, 3), (2, 3, 4)]), 0),
        ("two_components", gg.from_arcs(6, [(0, 1, 2), (1, 2, 2), (3, 4, 1), (4, 5, 1)]), 0),
        ("self_loops_parallel_zero", gg.from_arcs(4, [(0, 0, 0), (0, 1, 9), (0, 1, 4), (1, 1, 3), (1, 2, 0),
                                                       (2, 0, 0), (2, 3, 0), (3, 2, 5)]), 3),
        ("u32_saturation", gg.from_arcs(4, [(0, 1, 0xFFFFFFFF - 5), (1, 2, 3), (2, 3, 7)]), 0),
        ("f32_rounding", gg.from_arcs(4, [(0, 1, 1.0), (1, 2, 2.0 ** -24), (2, 3, 2.0 ** -24), (0, 3, 1.0 + 2.0 ** -23)],
                                      wtype=gg.W_F32), 0),
        ("f32_overflow", gg.from_arcs(3, [(0, 1, 3.0e38), (1, 2, 3.0e38)], wtype=gg.W_F32), 0),
        # one hub: block-mapped expansion of a 70,000-arc list
        ("star_hub", gg.from_arcs(70001, [(0, i, i % 97 + 1) for i in range(1, 70001)]), 0),
    ]
    for name, g, s in cases:
        check(g, [s], name)


def test_async_worklist_overflow_phases(monkeypatch):
    # appends past the list's capacity spill and continue in later phases;
    # GR_ASYNC_LIST_CAP shrinks the list so that every query here overflows,
    # down to one entry (each phase then expands a single vertex)
    cases = [("grid64", gg.workload("grid64")[0], 64, 0),
             ("rmat12", gg.rmat(12, 16, gseed=61, pseed=62, wseed=63), 256, None),
             ("road200", gg.grid(200, wseed=71, wtype=gg.W_U32, wlo=1, whi=1000, shortcuts=40, sseed=72), 4096, 0),
             ("grid12_f32", gg.grid(12, wseed=9, wtype=gg.W_F32), 1, 0)]
    for tag, g, cap, s in cases:
        s = int(gg.pick_sources(g, 65, 1)[0]) if s is None else s
        monkeypatch.setenv("GR_ASYNC_LIST_CAP", str(cap))
        G = gr.Graph.from_csr(g)
        try:
            want = oracle.dijkstra(g, s)
            say("async overflow %s cap=%d" % (tag, cap))
            got, st = run(G, g.n, s)
            assert np.array_equal(got, want), tag
            say("  phases=%d expansions=%d relaxations=%d" % (st["iterations"], st["frontier_sum"],
                                                              st["edges_pushed"]))
            assert st["iterations"] > 1
        finally:
            G.close()
    monkeypatch.delenv("GR_ASYNC_LIST_CAP")
    # the default capacity (4 n + 1024 entries) on the same road-like graph
    g = cases[2][1]
    G = gr.Graph.from_csr(g)
    try:
        got, st = run(G, g.n, 0)
        assert np.array_equal(got, oracle.dijkstra(g, 0))
        say("road200 default list: phases=%d expansions=%d" % (st["iterations"], st["frontier_sum"]))
    finally:
        G.close()


def test_async_configs_sampled():
    for name in ("rmat20", "road2048"):
        g, srcs = gg.workload(name)
        check(g, [int(srcs[0])], name)


def test_async_bfs():
    check(gg.grid(40, wseed=3), [0, 40 * 40 - 1], "grid40", bfs=True)
    g = gg.rmat(13, 16, gseed=5, pseed=6, wseed=7)
    check(g, gg.pick_sources(g, 8, 2), "rmat13", bfs=True)


def test_async_rejects_and_times_out():
    g = gg.grid(64, wseed=2)
    G = gr.Graph.from_csr(g)
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    try:
        for d in (gr.GR_DIR_PULL, gr.GR_DIR_ALTERNATE):
            with pytest.raises(gr.GrError) as ei:
                gr.gr_sssp_ex(G.handle, 0, dist, loop=gr.GR_LOOP_ASYNC, direction=d)
            assert ei.value.status == gr.GR_ERR_INVALID_ARG
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_ex(G.handle, 0, dist, loop=gr.GR_LOOP_ASYNC, delta=50)
        assert ei.value.status == gr.GR_ERR_INVALID_ARG
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_ex(G.handle, 0, dist, loop=6)  # past the last loop mode
        assert ei.value.status == gr.GR_ERR_INVALID_ARG
        # a 1 us bound on a worklist wait: idle blocks give up, the query
        # reports the failure, and the next query on the graph is exact
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_ex(G.handle, 0, dist, loop=gr.GR_LOOP_ASYNC, barrier_timeout_us=1)
        assert ei.value.status == gr.GR_ERR_HIP
        got, _ = run(G, g.n, 0)
        assert np.array_equal(got, oracle.dijkstra(g, 0))
    finally:
        G.close()


def test_async_is_the_small_mesh_default():
    # bounded degree and n <= 65,536, too large for one workgroup's LDS: AUTO
    # runs the asynchronous loop, except for requests it cannot serve (pull,
    # near-far), which take the queued loop
    g = gg.grid(128, wseed=2)
    want = oracle.dijkstra(g, 0)
    G = gr.Graph.from_csr(g)
    try:
        for kw, loop in ((dict(), gr.GR_LOOP_ASYNC), (dict(direction=gr.GR_DIR_ALTERNATE), gr.GR_LOOP_QUEUED),
                         (dict(delta=50), gr.GR_LOOP_QUEUED)):
            d = torch.full((g.n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
            st = gr.gr_sssp_ex(G.handle, 0, d, **kw)
            torch.cuda.synchronize()
            assert st["loop"] == loop, kw
            assert np.array_equal(d.cpu().numpy().view(np.uint32), want), kw
    finally:
        G.close()
    g = gg.rmat(14, 16, gseed=31, pseed=32, wseed=33)  # skewed degrees: queued
    G = gr.Graph.from_csr(g)
    try:
        s = int(gg.pick_sources(g, 3, 1)[0])
        d = torch.empty(g.n, dtype=torch.int32, device="cuda")
        st = gr.gr_sssp_ex(G.handle, s, d)
        torch.cuda.synchronize()
        assert st["loop"] == gr.GR_LOOP_QUEUED
        assert np.array_equal(d.cpu().numpy().view(np.uint32), oracle.dijkstra(g, s))
    finally:
        G.close()
