"""GPU parity of breadth-first search (gr_bfs / gr_bfs_ex): hop depths from the
same operators with unit steps, compared element by element with the CPU
oracle's FIFO BFS (tolerance 0) for every direction policy, both push
layouts and both loops that run it."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
gr = pytest.importorskip("paper_2212_08200_amd")

DIRS = {"auto": gr.GR_DIR_AUTO, "push": gr.GR_DIR_PUSH, "pull": gr.GR_DIR_PULL, "alternate": gr.GR_DIR_ALTERNATE}
LOOPS = {"host": gr.GR_LOOP_HOST, "queued": gr.GR_LOOP_QUEUED}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def bfs(G, n, src, **kw):
    d = torch.full((n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    st = gr.gr_bfs_ex(G.handle, int(src), d, **kw)
    torch.cuda.synchronize()
    return d.cpu().numpy().view(np.uint32), st


def check(g, srcs, tag, flags=gr.GR_FORCE_PARTITION, dirs=tuple(DIRS), loops=tuple(LOOPS)):
    G = gr.Graph.from_csr(g, flags=flags)
    info = G.info()
    layouts = [gr.GR_LAYOUT_PLAIN] + ([gr.GR_LAYOUT_PARTITIONED] if info["partitions"] > 1 else [])
    try:
        for s in srcs:
            want = oracle.bfs(g, int(s))
            for lay in layouts:
                for d in dirs:
                    if d in ("pull", "alternate") and not info["pull_enabled"]:
                        continue
                    for lp in loops:
                        rf = gr.GR_RELAX_BOUND if (lay + len(lp)) % 2 else 0  # the bound filter on some cases
                        say("bfs %s src=%d dir=%s layout=%d loop=%s relax=%d" % (tag, s, d, lay, lp, rf))
                        got, st = bfs(G, g.n, s, direction=DIRS[d], layout=lay, loop=LOOPS[lp], relax_filter=rf)
                        if not np.array_equal(got, want):
                            v = int(np.flatnonzero(got != want)[0])
                            raise AssertionError("%s src %d dir %s layout %d loop %s: vertex %d got %d want %d" % (
                                tag, s, d, lay, lp, v, int(got[v]), int(want[v])))
    finally:
        G.close()


def test_bfs_small_graphs():
    check(gg.grid(40, wseed=3), [0, 40 * 40 - 1, 777], "grid40")
    check(gg.rmat(13, 16, gseed=5, pseed=6, wseed=7), gg.pick_sources(gg.rmat(13, 16, gseed=5, pseed=6, wseed=7), 8, 3),
          "rmat13")
    g = gg.uniform(5000, 20000, gseed=9, wseed=10)  # directed, some vertices unreachable
    check(g, [0, 4999], "uniform")
    g = gg.from_arcs(7, [(0, 1, 5), (1, 2, 5), (2, 3, 5), (3, 0, 5), (5, 6, 1)])
    check(g, [0, 5, 4], "cycle+isolated", flags=0)


def test_bfs_f32_graph_ignores_weights():
    g = gg.rmat(12, 16, gseed=11, pseed=12, wseed=13, wtype=gg.W_F32)
    check(g, gg.pick_sources(g, 14, 2), "rmat12f", dirs=("auto", "push"))


def test_bfs_errors():
    g = gg.grid(8, wseed=1)
    G = gr.Graph.from_csr(g)
    d = torch.empty(g.n, dtype=torch.int32, device="cuda")
    try:
        with pytest.raises(gr.GrError) as ei:
            gr.gr_bfs_ex(G.handle, 0, d, loop=gr.GR_LOOP_PERSISTENT)
        assert ei.value.status == gr.GR_ERR_INVALID_ARG
        with pytest.raises(gr.GrError) as ei:
            gr.gr_bfs(G.handle, g.n, d)
        assert ei.value.status == gr.GR_ERR_SOURCE_RANGE
        o = gr.gr_sssp_opts(delta=5)
        rc = gr.lib().gr_bfs_ex(G.handle, 0, gr._ptr(d), None, gr.ctypes.byref(o), None)
        assert rc == gr.GR_ERR_INVALID_ARG
    finally:
        G.close()


def test_bfs_rmat20_rmat22_configs():
    for name in ("rmat20", "rmat22"):
        g, srcs = gg.workload(name)
        G = gr.Graph.from_csr(g)
        try:
            for s in list(srcs)[:2]:
                want = oracle.bfs(g, int(s))
                for d in ("auto", "push"):
                    say("bfs %s src=%d dir=%s" % (name, s, d))
                    got, st = bfs(G, g.n, s, direction=DIRS[d])
                    assert np.array_equal(got, want), (name, s, d)
                    assert st["loop"] == gr.GR_LOOP_HOST  # AUTO on a skewed graph
                    if d == "auto":
                        assert st["pull_iterations"] > 0  # the middle levels pull
        finally:
            G.close()


def test_bfs_default_loop_on_a_mesh():
    # bounded degree: the single-workgroup loop when the mesh fits one
    # workgroup's LDS, else the queued loop
    for side, loop in ((48, gr.GR_LOOP_LDS), (96, gr.GR_LOOP_QUEUED)):
        g = gg.grid(side, wseed=3)
        G = gr.Graph.from_csr(g)
        try:
            got, st = bfs(G, g.n, 0)
            assert np.array_equal(got, oracle.bfs(g, 0))
            assert st["loop"] == loop, side
        finally:
            G.close()
