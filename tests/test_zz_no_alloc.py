"""The allocation-free entry point gr_sssp_noalloc against gr_sssp, through the
C ABI: two calls in a row on the fixed per-device workspace, the second on a
smaller graph (the array keeps the first call's contents, so the second must
clear what it reads), both compared element by element with gr_sssp and with
the CPU oracle (tolerance 0); then a graph whose workspace exceeds the array
is refused before anything runs."""
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


def both(G, src, n):
    ref = torch.full((n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    got = torch.full((n,), 0x3C3C3C3C, dtype=torch.int32, device="cuda")
    gr.gr_sssp(G.handle, int(src), ref)
    torch.cuda.synchronize()
    gr.gr_sssp_noalloc(G.handle, int(src), got)
    torch.cuda.synchronize()
    return got.cpu().numpy().view(np.uint32), ref.cpu().numpy().view(np.uint32)


def test_noalloc_matches_gr_sssp_twice_then_smaller():
    cases = [("rmat16 u32", gg.rmat(16, gseed=11, pseed=12, wseed=13, wlo=1, whi=255)),
             ("road256 u32", gg.grid(256, 15, whi=1000, shortcuts=65, sseed=14)),
             ("rmat12 f32", gg.rmat(12, gseed=21, pseed=22, wseed=23, wtype=gg.W_F32)),
             ("grid40 u32", gg.grid(40, 31))]
    for tag, g in cases:
        G = gr.Graph.from_csr(g)
        try:
            srcs = [int(s) for s in gg.pick_sources(g, 5, 2)]
            for s in srcs:
                say("noalloc: %s n=%d m=%d src=%d" % (tag, g.n, g.m, s))
                got, ref = both(G, s, g.n)
                want = oracle.dijkstra(g, s)
                assert np.array_equal(ref, want), "%s src %d: gr_sssp differs from the oracle" % (tag, s)
                if not np.array_equal(got, ref):
                    bad = np.flatnonzero(got != ref)
                    raise AssertionError("%s src %d: %d mismatches, first vertex %d got 0x%08x want 0x%08x" % (
                        tag, s, len(bad), bad[0], got[bad[0]], ref[bad[0]]))
        finally:
            G.close()


def test_noalloc_refuses_a_graph_too_large_for_the_array():
    # a directed path of 8M vertices: its workspace (about 15 bytes per vertex) exceeds 96 MiB
    n = 8 << 20
    ro = np.arange(n + 1, dtype=np.int32)
    ro[-1] = n - 1
    col = np.arange(1, n, dtype=np.int32)
    w = np.ones(n - 1, dtype=np.uint32)
    G = gr.Graph(n, ro, col, w, gr.GR_W_U32, flags=gr.GR_NO_PULL | gr.GR_NO_PARTITION)
    try:
        out = torch.zeros(n, dtype=torch.int32, device="cuda")
        say("noalloc: oversized path n=%d" % n)
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_noalloc(G.handle, 0, out)
        assert ei.value.status == gr.GR_ERR_NO_CAPACITY
        torch.cuda.synchronize()
        assert int(out.abs().sum().item()) == 0  # nothing ran
    finally:
        G.close()


def test_noalloc_argument_errors():
    g = gg.grid(8, 3)
    G = gr.Graph.from_csr(g)
    try:
        out = torch.zeros(g.n, dtype=torch.int32, device="cuda")
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_noalloc(G.handle, g.n, out)
        assert ei.value.status == gr.GR_ERR_SOURCE_RANGE
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_noalloc(G.handle, 0, torch.zeros(g.n - 1, dtype=torch.int32, device="cuda"))
        assert ei.value.status == gr.GR_ERR_INVALID_ARG
    finally:
        G.close()
