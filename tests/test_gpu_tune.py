"""GPU tests of the schedule autotuner (gr_graph_tune): the chosen schedule is
one of the candidates, queries under it stay bit-identical to the oracle, and
the signature-keyed cache returns the stored choice without timing again."""
import os
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


def run(G, s, n):
    d = torch.empty(n, dtype=torch.int32, device="cuda")
    gr.gr_sssp(G.handle, int(s), d)
    torch.cuda.synchronize()
    return d.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("flags", [0, gr.GR_FORCE_PARTITION])
def test_tune_then_query(flags, tmp_path, monkeypatch):
    monkeypatch.setenv("GR_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    g = gg.rmat(14, 16, gseed=31, pseed=32, wseed=33)
    srcs = gg.pick_sources(g, 34, 3)
    with gr.Graph.from_csr(g, flags=flags) as G:
        say("tune rmat14 flags=%d" % flags)
        r = G.tune(srcs, reps=2)
        assert r["from_cache"] == 0 and r["trials"] >= 4
        assert r["layout"] in (gr.GR_LAYOUT_PLAIN, gr.GR_LAYOUT_PARTITIONED)
        if not G.info()["partitions"] > 1:
            assert r["layout"] == gr.GR_LAYOUT_PLAIN
        assert r["loop"] in (gr.GR_LOOP_HOST, gr.GR_LOOP_PERSISTENT, gr.GR_LOOP_QUEUED, gr.GR_LOOP_ASYNC,
                             gr.GR_LOOP_LDS)
        assert r["dense_ratio"] in (8, 64, 512) and r["alpha_x16"] in (0, 8, 32)
        assert r["relax_filter"] in (gr.GR_RELAX_DIST, gr.GR_RELAX_BOUND)
        assert 0 < r["best_ms"] <= r["default_ms"]
        for s in srcs:
            assert np.array_equal(run(G, s, g.n), oracle.dijkstra(g, int(s)))
    with gr.Graph.from_csr(g, flags=flags) as G2:
        r2 = G2.tune(srcs, reps=2)
        assert r2["from_cache"] == 1
        for k in ("layout", "loop", "dense_ratio", "alpha_x16", "delta", "small", "relax_filter", "async_blocks"):
            assert r2[k] == r[k]
        assert np.array_equal(run(G2, srcs[0], g.n), oracle.dijkstra(g, int(srcs[0])))
    lines = open(tmp_path / "tune.jsonl").read().splitlines()
    assert len(lines) == 1 and '"sig": "n16384_' in lines[0]


def test_tune_argument_errors(monkeypatch):
    monkeypatch.delenv("GR_TUNE_CACHE", raising=False)
    g = gg.grid(16, wseed=3)
    with gr.Graph.from_csr(g) as G:
        with pytest.raises(gr.GrError) as ei:
            G.tune([])
        assert ei.value.status == gr.GR_ERR_INVALID_ARG
        with pytest.raises(gr.GrError) as ei:
            G.tune([0, g.n])
        assert ei.value.status == gr.GR_ERR_SOURCE_RANGE
        r = G.tune([0], reps=1)
        assert r["from_cache"] == 0
        assert np.array_equal(run(G, 5, g.n), oracle.dijkstra(g, 5))
