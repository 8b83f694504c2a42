"""GPU parity of batched multi-source queries (gr_sssp_batch) and of the query
server (gr_serve_submit / gr_serve_poll) against the CPU oracle: every row and
every served result passes the oracle's shortest-path certificate, and rows on
every graph (all of them on the small graphs, at least four on the large
ones) equal the oracle's Dijkstra bit for bit.  As a second check, batched
rows and served results also equal the same query run alone."""
import sys
import time

import numpy as np
import pytest

import graphgen as gg
import oracle
from certify_rows import certify_all, dijkstra_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
gr = pytest.importorskip("paper_2212_08200_amd")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def batch(G, g, srcs):
    out = torch.full((len(srcs), g.n), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    gr.gr_sssp_batch(G.handle, np.asarray(srcs, np.int32), out)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def single(G, g, s):
    d = torch.empty(g.n, dtype=torch.int32, device="cuda")
    gr.gr_sssp(G.handle, int(s), d)
    torch.cuda.synchronize()
    return d.cpu().numpy().view(np.uint32)


def check_rows(g, srcs, rows, tag):
    for i, s in enumerate(srcs):
        want = oracle.dijkstra(g, int(s))
        if not np.array_equal(rows[i], want):
            v = int(np.flatnonzero(rows[i] != want)[0])
            raise AssertionError("%s row %d (src %d): vertex %d got 0x%08x want 0x%08x" % (
                tag, i, s, v, int(rows[i][v]), int(want[v])))


@pytest.mark.parametrize("wtype", [gg.W_U32, gg.W_F32])
def test_batch_rmat12(wtype):
    g = gg.rmat(12, 16, gseed=71, pseed=72, wseed=73, wtype=wtype)
    G = gr.Graph.from_csr(g)
    try:
        for k in (1, 7, 64):
            srcs = gg.pick_sources(g, 74 + k, k)
            say("batch rmat12 w%d k=%d" % (wtype, k))
            check_rows(g, srcs, batch(G, g, srcs), "rmat12 k=%d" % k)
    finally:
        G.close()


def test_batch_duplicates_isolated_and_directed():
    g = gg.uniform(3000, 15000, gseed=3, wseed=4, wtype=gg.W_U32, wlo=0, whi=5)
    deg = np.diff(g.ro)
    iso = int(np.flatnonzero(deg == 0)[0]) if (deg == 0).any() else 0
    srcs = [0, 0, 5, iso, 2999, 5, 17]
    G = gr.Graph.from_csr(g)
    try:
        say("batch uniform dup/isolated")
        check_rows(g, srcs, batch(G, g, srcs), "uniform")
    finally:
        G.close()


def test_batch_grid64_config_and_ragged():
    g, _ = gg.workload("grid64")
    G = gr.Graph.from_csr(g)
    try:
        srcs = list(range(0, 4096, 97))[:40]
        check_rows(g, srcs, batch(G, g, srcs), "grid64")
    finally:
        G.close()
    g = gg.grid(65, wseed=9)  # n = 4225: ragged against 64-vertex output tiles and 4096-vertex groups
    G = gr.Graph.from_csr(g)
    try:
        check_rows(g, [0, 4224, 2000], batch(G, g, [0, 4224, 2000]), "grid65")
    finally:
        G.close()


def test_batch_argument_errors():
    g = gg.grid(8, wseed=1)
    G = gr.Graph.from_csr(g)
    out = torch.empty((65, g.n), dtype=torch.int32, device="cuda")
    try:
        for bad in ([], list(range(65))):
            with pytest.raises(gr.GrError) as ei:
                gr.gr_sssp_batch(G.handle, np.asarray(bad, np.int32), out)
            assert ei.value.status == gr.GR_ERR_INVALID_ARG
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_batch(G.handle, np.asarray([0, 64], np.int32), out)
        assert ei.value.status == gr.GR_ERR_SOURCE_RANGE
    finally:
        G.close()


def test_batch_rmat20_config():
    g, _ = gg.workload("rmat20")
    srcs = gg.pick_sources(g, 55, 16)
    G = gr.Graph.from_csr(g)
    try:
        say("batch rmat20 k=16")
        rows = batch(G, g, srcs)
        say("batch rmat20: certificate on all 16 rows, Dijkstra on 4")
        certify_all(g, srcs, rows, "rmat20")
        dijkstra_rows(g, srcs, rows, (0, 5, 10, 15), "rmat20")
        for i in (3, 8):  # second check: the same query alone
            assert np.array_equal(rows[i], single(G, g, srcs[i])), "rmat20 row %d" % i
    finally:
        G.close()


def test_batch_rmat22_64_sources_config():
    g, srcs = gg.workload("rmat22")
    G = gr.Graph.from_csr(g)
    try:
        say("batch rmat22 k=64")
        rows = batch(G, g, srcs)
        inf = np.uint32(gr.GR_DIST_INF_U32)
        assert all(rows[i][srcs[i]] == 0 for i in range(64))
        assert (rows != inf).sum(axis=1).min() > 1000
        say("batch rmat22: certificate on all 64 rows")
        certify_all(g, srcs, rows, "rmat22", workers=12)
        say("batch rmat22: Dijkstra on 4 rows")
        dijkstra_rows(g, srcs, rows, (0, 21, 42, 63), "rmat22")
        for i in (7, 50):  # second check: the same query alone
            assert np.array_equal(rows[i], single(G, g, srcs[i])), "rmat22 row %d" % i
    finally:
        G.close()


# ------------------------------------------------------------------- server

def poll_all(server, tickets, timeout=60.0):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for t in tickets:
            if t not in done:
                r = gr.gr_serve_poll(server, t)
                if r is not None:
                    done[t] = r
        if time.time() - t0 > timeout:
            raise TimeoutError("%d of %d queries pending" % (len(tickets) - len(done), len(tickets)))
        time.sleep(0.0005)
    return done


def test_server_mixed_stream_matches_alone():
    graphs = [gg.rmat(13, 16, gseed=i, pseed=i + 1, wseed=i + 2) for i in (1, 11)] + \
             [gg.grid(96, wseed=5), gg.rmat(12, 16, gseed=7, pseed=8, wseed=9, wtype=gg.W_F32)]
    Gs = [gr.Graph.from_csr(g) for g in graphs]
    server = gr.gr_server_create(8 << 30, max_batch=16, num_streams=3, max_wait_us=300)
    try:
        gids = [gr.gr_server_add_graph(server, G.handle) for G in Gs]
        rng = np.random.default_rng(5)
        reqs = []
        for i in range(120):
            gi = int(rng.integers(0, len(graphs)))
            s = int(gg.pick_sources(graphs[gi], 1000 + i, 1)[0])
            out = torch.full((graphs[gi].n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
            reqs.append((gi, s, out))
        say("server: 120 queries over 4 graphs")
        tickets = []
        for j, (gi, s, out) in enumerate(reqs):
            tickets.append(gr.gr_serve_submit(server, gids[gi], s, out))
            if j % 10 == 0:
                time.sleep(0.001)  # arrivals spread while earlier batches run
        res = poll_all(server, tickets)
        sizes = [res[t]["batch_size"] for t in tickets]
        assert max(sizes) > 1, "no query was batched"
        served = {}
        for t, (gi, s, out) in zip(tickets, reqs):
            r = res[t]
            assert r["status"] == gr.GR_OK and r["graph_id"] == gids[gi] and r["src"] == s
            assert r["t_submit_ns"] <= r["t_start_ns"] <= r["t_done_ns"]
            assert r["iterations"] >= 1
            got = out.cpu().numpy().view(np.uint32)
            served.setdefault(gi, []).append((s, got))
            assert np.array_equal(got, single(Gs[gi], graphs[gi], s)), "served != alone"
        say("server: certificate on all 120 results, Dijkstra on 4 per graph")
        for gi, lst in served.items():
            srcs = [s for s, _ in lst]
            rows = [d for _, d in lst]
            certify_all(graphs[gi], srcs, rows, "served graph %d" % gi)
            dijkstra_rows(graphs[gi], srcs, rows, range(min(4, len(lst))), "served graph %d" % gi)
        with pytest.raises(gr.GrError) as ei:
            gr.gr_serve_poll(server, tickets[0])  # retired
        assert ei.value.status == gr.GR_ERR_UNKNOWN_TICKET
    finally:
        gr.gr_server_destroy(server)
        for G in Gs:
            G.close()


def test_server_errors_and_drain():
    g = gg.rmat(12, 16, gseed=3, pseed=4, wseed=5)
    G = gr.Graph.from_csr(g)
    try:
        small = gr.gr_server_create(64 << 10)  # 64 KiB: a query on this graph needs more
        gid = gr.gr_server_add_graph(small, G.handle)
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        with pytest.raises(gr.GrError) as ei:
            gr.gr_serve_submit(small, gid, 0, out)
        assert ei.value.status == gr.GR_ERR_NO_CAPACITY
        with pytest.raises(gr.GrError) as ei:
            gr.gr_serve_submit(small, gid + 1, 0, out)
        assert ei.value.status == gr.GR_ERR_INVALID_ARG
        with pytest.raises(gr.GrError) as ei:
            gr.gr_serve_submit(small, gid, g.n, out)
        assert ei.value.status == gr.GR_ERR_SOURCE_RANGE
        with pytest.raises(gr.GrError) as ei:
            gr.gr_serve_poll(small, 12345)
        assert ei.value.status == gr.GR_ERR_UNKNOWN_TICKET
        gr.gr_server_destroy(small)
        # destroy with queries still queued: they are drained first
        srv = gr.gr_server_create(4 << 30, max_batch=4, num_streams=1, max_wait_us=100000)
        gid = gr.gr_server_add_graph(srv, G.handle)
        srcs = gg.pick_sources(g, 9, 10)
        outs = [torch.full((g.n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda") for _ in srcs]
        for s, o in zip(srcs, outs):
            gr.gr_serve_submit(srv, gid, int(s), o)
        gr.gr_server_destroy(srv)
        torch.cuda.synchronize()
        for s, o in zip(srcs, outs):
            assert np.array_equal(o.cpu().numpy().view(np.uint32), oracle.dijkstra(g, int(s)))
    finally:
        G.close()
