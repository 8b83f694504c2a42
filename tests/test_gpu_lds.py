"""GPU parity of the single-workgroup loop (GR_LOOP_LDS): one 1024-thread
workgroup holds the distances, row offsets, arcs and frontier lists of a small
graph in LDS and runs every round there.  Distances are compared with the CPU
oracle element by element (tolerance 0: the fixed point is unique), for SSSP
and for BFS, on the small-mesh configuration, on skewed and directed graphs,
on the degenerate cases (one vertex, isolated source, unreachable parts), at
the 16-bit weight limit and at the LDS size limit, for the argument errors
and the round cap, and for batches and served queries (one workgroup per
query)."""
import sys
import time

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
    st = f(G.handle, int(src), d, loop=gr.GR_LOOP_LDS, **kw)
    torch.cuda.synchronize()
    return d.cpu().numpy().view(np.uint32), st


def check(g, srcs, bfs=True):
    G = gr.Graph.from_csr(g)
    try:
        for s in srcs:
            say("lds %s n=%d m=%d src=%d" % (g.name, g.n, g.m, s))
            got, st = run(G, g.n, s)
            np.testing.assert_array_equal(got, oracle.dijkstra(g, int(s)), err_msg="%s src=%d" % (g.name, s))
            assert st["loop"] == gr.GR_LOOP_LDS and st["launches"] == 1 and st["iterations"] >= 1
            code, v = oracle.certify(g, int(s), got)
            assert code == 0, (code, v)
            if bfs:
                got, st = run(G, g.n, s, bfs=True)
                np.testing.assert_array_equal(got, oracle.bfs(g, int(s)), err_msg="bfs %s src=%d" % (g.name, s))
    finally:
        G.close()


def test_lds_small_mesh_config():
    g, srcs = gg.workload("grid64")
    check(g, list(srcs) + [4095, 2080])


def test_lds_road_like_and_random():
    check(gg.grid(60, 5, whi=1000, shortcuts=4, sseed=9, name="road60"), [0, 1234, 3599])
    g = gg.uniform(3000, 9000, gseed=3, wseed=4, whi=500, name="uniform3000")  # directed, with unreachable vertices
    check(g, [int(x) for x in gg.pick_sources(g, 5, 3)])


def test_lds_skewed_graph():
    # hubs: a group of 16 lanes walks a hub's arcs (the row-offset layout:
    # degrees above 16 are not padded); AUTO picks the loop here too
    g = gg.rmat(11, 8, gseed=41, pseed=42, wseed=43, name="rmat11")
    check(g, [int(x) for x in gg.pick_sources(g, 44, 3)])
    G = gr.Graph.from_csr(g)
    try:
        d = torch.empty(g.n, dtype=torch.int32, device="cuda")
        st = gr.gr_sssp_ex(G.handle, 7, d)
        torch.cuda.synchronize()
        assert st["loop"] == gr.GR_LOOP_LDS
        np.testing.assert_array_equal(d.cpu().numpy().view(np.uint32), oracle.dijkstra(g, 7))
    finally:
        G.close()


def test_lds_degenerate_graphs():
    check(gg.from_arcs(1, [], name="one"), [0])
    check(gg.from_arcs(5, [(0, 1, 7), (1, 2, 65535), (3, 4, 1)], name="parts"), [0, 2, 3, 4])
    # isolated source, self-loops and parallel arcs kept as given
    check(gg.from_arcs(4, [(1, 1, 3), (1, 2, 9), (1, 2, 4), (2, 3, 1)], name="loops"), [0, 1])


def test_lds_weight_limit():
    g = gg.grid(40, 6, wlo=60000, whi=65535, name="grid40w")  # weights up to 2^16 - 1 pack
    check(g, [0, 799])
    g = gg.from_arcs(3, [(0, 1, 65535), (1, 2, 65536)], name="w17")  # a weight of 2^16 does not
    G = gr.Graph.from_csr(g)
    try:
        with pytest.raises(gr.GrError) as ei:
            run(G, g.n, 0)
        assert ei.value.status == gr.GR_ERR_INVALID_ARG
        got, _ = run(G, g.n, 0, bfs=True)  # unit steps ignore the weights
        np.testing.assert_array_equal(got, oracle.bfs(g, 0))
        d = torch.empty(g.n, dtype=torch.int32, device="cuda")
        st = gr.gr_sssp_ex(G.handle, 0, d)  # AUTO: another loop
        torch.cuda.synchronize()
        assert st["loop"] != gr.GR_LOOP_LDS
        np.testing.assert_array_equal(d.cpu().numpy().view(np.uint32), oracle.dijkstra(g, 0))
    finally:
        G.close()


def test_lds_long_path_distances():
    # distances are kept in 31 bits: a 9,000-vertex chain of 65,535-weight arcs
    # (the longest that fits) reaches 589,749,465 = (n - 1) * (2^16 - 1)
    n = 9000
    g = gg.from_arcs(n, [(i, i + 1, 65535) for i in range(n - 1)], name="chain9000")
    check(g, [0, 4321, n - 1])
    # both directions (groups of 2 lanes): 3,000 vertices, weights U[1, 1000]
    rng = np.random.default_rng(23)
    w = rng.integers(1, 1001, size=2999)
    arcs = [(i, i + 1, int(w[i])) for i in range(2999)] + [(i + 1, i, int(w[i])) for i in range(2999)]
    check(gg.from_arcs(3000, arcs, name="path3000"), [0, 1500, 2999])


def test_lds_size_limit():
    # row offsets: 3 n + m + 1 words must fit 39,936 (a 75 x 75 grid does);
    # padded arcs: 6 n words for a grid (4 slots per vertex), so 76 x 76 to
    # 81 x 81 fit only that way (uint32 weights: the padded copy holds
    # 16-bit weights), and 82 x 82 fits neither
    check(gg.grid(75, 7, name="grid75"), [0, 75 * 75 - 1], bfs=False)
    for side in (76, 81):
        g = gg.grid(side, 7, name="grid%d" % side)
        check(g, [0, g.n - 1, 1234])
        G = gr.Graph.from_csr(g)
        try:
            d = torch.empty(g.n, dtype=torch.int32, device="cuda")
            st = gr.gr_sssp_ex(G.handle, 5, d)
            torch.cuda.synchronize()
            assert st["loop"] == gr.GR_LOOP_LDS
            np.testing.assert_array_equal(d.cpu().numpy().view(np.uint32), oracle.dijkstra(g, 5))
        finally:
            G.close()
    for over in (gg.grid(82, 7, name="grid82"), gg.grid(76, 7, wtype=gg.W_F32, name="grid76f")):
        G = gr.Graph.from_csr(over)
        try:
            with pytest.raises(gr.GrError) as ei:
                run(G, over.n, 0, bfs=True)
            assert ei.value.status == gr.GR_ERR_INVALID_ARG
            d = torch.empty(over.n, dtype=torch.int32, device="cuda")
            st = gr.gr_sssp_ex(G.handle, 0, d)  # AUTO takes another loop
            torch.cuda.synchronize()
            assert st["loop"] != gr.GR_LOOP_LDS
            np.testing.assert_array_equal(d.cpu().numpy().view(np.uint32), oracle.dijkstra(over, 0))
        finally:
            G.close()


def test_lds_padded_only_graph_in_batches():
    # a graph that fits only the padded layout: same-graph batches use it;
    # multi-graph launches use it when every graph has the same slot count,
    # and fall back to the multi-query engine when the layouts differ
    g76, g64 = gg.grid(76, 7, name="grid76"), gg.workload("grid64")[0]
    road = gg.grid(60, 5, whi=1000, shortcuts=4, sseed=9, name="road60")  # 8 slots
    Gs = [gr.Graph.from_csr(x) for x in (g76, g64, road)]
    try:
        srcs = np.asarray(gg.pick_sources(g76, 61, 8), np.int32)
        out = torch.full((8, g76.n), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
        say("lds batch grid76 k=8")
        st = gr.gr_sssp_batch_ex(Gs[0].handle, srcs, out)
        torch.cuda.synchronize()
        rows = out.cpu().numpy().view(np.uint32)
        for i, s in enumerate(srcs):
            np.testing.assert_array_equal(rows[i], oracle.dijkstra(g76, int(s)))
        assert st["replays"] == 0
        for members, lds in (((0, 1), True), ((0, 2), False)):
            gs = [(g76, g64, road)[i] for i in members]
            ss = [3, 7]
            outs = [torch.full((x.n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda") for x in gs]
            say("lds multi %s" % [x.name for x in gs])
            st = gr.gr_sssp_multi([Gs[i].handle for i in members], ss, outs)
            torch.cuda.synchronize()
            for x, s, o in zip(gs, ss, outs):
                np.testing.assert_array_equal(o.cpu().numpy().view(np.uint32), oracle.dijkstra(x, s))
            assert (st["replays"] == 0) == lds
    finally:
        for G in Gs:
            G.close()


def test_lds_is_the_small_mesh_default_and_errors():
    g = gg.grid(64, wseed=2)
    want = oracle.dijkstra(g, 0)
    G = gr.Graph.from_csr(g)
    try:
        for kw, loop in ((dict(), gr.GR_LOOP_LDS), (dict(direction=gr.GR_DIR_ALTERNATE), gr.GR_LOOP_QUEUED),
                         (dict(delta=50), gr.GR_LOOP_QUEUED)):
            d = torch.full((g.n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
            st = gr.gr_sssp_ex(G.handle, 0, d, **kw)
            torch.cuda.synchronize()
            assert st["loop"] == loop, kw
            np.testing.assert_array_equal(d.cpu().numpy().view(np.uint32), want, err_msg=str(kw))
        d = torch.empty(g.n, dtype=torch.int32, device="cuda")
        st = gr.gr_bfs_ex(G.handle, 0, d)
        torch.cuda.synchronize()
        assert st["loop"] == gr.GR_LOOP_LDS
        np.testing.assert_array_equal(d.cpu().numpy().view(np.uint32), oracle.bfs(g, 0))
        for kw in (dict(direction=gr.GR_DIR_PULL), dict(delta=50)):
            with pytest.raises(gr.GrError) as ei:
                gr.gr_sssp_ex(G.handle, 0, d, loop=gr.GR_LOOP_LDS, **kw)
            assert ei.value.status == gr.GR_ERR_INVALID_ARG
        # the round cap ends the query with an error
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_ex(G.handle, 0, d, loop=gr.GR_LOOP_LDS, max_iters=3)
        assert ei.value.status == gr.GR_ERR_ITER_LIMIT
    finally:
        G.close()
    gf = gg.grid(32, 3, wtype=gg.W_F32, name="grid32f")  # binary32 weights do not pack
    G = gr.Graph.from_csr(gf)
    try:
        d = torch.empty(gf.n, dtype=torch.int32, device="cuda")
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_ex(G.handle, 0, d, loop=gr.GR_LOOP_LDS)
        assert ei.value.status == gr.GR_ERR_INVALID_ARG
        st = gr.gr_sssp_ex(G.handle, 0, d)  # AUTO: another loop
        torch.cuda.synchronize()
        assert st["loop"] != gr.GR_LOOP_LDS
        np.testing.assert_array_equal(d.cpu().numpy().view(np.uint32), oracle.dijkstra(gf, 0))
    finally:
        G.close()


def test_lds_batch_one_workgroup_per_source():
    # gr_sssp_batch on a graph whose default is this loop: one workgroup per
    # source in one launch; every row certified, two compared in full
    for g in (gg.workload("grid64")[0], gg.grid(60, 5, whi=1000, shortcuts=4, sseed=9, name="road60")):
        G = gr.Graph.from_csr(g)
        try:
            for k in (2, 17, 64):
                srcs = np.asarray(gg.pick_sources(g, 90 + k, k), np.int32)
                if k == 64:
                    srcs[10] = srcs[3]  # a duplicate source
                out = torch.full((k, g.n), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
                say("lds batch %s k=%d" % (g.name, k))
                st = gr.gr_sssp_batch_ex(G.handle, srcs, out)
                torch.cuda.synchronize()
                rows = out.cpu().numpy().view(np.uint32)
                for i, s in enumerate(srcs):
                    code, v = oracle.certify(g, int(s), rows[i])
                    assert code == 0, (g.name, k, i, code, v)
                for i in (0, k - 1):
                    np.testing.assert_array_equal(rows[i], oracle.dijkstra(g, int(srcs[i])))
                assert st["replays"] == 0 and st["rounds"] >= 1
                assert st["source_relaxations"] == st["edges_pushed"] > 0
        finally:
            G.close()


def test_lds_multi_graph_batch():
    # gr_sssp_multi over graphs that all default to this loop (different sizes,
    # weights and group sizes): one workgroup per query; every result
    # certified, iterations reported per query
    gs = [gg.workload("grid64")[0], gg.grid(60, 5, whi=1000, shortcuts=4, sseed=9, name="road60"),
          gg.grid(20, 3, name="grid20"), gg.from_arcs(1, [], name="one"),
          gg.uniform(2000, 8000, 11, 12, symmetric=True, name="uni2000")]
    Gs = [gr.Graph.from_csr(g) for g in gs]
    try:
        idx = [i % len(gs) for i in range(23)]
        srcs = [int(gg.pick_sources(gs[i], 200 + j, 1)[0]) if gs[i].n > 1 else 0 for j, i in enumerate(idx)]
        outs = [torch.full((gs[i].n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda") for i in idx]
        say("lds multi k=%d" % len(idx))
        st = gr.gr_sssp_multi([Gs[i].handle for i in idx], srcs, outs)
        torch.cuda.synchronize()
        iters = st["iterations"]
        for j, i in enumerate(idx):
            d = outs[j].cpu().numpy().view(np.uint32)
            np.testing.assert_array_equal(d, oracle.dijkstra(gs[i], srcs[j]), err_msg="%s src=%d" % (gs[i].name, srcs[j]))
            assert iters[j] >= 1
        assert st["replays"] == 0 and st["rounds"] == max(iters)
    finally:
        for G in Gs:
            G.close()


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


def test_lds_served_queries_beside_the_session():
    # a server holding graphs that fit one workgroup's LDS (run directly, one
    # workgroup per query) and graphs that do not (the multi-query session):
    # every result equals the oracle's, and the direct ones were batched
    graphs = [gg.workload("grid64")[0], gg.grid(60, 5, whi=1000, shortcuts=4, sseed=9, name="road60"),
              gg.rmat(12, 16, gseed=7, pseed=8, wseed=9, name="rmat12"), gg.grid(96, 5, name="grid96")]
    Gs = [gr.Graph.from_csr(g) for g in graphs]
    server = gr.gr_server_create(4 << 30, max_batch=16, num_streams=2, max_wait_us=300)
    late, outs = [], []
    try:
        gids = [gr.gr_server_add_graph(server, G.handle) for G in Gs]
        rng = np.random.default_rng(17)
        reqs = []
        for i in range(160):
            gi = int(rng.integers(0, len(graphs)))
            s = int(gg.pick_sources(graphs[gi], 500 + i, 1)[0])
            reqs.append((gi, s, torch.full((graphs[gi].n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")))
        say("lds server: 160 queries over 4 graphs (2 direct)")
        tickets = [gr.gr_serve_submit(server, gids[gi], s, out) for gi, s, out in reqs]
        res = poll_all(server, tickets)
        direct_sizes = []
        for t, (gi, s, out) in zip(tickets, reqs):
            r = res[t]
            assert r["status"] == gr.GR_OK and r["src"] == s and r["iterations"] >= 1
            assert r["t_submit_ns"] <= r["t_start_ns"] <= r["t_done_ns"]
            got = out.cpu().numpy().view(np.uint32)
            np.testing.assert_array_equal(got, oracle.dijkstra(graphs[gi], s), err_msg="%s src=%d" % (graphs[gi].name, s))
            if gi < 2:
                direct_sizes.append(r["batch_size"])
        assert direct_sizes and max(direct_sizes) > 1, "no direct batch held two queries"
        # queries still queued when the server is destroyed are run first
        late += [(0, 5), (1, 7), (2, 3), (0, 9)]
        outs += [torch.full((graphs[gi].n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda") for gi, _ in late]
        for (gi, s), out in zip(late, outs):
            gr.gr_serve_submit(server, gids[gi], s, out)
    finally:
        gr.gr_server_destroy(server)
    try:
        torch.cuda.synchronize()
        for (gi, s), out in zip(late, outs):
            np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), oracle.dijkstra(graphs[gi], s))
    finally:
        for G in Gs:
            G.close()

