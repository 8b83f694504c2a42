"""GPU results on the hand-derived fixtures of tests/golden/, compared with the
values written in the files (not with the oracle): every direction policy,
push layout, loop driver (the asynchronous one included) and relaxation
filter for SSSP, the batched call over all of a fixture's sources, BFS hop
counts, and queries served together by one query server."""
import sys

import numpy as np
import pytest

import golden_fixtures

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
gr = pytest.importorskip("paper_2212_08200_amd")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def fresh(n):
    return torch.full((n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("name", golden_fixtures.names())
def test_golden_fixture_on_gpu(name):
    g, queries = golden_fixtures.load(name)
    G = gr.Graph.from_csr(g, flags=gr.GR_FORCE_PARTITION)
    try:
        info = G.info()
        layouts = [gr.GR_LAYOUT_PLAIN] + ([gr.GR_LAYOUT_PARTITIONED] if info["partitions"] > 1 else [])
        dirs = [gr.GR_DIR_PUSH, gr.GR_DIR_AUTO] + (
            [gr.GR_DIR_PULL, gr.GR_DIR_ALTERNATE] if info["pull_enabled"] else [])
        # the single-workgroup loop packs uint32 weights below 2^16 (every fixture fits its LDS)
        lds = g.wtype == gr.GR_W_U32 and (g.m == 0 or int(np.max(g.w)) < 65536)
        loops = (gr.GR_LOOP_HOST, gr.GR_LOOP_PERSISTENT, gr.GR_LOOP_QUEUED, gr.GR_LOOP_ASYNC) + (
            (gr.GR_LOOP_LDS,) if lds else ())
        for src, dist, hops in queries:
            for lay in layouts:
                for d in dirs:
                    for lp in loops:
                        if lp in (gr.GR_LOOP_ASYNC, gr.GR_LOOP_LDS) and d not in (gr.GR_DIR_PUSH, gr.GR_DIR_AUTO):
                            continue  # the asynchronous and single-workgroup loops are push-only
                        for rf in (gr.GR_RELAX_DIST, gr.GR_RELAX_BOUND):
                            tag = "%s src=%d layout=%d dir=%d loop=%d relax=%d" % (name, src, lay, d, lp, rf)
                            say("golden " + tag)
                            out = fresh(g.n)
                            kw = dict(barrier_timeout_us=5_000_000) if lp != gr.GR_LOOP_HOST else {}
                            gr.gr_sssp_ex(G.handle, src, out, loop=lp, direction=d, layout=lay, relax_filter=rf,
                                          **kw)
                            np.testing.assert_array_equal(host(out), dist, err_msg=tag)
            for lp in (gr.GR_LOOP_HOST, gr.GR_LOOP_QUEUED, gr.GR_LOOP_ASYNC, gr.GR_LOOP_LDS):
                say("golden bfs %s src=%d loop=%d" % (name, src, lp))
                out = fresh(g.n)
                kw = dict(barrier_timeout_us=5_000_000) if lp != gr.GR_LOOP_HOST else {}
                gr.gr_bfs_ex(G.handle, src, out, loop=lp, **kw)
                np.testing.assert_array_equal(host(out), hops, err_msg="bfs %s src=%d loop=%d" % (name, src, lp))
        srcs = [q[0] for q in queries]
        say("golden batch %s sources=%s" % (name, srcs))
        out = torch.full((len(srcs), g.n), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
        gr.gr_sssp_batch(G.handle, np.asarray(srcs, np.int32), out)
        got = host(out)
        for i, (src, dist, _) in enumerate(queries):
            np.testing.assert_array_equal(got[i], dist, err_msg="batch %s src=%d" % (name, src))
    finally:
        G.close()


def test_golden_fixtures_served():
    # every fixture query, submitted four times over in an interleaved stream to
    # one server holding all fixture graphs, so that queries can share batches
    import time
    loaded = [golden_fixtures.load(nm) for nm in golden_fixtures.names()]
    Gs = [gr.Graph.from_csr(g) for g, _ in loaded]
    server = gr.gr_server_create(1 << 30, max_batch=8, num_streams=2, max_wait_us=500)
    try:
        gids = [gr.gr_server_add_graph(server, G.handle) for G in Gs]
        reqs = []
        for rep in range(4):
            for gi, (g, queries) in enumerate(loaded):
                for src, dist, _ in queries:
                    out = fresh(g.n)
                    reqs.append((gr.gr_serve_submit(server, gids[gi], src, out), gi, src, dist, out))
        say("golden served: %d queries on %d graphs" % (len(reqs), len(Gs)))
        pending = {r[0] for r in reqs}
        res = {}
        t0 = time.time()
        while pending:
            for t in list(pending):
                r = gr.gr_serve_poll(server, t)
                if r is not None:
                    res[t] = r
                    pending.discard(t)
            assert time.time() - t0 < 60, "%d served queries pending" % len(pending)
            time.sleep(0.0005)
        for t, gi, src, dist, out in reqs:
            assert res[t]["status"] == gr.GR_OK and res[t]["graph_id"] == gids[gi] and res[t]["src"] == src
            np.testing.assert_array_equal(host(out), dist, err_msg="served %s src=%d" % (loaded[gi][0].name, src))
    finally:
        gr.gr_server_destroy(server)
        for G in Gs:
            G.close()
