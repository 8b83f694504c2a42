"""GPU parity: distances from the HIP path through the C ABI equal the CPU
oracle bit for bit (tolerance 0, for uint32 and binary32 weights alike --
the shortest-path vector is unique, see ``include/gr.h``), for every traversal
schedule, on the benchmark configurations and on edge cases.
"""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from certify_rows import certify_all, dijkstra_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
gr = pytest.importorskip("paper_2212_08200_amd")

DIRS = {"push": 1, "auto": 0, "pull": 2, "alternate": 3}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run(G, src, direction=0, loop=0, n=None, layout=0, filt=0, delta=0, relax=0, hops=0):
    dist = torch.full((n or G.n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    st = gr.gr_sssp_ex(G.handle, int(src), dist, direction=direction, loop=loop, layout=layout, filter=filt,
                       delta=delta, relax_filter=relax, local_hops=hops)
    torch.cuda.synchronize()
    return dist.cpu().numpy().view(np.uint32), st


def assert_same(got, want, tag):
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        v = int(bad[0])
        raise AssertionError("%s: %d mismatches, first vertex %d got 0x%08x want 0x%08x" % (
            tag, len(bad), v, int(got[v]), int(want[v])))


LOOPS = {"host": 1, "persistent": 2, "queued": 3}
RELAX = (gr.GR_RELAX_DIST, gr.GR_RELAX_BOUND)


def check_all_dirs(g, srcs, tag, dirs=("push", "auto", "pull", "alternate"), flags=gr.GR_FORCE_PARTITION,
                   loops=("host", "persistent", "queued")):
    """Every direction policy, with both push layouts (plain CSR and partitioned),
    every loop driver (host-driven, device-driven persistent, queued) and both
    relaxation filters of push."""
    G = gr.Graph.from_csr(g, flags=flags)
    info = G.info()
    layouts = [gr.GR_LAYOUT_PLAIN] + ([gr.GR_LAYOUT_PARTITIONED] if info["partitions"] > 1 else [])
    try:
        for s in srcs:
            want = oracle.dijkstra(g, int(s))
            for lay in layouts:
                for d in dirs:
                    if d in ("pull", "alternate") and not info["pull_enabled"]:
                        continue
                    for lp in loops:
                        for rf in RELAX if d != "pull" else RELAX[:1]:
                            say("case %s src=%d dir=%s layout=%d loop=%s relax=%d n=%d m=%d" % (
                                tag, s, d, lay, lp, rf, g.n, g.m))
                            got, st = run(G, s, DIRS[d], layout=lay, loop=LOOPS[lp], relax=rf)
                            assert_same(got, want, "%s src %d dir %s layout %d loop %s relax %d" % (
                                tag, s, d, lay, lp, rf))
                            assert st["loop"] == LOOPS[lp]
    finally:
        G.close()


# ------------------------------------------------------------------ small cases

def test_grid64_config():
    g, srcs = gg.workload("grid64")
    check_all_dirs(g, [int(srcs[0]), 4095, 2080], "grid64")


@pytest.mark.parametrize("wtype", [gg.W_U32, gg.W_F32])
def test_rmat12_both_types(wtype):
    g = gg.rmat(12, 16, gseed=61, pseed=62, wseed=63, wtype=wtype)
    srcs = gg.pick_sources(g, 64, 3)
    check_all_dirs(g, srcs, "rmat12_w%d" % wtype)


@pytest.mark.parametrize("seed", [1, 2])
def test_uniform_directed_with_zero_weights(seed):
    g = gg.uniform(5000, 30000, gseed=seed, wseed=seed + 10, wtype=gg.W_U32, wlo=0, whi=3)
    check_all_dirs(g, [0, 17, 4999], "uniform%d" % seed)


def test_uniform_directed_f32():
    g = gg.uniform(3000, 20000, gseed=5, wseed=6, wtype=gg.W_F32)
    check_all_dirs(g, [0, 1234], "uniform_f32")


def test_road_like_small():
    g = gg.grid(200, wseed=71, wtype=gg.W_U32, wlo=1, whi=1000, shortcuts=40, sseed=72)
    check_all_dirs(g, [0, 199 * 200 + 199], "road200")


def test_edge_cases():
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
        ("f32_negzero", gg.from_arcs(3, [(0, 1, -0.0), (1, 2, 0.5)], wtype=gg.W_F32), 0),
        ("star_hub", gg.from_arcs(70001, [(0, i, i % 97 + 1) for i in range(1, 70001)]), 0),
    ]
    for name, g, s in cases:
        check_all_dirs(g, [s], name)


def test_ragged_group_boundaries():
    # n just above multiples of the 4096-vertex bitmap group and the 256-vertex pull block
    for n in (4097, 8191, 257):
        g = gg.uniform(n, 6 * n, gseed=n, wseed=n + 1, wtype=gg.W_U32, wlo=1, whi=9)
        check_all_dirs(g, [0, n - 1], "ragged%d" % n)


def test_repeat_determinism():
    g = gg.rmat(13, 16, gseed=81, pseed=82, wseed=83, wtype=gg.W_F32)
    s = int(gg.pick_sources(g, 84, 1)[0])
    want = oracle.dijkstra(g, s)
    G = gr.Graph.from_csr(g, flags=gr.GR_FORCE_PARTITION)
    try:
        for i in range(10):
            got, _ = run(G, s, DIRS["auto"], layout=gr.GR_LAYOUT_PARTITIONED if i % 2 else gr.GR_LAYOUT_PLAIN)
            assert_same(got, want, "repeat %d" % i)
    finally:
        G.close()


def test_device_input_graph():
    g = gg.rmat(11, 16, gseed=91, pseed=92, wseed=93, wtype=gg.W_U32)
    ro = torch.from_numpy(g.ro.copy()).cuda()
    col = torch.from_numpy(g.col.copy()).cuda()
    w = torch.from_numpy(g.w.view(np.int32).copy()).cuda()
    h = gr.gr_graph_create_csr(g.n, g.m, ro, col, w, g.wtype, gr.GR_INPUT_DEVICE)
    try:
        s = int(gg.pick_sources(g, 94, 1)[0])
        dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
        gr.gr_sssp(h, s, dist)
        torch.cuda.synchronize()
        assert_same(dist.cpu().numpy().view(np.uint32), oracle.dijkstra(g, s), "device input")
    finally:
        gr.gr_graph_destroy(h)
    bad = torch.from_numpy(np.array([0, 1, 5], np.int32)).cuda()
    with pytest.raises(gr.GrError) as ei:
        gr.gr_graph_create_csr(2, 2, bad, col[:2], w[:2], 0, gr.GR_INPUT_DEVICE)
    assert ei.value.status == gr.GR_ERR_INVALID_ARG


def test_persistent_loop_stats_match_host_loop():
    # both drivers run the same rounds on a deterministic-size workload (a directed path)
    L = 300
    g = gg.from_arcs(L + 1, [(i, i + 1, 1 + i % 7) for i in range(L)])
    G = gr.Graph.from_csr(g)
    try:
        a = run(G, 0, DIRS["push"], loop=LOOPS["host"])[1]
        for lp, filt in (("persistent", 0), ("queued", 0), ("queued", 3), ("queued", 3)):
            # queued twice with small rounds: the second starts from a predicted chunk;
            # one hop per round, so that every round is one level of the path
            b = run(G, 0, DIRS["push"], loop=LOOPS[lp], filt=filt, hops=1)[1]
            assert a["iterations"] == b["iterations"] == L, lp
            assert a["edges_pushed"] == b["edges_pushed"] == L, lp
            assert a["frontier_sum"] == b["frontier_sum"] == L, lp
            assert a["push_frontier_sum"] == b["push_frontier_sum"] == L, lp
            if filt == 3:  # one improved vertex per round: rounds after the first skip the filter
                assert b["small_rounds"] >= L - 2
        # four local hops per small round: the path takes a quarter of the rounds,
        # every arc still relaxed once
        c = run(G, 0, DIRS["push"], loop=LOOPS["queued"], filt=3, hops=4)[1]
        assert c["edges_pushed"] == L
        assert L // 4 <= c["iterations"] <= L // 4 + 4, c["iterations"]
        dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
        for lp in ("host", "persistent", "queued"):
            st = gr.gr_sssp_ex(G.handle, 0, dist, loop=LOOPS[lp], timing=1, local_hops=1)
            torch.cuda.synchronize()
            assert st["push_us"] > 0 and st["iterations"] == L, lp
    finally:
        G.close()


def test_direction_switch_alpha_beta_rules():
    """AUTO switching (Beamer et al.'s two rules): push -> pull once the frontier's
    out-arcs reach m / alpha, pull -> push once the frontier holds fewer than
    n / beta vertices.  beta = 1 leaves pull after every pull round; a huge beta
    keeps pulling to the end.  Both pulls (over the partitioned layout and over
    the transposed copy) and every loop driver give the oracle's distances."""
    g = gg.rmat(14, 16, gseed=41, pseed=42, wseed=43)
    G = gr.Graph.from_csr(g, flags=gr.GR_FORCE_PARTITION)
    try:
        dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
        for s in [int(x) for x in gg.pick_sources(g, 44, 2)]:
            want = oracle.dijkstra(g, s)
            for lay in (gr.GR_LAYOUT_PLAIN, gr.GR_LAYOUT_PARTITIONED):
                for lp in ("host", "persistent", "queued"):
                    pulls = {}
                    for beta in (1, 1 << 30):
                        say("alpha/beta rmat14 src=%d layout=%d loop=%s beta=%d" % (s, lay, lp, beta))
                        st = gr.gr_sssp_ex(G.handle, s, dist, loop=LOOPS[lp], layout=lay, alpha_x16=64, beta=beta)
                        torch.cuda.synchronize()
                        assert_same(dist.cpu().numpy().view(np.uint32), want, "alpha/beta %s beta %d" % (lp, beta))
                        pulls[beta] = (st["pull_iterations"], st["iterations"])
                    p1, it1 = pulls[1]
                    pb, itb = pulls[1 << 30]
                    assert p1 >= 1, "the alpha rule never switched to pull"
                    assert p1 <= (it1 + 1) // 2, "beta = 1 pulled twice in a row"
                    assert pb >= p1 and pb >= 2  # a huge beta keeps pulling once it started
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_ex(G.handle, 0, dist, beta=-1)
        assert ei.value.status == gr.GR_ERR_INVALID_ARG
    finally:
        G.close()


def test_persistent_barrier_timeout_reports_error_then_recovers():
    # a 1 us bound on each grid-barrier wait cannot be met by a real round: the
    # device-driven loop must end (every block leaves) and report GR_ERR_HIP
    g = gg.grid(300, wseed=3)
    want = oracle.dijkstra(g, 0)
    G = gr.Graph.from_csr(g)
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    try:
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_ex(G.handle, 0, dist, loop=LOOPS["persistent"], barrier_timeout_us=1)
        assert ei.value.status == gr.GR_ERR_HIP and "barrier" in ei.value.message
        got, _ = run(G, 0, DIRS["push"], loop=LOOPS["persistent"])
        assert_same(got, want, "after a timed-out query")
    finally:
        G.close()


def test_errors_on_gpu():
    g = gg.grid(8, wseed=1)
    G = gr.Graph.from_csr(g)
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    try:
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp(G.handle, g.n, dist)
        assert ei.value.status == gr.GR_ERR_SOURCE_RANGE
        for lp in (1, 2, 3):
            with pytest.raises(gr.GrError) as ei:
                gr.gr_sssp_ex(G.handle, 0, dist, max_iters=3, loop=lp)
            assert ei.value.status == gr.GR_ERR_ITER_LIMIT
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_ex(G.handle, 0, dist, loop=6)  # past the last loop mode
        assert ei.value.status == gr.GR_ERR_INVALID_ARG
        for rf in (-1, 3):
            with pytest.raises(gr.GrError) as ei:
                gr.gr_sssp_ex(G.handle, 0, dist, relax_filter=rf)
            assert ei.value.status == gr.GR_ERR_INVALID_ARG
    finally:
        G.close()
    Gp = gr.Graph.from_csr(g, flags=gr.GR_NO_PULL)
    try:
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_ex(Gp.handle, 0, dist, direction=gr.GR_DIR_PULL)
        assert ei.value.status == gr.GR_ERR_INVALID_ARG
    finally:
        Gp.close()


@pytest.mark.parametrize("wtype", [gg.W_U32, gg.W_F32])
def test_both_filters_both_layouts(wtype):
    # the group filter and the streaming filter build the same frontiers
    g = gg.rmat(14, 16, gseed=31 + wtype, pseed=32, wseed=33, wtype=wtype)
    G = gr.Graph.from_csr(g, flags=gr.GR_FORCE_PARTITION)
    try:
        for s in gg.pick_sources(g, 34, 2):
            want = oracle.dijkstra(g, int(s))
            for lay in (gr.GR_LAYOUT_PLAIN, gr.GR_LAYOUT_PARTITIONED):
                for filt in (1, 2):
                    for d in (DIRS["push"], DIRS["alternate"]):
                        say("filters rmat14 w%d src=%d layout=%d filter=%d dir=%d" % (wtype, s, lay, filt, d))
                        got, _ = run(G, s, d, layout=lay, filt=filt)
                        assert_same(got, want, "filter %d layout %d dir %d" % (filt, lay, d))
    finally:
        G.close()


def test_partition_layout_default_choice():
    # random ids (R-MAT) and large n: partitioned; grid: neighbours are close, plain only
    g = gg.rmat(17, 8, gseed=5, pseed=6, wseed=7)
    G = gr.Graph.from_csr(g)
    assert G.info()["partitions"] == 8
    G.close()
    g = gg.grid(400, wseed=8)
    G = gr.Graph.from_csr(g)
    assert G.info()["partitions"] == 1
    G.close()
    G = gr.Graph.from_csr(gg.grid(8, wseed=1), flags=gr.GR_NO_PARTITION)
    dist = torch.empty(64, dtype=torch.int32, device="cuda")
    with pytest.raises(gr.GrError) as ei:
        gr.gr_sssp_ex(G.handle, 0, dist, layout=gr.GR_LAYOUT_PARTITIONED)
    assert ei.value.status == gr.GR_ERR_INVALID_ARG
    G.close()


def test_symmetry_detection():
    sym = gg.rmat(10, 8, gseed=1, pseed=2, wseed=3)
    G = gr.Graph.from_csr(sym)
    assert G.info()["has_csc"] is False and G.info()["pull_enabled"]
    G.close()
    asym = gg.grid(16, wseed=4)  # one weight per directed arc: not symmetric
    G = gr.Graph.from_csr(asym)
    assert G.info()["has_csc"] is True
    G.close()


# ------------------------------------------------------------- benchmark configs

def test_rmat20_config_f32():
    g, srcs = gg.workload("rmat20")
    check_all_dirs(g, srcs, "rmat20", dirs=("auto", "push", "pull"), flags=0)


def test_road2048_config():
    g, srcs = gg.workload("road2048")
    check_all_dirs(g, srcs, "road2048", dirs=("auto",), flags=0)


def test_grid2048_config_device_loops():
    g, srcs = gg.workload("grid2048")
    check_all_dirs(g, srcs, "grid2048", dirs=("push",), flags=0, loops=("persistent", "queued"))


def test_rmat22_config_sampled_sources():
    g, srcs = gg.workload("rmat22")
    check_all_dirs(g, srcs[:2], "rmat22", dirs=("auto", "push"), flags=0)


def test_rmat22_all_bench_sources_tuned_schedule():
    """The benchmark's workload exactly: the graph tuned as the benchmark tunes
    it, then every one of its 64 sources through gr_sssp (the tuned AUTO
    schedule), each result certified; four also equal the oracle's Dijkstra."""
    g, srcs = gg.workload("rmat22")
    G = gr.Graph.from_csr(g)
    try:
        tuned = G.tune([int(s) for s in srcs[:4]], reps=2)
        say("rmat22 tuned schedule: %s" % tuned)
        rows = []
        for i, s in enumerate(srcs):
            d = torch.full((g.n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
            gr.gr_sssp(G.handle, int(s), d)
            torch.cuda.synchronize()
            rows.append(d.cpu().numpy().view(np.uint32))
        say("rmat22: certificate on all 64 tuned results")
        certify_all(g, srcs, rows, "rmat22 tuned", workers=12)
        say("rmat22: Dijkstra on 4 tuned results")
        dijkstra_rows(g, srcs, rows, (0, 17, 38, 63), "rmat22 tuned")
    finally:
        G.close()


def test_rmat22_asynchronous_loop():
    g, srcs = gg.workload("rmat22")
    G = gr.Graph.from_csr(g)
    try:
        rows = []
        for s in srcs[:3]:
            say("rmat22 asynchronous loop src=%d" % int(s))
            got, st = run(G, s, DIRS["push"], loop=gr.GR_LOOP_ASYNC)
            assert st["loop"] == gr.GR_LOOP_ASYNC
            rows.append(got)
        certify_all(g, srcs[:3], rows, "rmat22 async")
        dijkstra_rows(g, srcs[:3], rows, (0, 2), "rmat22 async")
    finally:
        G.close()


# ------------------------------------------------------------ near-far split

@pytest.mark.parametrize("wtype", [gg.W_U32, gg.W_F32])
def test_near_far_split_all_loops_filters(wtype):
    # held-back vertices, threshold raises and both filters, under every loop
    # driver; widths from below one weight to above the diameter
    graphs = [("rmat13", gg.rmat(13, 16, gseed=41, pseed=42, wseed=43, wtype=wtype), gr.GR_FORCE_PARTITION),
              ("grid48", gg.grid(48, wseed=44, wtype=wtype), 0)]
    for tag, g, flags in graphs:
        G = gr.Graph.from_csr(g, flags=flags)
        info = G.info()
        layouts = [gr.GR_LAYOUT_PLAIN] + ([gr.GR_LAYOUT_PARTITIONED] if info["partitions"] > 1 else [])
        mean_w = float(np.mean(g.w.view(np.float32))) if wtype == gg.W_F32 else float(np.mean(g.w))
        try:
            for s in gg.pick_sources(g, 45, 2):
                want = oracle.dijkstra(g, int(s))
                for f in (0.5, 4.0, 1e6):
                    d = gr.delta_bits(mean_w * f if wtype == gg.W_F32 else max(1, int(mean_w * f)), wtype)
                    for lay in layouts:
                        for lp in ("host", "persistent", "queued"):
                            for filt in (0, 1, 2):
                                rf = RELAX[filt % 2]
                                say("near-far %s w%d src=%d delta=%#x layout=%d loop=%s filter=%d relax=%d" % (
                                    tag, wtype, s, d, lay, lp, filt, rf))
                                got, st = run(G, s, DIRS["push"], layout=lay, loop=LOOPS[lp], filt=filt, delta=d,
                                              relax=rf)
                                assert_same(got, want, "near-far %s delta %#x layout %d loop %s filter %d" % (
                                    tag, d, lay, lp, filt))
        finally:
            G.close()


def test_near_far_cuts_relaxations_and_rejects_bad_widths():
    g = gg.grid(64, wseed=2)  # uint32 U[1,100]
    G = gr.Graph.from_csr(g)
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    try:
        base = run(G, 0, DIRS["push"], loop=LOOPS["host"])[1]
        split = run(G, 0, DIRS["push"], loop=LOOPS["host"], delta=50)[1]
        assert split["edges_pushed"] < base["edges_pushed"]
        assert split["iterations"] > base["iterations"]
        off = run(G, 0, DIRS["push"], loop=LOOPS["host"], delta=gr.GR_DELTA_OFF)[1]
        assert off["edges_pushed"] == base["edges_pushed"]
        for d in (gr.GR_DIR_PULL, gr.GR_DIR_ALTERNATE):
            with pytest.raises(gr.GrError) as ei:
                gr.gr_sssp_ex(G.handle, 0, dist, direction=d, delta=50)
            assert ei.value.status == gr.GR_ERR_INVALID_ARG
    finally:
        G.close()
    gf = gg.grid(16, wseed=3, wtype=gg.W_F32)
    Gf = gr.Graph.from_csr(gf)
    try:
        for bits in (0x7FC00000, 0x7F800000, 0x80000001):  # NaN, +inf, -denormal
            with pytest.raises(gr.GrError) as ei:
                gr.gr_sssp_ex(Gf.handle, 0, dist[:gf.n], delta=bits)
            assert ei.value.status == gr.GR_ERR_INVALID_ARG
    finally:
        Gf.close()


def test_near_far_configs():
    g, srcs = gg.workload("road2048")
    G = gr.Graph.from_csr(g)
    try:
        want = oracle.dijkstra(g, int(srcs[0]))
        for lp in ("host", "queued"):
            say("near-far road2048 loop=%s" % lp)
            got, st = run(G, srcs[0], DIRS["push"], loop=LOOPS[lp], delta=2000)
            assert_same(got, want, "road2048 near-far loop %s" % lp)
    finally:
        G.close()
    g, srcs = gg.workload("rmat20")  # fp32 weights in (0, 1]
    G = gr.Graph.from_csr(g)
    try:
        want = oracle.dijkstra(g, int(srcs[0]))
        for lp in ("host", "queued"):
            say("near-far rmat20 loop=%s" % lp)
            got, _ = run(G, srcs[0], DIRS["push"], loop=LOOPS[lp], delta=gr.delta_bits(0.25, gg.W_F32))
            assert_same(got, want, "rmat20 near-far loop %s" % lp)
    finally:
        G.close()


# ------------------------------------------------- queued loop: small rounds

def test_small_rounds_thread_and_block_mapped():
    # grids: every vertex thread-mapped; R-MAT: hubs go to the block-mapped
    # path; filter 1 / 2 turn small rounds off and must agree
    cases = [("grid300", gg.grid(300, wseed=21)), ("rmat14", gg.rmat(14, 16, gseed=22, pseed=23, wseed=24)),
             ("rmat13f", gg.rmat(13, 16, gseed=25, pseed=26, wseed=27, wtype=gg.W_F32)),
             ("road", gg.grid(200, wseed=29, whi=1000, shortcuts=40, sseed=28))]
    for tag, g in cases:
        G = gr.Graph.from_csr(g, flags=gr.GR_FORCE_PARTITION)
        try:
            for s in gg.pick_sources(g, 30, 2):
                want = oracle.dijkstra(g, int(s))
                for filt, rf in ((3, 1), (3, 2), (0, 0), (1, 2), (2, 1)):
                    say("small rounds %s src=%d filter=%d relax=%d" % (tag, s, filt, rf))
                    got, st = run(G, s, DIRS["push"], loop=LOOPS["queued"], filt=filt, relax=rf)
                    assert_same(got, want, "%s src %d filter %d relax %d" % (tag, s, filt, rf))
                    if filt in (1, 2):
                        assert st["small_rounds"] == 0
                    elif tag.startswith("grid"):  # bounded degree: small rounds by default too
                        assert st["small_rounds"] > st["iterations"] // 2
        finally:
            G.close()


def test_small_rounds_candidate_overflow():
    # a tree with fan-out 64, then 2: its last round improves 524,288 vertices,
    # more than a candidate list holds (2^18), so that round's next frontier
    # comes from the flag scan; earlier rounds run as small rounds
    rng = np.random.default_rng(7)
    src, dst = [], []
    level, nxt = [0], 1
    for fan in (64, 64, 64, 2):
        for u in level:
            src.extend([u] * fan)
            dst.extend(range(nxt, nxt + fan))
            nxt += fan
        level = list(range(nxt - len(level) * fan, nxt))
    n = nxt
    w = rng.integers(1, 50, size=len(src))
    g = gg.from_arcs(n, list(zip(src, dst, w.tolist())))
    G = gr.Graph.from_csr(g)
    try:
        want = oracle.dijkstra(g, 0)
        got, st = run(G, 0, DIRS["push"], loop=LOOPS["queued"], filt=3, hops=1)
        assert_same(got, want, "tree overflow")
        got4, _ = run(G, 0, DIRS["push"], loop=LOOPS["queued"], filt=3, hops=4)
        assert_same(got4, want, "tree overflow, local hops")
        ref = run(G, 0, DIRS["push"], loop=LOOPS["host"])[1]
        assert st["iterations"] == ref["iterations"] and st["edges_pushed"] == ref["edges_pushed"]
        assert st["small_rounds"] >= 1
    finally:
        G.close()


@pytest.mark.parametrize("hops", [2, 5, 16])
def test_small_rounds_local_hops(hops):
    """Small rounds with local hops (a block expands the vertices it improved
    again, with the improving distance, before the next round): oracle
    distances on bounded-degree graphs (grids with and without shortcuts,
    directed graphs with zero weights, binary32), fewer rounds than without."""
    cases = [("grid96", gg.grid(96, 51, whi=1000)),
             ("road256", gg.grid(256, 52, whi=1000, shortcuts=65, sseed=53)),
             ("uniform", gg.uniform(5000, 15000, 54, 55, wlo=0, whi=4)),
             ("grid80 f32", gg.grid(80, 56, wtype=gg.W_F32))]
    for tag, g in cases:
        G = gr.Graph.from_csr(g)
        try:
            for s in [0] + [int(x) for x in gg.pick_sources(g, 57, 2)]:
                want = oracle.dijkstra(g, s)
                say("local hops %d: %s src=%d" % (hops, tag, s))
                got1, st1 = run(G, s, DIRS["push"], loop=LOOPS["queued"], filt=3, hops=1)
                dist = torch.full((g.n,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
                st = gr.gr_sssp_ex(G.handle, s, dist, loop=LOOPS["queued"], direction=DIRS["push"], filter=3,
                                   local_hops=hops)
                torch.cuda.synchronize()
                assert_same(dist.cpu().numpy().view(np.uint32), want, "%s src %d hops %d" % (tag, s, hops))
                assert_same(got1, want, "%s src %d hops 1" % (tag, s))
                if tag.startswith("grid") and s == 0:
                    assert st["iterations"] < st1["iterations"], (st["iterations"], st1["iterations"])
        finally:
            G.close()
    g = gg.grid(8, 3)
    G = gr.Graph.from_csr(g)
    try:
        dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
        with pytest.raises(gr.GrError) as ei:
            gr.gr_sssp_ex(G.handle, 0, dist, local_hops=65)
        assert ei.value.status == gr.GR_ERR_INVALID_ARG
    finally:
        G.close()
