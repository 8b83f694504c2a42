"""Pins for the CPU oracle: closed forms, exhaustive enumeration, independent
brute force, library routines and the invariant certificate.

The shortest-path vector is the definition the paper's SSSP reaches
(Section IV-D, Listing 4): dist[v] = min over paths of the left fold
((0 + w1) + w2) ... in the weight type, dist[src] = 0, INF when unreachable.
"""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import golden_fixtures
import graphgen as gg
import oracle
from oracle import brute

INF = oracle.INF_U32
FINF = oracle.INF_F32_BITS


def f32bits(x):
    return int(np.array([x], dtype=np.float32).view(np.uint32)[0])


def as_f32(bits):
    return np.asarray(bits, dtype=np.uint32).view(np.float32)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("side", [1, 2, 5, 17])
def test_unit_grid_is_manhattan(side):
    g = gg.grid(side, wseed=0, wtype=gg.W_U32, wlo=1, whi=1)
    for src in {0, side * side - 1, (side // 2) * side + side // 3}:
        d = oracle.dijkstra(g, src)
        sr, sc = divmod(src, side)
        r, c = np.divmod(np.arange(side * side), side)
        np.testing.assert_array_equal(d, np.abs(r - sr) + np.abs(c - sc))


def test_constant_grid_is_scaled_manhattan_u32_and_f32():
    side = 12
    gu = gg.grid(side, wseed=0, wtype=gg.W_U32, wlo=7, whi=7)
    r, c = np.divmod(np.arange(side * side), side)
    np.testing.assert_array_equal(oracle.dijkstra(gu, 0), 7 * (r + c))
    # binary32 weight 2^-3: every prefix k/8 is exact, so the fold is k/8 exactly
    arcs = [(u, int(gu.col[e]), 0.125) for u in range(gu.n) for e in range(gu.ro[u], gu.ro[u + 1])]
    gf = gg.from_arcs(gu.n, arcs, wtype=gg.W_F32)
    np.testing.assert_array_equal(as_f32(oracle.dijkstra(gf, 0)), ((r + c) * 0.125).astype(np.float32))


def test_path_graph_is_prefix_fold_f32():
    # directed path 0 -> 1 -> ... -> L; only one path per vertex, so dist is the running
    # binary32 sum in path order (np.cumsum on float32 accumulates sequentially in float32)
    rng = np.random.default_rng(11)
    L = 300
    w = rng.random(L, dtype=np.float32) * np.float32(3.0) + np.float32(1e-3)
    g = gg.from_arcs(L + 1, [(i, i + 1, w[i]) for i in range(L)], wtype=gg.W_F32)
    want = np.concatenate([[np.float32(0)], np.cumsum(w, dtype=np.float32)])
    np.testing.assert_array_equal(as_f32(oracle.dijkstra(g, 0)), want)
    # a binary64 accumulation differs somewhere, so this pins the precision of (+)
    want64 = np.concatenate([[0.0], np.cumsum(w.astype(np.float64))]).astype(np.float32)
    assert (want64 != want).any()


def test_fp32_rounding_order_hand_example():
    # 0 -> 1 (1.0), 1 -> 2 (2^-24), 2 -> 3 (2^-24), and a direct arc 0 -> 3 of 1 + 2^-23.
    # Along the path: 1 + 2^-24 is a tie between 1 and 1 + 2^-23 and rounds to even (1.0),
    # twice, so the fold is exactly 1.0 and beats the direct arc.  An exact (or binary64)
    # sum would give 1 + 2^-23, a tie with the direct arc.
    e24 = 2.0 ** -24
    g = gg.from_arcs(4, [(0, 1, 1.0), (1, 2, e24), (2, 3, e24), (0, 3, 1.0 + 2 * e24)], wtype=gg.W_F32)
    d = as_f32(oracle.dijkstra(g, 0))
    assert d[3] == np.float32(1.0)
    assert d[2] == np.float32(1.0)
    assert d[1] == np.float32(1.0)
    # (1 + 2^-23) + 2^-24 is a tie between 1 + 2^-23 (odd) and 1 + 2^-22 (even): rounds up
    g2 = gg.from_arcs(3, [(0, 1, 1.0 + 2 * e24), (1, 2, e24)], wtype=gg.W_F32)
    assert as_f32(oracle.dijkstra(g2, 0))[2] == np.float32(1.0 + 4 * e24)


@pytest.mark.parametrize("name", golden_fixtures.names())
def test_hand_derived_golden_fixtures(name):
    # distances and hop counts worked out by hand in tests/golden/ (the paper
    # prints no numeric example); the BSP loop must reach the same fixed point
    g, queries = golden_fixtures.load(name)
    assert queries
    for src, dist, hops in queries:
        np.testing.assert_array_equal(oracle.dijkstra(g, src), dist, err_msg="%s from %d" % (name, src))
        np.testing.assert_array_equal(oracle.bsp(g, src)[0], dist, err_msg="bsp %s from %d" % (name, src))
        np.testing.assert_array_equal(oracle.bfs(g, src), hops, err_msg="bfs %s from %d" % (name, src))


def test_golden_fixture_inf_encodings_match_the_oracle():
    assert golden_fixtures.INF_U32 == oracle.inf_bits(gg.W_U32)
    assert golden_fixtures.INF_F32_BITS == oracle.inf_bits(gg.W_F32)


def test_star_and_components_and_isolated_source():
    # star: 0 -> i with weight i; vertices 6..9 form a separate component
    arcs = [(0, i, i) for i in range(1, 6)] + [(6, 7, 1), (7, 8, 1), (8, 9, 1), (9, 6, 1)]
    g = gg.from_arcs(10, arcs)
    d = oracle.dijkstra(g, 0)
    np.testing.assert_array_equal(d[:6], np.arange(6))
    assert (d[6:] == INF).all()
    # a source with out-degree 0 reaches only itself
    d5 = oracle.dijkstra(g, 5)
    assert d5[5] == 0 and (np.delete(d5, 5) == INF).all()
    # single vertex
    g1 = gg.from_arcs(1, [])
    np.testing.assert_array_equal(oracle.dijkstra(g1, 0), [0])


def test_self_loops_parallel_arcs_zero_weights():
    arcs = [(0, 0, 0), (0, 1, 9), (0, 1, 4), (1, 1, 3), (1, 2, 0), (2, 0, 0), (2, 3, 0), (3, 2, 5)]
    g = gg.from_arcs(4, arcs)
    np.testing.assert_array_equal(oracle.dijkstra(g, 0), [0, 4, 4, 4])
    np.testing.assert_array_equal(oracle.dijkstra(g, 3), [5, 9, 5, 0])


def test_u32_saturation_reports_inf():
    big = INF - 5
    g = gg.from_arcs(4, [(0, 1, big), (1, 2, 3), (2, 3, 7)])
    d = oracle.dijkstra(g, 0)
    assert d[1] == big and d[2] == big + 3
    assert d[3] == INF  # fold passes 2^32 - 1: reported unreachable


def test_f32_overflow_reports_inf():
    fm = float(np.finfo(np.float32).max)
    g = gg.from_arcs(3, [(0, 1, fm / 2), (1, 2, fm)], wtype=gg.W_F32)
    d = oracle.dijkstra(g, 0)
    assert as_f32(d)[1] == np.float32(fm / 2)
    assert d[2] == FINF


def test_bsp_rounds_on_directed_path():
    L = 20
    g = gg.from_arcs(L + 1, [(i, i + 1, 1) for i in range(L)])
    d, stt = oracle.bsp(g, 0)
    np.testing.assert_array_equal(d, np.arange(L + 1))
    assert stt["rounds"] == L + 1  # {0}, {1}, ..., {L}, then empty
    assert stt["relaxations"] == L
    assert stt["frontier_max"] == 1


# ------------------------------------------------------- exhaustive / brute force

@st.composite
def tiny_graphs(draw, max_n=7, wtype=gg.W_U32):
    n = draw(st.integers(1, max_n))
    k = draw(st.integers(0, 3 * n))
    if wtype == gg.W_U32:
        wst = st.one_of(st.integers(0, 5), st.integers(0, 1000))
    else:
        wst = st.one_of(st.sampled_from([0.0, 2.0 ** -24, 0.1, 1.0, 1.0 + 2.0 ** -23]),
                        st.floats(0.0, 10.0, width=32))
    arcs = [(draw(st.integers(0, n - 1)), draw(st.integers(0, n - 1)), draw(wst)) for _ in range(k)]
    src = draw(st.integers(0, n - 1))
    return gg.from_arcs(n, arcs, wtype=wtype), src


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_graphs(wtype=gg.W_U32))
def test_dijkstra_equals_path_enumeration_u32(case):
    g, src = case
    want = brute.paths_min(g, src)
    np.testing.assert_array_equal(oracle.dijkstra(g, src), want)
    np.testing.assert_array_equal(brute.bellman_ford(g, src), want)
    np.testing.assert_array_equal(oracle.bsp(g, src)[0], want)
    assert oracle.certify(g, src, want)[0] == 0


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(tiny_graphs(wtype=gg.W_F32))
def test_dijkstra_equals_path_enumeration_f32(case):
    g, src = case
    want = brute.paths_min(g, src)
    np.testing.assert_array_equal(oracle.dijkstra(g, src), want)
    np.testing.assert_array_equal(brute.bellman_ford(g, src), want)
    np.testing.assert_array_equal(oracle.bsp(g, src)[0], want)
    assert oracle.certify(g, src, want)[0] == 0


@pytest.mark.parametrize("seed", range(6))
def test_dijkstra_equals_floyd_warshall(seed):
    gu = gg.uniform(40, 160, gseed=seed, wseed=100 + seed, wtype=gg.W_U32, wlo=0, whi=50)
    fw = brute.floyd_warshall(gu)
    for s in range(0, 40, 7):
        np.testing.assert_array_equal(oracle.dijkstra(gu, s), fw[s])
    # binary32 with integer-valued weights: every partial sum exact, so re-association is harmless
    ints = gu.w.astype(np.float32)
    gf = gg.CSR(n=gu.n, ro=gu.ro, col=gu.col, w=ints.view(np.uint32).copy(), wtype=gg.W_F32)
    fwf = brute.floyd_warshall(gf)
    for s in range(0, 40, 7):
        np.testing.assert_array_equal(oracle.dijkstra(gf, s), fwf[s])


def test_brute_bellman_ford_on_medium_random():
    g = gg.uniform(60, 400, gseed=7, wseed=8, wtype=gg.W_F32)
    for s in (0, 13, 59):
        np.testing.assert_array_equal(oracle.dijkstra(g, s), brute.bellman_ford(g, s))


# ---------------------------------------------------------------- library routines

def _scipy_dist(g, src):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import dijkstra as sdij
    w = g.weights().astype(np.float64)
    # scipy drops explicit zeros from sparse matrices; shift so that all stored weights are > 0
    A = sp.csr_matrix((w + 1.0, g.col, g.ro), shape=(g.n, g.n))
    A.data -= 1.0
    A.data[A.data == 0] = 0.0
    return sdij(A, directed=True, indices=src)


def test_scipy_dijkstra_bit_exact_u32_grid64():
    g, srcs = gg.workload("grid64")
    d = oracle.dijkstra(g, int(srcs[0]))
    ref = _scipy_dist(g, int(srcs[0]))
    assert np.isfinite(ref).all()
    np.testing.assert_array_equal(d.astype(np.float64), ref)


def test_scipy_dijkstra_bit_exact_u32_rmat12():
    g = gg.rmat(12, 16, gseed=21, pseed=22, wseed=23, wtype=gg.W_U32, wlo=1, whi=255)
    s = int(gg.pick_sources(g, 24, 1)[0])
    d = oracle.dijkstra(g, s)
    ref = _scipy_dist(g, s)
    fin = np.isfinite(ref)
    np.testing.assert_array_equal(d[fin].astype(np.float64), ref[fin])
    assert (d[~fin] == INF).all()


def test_scipy_dijkstra_tolerance_f32_rmat12():
    # binary64 library distances are a tolerance check only: |fold32 - exact| <= hops * ulp
    g = gg.rmat(12, 16, gseed=31, pseed=32, wseed=33, wtype=gg.W_F32)
    s = int(gg.pick_sources(g, 34, 1)[0])
    d = as_f32(oracle.dijkstra(g, s)).astype(np.float64)
    ref = _scipy_dist(g, s)
    fin = np.isfinite(ref)
    assert ((d == np.float32(np.finfo(np.float32).max)) == ~fin).all()
    hops = 64  # R-MAT 12 shortest-path hop counts are far below this
    tol = hops * np.spacing(np.maximum(ref[fin], 1.0).astype(np.float32)).astype(np.float64)
    assert (np.abs(d[fin] - ref[fin]) <= tol).all()


def test_networkx_tiny():
    import networkx as nx
    g = gg.uniform(30, 90, gseed=5, wseed=6, wtype=gg.W_U32, wlo=0, whi=9)
    G = nx.DiGraph()
    G.add_nodes_from(range(g.n))
    for u in range(g.n):
        for e in range(g.ro[u], g.ro[u + 1]):
            G.add_edge(u, int(g.col[e]), weight=int(g.w[e]))
    for s in (0, 7, 29):
        ref = nx.single_source_dijkstra_path_length(G, s)
        d = oracle.dijkstra(g, s)
        for v in range(g.n):
            assert d[v] == (ref[v] if v in ref else INF)


# ---------------------------------------------------------------- certificate

def test_certificate_accepts_oracle_and_rejects_mutations():
    g = gg.rmat(11, 16, gseed=41, pseed=42, wseed=43, wtype=gg.W_U32, wlo=1, whi=255)
    s = int(gg.pick_sources(g, 44, 1)[0])
    d = oracle.dijkstra(g, s)
    assert oracle.certify(g, s, d) == (0, -1)
    fin = np.flatnonzero((d != INF) & (np.arange(g.n) != s))
    v = int(fin[len(fin) // 2])
    bad = d.copy(); bad[v] -= 1
    assert oracle.certify(g, s, bad)[0] in (2, 3)     # too small: no tight path, or a successor breaks
    bad = d.copy(); bad[v] += 1
    assert oracle.certify(g, s, bad)[0] == 2          # too large: an in-arc is violated
    bad = d.copy(); bad[v] = INF
    assert oracle.certify(g, s, bad)[0] == 2          # reachable vertex reported unreachable
    bad = d.copy(); bad[s] = 1
    assert oracle.certify(g, s, bad)[0] == 1
    unreached = np.flatnonzero(d == INF)
    if len(unreached):
        bad = d.copy(); bad[unreached[0]] = 5
        assert oracle.certify(g, s, bad)[0] == 3      # unreachable vertex given a value


def test_certificate_rejects_zero_weight_cycle_fake():
    # 0 -> 1 (5); 2 <-> 3 with weight 0, unreachable from 0.  Giving 2 and 3 a common finite
    # value makes their arcs tight to each other but not connected to the source.
    g = gg.from_arcs(4, [(0, 1, 5), (2, 3, 0), (3, 2, 0)])
    assert oracle.certify(g, 0, np.array([0, 5, INF, INF], np.uint32))[0] == 0
    assert oracle.certify(g, 0, np.array([0, 5, 3, 3], np.uint32))[0] == 3


def test_certificate_f32_value_checks():
    g = gg.from_arcs(3, [(0, 1, 0.5), (1, 2, 0.25)], wtype=gg.W_F32)
    good = np.array([f32bits(0), f32bits(0.5), f32bits(0.75)], np.uint32)
    assert oracle.certify(g, 0, good)[0] == 0
    negzero = good.copy(); negzero[0] = 0x80000000
    assert oracle.certify(g, 0, negzero)[0] == 10
    nan = good.copy(); nan[2] = 0x7FC00000
    assert oracle.certify(g, 0, nan)[0] == 10
    pinf = good.copy(); pinf[2] = 0x7F800000
    assert oracle.certify(g, 0, pinf)[0] == 10
    off = good.copy(); off[2] = f32bits(np.nextafter(np.float32(0.75), np.float32(1)))
    assert oracle.certify(g, 0, off)[0] == 2


@pytest.mark.parametrize("name", ["grid64"])
def test_bsp_matches_dijkstra_on_workload(name):
    g, srcs = gg.workload(name)
    d, stt = oracle.bsp(g, int(srcs[0]))
    np.testing.assert_array_equal(d, oracle.dijkstra(g, int(srcs[0])))
    assert stt["rounds"] > 60  # high-diameter grid: many BSP rounds


def test_rmat16_f32_oracle_certified():
    g = gg.rmat(16, 16, gseed=51, pseed=52, wseed=53, wtype=gg.W_F32)
    s = int(gg.pick_sources(g, 54, 1)[0])
    d = oracle.dijkstra(g, s)
    assert oracle.certify(g, s, d)[0] == 0
    np.testing.assert_array_equal(oracle.bsp(g, s)[0], d)


# ------------------------------------------------------------------ BFS pins

def _unit(g):
    """The same arcs with every weight 1 (uint32)."""
    return gg.CSR(n=g.n, ro=g.ro.copy(), col=g.col.copy(), w=np.ones(g.m, dtype=np.uint32), wtype=gg.W_U32,
                  name=g.name + "_unit")


@pytest.mark.parametrize("side,src", [(7, 0), (12, 5 * 12 + 7), (1, 0)])
def test_bfs_grid_is_manhattan(side, src):
    g = gg.grid(side, wseed=3)
    d = oracle.bfs(g, src)
    r0, c0 = divmod(src, side)
    want = np.array([abs(r - r0) + abs(c - c0) for r in range(side) for c in range(side)], dtype=np.uint32)
    assert np.array_equal(d, want)


def test_bfs_directed_path_and_unreachable():
    g = gg.from_arcs(6, [(0, 1, 7), (1, 2, 7), (2, 3, 7), (5, 4, 1)])
    d = oracle.bfs(g, 0)
    assert d.tolist() == [0, 1, 2, 3, oracle.INF_U32, oracle.INF_U32]
    assert oracle.bfs(g, 3).tolist() == [oracle.INF_U32] * 3 + [0] + [oracle.INF_U32] * 2


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(min_value=1, max_value=12), st.integers(min_value=0, max_value=10 ** 6))
def test_bfs_equals_floyd_warshall_on_unit_weights(n, seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(0, 3 * n + 1))
    arcs = [(int(rng.integers(0, n)), int(rng.integers(0, n)), int(rng.integers(1, 9))) for _ in range(k)]
    g = gg.from_arcs(n, arcs)
    fw = brute.floyd_warshall(_unit(g))
    for s in range(n):
        assert np.array_equal(oracle.bfs(g, s), fw[s].astype(np.uint32)), (arcs, s)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_bfs_equals_unit_weight_dijkstra(seed):
    g = gg.rmat(12, 8, gseed=seed, pseed=seed + 10, wseed=seed + 20)
    u = _unit(g)
    for s in gg.pick_sources(g, seed, 3):
        assert np.array_equal(oracle.bfs(g, int(s)), oracle.dijkstra(u, int(s)))
