"""The oracle's pins must catch plausible mistakes in the oracle.

Each case copies ``oracle/oracle.c``, plants one mistake (a dropped term, a
wrong comparison, a shifted index, a transposed operand), compiles the copy on
the CPU and runs a compact version of the pin battery against it: closed forms,
exhaustive path enumeration, the binary32 rounding example and saturation.
Every mutant must fail at least one pin; the unmodified source must pass all.
"""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

import graphgen as gg
from oracle import brute

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

DIJKSTRA_MUTANTS = {
    "drop_last_edge": ("for (int32_t e = ro[u]; e < ro[u + 1]; ++e) {\n                int32_t v = col[e];\n                uint32_t nd",
                       "for (int32_t e = ro[u]; e < ro[u + 1] - 1; ++e) {\n                int32_t v = col[e];\n                uint32_t nd"),
    "off_by_one_compare": ("if (nd < dist_out[v]) {", "if (nd < dist_out[v] && nd + 1 != dist_out[v]) {"),
    "no_saturation": ("return s >= (uint64_t)INF_U32 ? INF_U32 : (uint32_t)s;", "return (uint32_t)s;"),
    "f32_no_clamp_and_wrong_zero": ("dist[src] = 0.0f;\n        if (heap_push(&h, 0.0, src))",
                                    "dist[src] = 1.0f;\n        if (heap_push(&h, 1.0, src))"),
    "stale_skip_inverted": ("if (d > dist_out[u]) continue; /* stale entry */",
                            "if (d >= dist_out[u] && u != src) continue; /* stale entry */"),
    "shifted_index": ("int32_t v = col[e];\n                uint32_t nd = add_u32(d, w[e]);",
                      "int32_t v = col[e];\n                uint32_t nd = add_u32(d, w[ro[u]]);"),
    "f32_weight_of_wrong_edge": ("float nd = add_f32(d, bits_to_f(w[e]));",
                                 "float nd = add_f32(d, bits_to_f(w[e == ro[u] ? e : e - 1]));"),
    "f32_fold_in_binary64": [
        ("float *dist = (float *)malloc((size_t)n * sizeof(float));", "double *dist = (double *)malloc((size_t)n * sizeof(double));"),
        ("float d = (float)it.key;", "double d = it.key;"),
        ("float nd = add_f32(d, bits_to_f(w[e]));", "double nd = d + (double)bits_to_f(w[e]);"),
        ("dist_out[v] = f_to_bits(dist[v]);\n        free(dist);", "dist_out[v] = f_to_bits((float)dist[v]);\n        free(dist);"),
    ],
    "u32_source_not_zero": ("dist_out[src] = 0;\n        if (heap_push(&h, 0.0, src)) return -1;",
                            "dist_out[src] = 0;\n        if (heap_push(&h, 1.0, src)) return -1;"),
}

CERTIFY_MUTANTS = {
    "skip_tight_reachability": ("if (dist[v] != INF && !seen[v]) { if (bad) *bad = v; rc = 3; break; }",
                                "if (0) { rc = 3; }"),
    "triangle_strict_reversed": ("if (wtype == 0) ok = dist[v] <= add_u32(dist[u], w[e]);",
                                 "if (wtype == 0) ok = dist[v] >= add_u32(dist[u], w[e]) || 1;"),
    "tight_uses_wrong_endpoint": ("if (wtype == 0) tight = add_u32(dist[u], w[e]) == dist[v];",
                                  "if (wtype == 0) tight = add_u32(dist[u], w[e]) >= dist[v];"),
}


BFS_MUTANTS = {
    "two_hops_per_arc": ("depth[v] = depth[u] + 1u;", "depth[v] = depth[u] + 2u;"),
    "revisit_allowed": ("if (depth[v] == INF_U32) {\n                depth[v] = depth[u] + 1u;",
                        "if (depth[v] >= depth[u]) {\n                depth[v] = depth[u] + 1u;"),
    "skip_last_arc": ("for (int32_t e = ro[u]; e < ro[u + 1]; ++e) {\n            const int32_t v = col[e];\n            if (depth[v]",
                      "for (int32_t e = ro[u]; e < ro[u + 1] - 1; ++e) {\n            const int32_t v = col[e];\n            if (depth[v]"),
    "lifo_order": ("const int32_t u = q[head++];", "const int32_t u = q[--tail];"),
}


def _mutate(text, spec, name):
    pairs = spec if isinstance(spec, list) else [spec]
    for old, new in pairs:
        assert text.count(old) >= 1, "mutation anchor not found: %s: %r" % (name, old)
        text = text.replace(old, new, 1)
    return text


def _compile(tmp_path, text, tag):
    src = tmp_path / ("m_%s.c" % tag)
    so = tmp_path / ("m_%s.so" % tag)
    src.write_text(text)
    subprocess.run(["gcc", "-O1", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", str(src), "-o", str(so)],
                   check=True, capture_output=True)
    lib = ctypes.CDLL(str(so))
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.oracle_dijkstra.argtypes = [i32, vp, vp, vp, ctypes.c_int, i32, vp]
    lib.oracle_certify.argtypes = [i32, vp, vp, vp, ctypes.c_int, i32, vp, vp]
    lib.oracle_bfs.argtypes = [i32, vp, vp, i32, vp]
    return lib


def _dij(lib, g, s):
    ro = np.ascontiguousarray(g.ro, np.int32)
    col = np.ascontiguousarray(g.col if g.m else np.zeros(1, np.int32), np.int32)
    w = np.ascontiguousarray(g.w if g.m else np.zeros(1, np.uint32), np.uint32)
    out = np.empty(max(g.n, 1), np.uint32)
    lib.oracle_dijkstra(g.n, ro.ctypes.data, col.ctypes.data, w.ctypes.data, g.wtype, s, out.ctypes.data)
    return out[:g.n]


def _cert(lib, g, s, d):
    ro = np.ascontiguousarray(g.ro, np.int32)
    col = np.ascontiguousarray(g.col, np.int32)
    w = np.ascontiguousarray(g.w, np.uint32)
    d = np.ascontiguousarray(d, np.uint32)
    bad = ctypes.c_int32(-1)
    return lib.oracle_certify(g.n, ro.ctypes.data, col.ctypes.data, w.ctypes.data, g.wtype, s, d.ctypes.data,
                              ctypes.byref(bad))


def _tiny_cases():
    rng = np.random.default_rng(2024)
    cases = []
    for wt in (gg.W_U32, gg.W_F32):
        for _ in range(150):
            n = int(rng.integers(2, 7))
            k = int(rng.integers(1, 3 * n))
            arcs = []
            for _ in range(k):
                u, v = int(rng.integers(0, n)), int(rng.integers(0, n))
                w = int(rng.integers(0, 6)) if wt == gg.W_U32 else float(rng.choice([0.0, 2.0 ** -24, 0.1, 1.0, 3.5]))
                arcs.append((u, v, w))
            cases.append((gg.from_arcs(n, arcs, wtype=wt), int(rng.integers(0, n))))
    return cases


def dijkstra_pins_fail(lib):
    """Returns the list of failed pins (empty when all pass)."""
    failed = []
    for g, s in _tiny_cases():
        if not np.array_equal(_dij(lib, g, s), brute.paths_min(g, s)):
            failed.append("paths_min")
            break
    g = gg.grid(9, wseed=0, wtype=gg.W_U32, wlo=1, whi=1)
    r, c = np.divmod(np.arange(81), 9)
    if not np.array_equal(_dij(lib, g, 0), r + c):
        failed.append("manhattan")
    e24 = 2.0 ** -24
    g = gg.from_arcs(4, [(0, 1, 1.0), (1, 2, e24), (2, 3, e24), (0, 3, 1.0 + 2 * e24)], wtype=gg.W_F32)
    if _dij(lib, g, 0).view(np.float32)[3] != np.float32(1.0):
        failed.append("f32_rounding")
    rng = np.random.default_rng(11)
    w = rng.random(300, dtype=np.float32) * np.float32(3.0) + np.float32(1e-3)
    g = gg.from_arcs(301, [(i, i + 1, w[i]) for i in range(300)], wtype=gg.W_F32)
    want = np.concatenate([[np.float32(0)], np.cumsum(w, dtype=np.float32)])
    if not np.array_equal(_dij(lib, g, 0).view(np.float32), want):
        failed.append("f32_prefix_fold")
    g = gg.from_arcs(4, [(0, 1, 0xFFFFFFFF - 5), (1, 2, 3), (2, 3, 7)])
    if _dij(lib, g, 0)[3] != 0xFFFFFFFF:
        failed.append("saturation")
    return failed


def _bfs(lib, g, s):
    ro = np.ascontiguousarray(g.ro, np.int32)
    col = np.ascontiguousarray(g.col if g.m else np.zeros(1, np.int32), np.int32)
    out = np.empty(max(g.n, 1), np.uint32)
    lib.oracle_bfs(g.n, ro.ctypes.data, col.ctypes.data, s, out.ctypes.data)
    return out[:g.n]


def bfs_pins_fail(lib):
    """BFS pins: grid closed form, Floyd-Warshall on unit weights for tiny graphs."""
    failed = []
    g = gg.grid(9, wseed=0)
    r, c = np.divmod(np.arange(81), 9)
    if not np.array_equal(_bfs(lib, g, 0), r + c):
        failed.append("manhattan")
    for g, s in _tiny_cases()[:150]:
        unit = gg.CSR(n=g.n, ro=g.ro, col=g.col, w=np.ones(g.m, np.uint32), wtype=gg.W_U32)
        if not np.array_equal(_bfs(lib, g, s), brute.floyd_warshall(unit)[s].astype(np.uint32)):
            failed.append("floyd_warshall")
            break
    return failed


def certify_pins_fail(lib):
    failed = []
    g = gg.from_arcs(4, [(0, 1, 5), (2, 3, 0), (3, 2, 0)])
    if _cert(lib, g, 0, np.array([0, 5, 3, 3], np.uint32)) == 0:
        failed.append("zero_cycle_fake")
    g = gg.from_arcs(3, [(0, 1, 2), (1, 2, 2)])
    if _cert(lib, g, 0, np.array([0, 2, 5], np.uint32)) == 0:
        failed.append("too_large")
    if _cert(lib, g, 0, np.array([0, 2, 3], np.uint32)) == 0:
        failed.append("too_small")
    if _cert(lib, g, 0, np.array([0, 2, 4], np.uint32)) != 0:
        failed.append("accept_valid")
    # a value explained by a tight arc (0 -> 2, weight 10) yet beaten by another path
    g = gg.from_arcs(3, [(0, 1, 2), (1, 2, 2), (0, 2, 10)])
    if _cert(lib, g, 0, np.array([0, 2, 10], np.uint32)) == 0:
        failed.append("tight_but_not_minimal")
    return failed


def _run_battery(tmp_path, text, tag, kind):
    """Compiles the source and runs one battery in a child process (a mutant may loop
    forever, e.g. by re-queueing equal keys around a zero-weight cycle: a time-out
    counts as caught).  Returns the failed pins, or ["timeout"]."""
    _compile(tmp_path, text, tag)
    so = str(tmp_path / ("m_%s.so" % tag))
    try:
        env = dict(os.environ, PYTHONPATH=ROOT)
        r = subprocess.run([sys.executable, __file__, so, kind], capture_output=True, text=True, timeout=60,
                           cwd=ROOT, env=env)
    except subprocess.TimeoutExpired:
        return ["timeout"]
    if r.returncode not in (0, 3):
        return ["crash:%d:%s" % (r.returncode, r.stderr[-300:])]
    return [x for x in r.stdout.split() if x]


def test_unmodified_oracle_passes_battery(tmp_path):
    lib = _compile(tmp_path, open(SRC).read(), "orig")
    assert dijkstra_pins_fail(lib) == []
    assert certify_pins_fail(lib) == []
    # the same child-process route the mutants take reports no failure either
    assert _run_battery(tmp_path, open(SRC).read(), "orig_child", "dijkstra") == []
    assert _run_battery(tmp_path, open(SRC).read(), "orig_child2", "certify") == []
    assert bfs_pins_fail(lib) == []
    assert _run_battery(tmp_path, open(SRC).read(), "orig_child3", "bfs") == []


@pytest.mark.parametrize("name", sorted(DIJKSTRA_MUTANTS))
def test_dijkstra_mutant_is_caught(tmp_path, name):
    text = _mutate(open(SRC).read(), DIJKSTRA_MUTANTS[name], name)
    assert _run_battery(tmp_path, text, name, "dijkstra"), "mutant %s survived the pins" % name


@pytest.mark.parametrize("name", sorted(CERTIFY_MUTANTS))
def test_certify_mutant_is_caught(tmp_path, name):
    text = _mutate(open(SRC).read(), CERTIFY_MUTANTS[name], name)
    assert _run_battery(tmp_path, text, name, "certify"), "mutant %s survived the pins" % name


@pytest.mark.parametrize("name", sorted(BFS_MUTANTS))
def test_bfs_mutant_is_caught(tmp_path, name):
    text = _mutate(open(SRC).read(), BFS_MUTANTS[name], name)
    assert _run_battery(tmp_path, text, name, "bfs"), "mutant %s survived the pins" % name


if __name__ == "__main__":  # child process: python test_oracle_mutants.py <lib.so> <dijkstra|certify|bfs>
    sys.path.insert(0, ROOT)
    _lib = ctypes.CDLL(sys.argv[1])
    _vp, _i32 = ctypes.c_void_p, ctypes.c_int32
    _lib.oracle_dijkstra.argtypes = [_i32, _vp, _vp, _vp, ctypes.c_int, _i32, _vp]
    _lib.oracle_certify.argtypes = [_i32, _vp, _vp, _vp, ctypes.c_int, _i32, _vp, _vp]
    _lib.oracle_bfs.argtypes = [_i32, _vp, _vp, _i32, _vp]
    _failed = {"dijkstra": dijkstra_pins_fail, "certify": certify_pins_fail, "bfs": bfs_pins_fail}[sys.argv[2]](_lib)
    print(" ".join(_failed))
    sys.exit(3 if _failed else 0)
