"""CPU oracle for single-source shortest paths -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  It shares no code with the GPU
library and imports nothing from it.

Exports
-------
``dijkstra(g, src)``        textbook binary-heap Dijkstra (C, ``oracle.c``)
``bsp(g, src)``             the paper's bulk-synchronous push loop run
                            sequentially in the order of Listings 3-4 (C),
                            with round / relaxation / frontier statistics
``certify(g, src, dist)``   O(n+m) certificate that ``dist`` is the
                            shortest-path vector (conditions in ``oracle.c``)
``bfs(g, src)``             textbook FIFO breadth-first search depths (C)
``brute``                   tiny-input references written independently in
                            Python: Bellman-Ford, Floyd-Warshall and exhaustive
                            simple-path enumeration

Distances are returned as uint32 *bits* (uint32 values, or IEEE binary32
patterns for fp32 graphs).  INF is 0xFFFFFFFF (uint32) and FLT_MAX
(binary32), the initial value of Listing 4.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from . import brute  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

INF_U32 = 0xFFFFFFFF
INF_F32_BITS = int(np.array([np.finfo(np.float32).max], dtype=np.float32).view(np.uint32)[0])

CERT_OK = 0
CERT_REASONS = {
    0: "valid",
    1: "dist[src] != 0",
    2: "an arc violates dist[v] <= dist[u] (+) w",
    3: "a finite vertex is not reached along tight arcs",
    10: "a value is negative, -0, NaN or +inf",
}


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.run(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11", _SRC,
             "-o", tmp],
            check=True,
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            vp = ctypes.c_void_p
            i32 = ctypes.c_int32
            lib.oracle_dijkstra.argtypes = [i32, vp, vp, vp, ctypes.c_int, i32, vp]
            lib.oracle_bsp.argtypes = [i32, vp, vp, vp, ctypes.c_int, i32, ctypes.c_int64, vp, vp]
            lib.oracle_certify.argtypes = [i32, vp, vp, vp, ctypes.c_int, i32, vp, vp]
            lib.oracle_bfs.argtypes = [i32, vp, vp, i32, vp]
            _lib = lib
    return _lib


def _arrays(g):
    ro = np.ascontiguousarray(g.ro, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = np.ascontiguousarray(g.w, dtype=np.uint32)
    if col.size == 0:  # keep valid pointers for empty graphs
        col = np.zeros(1, dtype=np.int32)
        w = np.zeros(1, dtype=np.uint32)
    return ro, col, w


def inf_bits(wtype: int) -> int:
    return INF_F32_BITS if wtype == 1 else INF_U32


def dijkstra(g, src: int) -> np.ndarray:
    lib = _load()
    ro, col, w = _arrays(g)
    out = np.empty(max(g.n, 1), dtype=np.uint32)
    rc = lib.oracle_dijkstra(g.n, ro.ctypes.data, col.ctypes.data, w.ctypes.data, g.wtype, int(src),
                             out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_dijkstra failed (%d)" % rc)
    return out[: g.n]


def bfs(g, src: int) -> np.ndarray:
    """Hop depths from src (uint32; INF_U32 when unreachable); weights are ignored."""
    lib = _load()
    ro, col, _ = _arrays(g)
    out = np.empty(max(g.n, 1), dtype=np.uint32)
    if lib.oracle_bfs(g.n, ro.ctypes.data, col.ctypes.data, int(src), out.ctypes.data) != 0:
        raise MemoryError("oracle_bfs allocation failed")
    return out[: g.n]


def bsp(g, src: int, max_rounds: int | None = None):
    """Returns (dist_bits, stats) with stats = dict(rounds, relaxations, frontier_sum, frontier_max)."""
    lib = _load()
    ro, col, w = _arrays(g)
    out = np.empty(max(g.n, 1), dtype=np.uint32)
    st = np.zeros(4, dtype=np.int64)
    cap = g.n + 1 if max_rounds is None else max_rounds
    rc = lib.oracle_bsp(g.n, ro.ctypes.data, col.ctypes.data, w.ctypes.data, g.wtype, int(src), cap,
                        out.ctypes.data, st.ctypes.data)
    if rc == -2:
        raise RuntimeError("oracle_bsp exceeded %d rounds" % cap)
    if rc != 0:
        raise ValueError("oracle_bsp failed (%d)" % rc)
    return out[: g.n], dict(rounds=int(st[0]), relaxations=int(st[1]), frontier_sum=int(st[2]),
                            frontier_max=int(st[3]))


def certify(g, src: int, dist) -> tuple[int, int]:
    """Returns (code, vertex): code 0 when ``dist`` is the shortest-path vector."""
    lib = _load()
    ro, col, w = _arrays(g)
    d = np.ascontiguousarray(dist, dtype=np.uint32)
    if d.shape != (g.n,):
        raise ValueError("dist has shape %r, expected (%d,)" % (d.shape, g.n))
    bad = ctypes.c_int32(-1)
    rc = lib.oracle_certify(g.n, ro.ctypes.data, col.ctypes.data, w.ctypes.data, g.wtype, int(src),
                            d.ctypes.data if g.n else np.zeros(1, np.uint32).ctypes.data, ctypes.byref(bad))
    if rc < 0:
        raise MemoryError("oracle_certify allocation failed")
    return int(rc), int(bad.value)
