"""Seeded synthetic graph inputs, shared by the oracle's tests and the GPU path.

This module builds graphs only: it contains no shortest-path arithmetic.  The C
source (``graphgen.c``) documents the counter-based random generator and the
CSR conventions.  Graphs are returned as :class:`CSR` with int32
``row_offsets``/``col`` and uint32 weight *bits* (the value for uint32 weights,
the IEEE binary32 pattern for fp32 weights), matching the paper's ``csr_t``
(Section IV-A, Listing 1).

Named workloads (``workload(name)``) reproduce the benchmark configurations:

=============  ==============================================================
``grid64``     64x64 4-neighbour grid, uint32 weights U[1,100], source 0
``rmat20``     R-MAT scale 20, ef 16, (.57,.19,.19,.05), fp32 weights (0,1]
``road2048``   2048x2048 grid + floor(0.001 n) shortcuts, uint32 U[1,1000]
``grid2048``   the same grid without shortcuts (high-diameter stress case)
``rmat22``     R-MAT scale 22, same parameters, uint32 weights U[1,255]
=============  ==============================================================
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lock = threading.Lock()
_lib = None

W_U32 = 0
W_F32 = 1

RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = True) -> str:
    """Compile ``libgraphgen.so`` with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.run(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp],
            check=True,
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _CSR(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("m", ctypes.c_int64),
        ("ro", ctypes.POINTER(ctypes.c_int32)),
        ("col", ctypes.POINTER(ctypes.c_int32)),
        ("w", ctypes.POINTER(ctypes.c_uint32)),
    ]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.POINTER
            lib.gg_grid.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32,
                                    ctypes.c_uint32, ctypes.c_int64, ctypes.c_uint64, P(_CSR)]
            lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, P(_CSR)]
            lib.gg_uniform.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, P(_CSR)]
            lib.gg_pick_sources.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_uint64,
                                            ctypes.c_int32, ctypes.c_void_p]
            lib.gg_hash.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
            lib.gg_hash.restype = ctypes.c_uint64
            lib.gg_free.argtypes = [P(_CSR)]
            lib.gg_num_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


@dataclass
class CSR:
    """A directed graph in CSR form (paper's csr_t): arcs u -> col[e] for e in [ro[u], ro[u+1])."""

    n: int
    ro: np.ndarray  # int32[n+1]
    col: np.ndarray  # int32[m]
    w: np.ndarray  # uint32[m]: weight bits
    wtype: int  # W_U32 or W_F32
    name: str = ""
    symmetric: bool = False  # arcs and weights symmetric by construction

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def weights(self) -> np.ndarray:
        """Weights as numbers (uint32 or float32 view of the bits)."""
        return self.w.view(np.float32) if self.wtype == W_F32 else self.w

    def degrees(self) -> np.ndarray:
        return np.diff(self.ro)


def _take(lib, c: _CSR, wtype: int, name: str, symmetric: bool) -> CSR:
    try:
        n, m = int(c.n), int(c.m)
        ro = np.ctypeslib.as_array(c.ro, shape=(n + 1,)).copy()
        col = np.ctypeslib.as_array(c.col, shape=(max(m, 1),))[:m].copy()
        w = np.ctypeslib.as_array(c.w, shape=(max(m, 1),))[:m].copy()
    finally:
        lib.gg_free(ctypes.byref(c))
    return CSR(n=n, ro=ro, col=col, w=w, wtype=wtype, name=name, symmetric=symmetric)


def grid(side: int, wseed: int, wtype: int = W_U32, wlo: int = 1, whi: int = 100,
         shortcuts: int = 0, sseed: int = 0, name: str = "") -> CSR:
    lib = _load()
    c = _CSR()
    rc = lib.gg_grid(side, wseed, wtype, wlo, whi, shortcuts, sseed, ctypes.byref(c))
    if rc != 0:
        raise RuntimeError("gg_grid failed (%d)" % rc)
    return _take(lib, c, wtype, name or "grid%d" % side, False)


def rmat(scale: int, edge_factor: int = 16, abc=RMAT_ABC, gseed: int = 1, pseed: int = 2,
         wseed: int = 3, wtype: int = W_U32, wlo: int = 1, whi: int = 255, name: str = "") -> CSR:
    lib = _load()
    c = _CSR()
    a, b, cc = abc
    rc = lib.gg_rmat(scale, edge_factor, a, b, cc, gseed, pseed, wseed, wtype, wlo, whi, ctypes.byref(c))
    if rc != 0:
        raise RuntimeError("gg_rmat failed (%d)" % rc)
    return _take(lib, c, wtype, name or "rmat%d" % scale, True)


def uniform(n: int, arcs: int, gseed: int, wseed: int, wtype: int = W_U32, wlo: int = 1,
            whi: int = 100, symmetric: bool = False, name: str = "") -> CSR:
    """Random graph with `arcs` uniform (u, v) draws (self-loops/duplicates dropped)."""
    lib = _load()
    c = _CSR()
    rc = lib.gg_uniform(n, arcs, gseed, wseed, wtype, wlo, whi, int(symmetric), ctypes.byref(c))
    if rc != 0:
        raise RuntimeError("gg_uniform failed (%d)" % rc)
    return _take(lib, c, wtype, name or "uniform%d" % n, symmetric)


def from_arcs(n: int, arcs, wtype: int = W_U32, name: str = "custom") -> CSR:
    """CSR from an explicit list of (u, v, weight) arcs, kept as given (duplicates
    and self-loops included), ordered by source then by input position."""
    arcs = list(arcs)
    src = np.array([a[0] for a in arcs], dtype=np.int64)
    dst = np.array([a[1] for a in arcs], dtype=np.int32)
    if wtype == W_F32:
        w = np.array([a[2] for a in arcs], dtype=np.float32).view(np.uint32)
    else:
        w = np.array([a[2] for a in arcs], dtype=np.uint64).astype(np.uint32)
    order = np.argsort(src, kind="stable") if len(arcs) else np.zeros(0, dtype=np.int64)
    ro = np.zeros(n + 1, dtype=np.int64)
    if len(arcs):
        np.add.at(ro, src + 1, 1)
    ro = np.cumsum(ro).astype(np.int32)
    return CSR(n=n, ro=ro, col=dst[order].copy(), w=w[order].copy(), wtype=wtype, name=name)


def pick_sources(g: CSR, seed: int, k: int) -> np.ndarray:
    """k seeded sources drawn uniformly among vertices with out-degree > 0."""
    lib = _load()
    out = np.zeros(k, dtype=np.int32)
    ro = np.ascontiguousarray(g.ro, dtype=np.int32)
    rc = lib.gg_pick_sources(g.n, ro.ctypes.data, seed, k, out.ctypes.data)
    if rc != 0:
        raise RuntimeError("graph has no vertex with out-degree > 0")
    return out


def hash3(seed: int, a: int, b: int) -> int:
    return int(_load().gg_hash(seed, a, b))


def num_threads() -> int:
    return int(_load().gg_num_threads())


# --- named workloads -------------------------------------------------------

_PSEED_XOR = 0x5045524D  # permutation seed = graph seed ^ this constant


def workload(name: str):
    """Returns (graph, sources) for a named benchmark configuration."""
    if name == "grid64":
        g = grid(64, wseed=2, wtype=W_U32, wlo=1, whi=100, name=name)
        return g, np.array([0], dtype=np.int32)
    if name == "rmat20":
        g = rmat(20, 16, RMAT_ABC, gseed=3, pseed=3 ^ _PSEED_XOR, wseed=4, wtype=W_F32, name=name)
        return g, pick_sources(g, 5, 1)
    if name == "road2048":
        n = 2048 * 2048
        g = grid(2048, wseed=7, wtype=W_U32, wlo=1, whi=1000, shortcuts=n // 1000, sseed=6, name=name)
        return g, np.array([0], dtype=np.int32)
    if name == "grid2048":
        g = grid(2048, wseed=7, wtype=W_U32, wlo=1, whi=1000, name=name)
        return g, np.array([0], dtype=np.int32)
    if name == "rmat22":
        g = rmat(22, 16, RMAT_ABC, gseed=8, pseed=8 ^ _PSEED_XOR, wseed=9, wtype=W_U32, wlo=1, whi=255,
                 name=name)
        return g, pick_sources(g, 10, 64)
    if name.startswith("rmat") and name[4:].isdigit():
        s = int(name[4:])
        g = rmat(s, 16, RMAT_ABC, gseed=100 + s, pseed=(100 + s) ^ _PSEED_XOR, wseed=200 + s, wtype=W_U32,
                 wlo=1, whi=255, name=name)
        return g, pick_sources(g, 300 + s, 64)
    raise KeyError(name)


def serving_graphs():
    """The 32 resident graphs of the serving workload: ids 0-15 R-MAT scale
    14 + (i mod 7) (seed 100 + i), ids 16-31 grids of side 256/512/768/1024
    cycling; uint32 weights U[1,255]."""
    out = []
    for i in range(16):
        s = 14 + (i % 7)
        out.append(rmat(s, 16, RMAT_ABC, gseed=100 + i, pseed=(100 + i) ^ _PSEED_XOR, wseed=1100 + i,
                        wtype=W_U32, wlo=1, whi=255, name="srv_rmat%d_%d" % (s, i)))
    sides = [256, 512, 768, 1024]
    for j in range(16):
        out.append(grid(sides[j % 4], wseed=1200 + j, wtype=W_U32, wlo=1, whi=255,
                        name="srv_grid%d_%d" % (sides[j % 4], j)))
    return out
