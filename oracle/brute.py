"""Tiny-input references for the shortest-path definition -- TEST INFRASTRUCTURE.

Written independently of ``oracle.c`` (plain Python integers and numpy
binary32 scalars), to pin it:

* ``fold``            the left fold ((0 (+) w1) (+) w2) ... of one path
* ``paths_min``       the definition itself: min of ``fold`` over every simple
                      path from the source (exhaustive DFS; n <= ~9).  Simple
                      paths suffice: (+) never decreases a value and is
                      monotone in its left operand, so cutting a cycle out of a
                      path never increases its fold.
* ``bellman_ford``    n - 1 synchronous rounds of relaxation over all arcs
* ``floyd_warshall``  all-pairs relaxation d[i][j] = min(d[i][j], d[i][k] + d[k][j]);
                      equal to the fold definition for uint32, and for binary32
                      only when every partial sum is exact (integer weights),
                      because it re-associates the additions.

Values are uint32 bit patterns as in the rest of the oracle.
"""
from __future__ import annotations

import numpy as np

INF_U32 = 0xFFFFFFFF
FLT_MAX = np.float32(np.finfo(np.float32).max)
INF_F32_BITS = int(np.array([FLT_MAX], dtype=np.float32).view(np.uint32)[0])


def _to_val(bits: int, wtype: int):
    if wtype == 1:
        return np.array([bits], dtype=np.uint32).view(np.float32)[0]
    return int(bits)


def _to_bits(val, wtype: int) -> int:
    if wtype == 1:
        return int(np.array([val], dtype=np.float32).view(np.uint32)[0])
    return int(val)


def plus(d, w, wtype: int):
    """One (+) step on values (not bits)."""
    if wtype == 1:
        with np.errstate(over="ignore"):
            s = np.float32(d) + np.float32(w)  # binary32, round to nearest even
        return FLT_MAX if s >= FLT_MAX else s
    s = int(d) + int(w)
    return INF_U32 if s >= INF_U32 else s


def fold(weights, wtype: int):
    acc = np.float32(0.0) if wtype == 1 else 0
    for w in weights:
        acc = plus(acc, w, wtype)
    return acc


def _arcs(g):
    ws = g.w.view(np.float32) if g.wtype == 1 else g.w
    out = []
    for u in range(g.n):
        for e in range(int(g.ro[u]), int(g.ro[u + 1])):
            out.append((u, int(g.col[e]), ws[e]))
    return out


def paths_min(g, src: int) -> np.ndarray:
    """min over all simple paths of the fold, by exhaustive enumeration."""
    wt = g.wtype
    inf = FLT_MAX if wt == 1 else INF_U32
    best = [inf] * g.n
    best[src] = np.float32(0.0) if wt == 1 else 0
    adj = [[] for _ in range(g.n)]
    for u, v, w in _arcs(g):
        adj[u].append((v, w))
    on_path = [False] * g.n

    def dfs(u, acc):
        on_path[u] = True
        for v, w in adj[u]:
            if on_path[v]:
                continue
            nd = plus(acc, w, wt)
            if nd < best[v]:
                best[v] = nd
            dfs(v, nd)
        on_path[u] = False

    dfs(src, best[src])
    return np.array([_to_bits(b, wt) for b in best], dtype=np.uint32)


def bellman_ford(g, src: int) -> np.ndarray:
    wt = g.wtype
    inf = FLT_MAX if wt == 1 else INF_U32
    d = [inf] * g.n
    d[src] = np.float32(0.0) if wt == 1 else 0
    arcs = _arcs(g)
    for _ in range(max(g.n - 1, 0)):
        nxt = list(d)
        for u, v, w in arcs:
            if d[u] == inf:
                continue
            nd = plus(d[u], w, wt)
            if nd < nxt[v]:
                nxt[v] = nd
        if nxt == d:
            break
        d = nxt
    return np.array([_to_bits(x, wt) for x in d], dtype=np.uint32)


def floyd_warshall(g) -> np.ndarray:
    """All-pairs matrix of bit patterns (row i = distances from i)."""
    wt = g.wtype
    n = g.n
    if wt == 1:
        d = np.full((n, n), FLT_MAX, dtype=np.float32)
        np.fill_diagonal(d, 0)
        for u, v, w in _arcs(g):
            if u != v:
                d[u, v] = min(d[u, v], np.float32(w))
        for k in range(n):
            with np.errstate(over="ignore"):
                cand = np.minimum(d[:, k:k + 1] + d[k:k + 1, :], FLT_MAX).astype(np.float32)
            reach = (d[:, k:k + 1] < FLT_MAX) & (d[k:k + 1, :] < FLT_MAX)
            d = np.where(reach & (cand < d), cand, d)
        return d.view(np.uint32)
    d = np.full((n, n), INF_U32, dtype=np.uint64)
    np.fill_diagonal(d, 0)
    for u, v, w in _arcs(g):
        if u != v:
            d[u, v] = min(int(d[u, v]), int(w))
    for k in range(n):
        cand = np.minimum(d[:, k:k + 1] + d[k:k + 1, :], INF_U32)
        d = np.minimum(d, cand)
    return d.astype(np.uint32)
