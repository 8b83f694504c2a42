"""Checks of GPU results against the CPU oracle shared by the GPU tests:
``oracle.certify`` (the O(n + m) shortest-path certificate) on every row, run
on a few host threads (the oracle's C calls release the GIL), and
``oracle.dijkstra`` equality on the rows a test names."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def certify_all(g, srcs, rows, tag, workers=8):
    """Every rows[i] must pass the certificate for source srcs[i]."""
    def one(i):
        return i, oracle.certify(g, int(srcs[i]), np.ascontiguousarray(rows[i]))

    with ThreadPoolExecutor(max_workers=workers) as ex:
        for i, (code, v) in ex.map(one, range(len(srcs))):
            if code != oracle.CERT_OK:
                raise AssertionError("%s row %d (src %d): certificate fails at vertex %d: %s" % (
                    tag, i, int(srcs[i]), v, oracle.CERT_REASONS.get(code, code)))


def dijkstra_rows(g, srcs, rows, which, tag, workers=4):
    """rows[i] == oracle.dijkstra(g, srcs[i]) bit for bit, for i in which."""
    def one(i):
        return i, oracle.dijkstra(g, int(srcs[i]))

    with ThreadPoolExecutor(max_workers=workers) as ex:
        for i, want in ex.map(one, list(which)):
            got = np.asarray(rows[i])
            if not np.array_equal(got, want):
                v = int(np.flatnonzero(got != want)[0])
                raise AssertionError("%s row %d (src %d): vertex %d got 0x%08x want 0x%08x" % (
                    tag, i, int(srcs[i]), v, int(got[v]), int(want[v])))
