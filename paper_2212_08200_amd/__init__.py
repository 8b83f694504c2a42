"""Python binding of the gr C ABI (``include/gr.h``): frontier-driven SSSP on MI355X.

Argument marshalling only: every step of the computation runs in the HIP
library ``libgr.so``.  Importing succeeds without the library (so that CPU-only
tooling can inspect the package), but every call raises ``GrLibraryMissing``
until ``paper_2212_08200_amd.build.build()`` has produced it -- there is no
CPU fallback.

The functions carry the C names (``gr_graph_create_csr``, ``gr_sssp``,
``gr_sssp_ex``, ``gr_sssp_batch``, ``gr_server_create``, ``gr_server_add_graph``,
``gr_serve_submit``, ``gr_serve_poll``, ``gr_server_destroy``, ...).  Device
buffers may be given as torch tensors (their ``data_ptr()``) or raw integer
addresses; streams as ``torch.cuda.Stream``, raw ``hipStream_t`` integers, or
``None`` for torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgr.so")

GR_OK = 0
GR_ERR_INVALID_ARG = 1
GR_ERR_SOURCE_RANGE = 2
GR_ERR_OUT_OF_MEMORY = 3
GR_ERR_NO_CAPACITY = 4
GR_ERR_NOT_READY = 5
GR_ERR_ITER_LIMIT = 6
GR_ERR_HIP = 7
GR_ERR_UNKNOWN_TICKET = 8

GR_W_U32 = 0
GR_W_F32 = 1
GR_DIST_INF_U32 = 0xFFFFFFFF
GR_DIST_INF_F32_BITS = 0x7F7FFFFF
GR_NOALLOC_SCRATCH_BYTES = 96 << 20

GR_INPUT_DEVICE = 0x1
GR_NO_PULL = 0x2
GR_NO_PARTITION = 0x4
GR_FORCE_PARTITION = 0x8

GR_LAYOUT_AUTO = 0
GR_LAYOUT_PLAIN = 1
GR_LAYOUT_PARTITIONED = 2

GR_LOOP_AUTO = 0
GR_LOOP_HOST = 1
GR_LOOP_PERSISTENT = 2
GR_LOOP_QUEUED = 3
GR_LOOP_ASYNC = 4
GR_LOOP_LDS = 5
GR_DELTA_OFF = 0xFFFFFFFF
GR_RELAX_DIST = 1
GR_RELAX_BOUND = 2


def delta_bits(value, wt) -> int:
    """The gr_sssp_opts.delta encoding of a split width: the value for uint32
    weights, the binary32 bit pattern for fp32 weights."""
    if int(wt) == GR_W_F32:
        return int(np.array([value], np.float32).view(np.uint32)[0])
    return int(value)

GR_DIR_AUTO = 0
GR_DIR_PUSH = 1
GR_DIR_PULL = 2
GR_DIR_ALTERNATE = 3

EXPORTED = [
    "gr_graph_create_csr", "gr_graph_destroy", "gr_graph_info", "gr_graph_layout", "gr_graph_tune", "gr_sssp",
    "gr_sssp_ex", "gr_sssp_noalloc",
    "gr_bfs", "gr_bfs_ex", "gr_sssp_batch", "gr_sssp_batch_ex", "gr_sssp_multi",
    "gr_server_create", "gr_server_add_graph", "gr_serve_submit", "gr_serve_poll", "gr_server_destroy",
    "gr_status_string", "gr_last_error", "gr_version",
]


class GrLibraryMissing(RuntimeError):
    pass


class GrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_status_name(status), message))
        self.status = status
        self.message = message


class gr_sssp_opts(ctypes.Structure):
    _fields_ = [("loop", ctypes.c_int32), ("direction", ctypes.c_int32), ("alpha_x16", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("layout", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("filter", ctypes.c_int32), ("barrier_timeout_us", ctypes.c_int32), ("delta", ctypes.c_uint32),
                ("relax_filter", ctypes.c_int32), ("beta", ctypes.c_int32), ("local_hops", ctypes.c_int32)]


class gr_sssp_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("pull_iterations", ctypes.c_int32),
                ("edges_pushed", ctypes.c_int64), ("arcs_pulled", ctypes.c_int64),
                ("frontier_sum", ctypes.c_int64), ("push_frontier_sum", ctypes.c_int64),
                ("frontier_max", ctypes.c_int32), ("loop", ctypes.c_int32), ("push_launches", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("push_us", ctypes.c_double), ("pull_us", ctypes.c_double),
                ("filter_us", ctypes.c_double), ("small_rounds", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("relax_filter", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gr_tune_result(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_int32), ("loop", ctypes.c_int32), ("dense_ratio", ctypes.c_int32),
                ("alpha_x16", ctypes.c_int32), ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("trials", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("delta", ctypes.c_uint32),
                ("small", ctypes.c_int32), ("relax_filter", ctypes.c_int32), ("async_blocks", ctypes.c_int32),
                ("local_hops", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gr_multi_stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("replays", ctypes.c_int32), ("edges_pushed", ctypes.c_int64),
                ("frontier_sum", ctypes.c_int64), ("source_relaxations", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gr_server_config(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("num_streams", ctypes.c_int32), ("max_wait_us", ctypes.c_int32),
                ("local_hops", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


class gr_query_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("graph_id", ctypes.c_int32), ("src", ctypes.c_int32),
                ("batch_size", ctypes.c_int32), ("t_submit_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64), ("iterations", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lock = threading.Lock()
_lib = None


def lib():
    """The loaded ``libgr.so`` (raises ``GrLibraryMissing`` if it was never built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise GrLibraryMissing("libgr.so is not built (run paper_2212_08200_amd.build.build())")
            L = ctypes.CDLL(LIB_PATH)
            vp, i32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
            P = ctypes.POINTER
            sigs = {
                "gr_graph_create_csr": [P(vp), i32, i32, vp, vp, vp, ctypes.c_int, u32, vp],
                "gr_graph_destroy": [vp],
                "gr_graph_info": [vp, P(i32), P(i32), P(ctypes.c_int), P(ctypes.c_size_t)],
                "gr_graph_layout": [vp, P(i32), P(i32), P(i32)],
                "gr_graph_tune": [vp, vp, i32, i32, vp, P(gr_tune_result)],
                "gr_sssp": [vp, i32, vp, vp],
                "gr_sssp_ex": [vp, i32, vp, vp, P(gr_sssp_opts), P(gr_sssp_stats)],
                "gr_sssp_noalloc": [vp, i32, vp, vp],
                "gr_bfs": [vp, i32, vp, vp],
                "gr_bfs_ex": [vp, i32, vp, vp, P(gr_sssp_opts), P(gr_sssp_stats)],
                "gr_sssp_batch": [vp, vp, i32, vp, vp],
                "gr_sssp_batch_ex": [vp, vp, i32, vp, vp, P(gr_multi_stats)],
                "gr_sssp_multi": [vp, vp, i32, vp, vp, P(gr_multi_stats), vp],
                "gr_server_create": [P(vp), ctypes.c_size_t, P(gr_server_config)],
                "gr_server_add_graph": [vp, vp, P(i32)],
                "gr_serve_submit": [vp, i32, i32, vp, P(ctypes.c_uint64)],
                "gr_serve_poll": [vp, ctypes.c_uint64, P(gr_query_result)],
                "gr_server_destroy": [vp],
            }
            for name, args in sigs.items():
                if hasattr(L, name):
                    f = getattr(L, name)
                    f.argtypes = args
                    f.restype = ctypes.c_int
            L.gr_status_string.argtypes = [ctypes.c_int]
            L.gr_status_string.restype = ctypes.c_char_p
            L.gr_last_error.restype = ctypes.c_char_p
            L.gr_version.restype = ctypes.c_char_p
            _lib = L
    return _lib


def _status_name(s: int) -> str:
    try:
        return lib().gr_status_string(s).decode()
    except GrLibraryMissing:
        return "GR_STATUS_%d" % s


def _check(status: int, allow=(GR_OK,)) -> int:
    if status not in allow:
        raise GrError(status, lib().gr_last_error().decode())
    return status


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    if isinstance(x, np.ndarray):
        return int(x.ctypes.data)
    raise TypeError("cannot take the address of %r" % type(x))


def _stream(s) -> int | None:
    if s is None:
        try:
            import torch
            if torch.cuda.is_available():
                return int(torch.cuda.current_stream().cuda_stream) or None
        except ImportError:
            pass
        return None
    if isinstance(s, int):
        return s or None
    return int(s.cuda_stream) or None


# ---- graph ------------------------------------------------------------------

def gr_graph_create_csr(n, m, row_offsets, col_indices, weights, wt, flags=0, stream=None) -> int:
    """Returns a graph handle (int).  Host arrays are numpy arrays (int32, int32,
    uint32/float32); device arrays need ``flags |= GR_INPUT_DEVICE``."""
    keep = []
    if not (flags & GR_INPUT_DEVICE):
        ro = np.ascontiguousarray(row_offsets, dtype=np.int32)
        col = np.ascontiguousarray(col_indices, dtype=np.int32)
        w = np.ascontiguousarray(weights)
        if w.dtype == np.float32:
            w = w.view(np.uint32)
        w = np.ascontiguousarray(w, dtype=np.uint32)
        keep = [ro, col, w]
        a_ro, a_col, a_w = ro.ctypes.data, (col.ctypes.data if col.size else None), (w.ctypes.data if w.size else None)
    else:
        a_ro, a_col, a_w = _ptr(row_offsets), _ptr(col_indices), _ptr(weights)
    h = ctypes.c_void_p()
    _check(lib().gr_graph_create_csr(ctypes.byref(h), int(n), int(m), a_ro, a_col, a_w, int(wt), int(flags),
                                     _stream(stream)))
    del keep
    return h.value


def gr_graph_destroy(g: int) -> None:
    _check(lib().gr_graph_destroy(g))


def gr_graph_info(g: int) -> dict:
    """gr_graph_info and gr_graph_layout of one graph, as one dict."""
    n, m, hc, pe, pa = (ctypes.c_int32() for _ in range(5))
    wt = ctypes.c_int()
    db = ctypes.c_size_t()
    _check(lib().gr_graph_info(g, ctypes.byref(n), ctypes.byref(m), ctypes.byref(wt), ctypes.byref(db)))
    _check(lib().gr_graph_layout(g, ctypes.byref(hc), ctypes.byref(pe), ctypes.byref(pa)))
    return dict(n=n.value, m=m.value, wt=wt.value, dev_bytes=db.value, has_csc=bool(hc.value),
                pull_enabled=bool(pe.value), partitions=pa.value)


def gr_graph_layout(g: int) -> dict:
    hc, pe, pa = (ctypes.c_int32() for _ in range(3))
    _check(lib().gr_graph_layout(g, ctypes.byref(hc), ctypes.byref(pe), ctypes.byref(pa)))
    return dict(has_csc=bool(hc.value), pull_enabled=bool(pe.value), partitions=pa.value)


def _graph_n(g: int) -> int:
    n = ctypes.c_int32()
    _check(lib().gr_graph_info(g, ctypes.byref(n), None, None, None))
    return n.value


def _out_ptr(x, need: int, what: str) -> int | None:
    """Address of an output buffer of `need` 32-bit values.  Torch tensors are
    checked on the host (device memory, 4-byte elements, contiguous, large
    enough) so that a wrong buffer is an error instead of an out-of-bounds
    write on the device; raw integer addresses are the caller's promise."""
    if hasattr(x, "data_ptr") and hasattr(x, "is_cuda"):
        ok = (x.is_cuda and x.element_size() == 4 and x.is_contiguous() and x.numel() >= need)
        if not ok:
            raise GrError(GR_ERR_INVALID_ARG, "%s must be a contiguous device tensor of >= %d 4-byte elements "
                          "(got device %s, dtype %s, %d elements, contiguous %s)" % (
                              what, need, x.device, x.dtype, x.numel(), x.is_contiguous()))
        return int(x.data_ptr())
    return _ptr(x)


def gr_graph_tune(g: int, srcs, reps=3, stream=None) -> dict:
    """Times candidate schedules on queries from srcs and keeps the fastest as the graph's AUTO schedule."""
    s = np.ascontiguousarray(srcs, dtype=np.int32)
    r = gr_tune_result()
    _check(lib().gr_graph_tune(g, s.ctypes.data if s.size else None, int(s.size), int(reps), _stream(stream),
                               ctypes.byref(r)))
    return r.as_dict()


# ---- queries ----------------------------------------------------------------

def gr_sssp(g: int, src: int, dist_out, stream=None) -> None:
    _check(lib().gr_sssp(g, int(src), _out_ptr(dist_out, _graph_n(g), "dist_out"), _stream(stream)))


def gr_sssp_ex(g: int, src: int, dist_out, stream=None, loop=GR_LOOP_AUTO, direction=GR_DIR_AUTO, alpha_x16=0,
               max_iters=0, layout=GR_LAYOUT_AUTO, timing=0, filter=0, barrier_timeout_us=0, delta=0,
               relax_filter=0, beta=0, local_hops=0) -> dict:
    """delta: near-far split width as weight-type bits (see delta_bits), 0 = graph default, GR_DELTA_OFF = off.
    relax_filter: GR_RELAX_DIST / GR_RELAX_BOUND, 0 = graph default."""
    o = gr_sssp_opts(loop=loop, direction=direction, alpha_x16=alpha_x16, max_iters=max_iters, layout=layout,
                     timing=timing, filter=filter, barrier_timeout_us=barrier_timeout_us, delta=delta,
                     relax_filter=relax_filter, beta=beta, local_hops=local_hops)
    st = gr_sssp_stats()
    _check(lib().gr_sssp_ex(g, int(src), _out_ptr(dist_out, _graph_n(g), "dist_out"), _stream(stream),
                            ctypes.byref(o), ctypes.byref(st)))
    return st.as_dict()


def gr_sssp_noalloc(g: int, src: int, dist_out, stream=None) -> None:
    """gr_sssp without any allocation: the workspace is the library's fixed per-device array
    (GR_NOALLOC_SCRATCH_BYTES); calls that overlap on one GPU race."""
    _check(lib().gr_sssp_noalloc(g, int(src), _out_ptr(dist_out, _graph_n(g), "dist_out"), _stream(stream)))


def gr_bfs(g: int, src: int, depth_out, stream=None) -> None:
    _check(lib().gr_bfs(g, int(src), _out_ptr(depth_out, _graph_n(g), "depth_out"), _stream(stream)))


def gr_bfs_ex(g: int, src: int, depth_out, stream=None, loop=GR_LOOP_AUTO, direction=GR_DIR_AUTO, alpha_x16=0,
              max_iters=0, layout=GR_LAYOUT_AUTO, timing=0, filter=0, relax_filter=0, barrier_timeout_us=0,
              beta=0, local_hops=0) -> dict:
    o = gr_sssp_opts(loop=loop, direction=direction, alpha_x16=alpha_x16, max_iters=max_iters, layout=layout,
                     timing=timing, filter=filter, relax_filter=relax_filter, barrier_timeout_us=barrier_timeout_us,
                     beta=beta, local_hops=local_hops)
    st = gr_sssp_stats()
    _check(lib().gr_bfs_ex(g, int(src), _out_ptr(depth_out, _graph_n(g), "depth_out"), _stream(stream),
                           ctypes.byref(o), ctypes.byref(st)))
    return st.as_dict()


def gr_sssp_batch(g: int, srcs, dist_out, stream=None) -> None:
    s = np.ascontiguousarray(srcs, dtype=np.int32)
    out = _out_ptr(dist_out, _graph_n(g) * max(int(s.size), 1), "dist_out")
    _check(lib().gr_sssp_batch(g, s.ctypes.data if s.size else None, int(s.size), out, _stream(stream)))


def gr_sssp_batch_ex(g: int, srcs, dist_out, stream=None) -> dict:
    """gr_sssp_batch with its statistics (rounds, replays, edges_pushed, frontier_sum, source_relaxations)."""
    s = np.ascontiguousarray(srcs, dtype=np.int32)
    out = _out_ptr(dist_out, _graph_n(g) * max(int(s.size), 1), "dist_out")
    st = gr_multi_stats()
    _check(lib().gr_sssp_batch_ex(g, s.ctypes.data if s.size else None, int(s.size), out, _stream(stream),
                                  ctypes.byref(st)))
    return st.as_dict()


def gr_sssp_multi(graphs, srcs, dist_outs, stream=None) -> dict:
    """Queries (graphs[i], srcs[i]) advanced together; dist_outs[i] receives query i.  Returns the
    statistics plus 'iterations' (rounds with a non-empty frontier, per query)."""
    k = len(graphs)
    if len(srcs) != k or len(dist_outs) != k:
        raise GrError(GR_ERR_INVALID_ARG, "graphs, srcs and dist_outs differ in length")
    hs = (ctypes.c_void_p * max(k, 1))(*[int(g) for g in graphs])
    s = np.ascontiguousarray(srcs, dtype=np.int32)
    outs = (ctypes.c_void_p * max(k, 1))(*[_out_ptr(d, _graph_n(g), "dist_outs[%d]" % i)
                                           for i, (g, d) in enumerate(zip(graphs, dist_outs))])
    it = np.zeros(max(k, 1), dtype=np.int32)
    st = gr_multi_stats()
    _check(lib().gr_sssp_multi(ctypes.cast(hs, ctypes.c_void_p), s.ctypes.data if s.size else None, int(k),
                               ctypes.cast(outs, ctypes.c_void_p), _stream(stream), ctypes.byref(st),
                               it.ctypes.data))
    d = st.as_dict()
    d["iterations"] = [int(x) for x in it[:k]]
    return d


# ---- serving ----------------------------------------------------------------

def gr_server_create(hbm_budget_bytes: int, max_batch=0, num_streams=0, max_wait_us=0, local_hops=0) -> int:
    cfg = gr_server_config(max_batch=max_batch, num_streams=num_streams, max_wait_us=max_wait_us,
                           local_hops=local_hops)
    h = ctypes.c_void_p()
    _check(lib().gr_server_create(ctypes.byref(h), int(hbm_budget_bytes), ctypes.byref(cfg)))
    return h.value


_server_n = {}  # (server, graph id) -> vertex count, for the output checks of gr_serve_submit


def gr_server_add_graph(server: int, g: int) -> int:
    gid = ctypes.c_int32()
    _check(lib().gr_server_add_graph(server, g, ctypes.byref(gid)))
    _server_n[(server, gid.value)] = _graph_n(g)
    return gid.value


def gr_serve_submit(server: int, graph_id: int, src: int, dist_out) -> int:
    t = ctypes.c_uint64()
    need = _server_n.get((server, int(graph_id)), 0)
    _check(lib().gr_serve_submit(server, int(graph_id), int(src), _out_ptr(dist_out, need, "dist_out"),
                                 ctypes.byref(t)))
    return t.value


def gr_serve_poll(server: int, ticket: int):
    """Returns the result dict once done, or None while the query is pending."""
    r = gr_query_result()
    s = _check(lib().gr_serve_poll(server, int(ticket), ctypes.byref(r)), allow=(GR_OK, GR_ERR_NOT_READY))
    return r.as_dict() if s == GR_OK else None


def gr_server_destroy(server: int) -> None:
    _check(lib().gr_server_destroy(server))
    for key in [k for k in _server_n if k[0] == server]:
        del _server_n[key]


def gr_status_string(s: int) -> str:
    return lib().gr_status_string(int(s)).decode()


def gr_last_error() -> str:
    return lib().gr_last_error().decode()


def gr_version() -> str:
    return lib().gr_version().decode()


# ---- convenience --------------------------------------------------------------

class Graph:
    """Owning wrapper around a graph handle."""

    def __init__(self, n, row_offsets, col_indices, weights, wt, flags=0, stream=None):
        m = int(np.asarray(col_indices).shape[0]) if not (flags & GR_INPUT_DEVICE) else int(col_indices.numel())
        self.handle = gr_graph_create_csr(n, m, row_offsets, col_indices, weights, wt, flags, stream)
        self.n, self.m, self.wt = int(n), m, int(wt)

    @classmethod
    def from_csr(cls, csr, flags=0, stream=None):
        """From any object with n, ro, col, w (uint32 bits) and wtype attributes."""
        return cls(csr.n, csr.ro, csr.col, csr.w, csr.wtype, flags, stream)

    def info(self):
        return gr_graph_info(self.handle)

    def tune(self, srcs, reps=3, stream=None):
        return gr_graph_tune(self.handle, srcs, reps, stream)

    def close(self):
        if self.handle:
            gr_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
