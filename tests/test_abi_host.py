"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function ``include/gr.h`` declares, and rejects malformed input on the
host before any device call."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gr.h")

gr = pytest.importorskip("paper_2212_08200_amd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gr_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gr.LIB_PATH):
        from paper_2212_08200_amd import build
        build.build()
    return gr.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["gr_graph_create_csr", "gr_graph_destroy", "gr_graph_info", "gr_sssp", "gr_sssp_ex",
                 "gr_sssp_batch", "gr_server_create", "gr_server_add_graph", "gr_serve_submit", "gr_serve_poll",
                 "gr_server_destroy", "gr_status_string", "gr_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, "declared in gr.h but not exported: %s" % missing
    out = subprocess.run(["nm", "-D", "--defined-only", gr.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (gr_\w+)", out))
    assert set(declared_functions()) <= exported


def test_python_binding_names_match_the_c_abi():
    for n in declared_functions():
        assert hasattr(gr, n), "binding lacks %s" % n


STRUCTS = ["gr_sssp_opts", "gr_sssp_stats", "gr_tune_result", "gr_server_config", "gr_query_result",
           "gr_multi_stats"]


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct of gr.h has the size and field offsets the ctypes binding
    assumes: a C program compiled against the header prints them."""
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gr.h"', "int main(void) {"]
    for name in STRUCTS:
        cls = getattr(gr, name)
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for field, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, field, name, field))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for name in STRUCTS:
        cls = getattr(gr, name)
        assert int(got["%s size" % name]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got["%s.%s" % (name, field)]) == getattr(cls, field).offset, (name, field)
    # the served-query result carries the iteration count of the launch that served it
    assert "iterations" in dict(gr.gr_query_result._fields_)


def test_status_strings(lib):
    assert gr.gr_status_string(gr.GR_OK) == "GR_OK"
    assert gr.gr_status_string(gr.GR_ERR_SOURCE_RANGE) == "GR_ERR_SOURCE_RANGE"
    assert gr.gr_status_string(99) == "GR_ERR_UNKNOWN"
    assert gr.gr_version().startswith("gr ")


def _create(n, ro, col, w, wt=0, flags=0):
    return gr.gr_graph_create_csr(n, len(col), np.asarray(ro, np.int32), np.asarray(col, np.int32), w, wt, flags)


@pytest.mark.parametrize("case", [
    ("ro0", 3, [1, 1, 2, 2], [1, 2], np.array([1, 1], np.uint32), 0, "row_offsets[0]"),
    ("ron", 3, [0, 1, 2, 5], [1, 2], np.array([1, 1], np.uint32), 0, "row_offsets[n]"),
    ("decrease", 3, [0, 2, 1, 2], [1, 2], np.array([1, 1], np.uint32), 0, "decrease"),
    ("col_high", 3, [0, 1, 2, 2], [1, 3], np.array([1, 1], np.uint32), 0, "outside"),
    ("col_neg", 3, [0, 1, 2, 2], [1, -1], np.array([1, 1], np.uint32), 0, "outside"),
    ("neg_weight", 3, [0, 1, 2, 2], [1, 2], np.array([1.0, -1.0], np.float32), 1, "negative"),
    ("nan_weight", 3, [0, 1, 2, 2], [1, 2], np.array([1.0, np.nan], np.float32), 1, "not finite"),
    ("inf_weight", 3, [0, 1, 2, 2], [1, 2], np.array([np.inf, 1.0], np.float32), 1, "not finite"),
])
def test_malformed_csr_rejected_on_host(lib, case):
    _, n, ro, col, w, wt, text = case
    with pytest.raises(gr.GrError) as ei:
        _create(n, ro, col, w, wt)
    assert ei.value.status == gr.GR_ERR_INVALID_ARG
    assert text in ei.value.message


def test_bad_arguments_rejected(lib):
    L = gr.lib()
    h = ctypes.c_void_p()
    ro = np.array([0, 0], np.int32)
    assert L.gr_graph_create_csr(None, 1, 0, ro.ctypes.data, None, None, 0, 0, None) == gr.GR_ERR_INVALID_ARG
    assert L.gr_graph_create_csr(ctypes.byref(h), 0, 0, ro.ctypes.data, None, None, 0, 0, None) == gr.GR_ERR_INVALID_ARG
    assert L.gr_graph_create_csr(ctypes.byref(h), 1, 0, ro.ctypes.data, None, None, 7, 0, None) == gr.GR_ERR_INVALID_ARG
    assert "weight type" in gr.gr_last_error()
    assert L.gr_graph_create_csr(ctypes.byref(h), 1, 0, ro.ctypes.data, None, None, 0, 0x100, None) == gr.GR_ERR_INVALID_ARG
    assert L.gr_graph_create_csr(ctypes.byref(h), 1, 0, ro.ctypes.data, None, None, 0,
                                 gr.GR_NO_PARTITION | gr.GR_FORCE_PARTITION, None) == gr.GR_ERR_INVALID_ARG
    assert L.gr_graph_create_csr(ctypes.byref(h), 1, 2, ro.ctypes.data, None, None, 0, 0, None) == gr.GR_ERR_INVALID_ARG
    assert L.gr_sssp(None, 0, None, None) == gr.GR_ERR_INVALID_ARG
    assert L.gr_graph_destroy(None) == gr.GR_ERR_INVALID_ARG
    assert L.gr_graph_info(None, None, None, None, None) == gr.GR_ERR_INVALID_ARG
    assert L.gr_graph_layout(None, None, None, None) == gr.GR_ERR_INVALID_ARG


def test_last_error_is_per_thread(lib):
    import threading
    L = gr.lib()
    L.gr_graph_destroy(None)
    seen = {}

    def other():
        seen["t"] = gr.gr_last_error()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["t"] == ""
    assert "NULL" in gr.gr_last_error()


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import importlib
    mod = importlib.reload(gr)
    monkeypatch.setattr(mod, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(mod, "_lib", None)
    with pytest.raises(mod.GrLibraryMissing):
        mod.gr_version()
    importlib.reload(gr)
