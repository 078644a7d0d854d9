"""The C-ABI library loads and exports what include/kbisim.h declares; host-side
argument checks answer before any HIP call (runs without a GPU)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")
LIB = os.path.join(ROOT, "paper_2204_05821_amd", "libkbisim.so")


def declared_functions():
    names = []
    for fn in sorted(os.listdir(HEADER_DIR)):
        if fn.endswith(".h"):
            text = open(os.path.join(HEADER_DIR, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(kbisim_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libkbisim.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


class Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("nlabels", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("elabel", ctypes.c_void_p),
                ("vlabel_ptr", ctypes.c_void_p), ("vlabel", ctypes.c_void_p)]


def test_header_declares_the_core_api():
    names = declared_functions()
    for f in ["kbisim_workspace_bytes", "kbisim_create", "kbisim_initial", "kbisim_refine",
              "kbisim_refine_from", "kbisim_destroy", "kbisim_strerror"]:
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_workspace_bytes_argument_checks(lib):
    f = lib.kbisim_workspace_bytes
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    f.restype = ctypes.c_int
    out = ctypes.c_size_t(0)
    g = Graph(1000, 5000, 0, None, None, None, None, None)
    assert f(None, 10, ctypes.byref(out)) == -1
    assert f(ctypes.byref(g), 10, None) == -1
    assert f(ctypes.byref(g), -1, ctypes.byref(out)) == -1
    assert f(ctypes.byref(Graph(-1, 0, 0)), 10, ctypes.byref(out)) == -1
    assert f(ctypes.byref(Graph(1 << 31, 0, 0)), 10, ctypes.byref(out)) == -5
    assert f(ctypes.byref(g), 10, ctypes.byref(out)) == 0
    small = out.value
    assert small > 0
    assert f(ctypes.byref(Graph(100_000, 5000, 0)), 10, ctypes.byref(out)) == 0 and out.value > small
    assert f(ctypes.byref(Graph(1000, 500_000, 0)), 10, ctypes.byref(out)) == 0 and out.value > small


def test_create_rejects_bad_arguments_before_touching_the_device(lib):
    f = lib.kbisim_create
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    ctx = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails before a HIP call
    g = Graph(1000, 5000, 0, fake, fake, None, None, None)
    assert f(None, 4, fake, 1 << 30, None, ctypes.byref(ctx)) == -1
    assert f(ctypes.byref(g), 4, fake, 1 << 30, None, None) == -1
    assert f(ctypes.byref(g), -2, fake, 1 << 30, None, ctypes.byref(ctx)) == -1
    assert f(ctypes.byref(g), 4, None, 1 << 30, None, ctypes.byref(ctx)) == -1
    assert f(ctypes.byref(g), 4, fake, 16, None, ctypes.byref(ctx)) == -3           # workspace too small
    assert f(ctypes.byref(Graph(1000, 5000, 0, None, fake)), 4, fake, 1 << 30, None, ctypes.byref(ctx)) == -1
    assert f(ctypes.byref(Graph(1000, 5000, 0, fake, None)), 4, fake, 1 << 30, None, ctypes.byref(ctx)) == -1
    assert f(ctypes.byref(Graph(1 << 31, 5, 0, fake, fake)), 4, fake, 1 << 30, None, ctypes.byref(ctx)) == -5


def test_null_context_and_strerror(lib):
    lib.kbisim_refine.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.kbisim_refine.restype = ctypes.c_int
    assert lib.kbisim_refine(None, 3, None, None) == -1
    lib.kbisim_strerror.argtypes = [ctypes.c_int]
    lib.kbisim_strerror.restype = ctypes.c_char_p
    for code in range(-6, 1):
        assert lib.kbisim_strerror(code)
    lib.kbisim_destroy.argtypes = [ctypes.c_void_p]
    assert lib.kbisim_destroy(None) == 0


def test_transpose_argument_checks_before_touching_the_device(lib):
    wb = lib.kbisim_transpose_workspace_bytes
    wb.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
    wb.restype = ctypes.c_int
    out = ctypes.c_size_t(0)
    assert wb(100, 50, None) == -1
    assert wb(-1, 0, ctypes.byref(out)) == -1
    assert wb(1 << 31, 0, ctypes.byref(out)) == -5
    assert wb(1000, 5000, ctypes.byref(out)) == 0 and out.value >= 12 * 1000
    f = lib.kbisim_transpose
    f.argtypes = [ctypes.c_int64, ctypes.c_int64] + [ctypes.c_void_p] * 7 + [ctypes.c_size_t, ctypes.c_void_p]
    f.restype = ctypes.c_int
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails before a HIP call
    assert f(1000, 5000, None, fake, None, fake, fake, None, fake, 1 << 30, None) == -1
    assert f(1000, 5000, fake, None, None, fake, fake, None, fake, 1 << 30, None) == -1
    assert f(1000, 5000, fake, fake, None, fake, fake, None, None, 1 << 30, None) == -3
    assert f(1000, 5000, fake, fake, None, fake, fake, None, fake, 8, None) == -3
    assert f(1 << 31, 5, fake, fake, None, fake, fake, None, fake, 1 << 30, None) == -5


def test_the_two_billion_edge_graph_fits_one_gpu(lib):
    """The workspace of the 2B-edge RDF-like graph (2^28 vertices, about one label each), its CSR,
    labels and ten output arrays fit the 288 GB of one MI355X with room to spare, and the
    workspace grows linearly with the graph (the sizes are computed on the host)."""
    f = lib.kbisim_workspace_bytes
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    f.restype = ctypes.c_int
    out = ctypes.c_size_t(0)
    n, m = 1 << 28, 2_000_000_000
    assert f(ctypes.byref(Graph(n, m, n)), 10, ctypes.byref(out)) == 0
    ws = out.value
    csr = 8 * (n + 1) + 4 * m + 4 * m + 8 * (n + 1) + 4 * n   # row_ptr, col, elabel, label-set CSR
    outputs = 10 * 4 * n
    assert ws + csr + outputs < 0.5 * 288e9, (ws, csr, outputs)
    assert f(ctypes.byref(Graph(n // 2, m // 2, n // 2)), 10, ctypes.byref(out)) == 0
    assert 0.45 < out.value / ws < 0.55


def test_noalloc_rejects_graphs_beyond_its_scratch_before_touching_the_device(lib):
    lib.kbisim_noalloc_scratch_bytes.restype = ctypes.c_size_t
    limit = lib.kbisim_noalloc_scratch_bytes()
    assert limit == 128 << 20
    f = lib.kbisim_refine_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    fake = ctypes.c_void_p(0x1000)   # never dereferenced
    outs = (ctypes.c_void_p * 4)(fake, fake, fake, fake)
    counts = (ctypes.c_int64 * 4)()
    big = Graph(2_000_000, 4_000_000, 0, fake, fake, None, None, None)
    assert f(ctypes.byref(big), 4, outs, counts, None) == -3
    assert f(None, 4, outs, counts, None) == -1
    assert f(ctypes.byref(big), -1, outs, counts, None) == -1
    assert f(ctypes.byref(Graph(1000, 5000, 0, fake, fake, None, None, None)), 4, None, counts, None) == -1
