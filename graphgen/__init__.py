"""Seeded synthetic labeled graphs (inputs only).

This package generates the inputs that both the CPU reference (``oracle/``)
and the GPU library consume: CSR arrays, per-edge labels and per-vertex label
sets.  It contains no part of the refinement method itself.  Every draw is
counter based (see ``graphgen.c``), so a (config, seed) pair always yields the
same arrays, whatever the thread count.

The workload shapes follow the paper's datasets (Tab. statistics-datasets and
Tab. statistics-datasets-degree): about one type label per vertex, tens to
thousands of edge labels, heavy-tailed degrees.  RMAT with Graph500-style id
scrambling stands in for the paper's RDF crawls, which are not available here.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# KBISIM_SANITIZE=1 selects a copy built with AddressSanitizer and
# UndefinedBehaviorSanitizer (host code only; the process must preload libasan).
SANITIZE = os.environ.get("KBISIM_SANITIZE", "") == "1"
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
_LIB_PATH = os.path.join(_HERE, "libgraphgen_san.so" if SANITIZE else "libgraphgen.so")
_lib = None

ST_BATCH = 9


def build(force: bool = True, sanitize: Optional[bool] = None) -> str:
    """Compile libgraphgen.so (or the sanitizer copy libgraphgen_san.so) in place (gcc, OpenMP)."""
    san = SANITIZE if sanitize is None else sanitize
    lib = os.path.join(_HERE, "libgraphgen_san.so" if san else "libgraphgen.so")
    src = os.path.join(_HERE, "graphgen.c")
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        tmp = lib + ".tmp"
        flags = ["-O1"] + SAN_FLAGS if san else ["-O3"]
        subprocess.check_call(["gcc"] + flags + ["-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, src])
        os.replace(tmp, lib)
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    i64, i32p, i64p, u64, dbl = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double
    lib.gg_rmat_edges.argtypes = [u64, ctypes.c_int, i64, dbl, dbl, dbl, ctypes.c_int, i32p, i32p]
    lib.gg_rmat_edges.restype = None
    lib.gg_uniform_edges.argtypes = [u64, i64, i64, i32p, i32p]
    lib.gg_uniform_edges.restype = None
    lib.gg_edge_labels.argtypes = [u64, i64, i64, dbl, i32p]
    lib.gg_edge_labels.restype = ctypes.c_int
    lib.gg_vertex_labels.argtypes = [u64, i64, i64, dbl, i32p]
    lib.gg_vertex_labels.restype = ctypes.c_int
    lib.gg_vertex_set_sizes.argtypes = [u64, i64, ctypes.c_void_p, ctypes.c_int, i64p]
    lib.gg_vertex_set_sizes.restype = ctypes.c_int
    lib.gg_vertex_set_labels.argtypes = [u64, i64, i64p, i64, dbl, i32p]
    lib.gg_vertex_set_labels.restype = ctypes.c_int
    lib.gg_build_csr.argtypes = [i64, i64, i32p, i32p, i32p, i64p, i32p, i32p]
    lib.gg_build_csr.restype = ctypes.c_int
    lib.gg_draw.argtypes = [u64, u64, u64]
    lib.gg_draw.restype = u64
    lib.gg_scramble.argtypes = [u64, ctypes.c_int, u64]
    lib.gg_scramble.restype = u64
    lib.gg_num_threads.argtypes = []
    lib.gg_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


@dataclass
class Graph:
    """A labeled directed graph in CSR form (forward: row v lists v's out-edges).

    ``elabel`` is None when every edge carries the same label; ``vlabel_ptr``
    is None when each vertex has exactly one label ``vlabel[v]``; both
    ``vlabel_ptr`` and ``vlabel`` None means no vertex labels (P0 = {V}).
    """
    n: int
    row_ptr: np.ndarray            # int64 [n+1]
    col: np.ndarray                # int32 [m]
    elabel: Optional[np.ndarray]   # int32 [m] or None
    vlabel_ptr: Optional[np.ndarray] = None  # int64 [n+1] or None
    vlabel: Optional[np.ndarray] = None      # int32 [n] or [vlabel_ptr[n]] or None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def label_sets(self):
        """Per-vertex label lists as Python lists (small graphs only)."""
        if self.vlabel is None:
            return [[] for _ in range(self.n)]
        if self.vlabel_ptr is None:
            return [[int(x)] for x in self.vlabel]
        return [list(map(int, self.vlabel[self.vlabel_ptr[v]:self.vlabel_ptr[v + 1]])) for v in range(self.n)]


def num_threads() -> int:
    return int(_load().gg_num_threads())


def draw(seed: int, stream: int, i: int) -> int:
    return int(_load().gg_draw(seed, stream, i))


def scramble(seed: int, bits: int, x: int) -> int:
    return int(_load().gg_scramble(seed, bits, x))


def rmat_edges(scale: int, m: int, abcd=(0.57, 0.19, 0.19, 0.05), seed: int = 1, scramble_ids: bool = True):
    lib = _load()
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    a, b, c, _ = abcd
    lib.gg_rmat_edges(seed, scale, m, a, b, c, 1 if scramble_ids else 0, _p(src), _p(dst))
    return src, dst


def uniform_edges(n: int, m: int, seed: int = 1):
    lib = _load()
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    lib.gg_uniform_edges(seed, n, m, _p(src), _p(dst))
    return src, dst


def edge_labels(m: int, L: int, zipf_s: float = 0.0, seed: int = 1) -> np.ndarray:
    out = np.empty(m, dtype=np.int32)
    if m and _load().gg_edge_labels(seed, m, L, zipf_s, _p(out)) != 0:
        raise RuntimeError("edge label generation failed")
    return out


def vertex_labels(n: int, L: int, zipf_s: float = 0.0, seed: int = 1) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    if n and _load().gg_vertex_labels(seed, n, L, zipf_s, _p(out)) != 0:
        raise RuntimeError("vertex label generation failed")
    return out


def vertex_label_sets(n: int, size_probs, L: int, zipf_s: float = 0.0, seed: int = 1):
    lib = _load()
    probs = np.asarray(size_probs, dtype=np.float64)
    ptr = np.empty(n + 1, dtype=np.int64)
    if lib.gg_vertex_set_sizes(seed, n, _p(probs), len(probs), _p(ptr)) != 0:
        raise RuntimeError("label-set size generation failed")
    lab = np.empty(int(ptr[n]), dtype=np.int32)
    if n and lib.gg_vertex_set_labels(seed, n, _p(ptr), L, zipf_s, _p(lab)) != 0:
        raise RuntimeError("label-set generation failed")
    return ptr, lab


def build_csr(n: int, src: np.ndarray, dst: np.ndarray, lbl: Optional[np.ndarray]):
    """Stable CSR by source: row v keeps v's edges in edge-list order."""
    lib = _load()
    m = int(src.shape[0])
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    row_ptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(m, dtype=np.int32)
    el = np.empty(m, dtype=np.int32) if lbl is not None else None
    if lbl is not None:
        lbl = np.ascontiguousarray(lbl, dtype=np.int32)
    if lib.gg_build_csr(n, m, _p(src), _p(dst), _p(lbl) if lbl is not None else None,
                        _p(row_ptr), _p(col), _p(el) if el is not None else None) != 0:
        raise RuntimeError("CSR build failed")
    return row_ptr, col, el


def from_edges(n: int, src, dst, lbl=None, vlabel=None, vlabel_ptr=None, name="") -> Graph:
    src = np.asarray(src, dtype=np.int32)
    dst = np.asarray(dst, dtype=np.int32)
    lbl = None if lbl is None else np.asarray(lbl, dtype=np.int32)
    row_ptr, col, el = build_csr(n, src, dst, lbl)
    vl = None if vlabel is None else np.asarray(vlabel, dtype=np.int32)
    vp = None if vlabel_ptr is None else np.asarray(vlabel_ptr, dtype=np.int64)
    return Graph(n, row_ptr, col, el, vp, vl, name=name)


def prefix_subgraph(g: Graph, vs: int) -> Graph:
    """The rows of vertices [0, vs) of g, every vertex they name kept.

    Vertices [0, vs) keep their ids; the other targets of those rows get ids
    vs, vs + 1, ... in increasing order of their old id.  Every kept vertex
    keeps its label set (or label); the other vertices of g are dropped.  Rows
    of the renumbered targets are empty.
    """
    vs = max(0, min(int(vs), g.n))
    e_end = int(g.row_ptr[vs])
    cols = g.col[:e_end]
    mark = np.zeros(g.n, dtype=bool)
    mark[cols] = True
    mark[:vs] = False
    outside = np.flatnonzero(mark)
    del mark
    remap = np.arange(g.n, dtype=np.int64)
    remap[outside] = vs + np.arange(len(outside), dtype=np.int64)
    col = remap[cols].astype(np.int32)
    del remap
    ns = vs + len(outside)
    rp = np.empty(ns + 1, dtype=np.int64)
    rp[:vs + 1] = g.row_ptr[:vs + 1]
    rp[vs + 1:] = e_end
    keep = np.concatenate([np.arange(vs, dtype=np.int64), outside])
    vp = vl = None
    if g.vlabel_ptr is not None:
        lens = g.vlabel_ptr[keep + 1] - g.vlabel_ptr[keep]
        vp = np.zeros(ns + 1, dtype=np.int64)
        np.cumsum(lens, out=vp[1:])
        idx = np.repeat(g.vlabel_ptr[keep] - vp[:-1], lens) + np.arange(vp[-1], dtype=np.int64)
        vl = np.ascontiguousarray(g.vlabel[idx], dtype=np.int32)
    elif g.vlabel is not None:
        vl = np.ascontiguousarray(g.vlabel[keep], dtype=np.int32)
    el = None if g.elabel is None else g.elabel[:e_end].copy()
    return Graph(ns, rp, col, el, vp, vl, name=f"{g.name}_rows{vs}")


def transpose(g: Graph) -> Graph:
    """The inverse graph E^-1 with l_E^-1(y, x) = l_E(x, y) (Def. inverse-schema-element)."""
    src = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(g.row_ptr))
    return from_edges(g.n, g.col, src, g.elabel, g.vlabel, g.vlabel_ptr, name=g.name + "^T")


# ----------------------------------------------------------------------------
# Workload recipes.  Each mirrors one benchmark configuration; sizes, label
# distributions and seeds are stated here and in the design notes.
# ----------------------------------------------------------------------------

def tiny(seed: int = 1, n: int = 10_000, m: int = 50_000, vlabels: int = 4, elabels: int = 8) -> Graph:
    """Uniform random directed graph, uniform vertex and edge labels (10k vertices, 50k edges)."""
    src, dst = uniform_edges(n, m, seed)
    el = edge_labels(m, elabels, 0.0, seed)
    vl = vertex_labels(n, vlabels, 0.0, seed)
    g = from_edges(n, src, dst, el, vl, name=f"uniform_n{n}_m{m}")
    g.meta = dict(kind="uniform", n=n, m=m, vlabels=vlabels, elabels=elabels, seed=seed)
    return g


def rmat(scale: int, m: int, seed: int = 2, vlabels: int = 32, vzipf: float = 1.0,
         elabels: int = 64, ezipf: float = 1.1, abcd=(0.57, 0.19, 0.19, 0.05)) -> Graph:
    """RMAT graph with one Zipf vertex label per vertex and Zipf edge labels (the 100M-edge recipe)."""
    n = 1 << scale
    src, dst = rmat_edges(scale, m, abcd, seed)
    el = edge_labels(m, elabels, ezipf, seed)
    del_src = None
    row_ptr, col, el2 = build_csr(n, src, dst, el)
    del src, dst, el, del_src
    vl = vertex_labels(n, vlabels, vzipf, seed)
    g = Graph(n, row_ptr, col, el2, None, vl, name=f"rmat_s{scale}_m{m}")
    g.meta = dict(kind="rmat", scale=scale, m=m, abcd=list(abcd), vlabels=vlabels, vzipf=vzipf,
                  elabels=elabels, ezipf=ezipf, seed=seed)
    return g


def rmat_rdf(scale: int, m: int, seed: int = 3, types: int = 1000, tzipf: float = 1.0,
             size_probs=(0.25, 0.55, 0.15, 0.05), elabels: int = 1000, ezipf: float = 1.2,
             abcd=(0.57, 0.19, 0.19, 0.05)) -> Graph:
    """RDF-like RMAT: 0-3 distinct type labels per vertex (Zipf over types), Zipf edge labels."""
    n = 1 << scale
    src, dst = rmat_edges(scale, m, abcd, seed)
    el = edge_labels(m, elabels, ezipf, seed)
    row_ptr, col, el2 = build_csr(n, src, dst, el)
    del src, dst, el
    vp, vl = vertex_label_sets(n, size_probs, types, tzipf, seed)
    g = Graph(n, row_ptr, col, el2, vp, vl, name=f"rmat_rdf_s{scale}_m{m}")
    g.meta = dict(kind="rmat_rdf", scale=scale, m=m, abcd=list(abcd), types=types, tzipf=tzipf,
                  size_probs=list(size_probs), elabels=elabels, ezipf=ezipf, seed=seed)
    return g


def deep(seed: int = 7, n: int = 20_000, avg_degree: float = 1.0) -> Graph:
    """Sparse uniform graph, one shared vertex label and one shared edge label.

    Such graphs keep refining for many iterations, so they exercise k = 3..10.
    """
    m = int(round(n * avg_degree))
    src, dst = uniform_edges(n, m, seed)
    g = from_edges(n, src, dst, None, np.zeros(n, dtype=np.int32), name=f"deep_n{n}_d{avg_degree}")
    g.meta = dict(kind="deep", n=n, m=m, seed=seed)
    return g


def batch_sizes(num_graphs: int = 4096, seed: int = 5, lo: float = 1e3, hi: float = 2e6):
    """Edge counts m_g = round(exp(U(ln lo, ln hi))) drawn per graph index."""
    out = []
    for g in range(num_graphs):
        r = draw(seed, ST_BATCH, g)
        u = (r >> 11) * (1.0 / (1 << 53))
        out.append(int(round(math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo))))))
    return out


def batch_graph(g: int, m_g: int, seed: int = 5, vlabels: int = 16, elabels: int = 32) -> Graph:
    """Graph g of the batched workload: even g uniform (n = max(16, m/8)), odd g RMAT (scale = ceil(log2(m/8)))."""
    gseed = seed * 1_000_000 + g
    if g % 2 == 0:
        n = max(16, m_g // 8)
        src, dst = uniform_edges(n, m_g, gseed)
    else:
        scale = max(1, math.ceil(math.log2(max(2, m_g / 8))))
        n = 1 << scale
        src, dst = rmat_edges(scale, m_g, (0.57, 0.19, 0.19, 0.05), gseed)
    el = edge_labels(m_g, elabels, 0.0, gseed)
    vl = vertex_labels(n, vlabels, 0.0, gseed)
    gr = from_edges(n, src, dst, el, vl, name=f"batch{g}")
    gr.meta = dict(kind="batch", g=g, m=m_g, n=n, seed=gseed)
    return gr


def serving_pool_graph(j: int, seed: int = 6, lo: float = 1e4, hi: float = 5e7) -> Graph:
    """Pool graph j of the serving workload: RMAT, m log-uniform in [lo, hi], n = 2^ceil(log2(m/12)), labels as the 100M-edge recipe."""
    r = draw(seed, ST_BATCH, j)
    u = (r >> 11) * (1.0 / (1 << 53))
    m = int(round(math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))))
    scale = max(1, math.ceil(math.log2(max(2, m / 12))))
    g = rmat(scale, m, seed=seed * 1_000_000 + j)
    g.meta["pool_index"] = j
    return g


def example_graph() -> Graph:
    """The paper's worked example (Fig. simple_example_graph).

    Vertices 0 asc, 1 dri, 2 jra, 3 uess, 4 uulm, 5 "Ansgar Scherp",
    6 "David Richerby", 7 "Jannik Rau", 8 "University of Essex",
    9 "University of Ulm".  Vertex labels in Sigma_V order: Lecturer 0,
    Literal 1, Organization 2, Professor 3, Student 4.  Edge labels:
    name 0, worksAt 1.
    """
    edges = [(0, 0, 5), (0, 1, 4), (1, 0, 6), (1, 1, 3), (2, 0, 7), (2, 1, 4), (3, 0, 8), (4, 0, 9)]
    src = [e[0] for e in edges]
    lbl = [e[1] for e in edges]
    dst = [e[2] for e in edges]
    vl = [3, 0, 4, 2, 2, 1, 1, 1, 1, 1]
    return from_edges(10, src, dst, lbl, vl, name="paper_example")
