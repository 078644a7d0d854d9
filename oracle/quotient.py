"""Summary (quotient) graph of a partition chain — TEST INFRASTRUCTURE.

Sec. "Graph Summaries for Bisimulation": the summary graph has one vertex per
equivalence class, and summary vertices B and C are connected by label l when
all vertices of the input graph represented by B have an l-edge to a vertex
represented by C.  ``summary_graph`` follows that statement with source
classes from one partition and target classes from another (for a
k-bisimulation: P_k and P_{k-1}); ``require="some"`` gives the weaker "some
vertex of B" variant, for comparison.  ``summary_graph_brute`` states the same
with plain loops for tiny graphs.
"""
from __future__ import annotations

import numpy as np


def _entries(g):
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(np.asarray(g.row_ptr, dtype=np.int64)))
    lab = np.zeros(len(g.col), dtype=np.int64) if g.elabel is None else np.asarray(g.elabel, dtype=np.int64)
    return src, lab, np.asarray(g.col, dtype=np.int64)


def summary_graph(g, src_part, dst_part, require: str = "all") -> np.ndarray:
    """Sorted int64 array [E, 3] of summary edges (B, l, C)."""
    src_part = np.asarray(src_part, dtype=np.int64)
    dst_part = np.asarray(dst_part, dtype=np.int64)
    v, lab, w = _entries(g)
    if len(v) == 0:
        return np.zeros((0, 3), dtype=np.int64)
    # the distinct (l, C) pairs of every vertex
    pairs = np.unique(np.stack([v, lab, dst_part[w]], axis=1), axis=0)
    # how many vertices of B have the pair (l, C)
    keys, members = np.unique(np.stack([src_part[pairs[:, 0]], pairs[:, 1], pairs[:, 2]], axis=1), axis=0,
                              return_counts=True)
    if require == "some":
        return keys
    if require != "all":
        raise ValueError(require)
    size = np.bincount(src_part, minlength=int(src_part.max()) + 1 if len(src_part) else 0)
    return keys[members == size[keys[:, 0]]]


def summary_graph_brute(g, src_part, dst_part):
    """The same statement as plain loops over blocks, labels and target blocks (tiny graphs only)."""
    v, lab, w = _entries(g)
    edges_of = {}
    for a, l, b in zip(v.tolist(), lab.tolist(), w.tolist()):
        edges_of.setdefault(a, set()).add((l, b))
    blocks = {}
    for x in range(g.n):
        blocks.setdefault(int(src_part[x]), []).append(x)
    targets = {}
    for x in range(g.n):
        targets.setdefault(int(dst_part[x]), []).append(x)
    out = []
    labels = sorted(set(lab.tolist()))
    for B, members in sorted(blocks.items()):
        for l in labels:
            for C, tmembers in sorted(targets.items()):
                if all(any((l, y) in edges_of.get(u, ()) for y in tmembers) for u in members):
                    out.append((B, l, C))
    return np.array(sorted(out), dtype=np.int64).reshape(-1, 3)
