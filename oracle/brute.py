"""Brute-force k-bisimilarity from the definitions — TEST INFRASTRUCTURE.

For graphs of a dozen vertices: the relations ~0, ~1, ..., ~k are built as
boolean matrices exactly as Def. edge-labeled-fw-bisimulation and the base
case of Def. vertex-labeled-bw-bisimulation state them:

* u ~0 v  iff  l_V(u) = l_V(v)  (label SETS; with no vertex labels every pair
  is related, as in Def. fw-bisim);
* u ~(j+1) v  iff  u ~j v, and for every edge (u, l, u') there is an edge
  (v, l, v') with u' ~j v', and vice versa.

Edges are the CSR entries (one label each).  The relation is then turned into
ids by first vertex: v joins the block of the smallest u <= v with u ~ v.
Nothing here is shared with the main reference or the GPU path.
"""
from __future__ import annotations

from typing import List, Tuple


def _edges(g):
    out = [[] for _ in range(g.n)]
    for v in range(g.n):
        for e in range(int(g.row_ptr[v]), int(g.row_ptr[v + 1])):
            lab = int(g.elabel[e]) if g.elabel is not None else 0
            out[v].append((lab, int(g.col[e])))
    return out


def relations(g, k: int):
    """[R_0, ..., R_k] as lists of lists of bools."""
    n = g.n
    sets = [frozenset(s) for s in g.label_sets()]
    R = [[sets[u] == sets[v] for v in range(n)] for u in range(n)]
    out = [R]
    E = _edges(g)
    for _ in range(k):
        prev = out[-1]

        def covered(a, b):
            # every edge (a, l, a') is matched by some edge (b, l, b') with a' ~ b'
            return all(any(lb == la and prev[ta][tb] for (lb, tb) in E[b]) for (la, ta) in E[a])

        R = [[prev[u][v] and covered(u, v) and covered(v, u) for v in range(n)] for u in range(n)]
        out.append(R)
    return out


def ids_from_relation(R) -> Tuple[List[int], int]:
    n = len(R)
    ids = [-1] * n
    nxt = 0
    for v in range(n):
        for u in range(v):
            if R[u][v]:
                ids[v] = ids[u]
                break
        else:
            ids[v] = nxt
            nxt += 1
    return ids, nxt


def brute_force(g, k: int):
    """(ids, counts) for k' = 0..k, from the relations."""
    rels = relations(g, k)
    ids, counts = [], []
    for R in rels:
        i, c = ids_from_relation(R)
        ids.append(i)
        counts.append(c)
    return ids, counts


def is_equivalence(R) -> bool:
    n = len(R)
    for u in range(n):
        if not R[u][u]:
            return False
        for v in range(n):
            if R[u][v] != R[v][u]:
                return False
            if R[u][v]:
                for w in range(n):
                    if R[v][w] and not R[u][w]:
                        return False
    return True
