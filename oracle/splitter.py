"""Splitter-based refinement in the style of Alg. kaushik-alg — TEST INFRASTRUCTURE.

An independent mechanism for the same partitions: instead of building
signatures, each iteration copies the current partition (P^cp) and, for every
copied block B^cp not used before and every edge label l, splits each current
block B into the vertices that have an l-labelled edge into B^cp and those that
do not (Def. split-original, adapted to labelled splitters).  Blocks already
used as splitters are skipped in later iterations, since a partition stable
with respect to a set stays stable under refinement (the usedSplitters rule of
Alg. kaushik-alg).

Alg. kaushik-alg computes backward bisimulation with successor sets; the
forward relation of a graph is the backward relation of its inverse graph
(Def. inverse-schema-element), so here the split test uses predecessors.
The initial partition groups equal vertex label sets.
"""
from __future__ import annotations

from collections import defaultdict
from typing import List, Tuple

import numpy as np


def _canonical(block_of: List[int]) -> Tuple[List[int], int]:
    ren = {}
    out = []
    for b in block_of:
        if b not in ren:
            ren[b] = len(ren)
        out.append(ren[b])
    return out, len(ren)


def splitter_refine(g, k: int):
    """(ids, counts) for k' = 0..k."""
    n = g.n
    # predecessors with labels: pred[w] = [(v, l), ...] for every edge (v, l, w)
    pred = [[] for _ in range(n)]
    for v in range(n):
        for e in range(int(g.row_ptr[v]), int(g.row_ptr[v + 1])):
            lab = int(g.elabel[e]) if g.elabel is not None else 0
            pred[int(g.col[e])].append((v, lab))
    # partition V by label set
    keyed = {}
    block_of = []
    for s in g.label_sets():
        key = frozenset(s)
        if key not in keyed:
            keyed[key] = len(keyed)
        block_of.append(keyed[key])
    members = defaultdict(set)
    for v, b in enumerate(block_of):
        members[b].add(v)
    next_id = len(keyed)
    used = set()
    ids0, c0 = _canonical(block_of)
    all_ids, all_counts = [ids0], [c0]
    for _ in range(k):
        copy = [frozenset(s) for s in members.values()]
        for bcp in copy:
            if bcp in used:
                continue
            hit = defaultdict(set)
            for w in bcp:
                for (v, lab) in pred[w]:
                    hit[lab].add(v)
            for lab in sorted(hit):
                touched = defaultdict(list)
                for v in hit[lab]:
                    touched[block_of[v]].append(v)
                for b, vs in touched.items():
                    if len(vs) < len(members[b]):
                        nb = next_id
                        next_id += 1
                        for v in vs:
                            members[b].discard(v)
                            block_of[v] = nb
                        members[nb] = set(vs)
            used.add(bcp)
        ids, c = _canonical(block_of)
        all_ids.append(ids)
        all_counts.append(c)
    return all_ids, all_counts


def is_stable(g, ids) -> bool:
    """Every block is stable w.r.t. every (label, block) splitter (Def. partition-stable, labelled)."""
    ids = np.asarray(ids)
    n = g.n
    blocks = defaultdict(list)
    for v in range(n):
        blocks[int(ids[v])].append(v)
    hits = defaultdict(set)  # (label, target block) -> vertices with such an edge
    for v in range(n):
        for e in range(int(g.row_ptr[v]), int(g.row_ptr[v + 1])):
            lab = int(g.elabel[e]) if g.elabel is not None else 0
            hits[(lab, int(ids[int(g.col[e])]))].add(v)
    size = {b: len(vs) for b, vs in blocks.items()}
    for s in hits.values():
        touched = defaultdict(int)
        for v in s:
            touched[int(ids[v])] += 1
        for b, inside in touched.items():
            if inside < size[b]:
                return False
    return True
