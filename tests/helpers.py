"""Shared test helpers: fixtures parsing, small-graph makers, partition checks."""
from __future__ import annotations

import os
import random
from collections import defaultdict

import numpy as np

import graphgen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def parse_paper_example():
    """{mode: {k: canonical id list}} from the paper's printed partition tables."""
    names = None
    out = {}
    mode = None
    with open(os.path.join(GOLDEN, "paper_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("vertices"):
                names = line.split()[1:]
            elif line.startswith("mode"):
                mode = line.split()[1]
                out[mode] = {}
            elif line.startswith("k "):
                head, body = line.split(":", 1)
                k = int(head.split()[1])
                block_of = {}
                for b, blk in enumerate(body.split("|")):
                    for nm in blk.split():
                        assert nm not in block_of, nm
                        block_of[nm] = b
                assert sorted(block_of) == sorted(names), (mode, k)
                out[mode][k] = canonical([block_of[nm] for nm in names])
    return out


def canonical(labels):
    """Renumber any block labelling by first vertex."""
    ren = {}
    res = []
    for x in labels:
        x = int(x)
        if x not in ren:
            ren[x] = len(ren)
        res.append(ren[x])
    return res


def as_blocks(ids, perm=None):
    """Partition as a set of frozensets (optionally mapping vertex v -> perm[v])."""
    d = defaultdict(set)
    for v, b in enumerate(ids):
        d[int(b)].add(v if perm is None else int(perm[v]))
    return {frozenset(s) for s in d.values()}


def example_variant(mode: str) -> graphgen.Graph:
    """The worked example set up for one of the paper's bisimulation variants."""
    g = graphgen.example_graph()
    if mode in ("fw", "bw"):
        g = graphgen.Graph(g.n, g.row_ptr, g.col, None, None, None, name=mode)
    elif mode == "schaetzle":
        g = graphgen.Graph(g.n, g.row_ptr, g.col, g.elabel, None, None, name=mode)
    elif mode == "kaushik":
        g = graphgen.Graph(g.n, g.row_ptr, g.col, None, None, g.vlabel, name=mode)
    elif mode == "full_fw":
        pass
    elif mode == "full_bw":
        pass
    else:
        raise KeyError(mode)
    if mode in ("bw", "kaushik", "full_bw"):
        g = graphgen.transpose(g)
    return g


def random_small_graph(rng: random.Random, n_max=12, m_max=24, elabels_max=3, vlabels_max=3,
                       label_sets=True) -> graphgen.Graph:
    n = rng.randint(1, n_max)
    m = rng.randint(0, m_max)
    src = [rng.randrange(n) for _ in range(m)]
    dst = [rng.randrange(n) for _ in range(m)]
    L = rng.randint(1, elabels_max)
    lbl = [rng.randrange(L) for _ in range(m)] if rng.random() < 0.8 else None
    mode = rng.random()
    if not label_sets or mode < 0.2:
        vl, vp = None, None
    elif mode < 0.5:
        vl = [rng.randrange(vlabels_max) for _ in range(n)]
        vp = None
    else:
        sets = [[rng.randrange(vlabels_max + 1) for _ in range(rng.randint(0, 3))] for _ in range(n)]
        vp = np.zeros(n + 1, dtype=np.int64)
        vp[1:] = np.cumsum([len(s) for s in sets])
        vl = [x for s in sets for x in s]
    g = graphgen.from_edges(n, src, dst, lbl, vl, vp)
    if vl is not None and vp is not None and len(vl) == 0:
        g.vlabel = np.zeros(0, dtype=np.int32)
    return g


def check_canonical(ids, count):
    """First occurrences are 0, 1, 2, ... in vertex order; ids are dense."""
    seen = -1
    for x in ids:
        x = int(x)
        if x > seen:
            assert x == seen + 1, "ids not numbered by first vertex"
            seen = x
    assert seen + 1 == count


def check_refines(fine, coarse):
    """Every block of `fine` lies inside one block of `coarse` (Def. partition-refinement)."""
    f = np.asarray(fine)
    c = np.asarray(coarse)
    order = np.lexsort((c, f))
    fs, cs = f[order], c[order]
    same = fs[1:] == fs[:-1]
    assert np.all(cs[1:][same] == cs[:-1][same]), "partition does not refine its predecessor"
