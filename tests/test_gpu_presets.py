"""GPU tests of the device transpose and the paper's model presets.

The transpose must hold exactly the reversed entries of its input (row
order inside a row is free); the presets must reproduce the paper's printed
partitions of the worked example (Tabs. bisim-partition-schaetzle and
bisim-partition-kaushik) and match the CPU reference run on the host
transpose, bit for bit.
"""
from __future__ import annotations

import random

import numpy as np
import pytest

import graphgen
import oracle
from tests import helpers

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _kb():
    import paper_2204_05821_amd as kb
    return kb


def triples(n, row_ptr, col, elabel):
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    lab = np.zeros(len(col), dtype=np.int64) if elabel is None else elabel.astype(np.int64)
    return np.sort((src << 40) | (lab << 20) | col.astype(np.int64)) if n < (1 << 20) else None


@pytest.mark.parametrize("make", [
    lambda: graphgen.example_graph(),
    lambda: graphgen.tiny(seed=3, n=5000, m=30000),
    lambda: graphgen.rmat(14, 200_000, seed=4),
    lambda: graphgen.deep(seed=2, n=3000),
    lambda: graphgen.from_edges(1, [], []),
    lambda: graphgen.from_edges(7, [0, 0, 6, 6, 3], [6, 6, 0, 3, 3], [1, 1, 2, 0, 5]),
])
def test_transpose_matches_host(make):
    kb = _kb()
    g = make()
    rp, col, el, _, _ = kb.to_device(g)
    trp, tcol, tel = kb.transpose(rp, col, el)
    torch.cuda.synchronize()
    h = graphgen.transpose(g)
    assert np.array_equal(trp.cpu().numpy(), h.row_ptr)
    got = triples(g.n, h.row_ptr, tcol.cpu().numpy(), None if tel is None else tel.cpu().numpy())
    exp = triples(g.n, h.row_ptr, h.col, h.elabel)
    assert np.array_equal(got, exp)


def test_transpose_rejects_invalid_input():
    kb = _kb()
    g = graphgen.tiny(seed=3, n=100, m=400)
    rp, col, el, _, _ = kb.to_device(g)
    bad = col.clone()
    bad[3] = 100
    with pytest.raises(kb.KbisimError) as ei:
        kb.transpose(rp, bad, el)
    assert ei.value.code == kb.EGRAPH


def test_presets_reproduce_printed_tables():
    kb = _kb()
    from paper_2204_05821_amd import presets
    printed = helpers.parse_paper_example()
    g = graphgen.example_graph()
    rp, col, el, vl, _ = kb.to_device(g)
    for mode, r in [("schaetzle", presets.schaetzle(rp, col, el, kmax=3)),
                    ("kaushik", presets.kaushik(rp, col, vl, kmax=3))]:
        p0, _ = r.initial()
        ids, _ = r.refine(3)
        got = [p0.cpu().tolist()] + [t.cpu().tolist() for t in ids]
        for k, expect in printed[mode].items():
            assert got[k] == expect, (mode, k)
        r.close()


def test_presets_match_reference_on_random_graphs():
    kb = _kb()
    from paper_2204_05821_amd import presets
    rng = random.Random(21)
    graphs = [graphgen.tiny(seed=5, n=4000, m=16000), graphgen.rmat(13, 80_000, seed=6),
              graphgen.rmat_rdf(11, 20_000, seed=7, types=30, elabels=20)]
    graphs += [helpers.random_small_graph(rng) for _ in range(20)]
    for g in graphs:
        rp, col, el, vl, vp = kb.to_device(g)
        h = graphgen.transpose(g)
        cases = [
            ("schaetzle", presets.schaetzle(rp, col, el, kmax=5),
             graphgen.Graph(g.n, g.row_ptr, g.col, g.elabel, None, None)),
            ("kaushik", presets.kaushik(rp, col, vl, vp, kmax=5),
             graphgen.Graph(g.n, h.row_ptr, h.col, None, g.vlabel_ptr, g.vlabel)),
            ("full_bw", presets.full(rp, col, el, vl, vp, direction="bw", kmax=5), h),
        ]
        for name, r, ref_graph in cases:
            ids, counts = r.refine(5)
            exp, ec = oracle.refine(ref_graph, 5)
            assert counts == ec, (name, g.name)
            for a, b in zip(ids, exp):
                assert np.array_equal(a.cpu().numpy(), b), (name, g.name)
            r.close()
