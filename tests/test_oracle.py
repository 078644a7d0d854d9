"""Pins for the CPU reference (runs without a GPU).

The reference is checked against things other than itself:
* the paper's printed partitions of its worked example (tests/golden);
* brute-force relations built from the definitions on thousands of tiny graphs;
* an independent splitter-based refinement;
* closed forms (paths, cycles, complete binary trees, all-distinct labels, m = 0);
* refinement invariants and metamorphic relations;
* planted mistakes, each of which must fail at least one of the pins above.
"""
from __future__ import annotations

import random

import numpy as np
import pytest

import graphgen
import oracle
from oracle import brute, splitter
from tests import helpers


def oracle_all(g, k):
    """[P0, P1, ..., Pk] and counts from the reference."""
    p0, c0 = oracle.initial(g)
    ids, counts = oracle.refine(g, k)
    return [list(map(int, p0))] + [list(map(int, x)) for x in ids], [c0] + counts


# ---------------------------------------------------------------- worked example

PRINTED = helpers.parse_paper_example()


@pytest.mark.parametrize("mode", ["fw", "bw", "schaetzle", "kaushik"])
def test_paper_example_printed_tables(mode):
    """Tabs. bisim-partition-fw/-bw/-schaetzle/-kaushik, k = 0..2."""
    g = helpers.example_variant(mode)
    ids, counts = oracle_all(g, 3)
    for k, expect in PRINTED[mode].items():
        assert ids[k] == expect, (mode, k, ids[k], expect)
        assert counts[k] == max(expect) + 1


def test_paper_example_prose_facts():
    # Schaetzle's variant is stable from k = 1 on; Kaushik's is all singletons at k = 2.
    ids, counts = oracle_all(helpers.example_variant("schaetzle"), 4)
    assert ids[1] == ids[2] == ids[3] == ids[4]
    ids, counts = oracle_all(helpers.example_variant("kaushik"), 4)
    assert counts[2] == 10 and ids[2] == list(range(10))
    # Printed block counts: fw 1,2,3; bw 1,2,3; Schaetzle 1,3,3; Kaushik 5,9,10.
    for mode, exp in [("fw", [1, 2, 3]), ("bw", [1, 2, 3]), ("schaetzle", [1, 3, 3]), ("kaushik", [5, 9, 10])]:
        assert oracle_all(helpers.example_variant(mode), 2)[1] == exp


@pytest.mark.parametrize("mode", ["full_fw", "full_bw"])
def test_paper_example_labelled_modes_match_brute_force(mode):
    """Vertex- and edge-labelled modes (not printed in the paper): pinned by brute force."""
    g = helpers.example_variant(mode)
    ids, counts = oracle_all(g, 4)
    bids, bcounts = brute.brute_force(g, 4)
    assert ids == bids and counts == bcounts
    if mode == "full_fw":
        assert ids[0] == [0, 1, 2, 3, 3, 4, 4, 4, 4, 4] and ids[3] == ids[0]


# ---------------------------------------------------------------- brute force

def test_brute_force_relation_is_equivalence():
    rng = random.Random(11)
    for _ in range(60):
        g = helpers.random_small_graph(rng, n_max=8, m_max=14)
        for R in brute.relations(g, 3):
            assert brute.is_equivalence(R)


def test_is_equivalence_rejects_non_equivalences():
    """The relation check must fail on each way a relation can miss being an equivalence."""
    n = 4
    ident = [[u == v for v in range(n)] for u in range(n)]
    full = [[True] * n for _ in range(n)]
    assert brute.is_equivalence(ident) and brute.is_equivalence(full)
    two_blocks = [[(u < 2) == (v < 2) for v in range(n)] for u in range(n)]
    assert brute.is_equivalence(two_blocks)
    not_reflexive = [row[:] for row in two_blocks]
    not_reflexive[3][3] = False
    assert not brute.is_equivalence(not_reflexive)
    asymmetric = [row[:] for row in ident]
    asymmetric[0][2] = True            # 0 ~ 2 but not 2 ~ 0
    assert not brute.is_equivalence(asymmetric)
    not_transitive = [row[:] for row in ident]
    for u, v in [(0, 1), (1, 0), (1, 2), (2, 1)]:   # 0 ~ 1 ~ 2 but not 0 ~ 2
        not_transitive[u][v] = True
    assert not brute.is_equivalence(not_transitive)


@pytest.mark.parametrize("seed", range(8))
def test_oracle_matches_brute_force(seed):
    """Random graphs with n <= 12: empty label sets, parallel edges, self-loops, 1-3 edge labels."""
    rng = random.Random(1000 + seed)
    for _ in range(250):
        g = helpers.random_small_graph(rng)
        if rng.random() < 0.3:
            g = graphgen.transpose(g)
        k = rng.randint(0, 6)
        ids, counts = oracle_all(g, k)
        bids, bcounts = brute.brute_force(g, k)
        assert ids == bids, (g.n, g.m, k)
        assert counts == bcounts


def test_oracle_matches_brute_force_deep_chains():
    """Sparse unlabeled graphs that keep refining for many iterations, k up to 12."""
    rng = random.Random(77)
    for _ in range(150):
        n = rng.randint(4, 12)
        m = rng.randint(n // 2, n + 2)
        g = graphgen.from_edges(n, [rng.randrange(n) for _ in range(m)], [rng.randrange(n) for _ in range(m)])
        ids, counts = oracle_all(g, 12)
        bids, bcounts = brute.brute_force(g, 12)
        assert ids == bids and counts == bcounts


# ---------------------------------------------------------------- splitter oracle

@pytest.mark.parametrize("seed,n,m,L,V", [(1, 300, 900, 3, 2), (2, 2000, 5000, 4, 3), (3, 5000, 6000, 1, 1),
                                           (4, 3000, 12000, 8, 4)])
def test_oracle_matches_splitter_refinement(seed, n, m, L, V):
    src, dst = graphgen.uniform_edges(n, m, seed)
    el = graphgen.edge_labels(m, L, 0.0, seed)
    vl = graphgen.vertex_labels(n, V, 0.0, seed)
    g = graphgen.from_edges(n, src, dst, el, vl)
    ids, counts = oracle_all(g, 8)
    sids, scounts = splitter.splitter_refine(g, 8)
    assert counts == scounts
    for a, b in zip(ids, sids):
        assert a == b


def test_splitter_matches_on_deep_and_rmat():
    for g in [graphgen.deep(seed=8, n=3000, avg_degree=1.0), graphgen.rmat(11, 20000, seed=9)]:
        ids, counts = oracle_all(g, 10)
        sids, scounts = splitter.splitter_refine(g, 10)
        assert counts == scounts and ids == sids


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("L", [1, 2, 5, 17])
def test_directed_path(L):
    """Path 0->1->...->L-1, no labels: id_k(p) = max(0, p - max(0, L-1-k)), count_k = min(k, L-1) + 1."""
    g = graphgen.from_edges(L, list(range(L - 1)), list(range(1, L)))
    ids, counts = oracle_all(g, L + 2)
    for k in range(L + 3):
        assert ids[k] == [max(0, p - max(0, L - 1 - k)) for p in range(L)]
        assert counts[k] == min(k, L - 1) + 1


def test_disjoint_cycles_single_block():
    src, dst, n = [], [], 0
    for length in [1, 2, 3, 7, 11]:
        for i in range(length):
            src.append(n + i)
            dst.append(n + (i + 1) % length)
        n += length
    g = graphgen.from_edges(n, src, dst)
    ids, counts = oracle_all(g, 6)
    assert all(c == 1 for c in counts)


@pytest.mark.parametrize("height", [1, 3, 6])
def test_complete_binary_tree(height):
    """Edges parent -> children (heap order); a vertex's block is min(height above the leaves, k)."""
    n = 2 ** (height + 1) - 1
    src = [v for v in range(n) for c in (2 * v + 1, 2 * v + 2) if c < n]
    dst = [c for v in range(n) for c in (2 * v + 1, 2 * v + 2) if c < n]
    g = graphgen.from_edges(n, src, dst)
    hv = [height - int(np.floor(np.log2(v + 1))) for v in range(n)]
    ids, counts = oracle_all(g, height + 2)
    for k in range(height + 3):
        assert ids[k] == helpers.canonical([min(h, k) for h in hv])
        assert counts[k] == min(k, height) + 1


def test_all_distinct_labels_singletons():
    g = graphgen.tiny(seed=4, n=500, m=2000)
    g.vlabel = np.arange(g.n, dtype=np.int32)
    ids, counts = oracle_all(g, 3)
    for x in ids:
        assert x == list(range(g.n))


def test_no_edges_keeps_initial_partition():
    g = graphgen.from_edges(50, [], [], None, [i % 7 for i in range(50)])
    ids, counts = oracle_all(g, 5)
    assert all(x == ids[0] for x in ids) and counts == [7] * 6


def test_no_vertex_labels_single_initial_block():
    g = graphgen.tiny(seed=5, n=100, m=300)
    g.vlabel = None
    p0, c0 = oracle.initial(g)
    assert c0 == 1 and not p0.any()


def test_empty_graph():
    g = graphgen.from_edges(0, [], [])
    ids, counts = oracle.refine(g, 3)
    assert counts == [0, 0, 0]


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("maker", ["tiny", "rmat", "deep", "rdf"])
def test_refinement_invariants(maker):
    g = {"tiny": lambda: graphgen.tiny(seed=1),
         "rmat": lambda: graphgen.rmat(12, 40000, seed=2),
         "deep": lambda: graphgen.deep(seed=7, n=4000),
         "rdf": lambda: graphgen.rmat_rdf(12, 30000, seed=3, types=50, elabels=40)}[maker]()
    ids, counts = oracle_all(g, 10)
    fixed = None
    for k in range(len(ids)):
        helpers.check_canonical(ids[k], counts[k])
        if k:
            helpers.check_refines(ids[k], ids[k - 1])
            assert counts[k] >= counts[k - 1]
            if fixed is not None:
                assert ids[k] == ids[fixed]
            elif counts[k] == counts[k - 1]:
                fixed = k - 1
                assert ids[k] == ids[k - 1]
                assert splitter.is_stable(g, ids[k])


def test_is_stable_rejects_unstable_partitions():
    """Stability (Def. partition-stable, with labelled splitters) on hand-built cases.

    Vertex 0 has an a-edge into block {2}, vertex 1 a b-edge into it: the
    block {0, 1} is split by either splitter, so only the partition that
    separates 0 from 1 is stable.  A vertex without an edge into a block is
    split from one that has such an edge.
    """
    g = graphgen.from_edges(3, [0, 1], [2, 2], [0, 1])
    assert not splitter.is_stable(g, [0, 0, 1])
    assert splitter.is_stable(g, [0, 1, 2])
    g = graphgen.from_edges(3, [0, 1], [2, 2], [0, 0])
    assert splitter.is_stable(g, [0, 0, 1])           # same label: {0, 1} is stable
    assert not splitter.is_stable(g, [0, 0, 0])       # 2 has no edge into the block, 0 does
    g = graphgen.from_edges(2, [0], [1], [0])
    assert not splitter.is_stable(g, [0, 0])
    assert splitter.is_stable(g, [0, 1])


@pytest.mark.parametrize("mode", ["fw", "bw", "schaetzle", "kaushik"])
def test_is_stable_matches_printed_fixpoints(mode):
    """In the printed tables a partition is stable exactly when the next one repeats it."""
    g = helpers.example_variant(mode)
    printed = PRINTED[mode]
    for k in sorted(printed):
        if k + 1 in printed:
            assert splitter.is_stable(g, printed[k]) == (printed[k + 1] == printed[k]), (mode, k)


def test_is_stable_iff_brute_force_fixpoint():
    """On random tiny graphs: P_k is stable iff brute force gives P_{k+1} = P_k."""
    rng = random.Random(23)
    seen = {True: 0, False: 0}
    for _ in range(150):
        g = helpers.random_small_graph(rng, n_max=9, m_max=16)
        bids, _ = brute.brute_force(g, 5)
        for k in range(5):
            fix = bids[k + 1] == bids[k]
            assert splitter.is_stable(g, bids[k]) == fix, k
            seen[fix] += 1
    assert seen[True] > 50 and seen[False] > 50


def test_resume_from_intermediate_partition():
    g = graphgen.deep(seed=9, n=3000)
    ids, counts = oracle.refine(g, 8)
    ids2, counts2 = oracle.refine(g, 5, start=ids[2])
    for a, b in zip(ids[3:], ids2):
        assert np.array_equal(a, b)
    assert counts[3:] == counts2


# ---------------------------------------------------------------- metamorphic

def test_vertex_permutation_permutes_partition():
    g = graphgen.tiny(seed=3, n=2000, m=8000)
    rng = np.random.default_rng(5)
    perm = rng.permutation(g.n).astype(np.int32)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    h = graphgen.from_edges(g.n, perm[src], perm[g.col], g.elabel, None)
    vl = np.empty(g.n, dtype=np.int32)
    vl[perm] = g.vlabel
    h.vlabel = vl
    a, _ = oracle_all(g, 6)
    b, _ = oracle_all(h, 6)
    for x, y in zip(a, b):
        assert helpers.as_blocks(x, perm) == helpers.as_blocks(y)


def test_row_shuffle_and_duplicates_do_not_matter():
    g = graphgen.rmat(10, 8000, seed=4)
    rng = np.random.default_rng(6)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    dup = rng.random(g.m) < 0.3
    s2 = np.concatenate([src, src[dup]])
    d2 = np.concatenate([g.col, g.col[dup]])
    l2 = np.concatenate([g.elabel, g.elabel[dup]])
    order = rng.permutation(len(s2))
    h = graphgen.from_edges(g.n, s2[order], d2[order], l2[order], g.vlabel)
    a, ca = oracle_all(g, 6)
    b, cb = oracle_all(h, 6)
    assert a == b and ca == cb


@pytest.mark.parametrize("maker", ["tiny", "rmat", "rdf"])
def test_prefix_rows_keep_the_first_step(maker):
    """The rows of the first vs vertices, with all other targets renumbered, give the whole
    graph's P0 and P1 on those vertices: a step only reads a vertex's own row and its
    targets' previous blocks, and ids are numbered by first vertex."""
    g = {"tiny": lambda: graphgen.tiny(seed=4),
         "rmat": lambda: graphgen.rmat(12, 40000, seed=5),
         "rdf": lambda: graphgen.rmat_rdf(12, 30000, seed=6, types=50, elabels=40)}[maker]()
    full, fc = oracle_all(g, 2)
    for vs in (1, g.n // 7, g.n // 2, g.n):
        s = graphgen.prefix_subgraph(g, vs)
        assert s.m == int(g.row_ptr[vs])
        sub, _ = oracle_all(s, 1)
        assert sub[0][:vs] == full[0][:vs] and sub[1][:vs] == full[1][:vs], vs


def test_label_bijection_does_not_matter():
    g = graphgen.tiny(seed=6, n=3000, m=9000)
    h = graphgen.Graph(g.n, g.row_ptr, g.col, (g.elabel * 7919 + 13).astype(np.int32), None,
                       (1000 - g.vlabel).astype(np.int32))
    assert oracle_all(g, 5) == oracle_all(h, 5)


def test_disjoint_union_restricts_to_components():
    gs = [graphgen.tiny(seed=s, n=300 + 50 * s, m=900 + 100 * s) for s in range(4)]
    src, dst, lbl, vl, off = [], [], [], [], 0
    for g in gs:
        s = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        src.append(s + off)
        dst.append(g.col + off)
        lbl.append(g.elabel)
        vl.append(g.vlabel + 100 * len(vl))   # distinct label range per component
        off += g.n
    u = graphgen.from_edges(off, np.concatenate(src), np.concatenate(dst), np.concatenate(lbl), np.concatenate(vl))
    ui, _ = oracle_all(u, 6)
    off = 0
    for g in gs:
        gi, gc = oracle_all(g, 6)
        for k in range(7):
            part = ui[k][off:off + g.n]
            assert helpers.canonical(part) == gi[k]
            assert len(set(part)) == gc[k]
        off += g.n


# ---------------------------------------------------------------- planted mistakes

_PIN_CASES = []


def _pin_cases():
    """Random tiny graphs with their brute-force partitions (computed once; independent of the reference)."""
    if not _PIN_CASES:
        rng = random.Random(2024)
        for _ in range(300):
            g = helpers.random_small_graph(rng)
            k = rng.randint(1, 4)
            _PIN_CASES.append((g, k, brute.brute_force(g, k)))
    return _PIN_CASES


def _pins_pass() -> bool:
    """True iff the reference passes a compact set of the pins above."""
    cases = _pin_cases()
    try:
        for mode in ["fw", "bw", "schaetzle", "kaushik"]:
            ids, _ = oracle_all(helpers.example_variant(mode), 2)
            for k, expect in PRINTED[mode].items():
                if ids[k] != expect:
                    return False
        for g, k, expect in cases:
            if oracle_all(g, k) != expect:
                return False
        L = 9
        g = graphgen.from_edges(L, list(range(L - 1)), list(range(1, L)))
        ids, counts = oracle_all(g, 4)
        for k in range(5):
            if ids[k] != [max(0, p - max(0, L - 1 - k)) for p in range(L)]:
                return False
        return True
    except ValueError:
        return False


def test_pins_pass_on_the_reference():
    assert _pins_pass()


@pytest.mark.parametrize("mutation", sorted(oracle.MUTATIONS))
def test_planted_mistake_is_caught(mutation):
    with oracle.planted_mistake(mutation):
        caught = not _pins_pass()
    assert caught, f"planted mistake '{mutation}' passed every pin"
    assert _pins_pass()
