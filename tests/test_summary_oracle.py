"""Pins of the summary-graph reference (CPU).

The reference follows the statement of Sec. "Graph Summaries for
Bisimulation" (B --l--> C when every vertex of B has an l-edge into C).  It
is checked against a hand-derived fixture of the paper's worked example,
plain loops on tiny graphs, closed forms, and the fact that along a
refinement chain (source P_k, target P_{k-1}) "every vertex" and "some
vertex" give the same graph.
"""
from __future__ import annotations

import os
import random

import numpy as np
import pytest

import graphgen
import oracle
from oracle import quotient
from tests import helpers

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_example_summary.txt")


def golden():
    out, mode = {}, None
    for line in open(GOLDEN):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "mode":
            mode = f[1]
            out[mode] = {"edges": []}
        elif f[0] in ("p_src", "p_dst"):
            out[mode][f[0]] = np.array([int(x) for x in f[1:]])
        elif f[0] == "edge":
            out[mode]["edges"].append(tuple(int(x) for x in f[1:]))
    return out


def test_worked_example_fixture():
    gold = golden()
    for mode, d in gold.items():
        g = helpers.example_variant(mode)
        # the fixture's partitions are the reference's P1 and P0
        p0, _ = oracle.initial(g)
        ids, _ = oracle.refine(g, 1)
        assert np.array_equal(p0, d["p_dst"]) and np.array_equal(ids[0], d["p_src"]), mode
        got = quotient.summary_graph(g, d["p_src"], d["p_dst"])
        assert [tuple(x) for x in got.tolist()] == d["edges"], mode


def test_matches_plain_loops_on_tiny_graphs():
    rng = random.Random(3)
    for _ in range(400):
        g = helpers.random_small_graph(rng, n_max=8, m_max=16)
        p0, _ = oracle.initial(g)
        ids, _ = oracle.refine(g, 3)
        chain = [p0] + ids
        for a, b in [(1, 0), (2, 1), (3, 2), (2, 2), (0, 0)]:
            exp = quotient.summary_graph_brute(g, chain[a], chain[b])
            got = quotient.summary_graph(g, chain[a], chain[b])
            assert np.array_equal(got, exp), (a, b)


def test_singleton_partition_gives_the_graph_itself():
    g = graphgen.tiny(seed=2, n=500, m=2000)
    ident = np.arange(g.n)
    got = quotient.summary_graph(g, ident, ident)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    exp = np.unique(np.stack([src, g.elabel, g.col], axis=1), axis=0)
    assert np.array_equal(got, exp)


def test_single_block_keeps_labels_every_vertex_has():
    g = graphgen.from_edges(4, [0, 1, 2, 3, 0, 1], [1, 2, 3, 0, 2, 3], [5, 5, 5, 5, 7, 7])
    one = np.zeros(4, dtype=np.int64)
    assert quotient.summary_graph(g, one, one).tolist() == [[0, 5, 0]]
    assert quotient.summary_graph(g, one, one, require="some").tolist() == [[0, 5, 0], [0, 7, 0]]


def test_every_and_some_coincide_along_a_chain():
    rng = random.Random(11)
    differs = 0
    for _ in range(150):
        g = helpers.random_small_graph(rng, n_max=12, m_max=30)
        p0, _ = oracle.initial(g)
        ids, _ = oracle.refine(g, 4)
        chain = [p0] + ids
        for k in range(1, 5):
            a = quotient.summary_graph(g, chain[k], chain[k - 1])
            b = quotient.summary_graph(g, chain[k], chain[k - 1], require="some")
            assert np.array_equal(a, b), k
        # with the same partition on both sides the two can differ
        a = quotient.summary_graph(g, chain[1], chain[1])
        b = quotient.summary_graph(g, chain[1], chain[1], require="some")
        differs += not np.array_equal(a, b)
    assert differs > 0
