"""CPU tests of the property checker used for full-size parity.

The checker must accept every partition chain the reference produces and
reject each kind of wrong partition: ids not numbered by first vertex, a
block that crosses previous blocks, a block holding two signatures, two
blocks with one key, and the outputs of the reference's planted mistakes.
"""
from __future__ import annotations

import random

import numpy as np
import pytest

import graphgen
import oracle
from tests import helpers


def chain(g, k):
    p0, _ = oracle.initial(g)
    ids, counts = oracle.refine(g, k)
    return [p0] + ids


def canon(ids):
    """Renumber an id array by first vertex."""
    m = {}
    return np.array([m.setdefault(int(x), len(m)) for x in ids], dtype=np.int32)


GRAPHS = [
    lambda: graphgen.tiny(seed=4, n=3000, m=12000),
    lambda: graphgen.rmat(12, 50_000, seed=3),
    lambda: graphgen.deep(seed=7, n=5000, avg_degree=1.2),
    lambda: graphgen.rmat_rdf(11, 20_000, seed=5, types=40, elabels=30),
    lambda: helpers.example_variant("schaetzle"),
    lambda: helpers.example_variant("kaushik"),
    lambda: graphgen.from_edges(50, [], [], None, np.arange(50) % 4),
    lambda: graphgen.from_edges(0, [], []),
]


@pytest.mark.parametrize("make", GRAPHS)
def test_accepts_reference_chains(make):
    g = make()
    ch = chain(g, 8)
    assert oracle.check_initial(g, ch[0]) == len(set(ch[0].tolist()))
    for i in range(8):
        assert oracle.check_step(g, ch[i], ch[i + 1]) == len(set(ch[i + 1].tolist()))


def test_accepts_random_small_graphs():
    rng = random.Random(5)
    for _ in range(100):
        g = helpers.random_small_graph(rng)
        ch = chain(g, 5)
        oracle.check_initial(g, ch[0])
        for i in range(5):
            oracle.check_step(g, ch[i], ch[i + 1])


def _first_split_step(ch):
    for i in range(1, len(ch)):
        if len(set(ch[i].tolist())) > len(set(ch[i - 1].tolist())):
            return i
    raise AssertionError("no split")


def test_rejects_noncanonical_ids():
    g = graphgen.tiny(seed=4, n=3000, m=12000)
    ch = chain(g, 3)
    bad = ch[2].copy()
    a, b = bad == 0, bad == 1
    bad[a], bad[b] = 1, 0
    with pytest.raises(AssertionError, match="first vertex"):
        oracle.check_step(g, ch[1], bad)
    with pytest.raises(AssertionError, match="first vertex"):
        oracle.check_initial(g, np.where(ch[0] == 0, 99, ch[0]).astype(np.int32))


def test_rejects_block_across_previous_blocks():
    g = graphgen.tiny(seed=4, n=3000, m=12000)
    ch = chain(g, 3)
    cur, prev = ch[2].copy(), ch[1]
    # merge the blocks of vertices 0 and the first vertex with another previous block
    v = int(np.nonzero(prev != prev[0])[0][0])
    cur[cur == cur[v]] = cur[0]
    with pytest.raises(AssertionError, match="not a refinement"):
        oracle.check_step(g, prev, canon(cur))


def test_rejects_merged_signatures():
    g = graphgen.tiny(seed=4, n=3000, m=12000)
    ch = chain(g, 3)
    i = _first_split_step(ch)
    prev, cur = ch[i - 1], ch[i].copy()
    # two blocks of cur inside one block of prev, merged
    for b in range(int(prev.max()) + 1):
        blocks = np.unique(cur[prev == b])
        if len(blocks) >= 2:
            cur[cur == blocks[1]] = blocks[0]
            break
    with pytest.raises(AssertionError, match="two different signatures"):
        oracle.check_step(g, prev, canon(cur))


def test_rejects_split_block():
    g = graphgen.tiny(seed=4, n=3000, m=12000)
    ch = chain(g, 3)
    prev, cur = ch[1], ch[2].copy()
    sizes = np.bincount(cur)
    b = int(np.nonzero(sizes >= 2)[0][0])
    v = int(np.nonzero(cur == b)[0][-1])
    cur[v] = cur.max() + 1
    with pytest.raises(AssertionError, match="share one key"):
        oracle.check_step(g, prev, canon(cur))


def test_rejects_wrong_initial_partitions():
    g = graphgen.rmat_rdf(11, 20_000, seed=5, types=40, elabels=30)
    p0, _ = oracle.initial(g)
    merged = p0.copy()
    merged[merged == 1] = 0
    with pytest.raises(AssertionError):
        oracle.check_initial(g, canon(merged))
    split = p0.copy()
    v = int(np.nonzero(p0 == 0)[0][-1])
    split[v] = p0.max() + 1
    with pytest.raises(AssertionError):
        oracle.check_initial(g, canon(split))


@pytest.mark.parametrize("mutation", sorted(oracle.MUTATIONS))
def test_rejects_planted_mistakes_of_the_reference(mutation):
    """Every planted mistake, where it changes some partition, is rejected at the first wrong step."""
    rng = random.Random(17)
    graphs = [graphgen.tiny(seed=4, n=3000, m=12000), graphgen.deep(seed=7, n=3000, avg_degree=1.3),
              graphgen.rmat_rdf(10, 8000, seed=5, types=30, elabels=20)]
    graphs += [helpers.random_small_graph(rng) for _ in range(60)]
    caught = 0
    for g in graphs:
        good = chain(g, 5)
        with oracle.planted_mistake(mutation):
            bad = chain(g, 5)
        diff = [i for i in range(6) if not np.array_equal(good[i], bad[i])]
        if not diff:
            continue
        i = diff[0]
        with pytest.raises(AssertionError):
            if i == 0:
                oracle.check_initial(g, bad[0])
            else:
                oracle.check_step(g, bad[i - 1], bad[i])
        caught += 1
    assert caught > 0, "the mutation never changed a result on these graphs"
