"""GPU tests of the summary (quotient) graph against the CPU reference."""
from __future__ import annotations

import random

import numpy as np
import pytest

import graphgen
import oracle
from oracle import quotient
from tests import helpers
from tests.test_summary_oracle import golden

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _kb():
    import paper_2204_05821_amd as kb
    return kb


def gpu_summary(r, a, b):
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).cuda()
    s, l, d = r.quotient(t(a), t(b))
    return np.stack([s.cpu().numpy(), l.cpu().numpy(), d.cpu().numpy()], axis=1).astype(np.int64)


def test_worked_example():
    kb = _kb()
    for mode, d in golden().items():
        g = helpers.example_variant(mode)
        r = kb.refiner_for(g, kmax=2)
        got = gpu_summary(r, d["p_src"], d["p_dst"])
        assert [tuple(x) for x in got.tolist()] == d["edges"], mode
        r.close()


@pytest.mark.parametrize("make", [
    lambda: graphgen.tiny(seed=1),
    lambda: graphgen.rmat(14, 200_000, seed=2),
    lambda: graphgen.deep(seed=7, n=20_000, avg_degree=1.0),
    lambda: graphgen.rmat_rdf(12, 60_000, seed=3),
])
def test_chain_summaries_match_reference(make):
    kb = _kb()
    g = make()
    p0, _ = oracle.initial(g)
    ids, _ = oracle.refine(g, 4)
    chain = [p0] + ids
    r = kb.refiner_for(g, kmax=4)
    for a, b in [(1, 0), (2, 1), (4, 3)]:
        exp = quotient.summary_graph(g, chain[a], chain[b])
        got = gpu_summary(r, chain[a], chain[b])
        assert np.array_equal(got, exp), (g.name, a, b)
    # same partition on both sides: the union of the members' edges
    exp = quotient.summary_graph(g, chain[2], chain[2], require="some")
    assert np.array_equal(gpu_summary(r, chain[2], chain[2]), exp)
    r.close()


@pytest.mark.parametrize("kbits", [0, 64])
def test_summaries_over_every_tier(kbits):
    """Keys are built over the degree schedule: ranges, single-row ranges, staged hub chunks and
    the global-set hubs (rows past the staged limit); labels packed, separate and sorted with
    their rows."""
    kb = _kb()
    from tests.test_gpu_parity import giant_hub_graph, tier_graph
    wide = tier_graph(seed=14, labels=50, shared_targets=2000)
    wide.elabel = (((1 << 30) + 7) * (wide.elabel.astype(np.int64) + 1) % ((1 << 31) - 1)).astype(np.int32)
    seen = {"range": 0, "workgroup": 0, "hub": 0, "hub_global": 0}
    for g in [tier_graph(seed=12, labels=50, shared_targets=2000), wide, giant_hub_graph()]:
        ids, _ = oracle.refine(g, 2)
        r = kb.Refiner(*kb.to_device(g), kmax=2, tuning=kb.tuning(key_bits=kbits))
        for tier, v in r.schedule_info().items():
            seen[tier] += v["vertices"]
        exp = quotient.summary_graph(g, ids[1], ids[0])
        assert np.array_equal(gpu_summary(r, ids[1], ids[0]), exp), g.name
        r.close()
    assert all(v > 0 for v in seen.values()), seen


def test_singletons_and_random_small_graphs():
    kb = _kb()
    rng = random.Random(5)
    for _ in range(25):
        g = helpers.random_small_graph(rng, n_max=30, m_max=90)
        if g.m == 0:
            continue
        p0, _ = oracle.initial(g)
        ids, _ = oracle.refine(g, 2)
        r = kb.refiner_for(g, kmax=2)
        assert np.array_equal(gpu_summary(r, ids[1], ids[0]), quotient.summary_graph(g, ids[1], ids[0]))
        ident = np.arange(g.n)
        assert np.array_equal(gpu_summary(r, ident, ident), quotient.summary_graph(g, ident, ident))
        r.close()


def test_rejects_ids_out_of_range():
    kb = _kb()
    g = graphgen.tiny(seed=3, n=200, m=800)
    r = kb.refiner_for(g, kmax=1)
    bad = np.zeros(g.n, dtype=np.int32)
    bad[7] = g.n
    with pytest.raises(kb.KbisimError) as ei:
        gpu_summary(r, bad, np.zeros(g.n, dtype=np.int32))
    assert ei.value.code == kb.EINVAL
    r.close()
