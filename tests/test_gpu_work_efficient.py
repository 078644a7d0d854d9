"""GPU tests of the work-efficient mode: the same partitions as the CPU
reference (bit for bit) while singleton blocks are skipped and the loop
stops at the fixpoint."""
from __future__ import annotations

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


def check(g, k, label, start=None):
    kb = _kb()
    print(f"[work-efficient] {label} n={g.n} m={g.m} k={k}", flush=True)
    r = kb.refiner_for(g, kmax=k)
    r.work_efficient(True)
    for rep in range(2):
        ids, counts = r.refine(k, start=None if start is None else torch.from_numpy(start).cuda())
        exp, ec = oracle.refine(g, k, start=start)
        assert counts == list(ec), (label, counts, ec)
        for i, (a, b) in enumerate(zip(ids, exp)):
            assert np.array_equal(a.cpu().numpy(), b), (label, i)
    steps = r.work_efficient(None)
    r.close()
    return steps, ec


def first_fixpoint(counts, c0):
    prev = c0
    for i, c in enumerate(counts):
        if c == prev:
            return i + 1
        prev = c
    return len(counts)


@pytest.mark.parametrize("make,k", [
    (lambda: graphgen.tiny(seed=1), 10),
    (lambda: graphgen.rmat(14, 200_000, seed=2), 10),
    (lambda: graphgen.deep(seed=7, n=20_000, avg_degree=1.0), 10),
    (lambda: graphgen.deep(seed=8, n=20_000, avg_degree=1.5), 10),
    (lambda: graphgen.rmat_rdf(13, 80_000, seed=3), 8),
    (lambda: helpers.example_variant("full_fw"), 4),
    (lambda: helpers.example_variant("kaushik"), 4),
    (lambda: graphgen.from_edges(64, [], [], None, np.arange(64) % 5), 4),
])
def test_same_partitions_fewer_steps(make, k):
    g = make()
    steps, ec = check(g, k, g.name)
    p0, c0 = oracle.initial(g)
    assert steps == first_fixpoint(list(ec), c0)


def test_tiers_and_forced_collisions(monkeypatch):
    from tests.test_gpu_parity import giant_hub_graph, tier_graph
    check(tier_graph(seed=3), 6, "tiers")
    check(giant_hub_graph(seed=4), 4, "giant-hubs")
    monkeypatch.setenv("KBISIM_DEBUG_HASH_BITS", "6")
    check(tier_graph(seed=5), 5, "tiers-collide")
    check(graphgen.deep(seed=9, n=6000, avg_degree=1.2), 8, "deep-collide")


def test_resume_from_a_partition():
    g = graphgen.deep(seed=12, n=8000, avg_degree=1.3)
    exp, _ = oracle.refine(g, 4)
    check(g, 5, "resume", start=exp[3])


def test_batch_work_efficient():
    kb = _kb()
    from tests.test_gpu_batch import mixed_graphs
    graphs = mixed_graphs(seed=9, count=12) + [graphgen.deep(seed=3, n=4000, avg_degree=1.1)]
    graphs[-1].elabel = np.zeros(graphs[-1].m, dtype=np.int32)
    b = kb.batch_for(graphs, kmax=8)
    b.work_efficient(True)
    outs, counts = b.refine(8)
    got = [o.cpu().numpy() for o in outs]
    for gi, g in enumerate(graphs):
        exp, ec = oracle.refine(g, 8)
        assert counts[gi] == list(ec), gi
        for i in range(8):
            assert np.array_equal(got[i][b.vert_off[gi]:b.vert_off[gi + 1]], exp[i]), (gi, i)
    b.close()


def test_single_steps_with_skipping():
    kb = _kb()
    g = graphgen.deep(seed=11, n=10_000, avg_degree=1.2)
    exp, ec = oracle.refine(g, 7)
    r = kb.refiner_for(g, kmax=7)
    r.work_efficient(True)
    outs = r.alloc_outputs(7)
    counts = []
    for i in range(7):
        r.step_async(i, None if i == 0 else outs[i - 1], outs[i])
        counts.append(r.step_result(i, None if i == 0 else outs[i - 1], outs[i]))
    assert counts == list(ec)
    for a, b in zip(outs, exp):
        assert np.array_equal(a.cpu().numpy(), b)
    r.close()
