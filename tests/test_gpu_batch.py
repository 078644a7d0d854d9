"""GPU tests of the batched form, HIP-graph replay and launch-shape tunings.

Every graph of a batch must get exactly what it gets alone (the disjoint-union
property), every replay of a captured refinement loop must equal the eager
result, and every tuning must give identical outputs.  All comparisons are
against the CPU reference, bit-exact.
"""
from __future__ import annotations

import itertools

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


def ref(g, k):
    ids, counts = oracle.refine(g, k)
    return ids, counts


def check_batch(graphs, k, label, **kw):
    kb = _kb()
    print(f"[batch] {label}: {len(graphs)} graphs, k={k}", flush=True)
    b = kb.batch_for(graphs, kmax=k, **kw)
    outs, counts = b.refine(k)
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o in outs]
    off = b.vert_off
    for gi, g in enumerate(graphs):
        exp, ec = ref(g, k)
        assert counts[gi] == ec, (label, gi, counts[gi], ec)
        for i in range(k):
            part = got[i][off[gi]:off[gi + 1]]
            if not np.array_equal(part, exp[i]):
                bad = np.nonzero(part != exp[i])[0]
                raise AssertionError(f"{label}: graph {gi} P{i + 1} differs at {bad[:8]}")
    b.close()


def mixed_graphs(seed=0, count=24):
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        m = int(np.exp(rng.uniform(np.log(200), np.log(20000))))
        out.append(graphgen.batch_graph(j, m, seed=seed + 11))
    return out


def test_batch_equals_solo_mixed_sizes():
    check_batch(mixed_graphs(), 6, "mixed")


def test_batch_narrow_keys_with_separate_labels():
    """Labels of 19 bits: with the largest graph's 12 bits of block id they fit 32-bit set keys, but
    not above the union's 17 rank bits, so the labels stay in their own array (and move with the
    rank-sorted rows); the tier graph has rows in every tier up to 20,000 entries."""
    from tests.test_gpu_parity import tier_graph
    rng = np.random.default_rng(31)
    graphs = [tier_graph(seed=12, labels=3)]
    for j in range(40):
        graphs.append(graphgen.tiny(seed=100 + j, n=3000, m=12000))
    for g in graphs:
        g.elabel = ((1 << 18) + rng.integers(0, 4, size=g.m)).astype(np.int32)
    check_batch(graphs, 5, "narrow-separate")


def test_batch_with_degenerate_members():
    gs = [graphgen.batch_graph(1, 3000),
          graphgen.from_edges(1, [], [], None, [3]),
          graphgen.from_edges(40, [], [], None, np.arange(40) % 3),
          graphgen.from_edges(5, [0, 1, 2, 3, 4], [0, 1, 2, 3, 4], [0, 1, 0, 1, 0], [1, 1, 1, 1, 1]),
          graphgen.batch_graph(2, 2500),
          graphgen.from_edges(0, [], [], None, np.zeros(0, dtype=np.int32)),
          graphgen.batch_graph(3, 8000)]
    check_batch(gs, 5, "degenerate")


def test_batch_without_vertex_labels():
    gs = [graphgen.deep(seed=s, n=3000 + 500 * s, avg_degree=1.2) for s in range(5)]
    for g in gs:
        g.vlabel = None
    check_batch(gs, 8, "unlabelled")


def test_batch_with_label_sets():
    gs = [graphgen.rmat_rdf(10 + (s % 3), 8000 + 1000 * s, seed=20 + s, types=30, elabels=20) for s in range(6)]
    check_batch(gs, 5, "label-sets")


def test_batch_with_hubs_and_collisions(monkeypatch):
    monkeypatch.setenv("KBISIM_DEBUG_HASH_BITS", "12")
    from tests.test_gpu_parity import tier_graph
    gs = [tier_graph(seed=7), graphgen.tiny(seed=3, n=2000, m=9000), tier_graph(seed=8, labels=50)]
    check_batch(gs, 4, "hubs+collisions")


def test_batch_rejects_crossing_edges():
    kb = _kb()
    a = graphgen.tiny(seed=1, n=100, m=300)
    b = graphgen.tiny(seed=2, n=100, m=300)
    rp, col, el, vl, vp, off = kb.union_of([a, b])
    col = col.copy()
    col[5] = 150          # an entry of graph 0 pointing into graph 1
    t = lambda x: None if x is None else torch.from_numpy(x).cuda()
    with pytest.raises(kb.KbisimError) as ei:
        kb.Batch(t(rp), t(col), t(el), t(vl), t(vp), off, kmax=2)
    assert ei.value.code == kb.EGRAPH


def test_batch_graph_replay():
    check_batch(mixed_graphs(seed=3, count=16), 7, "batch-graphs", graphs_mode=True)


# ------------------------------------------------------------------ HIP graphs

def test_graph_replays_match_eager():
    kb = _kb()
    g = graphgen.deep(seed=21, n=12000, avg_degree=1.4)
    exp, ec = ref(g, 9)
    r = kb.refiner_for(g, kmax=9)
    kb._lib().kbisim_use_graphs(r._ctx, 0)
    rg = kb.Refiner(*kb.to_device(g), kmax=9, graphs=True)
    outs = rg.alloc_outputs(9)
    for rep in range(4):
        ids, counts = rg.refine(9, out=outs)          # capture once, then replay
        assert counts == ec
        for a, b in zip(ids, exp):
            assert np.array_equal(a.cpu().numpy(), b)
        # eager work on the same device between replays
        ids2, c2 = r.refine(3)
        assert c2 == ec[:3]
    # a different output set and k: a second captured graph
    ids, counts = rg.refine(4)
    assert counts == ec[:4]
    rg.close()
    r.close()


def test_graph_replay_with_collision_fallback(monkeypatch):
    monkeypatch.setenv("KBISIM_DEBUG_HASH_BITS", "5")
    kb = _kb()
    g = graphgen.tiny(seed=4, n=3000, m=12000)
    exp, ec = ref(g, 5)
    rg = kb.Refiner(*kb.to_device(g), kmax=5, graphs=True)
    outs = rg.alloc_outputs(5)
    for rep in range(3):
        ids, counts = rg.refine(5, out=outs)
        assert counts == ec
        for a, b in zip(ids, exp):
            assert np.array_equal(a.cpu().numpy(), b)
    rg.close()


def test_epochs_wrap_across_eager_and_replayed_calls(monkeypatch):
    """Table epochs cycle every 15 steps and a wrap clears the table on the device.  Many eager
    and replayed calls on two contexts, eager single steps after replays, and forced collisions
    (host-driven peeling rounds advance the peeling-table epoch too) cross several wraps and must
    all give the reference results."""
    monkeypatch.setenv("KBISIM_DEBUG_HASH_BITS", "6")
    kb = _kb()
    g = graphgen.tiny(seed=8, n=3000, m=12000)
    exp, ec = ref(g, 5)
    r = kb.refiner_for(g, kmax=5)
    rg = kb.Refiner(*kb.to_device(g), kmax=5, graphs=True)
    outs = rg.alloc_outputs(5)
    sout = rg.alloc_outputs(5)
    for rep in range(7):
        print(f"[epochs] round {rep}", flush=True)
        for ctx, o in ((r, None), (rg, outs)):
            ids, counts = ctx.refine(5, out=o)
            assert counts == ec, (rep, counts, ec)
            for a, b in zip(ids, exp):
                assert np.array_equal(a.cpu().numpy(), b)
        counts = []
        for i in range(5):
            rg.step_async(i, None if i == 0 else sout[i - 1], sout[i])
            counts.append(rg.step_result(i, None if i == 0 else sout[i - 1], sout[i]))
        assert counts == ec
        for a, b in zip(sout, exp):
            assert np.array_equal(a.cpu().numpy(), b)
    r.close()
    rg.close()


def test_set_stream_after_create():
    """A context moved to another stream right after create (whose last kernels are still queued
    on the first stream), and moved again between calls, gives the reference results."""
    kb = _kb()
    from tests.test_gpu_parity import tier_graph
    g = tier_graph(seed=19)
    exp, ec = ref(g, 5)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    r = kb.Refiner(*kb.to_device(g), kmax=5, stream=s1)
    r.set_stream(s2)
    ids, counts = r.refine(5)
    assert counts == ec
    for a, b in zip(ids, exp):
        assert np.array_equal(a.cpu().numpy(), b)
    r.set_stream(s1)
    ids, counts = r.refine(3)
    assert counts == ec[:3]
    r.close()
    graphs = mixed_graphs(seed=5, count=8)
    rp, col, el, vl, vp, off = kb.union_of(graphs)
    t = lambda a: None if a is None else torch.from_numpy(a).cuda()
    b = kb.Batch(t(rp), t(col), t(el), t(vl), t(vp), off, kmax=4, stream=s1)
    b.set_stream(s2)
    outs, counts = b.refine(4)
    torch.cuda.synchronize()
    off = b.vert_off
    for gi, gg in enumerate(graphs):
        e, c = ref(gg, 4)
        assert counts[gi] == c
        for i in range(4):
            assert np.array_equal(outs[i][off[gi]:off[gi + 1]].cpu().numpy(), e[i])
    b.close()


# ------------------------------------------------------------------ tunings

@pytest.mark.parametrize("re,hc,hp,kbits", list(itertools.product([1024, 2048], [2048, 4096], [1024, 2048],
                                                                   [0, 64])))
def test_every_tuning_gives_identical_results(re, hc, hp, kbits):
    kb = _kb()
    from tests.test_gpu_parity import tier_graph
    for g in [graphgen.rmat(14, 250_000, seed=5), tier_graph(seed=9)]:
        exp, ec = ref(g, 4)
        r = kb.Refiner(*kb.to_device(g), kmax=4, tuning=kb.tuning(re, hc, hp, kbits))
        ids, counts = r.refine(4)
        assert counts == ec
        for a, b in zip(ids, exp):
            assert np.array_equal(a.cpu().numpy(), b)
        r.close()


# ------------------------------------------------------------------ single steps

def _stepwise_batch(graphs, k):
    kb = _kb()
    b = kb.batch_for(graphs, kmax=k)
    outs = b.alloc_outputs(k)
    counts = []
    for i in range(k):
        b.step_async(i, outs[i])
        counts.append(b.step_result(i, outs[i]))
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o in outs]
    off = b.vert_off
    b.close()
    return got, counts, off


@pytest.mark.parametrize("bits", [None, "6"])
def test_batch_single_steps_equal_reference(bits, monkeypatch):
    if bits:
        monkeypatch.setenv("KBISIM_DEBUG_HASH_BITS", bits)
    graphs = mixed_graphs(seed=5, count=10)
    got, counts, off = _stepwise_batch(graphs, 6)
    for gi, g in enumerate(graphs):
        exp, ec = ref(g, 6)
        assert [counts[i][gi] for i in range(6)] == ec
        for i in range(6):
            assert np.array_equal(got[i][off[gi]:off[gi + 1]], exp[i]), (gi, i)


@pytest.mark.parametrize("bits", [None, "5"])
def test_solo_single_steps_equal_reference(bits, monkeypatch):
    if bits:
        monkeypatch.setenv("KBISIM_DEBUG_HASH_BITS", bits)
    kb = _kb()
    g = graphgen.tiny(seed=6, n=4000, m=20000)
    exp, ec = ref(g, 7)
    r = kb.refiner_for(g, kmax=7)
    outs = r.alloc_outputs(7)
    for rep in range(2):
        counts = []
        for i in range(7):
            r.step_async(i, None if i == 0 else outs[i - 1], outs[i])
            counts.append(r.step_result(i, None if i == 0 else outs[i - 1], outs[i]))
        assert counts == ec
        for a, b in zip(outs, exp):
            assert np.array_equal(a.cpu().numpy(), b)
    r.close()


def test_gather_probe_runs_on_small_and_empty_graphs():
    kb = _kb()
    for g in [graphgen.from_edges(3, [0, 1], [1, 2]), graphgen.tiny(seed=2, n=500, m=3000),
              graphgen.from_edges(5, [], [])]:
        r = kb.refiner_for(g, kmax=1)
        ids, _ = r.refine(1)
        assert r.gather_probe(ids[0], reps=2) >= 0.0
        ids2, _ = r.refine(1)                      # the context still refines correctly afterwards
        assert torch.equal(ids[0], ids2[0])
        r.close()


def test_batch_with_device_built_schedule(monkeypatch):
    """Batches with the degree schedule built on the device (graphs of every size in one union)."""
    monkeypatch.setenv("KBISIM_DEBUG_DEVICE_SCHEDULE", "1")
    check_batch(mixed_graphs(seed=8, count=24), 4, "device schedule")
