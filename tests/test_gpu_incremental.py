"""Incremental k-bisimulation on an edited graph (GPU) against a refinement
from scratch of the edited graph, on the GPU and in the CPU reference.

A context caches the chain of a refine call on the original graph; an update
gets the edited graph (edges deleted and inserted) and the vertices whose rows
changed, and recomputes P'_1..P'_k: only the vertices whose key inputs can
have changed are re-signed, the others reuse their cached key hashes.  The
result must equal, bit for bit, what refining the edited graph from scratch
gives.  Edits: single edges, a hundred, a few percent of all edges, rows
emptied and filled, a hub row, and several edits against one cached chain.
"""
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


def edited(g, rng, n_del, n_ins, empty_rows=(), fill_rows=(), touch_rows=()):
    """g with n_del random entries deleted, n_ins random edges inserted (labels drawn from g's),
    every entry of empty_rows deleted, a few edges added to each of fill_rows and, in each of
    touch_rows, one entry deleted and one edge added.
    Returns (edited graph, the vertices whose rows changed)."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    keep = np.ones(g.m, dtype=bool)
    if n_del:
        keep[rng.choice(g.m, size=n_del, replace=False)] = False
    for v in empty_rows:
        keep[g.row_ptr[v]:g.row_ptr[v + 1]] = False
    for v in touch_rows:
        keep[int(rng.integers(g.row_ptr[v], g.row_ptr[v + 1]))] = False
    ins_src = list(rng.integers(0, g.n, size=n_ins))
    for v in fill_rows:
        ins_src += [v] * 3
    ins_src += list(touch_rows)
    ins_src = np.asarray(ins_src, dtype=np.int64)
    ins_dst = rng.integers(0, g.n, size=len(ins_src))
    labs = g.elabel if g.elabel is not None else None
    ins_lab = rng.choice(labs, size=len(ins_src)) if labs is not None and g.m else None
    s2 = np.concatenate([src[keep], ins_src])
    d2 = np.concatenate([g.col[keep], ins_dst])
    l2 = None if labs is None else np.concatenate([labs[keep], ins_lab if ins_lab is not None else []])
    g2 = graphgen.from_edges(g.n, s2, d2, l2, g.vlabel, g.vlabel_ptr, name=g.name + "_edited")
    rows = np.unique(np.concatenate([src[~keep], ins_src])).astype(np.int32)
    return g2, rows


def fresh(g, k, tuning=None):
    kb = _kb()
    r = kb.Refiner(*kb.to_device(g), kmax=k, tuning=tuning)
    ids, counts = r.refine(k)
    out = [t.cpu().numpy() for t in ids]
    r.close()
    return out, counts


class Cached:
    """A context on g with its chain cached (one refine call)."""

    def __init__(self, g, k, tuning=None):
        kb = _kb()
        self.g, self.k = g, k
        self.dev = kb.to_device(g)
        self.r = kb.Refiner(*self.dev, kmax=k, tuning=tuning)
        self.r.incremental()
        self.base_ids, self.base_counts = self.r.refine(k)

    def update(self, g2, rows, k=None):
        k = self.k if k is None else k
        rp = torch.from_numpy(g2.row_ptr).cuda()
        col = torch.from_numpy(g2.col).cuda()
        el = None if g2.elabel is None else torch.from_numpy(g2.elabel).cuda()
        rw = torch.from_numpy(np.asarray(rows, dtype=np.int32)).cuda()
        ids, counts = self.r.update(rp, col, el, rw, k)
        torch.cuda.synchronize()
        return [t.cpu().numpy() for t in ids], counts

    def close(self):
        self.r.close()


def check_update(c, g2, rows, label, k=None, tuning=None, with_ref=True):
    k = c.k if k is None else k
    got, gc = c.update(g2, rows, k)
    exp, ec = fresh(g2, k, tuning)
    assert gc == ec, (label, gc, ec)
    for i in range(k):
        if not np.array_equal(got[i], exp[i]):
            bad = np.nonzero(got[i] != exp[i])[0]
            raise AssertionError(f"{label}: P{i + 1} differs at {bad[:8]} ({len(bad)}): {got[i][bad[:8]]} vs "
                                 f"{exp[i][bad[:8]]}")
    if with_ref:
        ref, rc = oracle.refine(g2, k)
        assert rc == gc, label
        for i in range(k):
            assert np.array_equal(ref[i], got[i]), (label, i)
    print(f"[incr] {label}: {len(rows)} edited rows, counts {gc}", flush=True)


GRAPHS = {
    "tiny": lambda: graphgen.tiny(seed=5),
    "rmat": lambda: graphgen.rmat(14, 200_000, seed=6),
    "rdf": lambda: graphgen.rmat_rdf(13, 90_000, seed=7, types=200, elabels=300),
    "deep": lambda: graphgen.deep(seed=8, n=20_000, avg_degree=1.3),
    # vertex counts that are not multiples of 4: a step's slice of the cached
    # chain starts unaligned, and the per-vertex passes take one vertex at a time
    "odd1": lambda: graphgen.tiny(seed=15, n=4_001, m=20_000),
    "odd2": lambda: graphgen.tiny(seed=16, n=4_094, m=30_000, elabels=60),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_update_equals_refine_from_scratch(name):
    g = GRAPHS[name]()
    k = 10 if name == "deep" else 6
    c = Cached(g, k)
    rng = np.random.default_rng(31)
    try:
        for n_del, n_ins in [(1, 0), (0, 1), (50, 50), (g.m // 40, g.m // 40)]:
            g2, rows = edited(g, rng, n_del, n_ins)
            check_update(c, g2, rows, f"{name} -{n_del}+{n_ins}")
        # no edit at all: the cached chain itself
        got, gc = c.update(g, np.zeros(0, dtype=np.int32))
        assert gc == c.base_counts
        for a, b in zip(got, c.base_ids):
            assert np.array_equal(a, b.cpu().numpy())
    finally:
        c.close()


@pytest.mark.parametrize("name", ["tiny", "rmat", "rdf"])
def test_update_with_global_dirty_filter(name, monkeypatch):
    """The global filter of dirty keys (taken with many dirty vertices) forced on every list
    step: clean vertices whose key or name bit is set there probe the table, the others not."""
    monkeypatch.setenv("KBISIM_DEBUG_GFILTER_MIN", "1")
    g = GRAPHS[name]()
    c = Cached(g, 6)
    rng = np.random.default_rng(51)
    try:
        for n_del, n_ins in [(1, 0), (0, 1), (50, 50), (400, 400)]:
            g2, rows = edited(g, rng, n_del, n_ins)
            check_update(c, g2, rows, f"{name} gfilter -{n_del}+{n_ins}")
    finally:
        c.close()


def test_outputs_off_16_byte_boundaries():
    """Output tensors that start 4, 8 or 12 bytes past a 16-byte boundary (views into one
    buffer): the per-vertex passes and the fixpoint copies then write them one id at a time;
    refine and update results equal those into fresh tensors."""
    g = GRAPHS["rmat"]()
    k = 6
    c = Cached(g, k)
    rng = np.random.default_rng(61)
    try:
        g2, rows = edited(g, rng, 20, 20)
        exp, ec = c.update(g2, rows)
        buf = torch.empty(k * g.n + 16, dtype=torch.int32, device="cuda")
        for off in (1, 2, 3):
            outs = [buf[off + i * g.n: off + (i + 1) * g.n] for i in range(k)]
            ids, counts = c.r.refine(k, out=outs)
            assert counts == c.base_counts
            for a, b in zip(ids, c.base_ids):
                assert bool((a == b).all())
            rp = torch.from_numpy(g2.row_ptr).cuda()
            col = torch.from_numpy(g2.col).cuda()
            el = torch.from_numpy(g2.elabel).cuda()
            rw = torch.from_numpy(np.asarray(rows, dtype=np.int32)).cuda()
            ids2, counts2 = c.r.update(rp, col, el, rw, k, out=outs)
            assert counts2 == ec
            for a, b in zip(ids2, exp):
                assert np.array_equal(a.cpu().numpy(), b), off
    finally:
        c.close()


def test_rows_emptied_filled_and_a_hub_row():
    g = graphgen.rmat(13, 150_000, seed=9)
    deg = np.diff(g.row_ptr)
    hub = int(np.argmax(deg))
    empty = [int(v) for v in np.nonzero(deg == 0)[0][:5]]
    full = [int(v) for v in np.nonzero(deg > 3)[0][:5]]
    c = Cached(g, 6)
    rng = np.random.default_rng(5)
    try:
        g2, rows = edited(g, rng, 10, 10, empty_rows=full + [hub], fill_rows=empty)
        assert hub in rows and all(v in rows for v in empty)
        check_update(c, g2, rows, "emptied/filled/hub")
    finally:
        c.close()


@pytest.mark.parametrize("kbits", [32, 64])
def test_update_with_other_key_forms(kbits):
    kb = _kb()
    g = graphgen.rmat_rdf(13, 80_000, seed=11, types=100, elabels=200)
    t = kb.tuning(key_bits=kbits)
    c = Cached(g, 5, tuning=t)
    rng = np.random.default_rng(kbits)
    try:
        for n_del, n_ins in [(3, 3), (2000, 2000)]:
            g2, rows = edited(g, rng, n_del, n_ins)
            check_update(c, g2, rows, f"keys{kbits} -{n_del}+{n_ins}", tuning=t)
    finally:
        c.close()


def test_update_with_wide_labels_and_hub_tiers():
    """Labels too wide to pack (hashed keys by default) and rows in every tier up to hubs."""
    from tests.test_gpu_parity import tier_graph
    g = tier_graph(seed=21, labels=200, shared_targets=3000)
    g.elabel = (((1 << 30) + 7) * (g.elabel.astype(np.int64) + 1) % ((1 << 31) - 1)).astype(np.int32)
    c = Cached(g, 4)
    rng = np.random.default_rng(2)
    try:
        for n_del, n_ins in [(5, 5), (3000, 3000)]:
            g2, rows = edited(g, rng, n_del, n_ins)
            check_update(c, g2, rows, f"wide-tiers -{n_del}+{n_ins}")
    finally:
        c.close()


@pytest.mark.parametrize("kbits", [0, 64])
def test_edited_long_rows(kbits):
    """Edited rows past 4096 entries (each one a global hash set of its own, or the list kernel's
    passes where no spare set space is left), with their twins left unedited."""
    kb = _kb()
    from tests.test_gpu_parity import tier_graph
    g = tier_graph(seed=17, labels=4, shared_targets=500)
    deg = np.diff(g.row_ptr)
    long_rows = [int(v) for v in np.nonzero(deg > 4096)[0] if v % 2 == 0]
    assert len(long_rows) >= 4
    t = kb.tuning(key_bits=kbits)
    c = Cached(g, 4, tuning=t)
    rng = np.random.default_rng(40 + kbits)
    try:
        g2, rows = edited(g, rng, 3, 3, touch_rows=long_rows)
        check_update(c, g2, rows, f"long rows keys{kbits}", tuning=t)
        g3, rows3 = edited(g, rng, 0, 0, empty_rows=long_rows[:1], touch_rows=long_rows[1:])
        check_update(c, g3, rows3, f"long rows emptied keys{kbits}", tuning=t)
    finally:
        c.close()


def test_edited_giant_hub_rows():
    """Edits to rows of 4.5M entries."""
    from tests.test_gpu_parity import giant_hub_graph
    g = giant_hub_graph()
    c = Cached(g, 3)
    rng = np.random.default_rng(77)
    try:
        g2, rows = edited(g, rng, 5, 5, touch_rows=[1, 2])
        check_update(c, g2, rows, "giant hubs", with_ref=False)
    finally:
        c.close()


def test_several_edits_against_one_cached_chain_and_shorter_k():
    g = graphgen.tiny(seed=12)
    c = Cached(g, 8)
    rng = np.random.default_rng(8)
    try:
        g2, rows2 = edited(g, rng, 30, 30)
        check_update(c, g2, rows2, "first")
        g3, rows3 = edited(g, rng, 400, 10)
        check_update(c, g3, rows3, "second, against the same chain")
        check_update(c, g3, rows3, "k=3", k=3)
        check_update(c, g2, np.concatenate([rows2, rows2[:5]]), "repeated rows")
    finally:
        c.close()


def test_update_with_forced_hash_collisions(monkeypatch):
    monkeypatch.setenv("KBISIM_DEBUG_HASH_BITS", "7")
    g = graphgen.tiny(seed=13, n=4000, m=16000)
    c = Cached(g, 5)
    rng = np.random.default_rng(3)
    try:
        for n_del, n_ins in [(2, 2), (800, 800)]:
            g2, rows = edited(g, rng, n_del, n_ins)
            check_update(c, g2, rows, f"collide -{n_del}+{n_ins}")
    finally:
        c.close()


def test_update_argument_errors():
    kb = _kb()
    g = graphgen.tiny(seed=14, n=2000, m=8000)
    r = kb.refiner_for(g, kmax=4)
    rp, col, el = (torch.from_numpy(x).cuda() for x in (g.row_ptr, g.col, g.elabel))
    v = int(np.nonzero(np.diff(g.row_ptr))[0][0])      # a vertex with entries
    rows = torch.tensor([v], dtype=torch.int32, device="cuda")
    with pytest.raises(kb.KbisimError):      # not enabled
        r.update(rp, col, el, rows, 2)
    r.incremental()
    with pytest.raises(kb.KbisimError):      # no cached chain yet
        r.update(rp, col, el, rows, 2)
    r.refine(3)
    with pytest.raises(kb.KbisimError):      # more steps than cached
        r.update(rp, col, el, rows, 4)
    with pytest.raises(kb.KbisimError):      # a listed vertex out of range
        r.update(rp, col, el, torch.tensor([2000], dtype=torch.int32, device="cuda"), 2)
    bad = el.clone()
    bad[int(g.row_ptr[v]):int(g.row_ptr[v + 1])] = int(g.elabel.max()) + 1
    with pytest.raises(kb.KbisimError):      # a label beyond the cached graph's
        r.update(rp, col, bad, rows, 2)
    with pytest.raises(kb.KbisimError):      # work-efficient mode needs every step, updates the cache
        r.work_efficient(True)
    ids, counts = r.update(rp, col, el, rows, 3)
    exp, ec = oracle.refine(g, 3)
    assert counts == ec and all(np.array_equal(a.cpu().numpy(), b) for a, b in zip(ids, exp))
    r.close()
