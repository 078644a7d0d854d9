"""GPU parity: the HIP path (through the C ABI) against the CPU reference, bit-exact.

Every test here needs an MI355X and the built libkbisim.so; the library is
called through its C ABI (ctypes binding), never through a fallback.
"""
from __future__ import annotations

import os
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


def gpu_all(g, k, kmax=None):
    """[P0, ..., Pk] (numpy int32) and counts from the GPU library."""
    kb = _kb()
    r = kb.refiner_for(g, kmax=max(k, 1) if kmax is None else kmax)
    p0, c0 = r.initial()
    ids, counts = r.refine(k)
    torch.cuda.synchronize()
    out = [p0.cpu().numpy()] + [t.cpu().numpy() for t in ids]
    r.close()
    return out, [c0] + counts


def ref_all(g, k):
    p0, c0 = oracle.initial(g)
    ids, counts = oracle.refine(g, k)
    return [p0] + ids, [c0] + counts


def assert_same(g, k, label=""):
    print(f"[parity] {label or g.name} n={g.n} m={g.m} k={k}", flush=True)
    got, gc = gpu_all(g, k)
    exp, ec = ref_all(g, k)
    assert gc == ec, (label, gc, ec)
    for i, (a, b) in enumerate(zip(got, exp)):
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{label}: P{i} differs at {bad[:10]} (of {len(bad)}): got {a[bad[:10]]} want {b[bad[:10]]}")


# ------------------------------------------------------------------ worked example

@pytest.mark.parametrize("mode", ["fw", "bw", "schaetzle", "kaushik", "full_fw", "full_bw"])
def test_paper_example(mode):
    g = helpers.example_variant(mode)
    got, gc = gpu_all(g, 3)
    if mode in helpers.parse_paper_example():
        for k, expect in helpers.parse_paper_example()[mode].items():
            assert list(got[k]) == expect
    assert_same(g, 3, "example-" + mode)


# ------------------------------------------------------------------ configurations

def test_tiny_config_k10():
    """Uniform 10k vertices / 50k edges, 4 vertex and 8 edge labels, k = 1..10."""
    assert_same(graphgen.tiny(seed=1), 10, "tiny")


@pytest.mark.parametrize("seed,avg", [(7, 1.0), (8, 1.5), (9, 2.0)])
def test_deep_graphs_k10(seed, avg):
    """Sparse unlabeled graphs that keep refining through k = 10."""
    g = graphgen.deep(seed=seed, n=20_000, avg_degree=avg)
    _, counts = ref_all(g, 10)
    assert counts[10] > counts[3]          # really deep
    assert_same(g, 10, f"deep{seed}")


@pytest.mark.parametrize("scale,m", [(12, 60_000), (14, 200_000), (16, 900_000)])
def test_rmat_k10(scale, m):
    assert_same(graphgen.rmat(scale, m, seed=2), 10, f"rmat{scale}")


def test_rdf_label_sets():
    """0-3 type labels per vertex (empty sets included), 1,000 edge labels."""
    assert_same(graphgen.rmat_rdf(14, 150_000, seed=3), 10, "rdf14")


def test_batch_style_graphs():
    for g_idx in [0, 1, 6, 7]:
        g = graphgen.batch_graph(g_idx, 5000 + 1000 * g_idx)
        assert_same(g, 6, f"batch{g_idx}")


# ------------------------------------------------------------------ degree tiers

def tier_graph(seed=3, labels=3, shared_targets=50):
    """Vertices at every tier boundary (0, 1, 15-17, 63-65, 511-513, the range capacities 1023-1025 and
    2047-2049, 4095-4097, 8191-8193, the 32-bit-key row limit 19455-19457, hubs up to 3 chunks),
    with few labels and targets so rows are full of duplicates, plus twin rows so the
    large-row exact check finds matches."""
    rng = np.random.default_rng(seed)
    degs = [0, 1, 2, 15, 16, 17, 63, 64, 65, 511, 512, 513, 1000, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096,
            4097, 8191, 8192, 8193, 19455, 19456, 19457, 20000]
    n_small = 3000
    n = len(degs) * 2 + n_small
    src, dst, lbl = [], [], []
    for i, d in enumerate(degs):
        a, b = 2 * i, 2 * i + 1            # twins: identical rows (same multiset, shuffled)
        tg = rng.integers(2 * len(degs), 2 * len(degs) + shared_targets, size=d)
        lb = rng.integers(0, labels, size=d)
        perm = rng.permutation(d)
        src += [a] * d + [b] * d
        dst += list(tg) + list(tg[perm])
        lbl += list(lb) + list(lb[perm])
    base = 2 * len(degs)
    for v in range(base, n):
        d = int(rng.integers(0, 5))
        src += [v] * d
        dst += list(rng.integers(base, n, size=d))
        lbl += list(rng.integers(0, labels, size=d))
    vl = np.zeros(n, dtype=np.int32)
    vl[base:] = rng.integers(0, 3, size=n - base)
    return graphgen.from_edges(n, np.array(src), np.array(dst), np.array(lbl), vl, name="tiers")


def test_degree_tier_boundaries():
    g = tier_graph()
    exp, _ = ref_all(g, 4)
    # twins must be in the same block in P1 (identical pair sets)
    for i in range(0, 40, 2):
        assert exp[1][i] == exp[1][i + 1]
    assert_same(g, 6, "tiers")


def test_degree_tiers_many_labels():
    assert_same(tier_graph(seed=4, labels=200, shared_targets=3000), 5, "tiers-many")


@pytest.mark.parametrize("kbits", [0, 32, 64])
def test_hub_partition_overflow_takes_sub_passes(kbits, monkeypatch):
    """One partition per staged hub (a test knob): a 20,000-entry hub row of ~19,000 distinct
    pairs overflows its partition set (8,192 slots, or 4,096 with 64-bit keys), and the reduce
    pass must redo that partition in sub-passes instead of failing; results stay exact."""
    kb = _kb()
    monkeypatch.setenv("KBISIM_DEBUG_HUB_PARTS", "1")
    g = tier_graph(seed=10, labels=200, shared_targets=3000)
    r = kb.Refiner(*kb.to_device(g), kmax=1, tuning=kb.tuning(key_bits=kbits))
    info = r.schedule_info()
    r.close()
    assert info["hub"]["vertices"] >= 2, info
    assert_same_tuned(g, 4, kb.tuning(key_bits=kbits), f"hub-overflow-{kbits}")


def test_wide_hub_partitions_overflow(monkeypatch):
    """Hubs of 2^20 distinct pairs cut into at most 4 partitions: each partition holds ~2^18
    distinct keys and is reduced in many sub-passes."""
    kb = _kb()
    monkeypatch.setenv("KBISIM_DEBUG_HUB_PARTS", "4")
    g = wide_hub_graph()
    assert_same(g, 2, "wide-hubs-overflow")
    assert_same_tuned(g, 2, kb.tuning(key_bits=64), "wide-hubs-overflow-64")


# ------------------------------------------------------------------ key width

def assert_same_tuned(g, k, tune, label):
    kb = _kb()
    print(f"[parity] {label} n={g.n} m={g.m} k={k} tuning={tune.as_dict()}", flush=True)
    exp, ec = ref_all(g, k)
    r = kb.Refiner(*kb.to_device(g), kmax=k, tuning=tune)
    ids, counts = r.refine(k)
    assert counts == ec[1:], label
    for i, (a, b) in enumerate(zip(ids, exp[1:])):
        assert np.array_equal(a.cpu().numpy(), b), (label, i + 1)
    r.close()


@pytest.mark.parametrize("kbits", [0, 32, 64])
def test_key_width_forced_and_automatic(kbits):
    """32-bit LDS keys: exact where (edge label, block) fits in 31 bits, else hashed; hashed keys
    (32) and 64-bit keys (64) forced on every graph."""
    kb = _kb()
    for g in [graphgen.rmat(14, 200_000, seed=2), tier_graph(seed=6), graphgen.rmat_rdf(12, 60_000, seed=8),
              graphgen.deep(seed=9, n=20_000, avg_degree=1.5)]:
        assert_same_tuned(g, 6, kb.tuning(key_bits=kbits), f"keys{kbits}-{g.name}")


@pytest.mark.parametrize("items", [8, 16])
def test_numbering_tiles(items):
    """Numbering through head words with tiles of 2,048 and 4,096 vertices: vertex counts below
    one word, below one tile, several tiles with a ragged tail, and counts that are not a
    multiple of 4 (the assign kernels then take the tail one vertex at a time)."""
    kb = _kb()
    for g in [graphgen.tiny(seed=21, n=37, m=120), graphgen.tiny(seed=22, n=1_999, m=9_000),
              graphgen.tiny(seed=23, n=12_289, m=60_000), graphgen.rmat(14, 150_000, seed=24),
              graphgen.deep(seed=25, n=20_003, avg_degree=1.2)]:
        assert_same_tuned(g, 5, kb.tuning(scan_items=items), f"scan{items}-{g.name}")


@pytest.mark.parametrize("kbits", [0, 64])
def test_device_built_schedule(kbits, monkeypatch):
    """The degree schedule built on the device (as for graphs of 16M+ vertices), forced on small
    graphs: every tier boundary, hubs, label-set rows, empty rows; the same tier totals as the
    host-built schedule and the reference's partitions."""
    kb = _kb()
    t = kb.tuning(key_bits=kbits)
    graphs = [tier_graph(seed=31, labels=50, shared_targets=2000), graphgen.rmat(14, 200_000, seed=32),
              graphgen.rmat_rdf(13, 90_000, seed=33, types=200, elabels=300),
              graphgen.deep(seed=34, n=20_000, avg_degree=1.1), graphgen.tiny(seed=35, n=3000, m=6000)]
    for g in graphs:
        monkeypatch.delenv("KBISIM_DEBUG_DEVICE_SCHEDULE", raising=False)
        r = kb.Refiner(*kb.to_device(g), kmax=1, tuning=t)
        host_tiers = r.schedule_info()
        r.close()
        monkeypatch.setenv("KBISIM_DEBUG_DEVICE_SCHEDULE", "1")
        r = kb.Refiner(*kb.to_device(g), kmax=1, tuning=t)
        assert r.schedule_info() == host_tiers, g.name
        r.close()
        assert_same_tuned(g, 5, t, f"device-schedule keys{kbits}-{g.name}")


@pytest.mark.parametrize("label_max", [(1 << 11) - 1, 1 << 11])
def test_key_width_boundary(label_max):
    """n = 2^20 gives 20 bits of block id; labels up to 2^11 - 1 fill 31 bits exactly (narrow keys),
    one more label bit needs 64-bit keys."""
    kb = _kb()
    rng = np.random.default_rng(label_max)
    n, m = 1 << 20, 3_000_000
    src = rng.integers(0, n, size=m)
    dst = rng.integers(0, n // 64, size=m)           # few targets: many equal pairs to merge
    lab = rng.integers(label_max - 3, label_max + 1, size=m)
    vl = rng.integers(0, 3, size=n)
    g = graphgen.from_edges(n, src, dst, lab, vl, name=f"bound{label_max}")
    assert_same_tuned(g, 4, kb.tuning(), f"boundary-{label_max}")


@pytest.mark.parametrize("key_bits", [2, 5, 12])
def test_hashed_keys_colliding_inside_rows(key_bits, monkeypatch):
    """Hashed set keys cut to a few bits collide inside rows, so rows with different pair sets
    share key sets and distinct-key counts; the two-sided exact check must keep every
    partition exact (tiers from single entries to hub chunks)."""
    kb = _kb()
    monkeypatch.setenv("KBISIM_DEBUG_KEY_BITS", str(key_bits))
    t = kb.tuning(key_bits=32)
    for mode in ["full_fw", "kaushik"]:
        assert_same_tuned(helpers.example_variant(mode), 3, t, f"kcollide{key_bits}-{mode}")
    for g in [graphgen.tiny(seed=3, n=2000, m=9000), graphgen.deep(seed=4, n=5000, avg_degree=1.4),
              graphgen.rmat(12, 60_000, seed=6), tier_graph(seed=8)]:
        assert_same_tuned(g, 5, t, f"kcollide{key_bits}-{g.name}")


def test_hashed_keys_with_forced_hash_collisions(monkeypatch):
    kb = _kb()
    monkeypatch.setenv("KBISIM_DEBUG_HASH_BITS", "5")
    monkeypatch.setenv("KBISIM_DEBUG_KEY_BITS", "6")
    t = kb.tuning(key_bits=32)
    assert_same_tuned(graphgen.tiny(seed=2, n=3000, m=12000), 4, t, "hcollide-tiny")
    assert_same_tuned(tier_graph(seed=9), 3, t, "hcollide-tiers")


# ------------------------------------------------------------------ hash collisions

@pytest.mark.parametrize("bits", [0, 3, 8])
def test_forced_collisions_small(bits, monkeypatch):
    """Truncated hashes make collisions routine; the exact check must keep results exact."""
    monkeypatch.setenv("KBISIM_DEBUG_HASH_BITS", str(bits))
    for mode in ["full_fw", "kaushik", "schaetzle"]:
        assert_same(helpers.example_variant(mode), 3, f"collide{bits}-{mode}")
    assert_same(graphgen.tiny(seed=2, n=300, m=900), 5, f"collide{bits}-tiny300")


@pytest.mark.parametrize("bits", [10, 16, 24])
def test_forced_collisions_tiny_config(bits, monkeypatch):
    monkeypatch.setenv("KBISIM_DEBUG_HASH_BITS", str(bits))
    assert_same(graphgen.tiny(seed=1), 4, f"collide{bits}-tiny")


def test_forced_collisions_tiers(monkeypatch):
    monkeypatch.setenv("KBISIM_DEBUG_HASH_BITS", "6")
    assert_same(tier_graph(seed=5), 3, "collide-tiers")


# ------------------------------------------------------------------ edge cases

def test_empty_and_degenerate_graphs():
    kb = _kb()
    cases = [graphgen.from_edges(1, [], []),
             graphgen.from_edges(1, [0, 0], [0, 0], [1, 1]),
             graphgen.from_edges(5, [0, 1, 2, 3, 4], [0, 1, 2, 3, 4], [0, 1, 0, 1, 0]),   # self-loops
             graphgen.from_edges(64, [], [], None, np.arange(64) % 5),                   # m = 0
             graphgen.from_edges(300, [], [], None, None)]                               # no labels at all
    for g in cases:
        assert_same(g, 4, f"degenerate n={g.n} m={g.m}")
    # n = 0
    g = graphgen.from_edges(0, [], [])
    r = kb.refiner_for(g, kmax=3)
    ids, counts = r.refine(3)
    assert counts == [0, 0, 0]


def test_empty_label_sets_and_repeats():
    rng = random.Random(3)
    for _ in range(30):
        g = helpers.random_small_graph(rng, n_max=40, m_max=120, vlabels_max=4)
        if g.vlabel is None:
            continue
        assert_same(g, 5, "small-random")


def test_random_small_graphs_against_brute_force_reference():
    rng = random.Random(9)
    for _ in range(40):
        g = helpers.random_small_graph(rng)
        if rng.random() < 0.5:
            g = graphgen.transpose(g)
        assert_same(g, 6, "brute-sized")


def test_repeated_calls_and_epoch_wrap():
    """More than 15 steps on one context: table epochs wrap and tables are cleared."""
    kb = _kb()
    g = graphgen.deep(seed=11, n=5000)
    exp, ec = ref_all(g, 10)
    r = kb.refiner_for(g, kmax=10)
    for rep in range(4):
        ids, counts = r.refine(10)
        assert counts == ec[1:]
        for a, b in zip(ids, exp[1:]):
            assert np.array_equal(a.cpu().numpy(), b)
    r.close()


def test_refine_from_resume():
    kb = _kb()
    g = graphgen.deep(seed=12, n=8000, avg_degree=1.3)
    exp, ec = ref_all(g, 9)
    r = kb.refiner_for(g, kmax=9)
    ids, counts = r.refine(4)
    start = ids[3].clone()
    ids2, counts2 = r.refine(5, start=start)
    for a, b in zip(ids2, exp[5:]):
        assert np.array_equal(a.cpu().numpy(), b)
    assert counts2 == ec[5:]
    # non-canonical start labels (another numbering of the same blocks): same partitions
    relab = (g.n - 1 - exp[2]).astype(np.int32)
    lab = torch.from_numpy(relab).cuda()
    ids3, c3 = r.refine(3, start=lab)
    ref3, rc3 = oracle.refine(g, 3, start=relab)
    assert c3 == rc3
    for a, b in zip(ids3, ref3):
        assert np.array_equal(a.cpu().numpy(), b)
    r.close()


def test_vertex_permutation_on_gpu():
    g = graphgen.rmat(13, 100_000, seed=5)
    perm = np.random.default_rng(1).permutation(g.n).astype(np.int32)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    vl = np.empty(g.n, dtype=np.int32)
    vl[perm] = g.vlabel
    h = graphgen.from_edges(g.n, perm[src], perm[g.col], g.elabel, vl)
    a, _ = gpu_all(g, 5)
    b, _ = gpu_all(h, 5)
    for x, y in zip(a, b):
        assert helpers.as_blocks(x, perm) == helpers.as_blocks(y)


# ------------------------------------------------------------------ errors through the ABI

def test_invalid_graphs_rejected():
    kb = _kb()
    g = graphgen.tiny(seed=3, n=100, m=400)
    rp, col, el, vl, _ = kb.to_device(g)
    bad_rp = rp.clone(); bad_rp[10] = bad_rp[11] + 1          # not monotone
    bad_col = col.clone(); bad_col[5] = 100                     # out of range
    bad_el = el.clone(); bad_el[7] = -1                         # negative label
    bad_vl = vl.clone(); bad_vl[3] = -2
    for args in [(bad_rp, col, el, vl), (rp, bad_col, el, vl), (rp, col, bad_el, vl), (rp, col, el, bad_vl)]:
        with pytest.raises(kb.KbisimError) as ei:
            kb.Refiner(*args, kmax=2)
        assert ei.value.code == kb.EGRAPH
    r = kb.Refiner(rp, col, el, vl, kmax=2)
    with pytest.raises(kb.KbisimError) as ei:
        r.refine(3)
    assert ei.value.code == kb.EINVAL
    neg = torch.full((g.n,), -1, dtype=torch.int32, device=rp.device)
    with pytest.raises(kb.KbisimError) as ei:
        r.refine(1, start=neg)
    assert ei.value.code == kb.EINVAL
    big = torch.full((g.n,), g.n, dtype=torch.int32, device=rp.device)
    with pytest.raises(kb.KbisimError) as ei:
        r.refine(1, start=big)
    assert ei.value.code == kb.EINVAL
    r.close()


def test_workspace_alignment():
    """The workspace must start at a 256-byte boundary: an offset one is refused with EINVAL,
    a caller-given aligned one gives the same partitions as the library-sized default."""
    kb = _kb()
    g = graphgen.tiny(seed=4, n=500, m=3000)
    d = kb.to_device(g)
    ref = kb.Refiner(*d, kmax=3)
    ids, counts = ref.refine(3)
    nbytes = ref.workspace_bytes
    ref.close()
    buf = torch.empty(nbytes + 512, dtype=torch.uint8, device=d[0].device)
    for off in (1, 8, 128):
        with pytest.raises(kb.KbisimError) as ei:
            kb.Refiner(*d, kmax=3, workspace=buf[off:])
        assert ei.value.code == kb.EINVAL
    r = kb.Refiner(*d, kmax=3, workspace=buf[256:])
    ids2, counts2 = r.refine(3)
    assert counts2 == counts and all(bool((a == b).all()) for a, b in zip(ids, ids2))
    r.close()


def test_range_checks_at_every_alignment():
    """Targets and labels are range-checked 16 bytes at a time over the aligned body of the
    array and one by one before and after it: a bad value is found in the head, the body and
    the tail, for arrays starting at each 4-byte offset and for arrays shorter than one group."""
    kb = _kb()
    for n, m in [(50, 1), (50, 3), (60, 7), (300, 4099)]:
        g = graphgen.tiny(seed=11, n=n, m=m)
        rp, col, el, vl, _ = kb.to_device(g)
        for off in range(4):
            cbuf = torch.zeros(g.m + off + 3, dtype=torch.int32, device=rp.device)
            ebuf = torch.zeros_like(cbuf)
            c, e = cbuf[off:off + g.m], ebuf[off:off + g.m]
            c.copy_(col)
            e.copy_(el)
            kb.Refiner(rp, c, e, vl, kmax=1).close()     # clean arrays pass
            for pos in sorted({0, 1, 2, 3, g.m // 2, g.m - 2, g.m - 1} & set(range(g.m))):
                for arr, bad in [(c, g.n), (c, -1), (e, -1)]:
                    old = arr[pos].item()
                    arr[pos] = bad
                    with pytest.raises(kb.KbisimError) as ei:
                        kb.Refiner(rp, c, e, vl, kmax=1)
                    assert ei.value.code == kb.EGRAPH, (n, m, off, pos, bad)
                    arr[pos] = old


def test_large_sparse_label_values():
    """Labels need not be dense: values up to 2^31 - 1 (no packing, 64-bit keys) and a mix of
    small graphs where labels pack above the target ranks."""
    rng = np.random.default_rng(17)
    g = graphgen.rmat(13, 90_000, seed=9)
    big = np.array([0, 5, 1 << 20, (1 << 31) - 1, 123456789, 77], dtype=np.int64)
    g.elabel = big[rng.integers(0, len(big), size=g.m)].astype(np.int32)
    g.vlabel = (big[rng.integers(0, len(big), size=g.n)] // 3).astype(np.int32)
    assert_same(g, 6, "large-labels")
    h = graphgen.rmat(13, 90_000, seed=9)
    h.elabel = (h.elabel * 1000).astype(np.int32)      # 16 label bits + 13 rank bits: packed
    assert_same(h, 6, "spread-labels")


def test_tiers_with_separate_labels():
    """Labels too wide to pack above the ranks: every tier (rows up to 20,000 entries, hub chunks)
    with the labels in their own array, sorted with their rows, in both key widths."""
    kb = _kb()
    g = tier_graph(seed=13, labels=3)
    g.elabel = (((1 << 30) + 7) * (g.elabel.astype(np.int64) + 1) % ((1 << 31) - 1)).astype(np.int32)
    assert_same(g, 5, "tiers-separate")
    assert_same_tuned(g, 5, kb.tuning(key_bits=64), "tiers-separate-64")
    assert_same_tuned(g, 5, kb.tuning(key_bits=32), "tiers-separate-32")


def giant_hub_graph(seed=23):
    """Two twin rows of 4.5M entries (same pairs, different order and duplicates), one slightly
    different, and small rows."""
    rng = np.random.default_rng(seed)
    n, d = 60_000, 4_500_000
    tg = rng.integers(10, 40_000, size=d)
    lb = rng.integers(0, 5, size=d)
    perm = rng.permutation(d)
    src = [np.zeros(d, np.int64), np.ones(d, np.int64), np.full(d, 2, np.int64)]
    dst = [tg, tg[perm], np.concatenate([tg[:-1], [50_000]])]
    lab = [lb, lb[perm], lb]
    m_small = 200_000
    src.append(rng.integers(3, n, size=m_small))
    dst.append(rng.integers(0, n, size=m_small))
    lab.append(rng.integers(0, 5, size=m_small))
    return graphgen.from_edges(n, np.concatenate(src), np.concatenate(dst), np.concatenate(lab),
                               rng.integers(0, 2, size=n), name="giant-hubs")


def test_giant_hubs_use_the_global_set_path():
    """Rows above 4M entries take the global-hash-set hub path."""
    kb = _kb()
    g = giant_hub_graph()
    r = kb.refiner_for(g, kmax=1)
    info = r.schedule_info()
    r.close()
    assert info["hub_global"]["vertices"] == 3, info
    exp, _ = ref_all(g, 3)
    assert exp[1][0] == exp[1][1] != exp[1][2]
    assert_same(g, 3, "giant-hubs")


def wide_hub_graph(seed=43):
    """Hub rows over 2^20 distinct targets whose P0 blocks all differ, so every pair of a row is
    distinct and 64-bit keys are needed (22 bits of block id, 10 of edge label): row 1 is row 0
    with one target replaced, row 2 holds row 0's pairs twice and one more copy (2^21 + 1
    entries, past the largest staged hub).  5M small random entries give the schedule room to
    stage the two shorter hubs."""
    rng = np.random.default_rng(seed)
    n, d, m_small = 2_200_000, 1 << 20, 5_000_000
    tg = rng.choice(np.arange(3, n), size=d + 1, replace=False)
    t, extra = tg[:d], tg[d]
    lb = rng.integers(0, 1000, size=d)
    t1 = t.copy()
    t1[-1] = extra
    perm = rng.permutation(2 * d + 1)
    t2 = np.concatenate([t, t, t[:1]])[perm]
    l2 = np.concatenate([lb, lb, lb[:1]])[perm]
    src = np.concatenate([np.zeros(d), np.ones(d), np.full(2 * d + 1, 2), rng.integers(3, n, size=m_small)])
    dst = np.concatenate([t, t1, t2, rng.integers(0, n, size=m_small)])
    lab = np.concatenate([lb, lb, l2, rng.integers(0, 1000, size=m_small)])
    vlabel = np.arange(n) - 2
    vlabel[:3] = 0
    return graphgen.from_edges(n, src.astype(np.int64), dst, lab, vlabel, name="wide-hubs")


def test_wide_key_hubs_fill_their_partition_sets():
    """With 64-bit keys a staged hub's partitions have 4,096-slot sets: a row of 2^20 distinct
    pairs has 512 partitions of about 2,048 pairs each, the most a partition is planned for.  A
    row past 2^21 entries takes the global set, and both paths must give the same signature
    for the same pair set."""
    kb = _kb()
    g = wide_hub_graph()
    t64 = kb.tuning(key_bits=64)
    r = kb.Refiner(*kb.to_device(g), kmax=1, tuning=t64)
    info = r.schedule_info()
    r.close()
    assert info["hub"]["vertices"] == 2 and info["hub_global"]["vertices"] == 1, info
    exp, _ = ref_all(g, 2)
    assert exp[1][0] == exp[1][2] != exp[1][1]
    assert_same_tuned(g, 2, t64, "wide-hubs-64")
    # default: hashed 32-bit keys (the pairs need 32 bits); the longest row has more
    # chunks than a hub can be staged in, so it keeps the global set
    r = kb.refiner_for(g, kmax=1)
    info = r.schedule_info()
    r.close()
    assert info["hub"]["vertices"] == 2 and info["hub_global"]["vertices"] == 1, info
    assert_same(g, 2, "wide-hubs-hashed")


def test_hashed_keys_agree_between_staged_and_global_hubs():
    """Hashed keys: a staged hub (2^20 distinct pairs) and a row past the staged limit holding
    the same pairs five times (global set) have one signature; a third row lacks one pair."""
    kb = _kb()
    rng = np.random.default_rng(51)
    n, d = 2_200_000, 1 << 20          # 22 bits of block id + 10 of edge label: hashed keys
    t = rng.choice(np.arange(3, n), size=d, replace=False)
    lb = rng.integers(0, 1000, size=d)
    perm = rng.permutation(5 * d)
    src = np.concatenate([np.zeros(d), np.ones(5 * d), np.full(d - 1, 2), rng.integers(3, n, size=2_000_000)])
    dst = np.concatenate([t, np.tile(t, 5)[perm], t[1:], rng.integers(0, n, size=2_000_000)])
    lab = np.concatenate([lb, np.tile(lb, 5)[perm], lb[1:], rng.integers(0, 1000, size=2_000_000)])
    vlabel = np.arange(n) - 2
    vlabel[:3] = 0
    g = graphgen.from_edges(n, src.astype(np.int64), dst, lab, vlabel, name="hashed-hubs")
    r = kb.refiner_for(g, kmax=1)
    info = r.schedule_info()
    r.close()
    assert info["hub"]["vertices"] == 2 and info["hub_global"]["vertices"] == 1, info
    exp, _ = ref_all(g, 2)
    assert exp[1][0] == exp[1][1] != exp[1][2]
    assert_same(g, 2, "hashed-hubs")
