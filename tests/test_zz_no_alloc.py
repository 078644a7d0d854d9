"""kbisim_refine_noalloc (scratch in a static per-GPU array, no allocation)
against the allocating entry points (kbisim_create + kbisim_refine) on the
same inputs: consecutive calls, each smaller than the one before, so every
call runs on whatever the previous one left in the scratch array."""
from __future__ import annotations

import ctypes

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


def refine_noalloc(g, k):
    kb = _kb()
    lib = kb._lib()
    f = lib.kbisim_refine_noalloc
    f.argtypes = [ctypes.POINTER(kb._Graph), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                  ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]
    f.restype = ctypes.c_int
    rp, col, el, vl, vp = kb.to_device(g, "cuda")
    nl = int(vl.numel()) if (vl is not None and vp is not None) else 0
    gs = kb._Graph(g.n, g.m, nl, kb._ptr(rp), kb._ptr(col), kb._ptr(el), kb._ptr(vp), kb._ptr(vl))
    outs = [torch.full((g.n,), -7, dtype=torch.int32, device="cuda") for _ in range(k)]
    ptrs = (ctypes.c_void_p * max(k, 1))(*[o.data_ptr() for o in outs])
    counts = (ctypes.c_int64 * max(k, 1))()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    rc = f(ctypes.byref(gs), k, ptrs, counts, ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0, (rc, lib.kbisim_strerror(rc))
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs], [int(counts[i]) for i in range(k)]


def refine_alloc(g, k):
    kb = _kb()
    r = kb.refiner_for(g, kmax=k)
    ids, counts = r.refine(k)
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in ids]
    r.close()
    return out, counts


def test_noalloc_matches_the_allocating_entry_points():
    graphs = [graphgen.rmat_rdf(17, 1_500_000, seed=12, types=200, elabels=300),   # label sets, hub rows
              graphgen.tiny(seed=2),                                               # 10k vertices, 50k edges
              helpers.example_variant("kaushik")]                                  # the worked example
    sizes = [(g.n, g.m) for g in graphs]
    assert sizes == sorted(sizes, reverse=True)
    for g in graphs:
        k = 6
        print(f"[no-alloc] {g.name} n={g.n} m={g.m} k={k}", flush=True)
        got, gc = refine_noalloc(g, k)
        exp, ec = refine_alloc(g, k)
        assert gc == ec, (g.name, gc, ec)
        for i in range(k):
            assert np.array_equal(got[i], exp[i]), (g.name, i)
        ref, rc = oracle.refine(g, k)
        assert gc == rc
        for i in range(k):
            assert np.array_equal(got[i], ref[i]), (g.name, i)


def test_noalloc_rejects_graphs_beyond_the_scratch_array():
    kb = _kb()
    lib = kb._lib()
    lib.kbisim_noalloc_scratch_bytes.restype = ctypes.c_size_t
    assert lib.kbisim_noalloc_scratch_bytes() == 128 << 20
    g = graphgen.tiny(seed=3, n=2_000_000, m=4_000_000, vlabels=4, elabels=8)
    f = lib.kbisim_refine_noalloc
    f.argtypes = [ctypes.POINTER(kb._Graph), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    fake = ctypes.c_void_p(0x1000)      # never dereferenced: the size check comes first
    gs = kb._Graph(g.n, g.m, 0, fake, fake, fake, None, fake)
    outs = (ctypes.c_void_p * 2)(fake, fake)
    counts = (ctypes.c_int64 * 2)()
    assert f(ctypes.byref(gs), 2, outs, counts, None) == kb.ENOSPACE
    # and the array is still usable afterwards
    small = graphgen.tiny(seed=4, n=3000, m=12000)
    got, gc = refine_noalloc(small, 3)
    exp, ec = refine_alloc(small, 3)
    assert gc == ec and all(np.array_equal(a, b) for a, b in zip(got, exp))
