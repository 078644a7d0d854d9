"""GPU tests of the served form: each job's result is the same alone and in the mix.

Jobs of mixed sizes and k arrive with Poisson gaps while others are on the
device; small ones share cohorts (one union refined by the batched entry
points), large ones run alone, and units at different iteration indices
overlap on a pool of streams.  Every job's counts and device ids must equal,
bit for bit, what the same graph gives when refined alone, and the CPU
reference.
"""
from __future__ import annotations

import random
import threading
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _kb():
    import paper_2204_05821_amd as kb
    return kb


def job_pool(seed=0, count=14):
    rng = np.random.default_rng(seed)
    gs = []
    for i in range(count):
        m = int(np.exp(rng.uniform(np.log(2_000), np.log(300_000))))
        scale = max(8, int(np.ceil(np.log2(m / 12))))
        g = graphgen.rmat(scale, m, seed=1000 + i)
        g.name = f"rmat{i}"
        gs.append(g)
    gs.append(graphgen.from_edges(1, [], [], None, [2], name="single"))
    gs.append(graphgen.deep(seed=5, n=4000, avg_degree=1.3))
    gs[-1].vlabel = gs[-1].vlabel.copy()
    gs[-1].elabel = np.zeros(gs[-1].m, dtype=np.int32)
    return gs


def alone(g, k):
    kb = _kb()
    if k == 0:
        return [], []
    r = kb.refiner_for(g, kmax=k)
    ids, counts = r.refine(k)
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in ids]
    r.close()
    return out, counts


def run_mix(graphs, ks, budget, cohort_edges, pin=False, gap_s=0.002, seed=0, burst=6, whole_edges=None):
    """The first `burst` jobs are queued before the loop starts (so they are admitted
    together and small ones share a cohort); the rest arrive with Poisson gaps while
    the earlier ones are on the device."""
    from paper_2204_05821_amd import serve
    be = serve.DeviceBackend(streams=4, keep_outputs=True)
    pool = [serve.DeviceBackend.pin(g) if pin else g for g in graphs]
    srv = serve.Server(be, budget_bytes=budget, workers=4, cohort_edges=cohort_edges, whole_edges=whole_edges)
    rnd = random.Random(seed)
    jobs = []
    for idx, (g, k) in enumerate(zip(pool, ks)):
        if idx == burst:
            srv.start()
        jobs.append(srv.submit(g, k))
        if idx >= burst:
            time.sleep(rnd.expovariate(1.0 / gap_s))
    if len(jobs) <= burst:
        srv.start()
    srv.stop()
    torch.cuda.synchronize()
    return srv, jobs


def check_jobs(graphs, ks, jobs, label):
    for i, (g, k, j) in enumerate(zip(graphs, ks, jobs)):
        assert j.error is None, (label, i, j.error)
        exp_ids, exp_counts = alone(g, k)
        assert j.counts == exp_counts, (label, i, j.counts, exp_counts)
        ref_ids, ref_counts = oracle.refine(g, k) if k else ([], [])
        assert j.counts == list(ref_counts)
        got = [o.cpu().numpy() for o in (j.outputs or [])]
        assert len(got) == k
        for step, (a, b, c) in enumerate(zip(got, exp_ids, ref_ids)):
            assert np.array_equal(a, b), (label, i, step)
            assert np.array_equal(a, c), (label, i, step)


def test_each_result_same_alone_and_in_the_mix():
    graphs = job_pool()
    rnd = random.Random(3)
    ks = [rnd.randint(1, 10) for _ in graphs]
    ks[3] = 0
    print(f"[serve] mix of {len(graphs)} jobs, k={ks}", flush=True)
    srv, jobs = run_mix(graphs, ks, budget=200 << 30, cohort_edges=60_000)
    st = srv.stats()
    print(f"[serve] stats {st}", flush=True)
    assert st["units"] < len(graphs)          # some jobs shared a cohort
    check_jobs(graphs, ks, jobs, "mix")


def test_large_jobs_refined_whole_beside_stepped_cohorts():
    """Jobs above the cohort limit refined in one call on workers while the cohorts step per tick."""
    graphs = job_pool()
    rnd = random.Random(9)
    ks = [rnd.randint(1, 10) for _ in graphs]
    print(f"[serve] whole mix of {len(graphs)} jobs, k={ks}", flush=True)
    srv, jobs = run_mix(graphs, ks, budget=200 << 30, cohort_edges=60_000, whole_edges=60_001, seed=4)
    st = srv.stats()
    print(f"[serve] stats {st}", flush=True)
    assert any(g.m > 60_000 for g in graphs) and any(g.m <= 60_000 for g in graphs)
    check_jobs(graphs, ks, jobs, "whole")


def test_mix_from_pinned_pool_with_mixed_label_forms():
    graphs = job_pool(seed=1, count=8)
    sets = graphgen.rmat_rdf(11, 20_000, seed=9, types=40, elabels=30)
    graphs = graphs[:4] + [sets] + graphs[4:]
    ks = [4, 7, 2, 9, 5, 3, 10, 6, 1, 8, 2][: len(graphs)]
    srv, jobs = run_mix(graphs, ks, budget=200 << 30, cohort_edges=1 << 40, pin=True)
    check_jobs(graphs, ks, jobs, "pinned")


def test_tiny_budget_forces_queueing_on_device():
    from paper_2204_05821_amd import serve
    graphs = job_pool(seed=2, count=8)
    ks = [3, 5, 2, 6, 4, 1, 7, 3, 2, 5][: len(graphs)]
    be = serve.DeviceBackend(streams=2)
    one = max(be.footprint([g], k) for g, k in zip(graphs, ks))
    srv, jobs = run_mix(graphs, ks, budget=one + 1024, cohort_edges=60_000, gap_s=0.0005)
    assert srv.peak_used <= one + 1024
    check_jobs(graphs, ks, jobs, "tiny-budget")


def test_serving_pool_jobs_up_to_24M_edges():
    """Jobs of the serving workload's own pool (RMAT, m log-uniform 10k-50M, labels as the
    100M-edge recipe): small pool graphs share cohorts, three jobs of 10-24M edges run
    beside them.  Every job equals its solo refinement; the small ones equal the plain
    reference, the large ones pass the property checker step by step."""
    oracle.check_threads(16)
    small = [1, 3, 8, 17, 20, 21, 26, 28, 41, 43]
    big = [11, 56, 44]
    order = [1, 11, 3, 8, 56, 17, 20, 44, 21, 26, 28, 41, 43]
    assert sorted(order) == sorted(small + big)
    graphs = [graphgen.serving_pool_graph(j) for j in order]
    rnd = random.Random(17)
    ks = [rnd.randint(1, 10) for _ in graphs]
    for i, j in enumerate(order):
        if j in big:
            ks[i] = 10 - i % 3
    print(f"[serve] pool jobs {order}, m={[g.m for g in graphs]}, k={ks}", flush=True)
    assert max(g.m for g in graphs) >= 20_000_000
    srv, jobs = run_mix(graphs, ks, budget=200 << 30, cohort_edges=2_000_000, pin=True, burst=4, gap_s=0.005)
    st = srv.stats()
    print(f"[serve] stats {st}", flush=True)
    assert st["units"] < len(graphs)
    for i, (g, k, j) in enumerate(zip(graphs, ks, jobs)):
        assert j.error is None, (i, j.error)
        got = [o.cpu().numpy() for o in (j.outputs or [])]
        assert len(got) == k
        exp_ids, exp_counts = alone(g, k)
        assert j.counts == exp_counts, (i, j.counts, exp_counts)
        for step in range(k):
            assert np.array_equal(got[step], exp_ids[step]), (i, step)
        if order[i] in small:
            ref_ids, ref_counts = oracle.refine(g, k)
            assert j.counts == list(ref_counts)
            for step in range(k):
                assert np.array_equal(got[step], ref_ids[step]), (i, step)
        else:
            p0, c0 = oracle.initial(g)
            prev = p0
            for step in range(k):
                assert oracle.check_step(g, prev, got[step]) == j.counts[step], (i, step)
                prev = got[step]
        print(f"[serve] job {order[i]} (m={g.m}, k={k}) checked", flush=True)
        j.outputs = None
