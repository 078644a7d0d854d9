"""CPU tests of the serving scheduler with a fake device and a fake clock.

The fake backend answers every step with the CPU reference's block counts
for each member graph, so these tests check the scheduler's bookkeeping
(admission by budget and slots, cohort membership, iteration-level progress,
completion, retirement, error handling), not the refinement itself.
"""
from __future__ import annotations

import random
import threading

import numpy as np
import pytest

import graphgen
import oracle
from paper_2204_05821_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0
        self.lock = threading.Lock()

    def __call__(self):
        with self.lock:
            return self.t

    def advance(self, dt):
        with self.lock:
            self.t += dt


class FakeBackend:
    """Footprint = 100 bytes per vertex + 10 per edge per member (+ 50 per graph in a cohort)."""

    def __init__(self, clock, fail_on=None):
        self.clock = clock
        self.fail_on = fail_on or set()
        self.prepared = []
        self.released = []
        self.live = set()
        self.max_live = 0
        self.steps_seen = []          # (tick index, uid, step) per advanced unit
        self.tick = 0
        self._ref = {}

    def footprint(self, graphs, kmax):
        return sum(100 * g.n + 10 * g.m for g in graphs) + (50 * len(graphs) if len(graphs) > 1 else 0)

    def ref_counts(self, g):
        key = id(g)
        if key not in self._ref:
            self._ref[key] = oracle.refine(g, 10)[1]
        return self._ref[key]

    def prepare(self, unit):
        for j in unit.jobs:
            if j.graph.name in self.fail_on:
                raise RuntimeError("prepare failed for " + j.graph.name)
        self.prepared.append(unit.uid)
        self.live.add(unit.uid)
        self.max_live = max(self.max_live, len(self.live))
        return {"uid": unit.uid}

    def step_async(self, unit):
        assert unit.handle["uid"] == unit.uid
        self.steps_seen.append((self.tick, unit.uid, unit.step))

    def step_result(self, unit):
        self.clock.advance(0.001)
        return [self.ref_counts(j.graph)[unit.step] for j in unit.jobs]

    def run_all(self, unit):
        self.clock.advance(0.001 * unit.kmax)
        return [self.ref_counts(unit.jobs[0].graph)[:unit.kmax]]

    def job_outputs(self, unit, member, k):
        return ("outputs", unit.uid, member, k)

    def release(self, unit):
        self.released.append(unit.uid)
        self.live.discard(unit.uid)


def small_graph(i, m=None):
    rng = np.random.default_rng(i)
    m = int(rng.integers(50, 600)) if m is None else m
    g = graphgen.tiny(seed=100 + i, n=max(8, m // 4), m=m)
    g.name = f"g{i}"
    return g


def drive(server, backend, max_ticks=10_000):
    for _ in range(max_ticks):
        if server.idle():
            return
        backend.tick += 1
        server.tick()
        server.clock.advance(0.0001) if hasattr(server.clock, "advance") else None
    raise AssertionError("did not finish")


def test_every_job_gets_its_own_counts():
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = serve.Server(be, budget_bytes=10**9, workers=0, cohort_edges=400, clock=clock)
    rnd = random.Random(1)
    jobs = [srv.submit(small_graph(i), rnd.randint(0, 10)) for i in range(40)]
    drive(srv, be)
    for j in jobs:
        assert j.error is None
        assert j.counts == be.ref_counts(j.graph)[: j.k], j.jid
        if j.k:
            assert j.outputs == ("outputs", j.unit.uid, j.member, j.k)
    assert sorted(be.prepared) == sorted(be.released)
    assert srv.used == 0
    st = srv.stats()
    assert st["jobs"] == 40 and st["errors"] == 0


def test_small_jobs_share_cohorts_and_large_jobs_run_alone():
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = serve.Server(be, budget_bytes=10**9, workers=0, cohort_edges=300, max_cohort=5, clock=clock)
    gs = [small_graph(i, m=100) for i in range(7)] + [small_graph(50, m=2000)] + [small_graph(60 + i, m=100)
                                                                                  for i in range(3)]
    jobs = [srv.submit(g, 3) for g in gs]
    drive(srv, be)
    units = {}
    for j in jobs:
        units.setdefault(j.unit.uid, []).append(j.jid)
    sizes = sorted(len(v) for v in units.values())
    assert sizes == [1, 2, 3, 5]            # 5 + 2 small, then the large one alone, then 3 small
    big = jobs[7]
    assert units[big.unit.uid] == [7]
    # cohort members are consecutive in arrival order (FIFO)
    for v in units.values():
        assert v == list(range(v[0], v[0] + len(v)))


def test_budget_forces_queueing_and_is_never_exceeded():
    clock = FakeClock()
    be = FakeBackend(clock)
    gs = [small_graph(i, m=400) for i in range(12)]
    one = max(be.footprint([g], 5) for g in gs)
    srv = serve.Server(be, budget_bytes=one + 10, workers=0, cohort_edges=10**9, clock=clock)
    jobs = [srv.submit(g, 5) for g in gs]
    drive(srv, be)
    assert be.max_live == 1
    assert srv.peak_used <= srv.budget
    fin = [j.finished for j in jobs]
    assert fin == sorted(fin)               # FIFO: no overtaking
    for j in jobs:
        assert j.counts == be.ref_counts(j.graph)[:5]


def test_slots_bound_concurrent_units():
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = serve.Server(be, budget_bytes=10**12, max_units=3, workers=0, cohort_edges=0, clock=clock)
    jobs = [srv.submit(small_graph(i), 4) for i in range(10)]
    drive(srv, be)
    assert be.max_live == 3
    assert all(j.counts == be.ref_counts(j.graph)[:4] for j in jobs)


def test_oversize_job_is_rejected_and_others_proceed():
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = serve.Server(be, budget_bytes=50_000, workers=0, clock=clock)
    ok1 = srv.submit(small_graph(1, m=200), 3)
    huge = srv.submit(small_graph(2, m=20_000), 3)
    ok2 = srv.submit(small_graph(3, m=200), 3)
    assert isinstance(huge.error, MemoryError) and huge.done.is_set()
    drive(srv, be)
    assert ok1.error is None and ok2.error is None
    assert srv.stats()["rejected"] == 1


def test_jobs_join_while_others_run_at_other_steps():
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = serve.Server(be, budget_bytes=10**9, workers=0, cohort_edges=0, clock=clock)
    a = srv.submit(small_graph(1), 10)
    for _ in range(4):
        be.tick += 1
        srv.tick()
    b = srv.submit(small_graph(2), 3)       # arrives while a is at step 4
    be.tick += 1
    srv.tick()
    last = [(u, s) for t, u, s in be.steps_seen if t == be.tick]
    assert sorted(last) == [(a.unit.uid, 4), (b.unit.uid, 0)]
    drive(srv, be)
    assert b.finished < a.finished          # the short job is not held behind the long one
    assert a.counts == be.ref_counts(a.graph)[:10] and b.counts == be.ref_counts(b.graph)[:3]


def test_member_with_smaller_k_finishes_before_its_cohort():
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = serve.Server(be, budget_bytes=10**9, workers=0, clock=clock)
    a = srv.submit(small_graph(1), 9)
    b = srv.submit(small_graph(2), 2)
    drive(srv, be)
    assert a.unit is b.unit
    assert b.finished < a.finished
    assert b.counts == be.ref_counts(b.graph)[:2]


def test_prepare_failure_is_reported_on_its_jobs_only():
    clock = FakeClock()
    be = FakeBackend(clock, fail_on={"g2"})
    srv = serve.Server(be, budget_bytes=10**9, workers=0, cohort_edges=0, clock=clock)
    jobs = [srv.submit(small_graph(i), 3) for i in range(4)]
    drive(srv, be)
    assert isinstance(jobs[2].error, RuntimeError)
    for i in (0, 1, 3):
        assert jobs[i].error is None and jobs[i].counts == be.ref_counts(jobs[i].graph)[:3]
    assert srv.used == 0


def test_fifo_baseline_same_counts():
    clock = FakeClock()
    be = FakeBackend(clock)
    srv = serve.FifoServer(be, budget_bytes=10**9, clock=clock)
    rnd = random.Random(4)
    jobs = [srv.submit(small_graph(i), rnd.randint(0, 10)) for i in range(15)]
    drive(srv, be)
    assert be.max_live == 1
    for j in jobs:
        assert j.error is None and j.counts == be.ref_counts(j.graph)[: j.k]


def test_threaded_loop_with_workers():
    be = FakeBackend(FakeClock())
    srv = serve.Server(be, budget_bytes=30_000, workers=4, cohort_edges=300).start()
    rnd = random.Random(7)
    jobs = []
    for i in range(30):
        jobs.append(srv.submit(small_graph(i), rnd.randint(1, 10)))
    srv.stop()
    for j in jobs:
        assert j.done.is_set()
        assert j.error is None, j.error
        assert j.counts == be.ref_counts(j.graph)[: j.k]
    assert srv.peak_used <= 30_000 and srv.used == 0


def test_large_jobs_run_whole_on_workers():
    """With whole_edges, a job of at least that many edges is refined in one call on a worker
    (never stepped per tick) while smaller ones are still stepped in cohorts; every job gets its
    own counts, and slots and memory are held until it is done."""
    be = FakeBackend(FakeClock())
    srv = serve.Server(be, budget_bytes=60_000, workers=4, cohort_edges=300, whole_edges=400).start()
    rnd = random.Random(11)
    jobs = [srv.submit(small_graph(i), rnd.randint(1, 10)) for i in range(40)]
    srv.stop()
    whole = {j.unit.uid for j in jobs if j.m >= 400}
    assert whole and any(j.m < 400 for j in jobs)
    stepped = {u for _, u, _ in be.steps_seen}
    assert not (whole & stepped)
    for j in jobs:
        assert j.done.is_set()
        assert j.error is None, j.error
        assert j.counts == be.ref_counts(j.graph)[: j.k]
    assert srv.peak_used <= 60_000 and srv.used == 0 and srv.idle()


def test_latency_percentiles():
    srv = serve.Server(FakeBackend(FakeClock()), budget_bytes=1, workers=0)
    for i in range(100):
        j = serve.Job(i, None, 1, arrival=0.0)
        j.finished = (i + 1) / 1000.0
        srv.finished.append(j)
    st = srv.stats()
    assert st["p50_s"] == pytest.approx(0.050)
    assert st["p99_s"] == pytest.approx(0.099)
