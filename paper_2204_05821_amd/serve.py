"""Served form: a request loop with continuous (iteration-level) batching.

Jobs (a graph and its k) arrive at any time.  At every scheduler tick the
queue head is admitted as long as a slot is free and the device footprint
(CSR, workspace, outputs) fits the HBM budget.  Small jobs admitted in the
same tick are packed into one *cohort*: their disjoint union, refined by the
batched library entry points, so one launch per kernel serves all of them.
A large job gets a context of its own.  Each admitted unit (cohort or solo
context) is prepared by a worker thread (CSR copied to the device from
pinned host memory, context created) and from then on advances by one
refinement step per tick: the steps of all units are enqueued back to back
over a small pool of HIP streams, so units at different iteration indices
run concurrently on the device, and are completed together afterwards.
A job completes at the tick where its unit reaches the job's k (its counts
are on the host, its ids on the device); the unit's memory returns to the
budget when its last job is done.  CSR arrays and partitions stay
device-resident from admission to retirement.

The scheduler talks to a small backend interface, so that admission and
progress can be exercised on the CPU with a fake clock and a fake device;
``DeviceBackend`` drives the GPU library.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Deque, Dict, List, Optional


@dataclass
class Job:
    jid: int
    graph: Any
    k: int
    arrival: float
    nbytes: int = 0
    unit: Any = None
    member: int = 0
    counts: List[int] = field(default_factory=list)
    admitted: float = 0.0
    started: float = 0.0
    ready: float = 0.0
    finished: float = 0.0
    outputs: Any = None
    error: Optional[BaseException] = None
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def m(self) -> int:
        return int(self.graph.m)


@dataclass
class Unit:
    """A solo context or a cohort: what one chain of steps advances."""
    uid: int
    jobs: List[Job]
    kmax: int
    nbytes: int
    handle: Any = None
    step: int = 0
    error: Optional[BaseException] = None

    @property
    def solo(self) -> bool:
        return len(self.jobs) == 1


def _same_form(graphs) -> bool:
    def form(g):
        return (g.elabel is not None, g.vlabel is not None, g.vlabel_ptr is not None)
    return len({form(g) for g in graphs}) == 1


class DeviceBackend:
    """Runs units on the GPU through the C ABI (a pool of streams, one context per unit).

    keep_outputs: give each finished job its device ids (views into its unit's
    output buffers); off for throughput runs so memory is recycled at once.
    """

    def __init__(self, device="cuda", streams: int = 4, keep_outputs: bool = True, tuning=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max(1, streams))]
        self._next = 0
        self._lock = threading.Lock()
        self.keep_outputs = keep_outputs
        self.tuning = tuning

    # ------------------------------------------------------------ host side
    @staticmethod
    def pin(graph):
        """A copy of a host graph whose arrays live in pinned memory (fast, truly asynchronous H2D)."""
        import torch

        class Pinned:
            pass
        p = Pinned()
        p.n, p.name = graph.n, getattr(graph, "name", "")
        p.m = int(graph.col.shape[0])
        for a in ("row_ptr", "col", "elabel", "vlabel", "vlabel_ptr"):
            x = getattr(graph, a)
            if x is None:
                setattr(p, a, None)
            else:
                t = torch.empty(tuple(x.shape), dtype=torch.from_numpy(x[:0]).dtype, pin_memory=True)
                t.numpy()[...] = x
                setattr(p, a, t)
        return p

    @staticmethod
    def _sizes(graphs):
        n = sum(int(g.n) for g in graphs)
        m = sum(int(g.col.shape[0]) for g in graphs)
        have_el = any(g.elabel is not None for g in graphs)
        sets = any(g.vlabel_ptr is not None for g in graphs)
        nl = 0
        if sets:
            for g in graphs:
                if g.vlabel_ptr is not None:
                    nl += int(g.vlabel.shape[0])
                elif g.vlabel is not None:
                    nl += int(g.n)
        lab = sum(int(g.vlabel.shape[0]) for g in graphs if g.vlabel is not None)
        return n, m, have_el, sets, nl, lab

    def footprint(self, graphs, kmax: int) -> int:
        import ctypes
        from . import _Graph, _lib, KbisimError
        n, m, have_el, sets, nl, lab = self._sizes(graphs)
        g = _Graph(n, m, nl, None, None, None, None, None)
        if sets:
            g.vlabel_ptr = ctypes.c_void_p(1)   # only the sizes are read
        ws = ctypes.c_size_t(0)
        if len(graphs) == 1:
            rc = _lib().kbisim_workspace_bytes(ctypes.byref(g), max(kmax, 1), ctypes.byref(ws))
        else:
            rc = _lib().kbisim_batch_workspace_bytes(ctypes.byref(g), len(graphs), max(kmax, 1), ctypes.byref(ws))
        if rc:
            raise KbisimError(rc, "workspace size query")
        gbytes = 8 * (n + 1) + 4 * m * (2 if have_el else 1) + 4 * lab + (8 * (n + 1) if sets else 0)
        return int(ws.value) + gbytes + 4 * n * max(kmax, 1)

    # ------------------------------------------------------------ device side
    def _stream(self):
        with self._lock:
            s = self.streams[self._next % len(self.streams)]
            self._next += 1
        return s

    def _t(self, a):
        torch = self.torch
        if a is None:
            return None
        if not isinstance(a, torch.Tensor):
            a = torch.from_numpy(a)
        return a.to(self.device, non_blocking=True)

    def _h(self, a):
        return a if isinstance(a, self.torch.Tensor) else self.torch.from_numpy(a)

    def _union_on_device(self, graphs):
        """Disjoint union built on the device: member arrays copied into slices, ids offset in place."""
        import numpy as np
        torch = self.torch
        n, m, have_el, sets, nl, lab = self._sizes(graphs)
        dev = self.device
        rp = torch.empty(n + 1, dtype=torch.int64, device=dev)
        col = torch.empty(m, dtype=torch.int32, device=dev)
        el = torch.empty(m, dtype=torch.int32, device=dev) if have_el else None
        vl = torch.empty(lab, dtype=torch.int32, device=dev) if graphs[0].vlabel is not None else None
        vp = torch.empty(n + 1, dtype=torch.int64, device=dev) if sets else None
        off = np.zeros(len(graphs) + 1, dtype=np.int64)
        v0 = e0 = l0 = 0
        rp[0:1].zero_()
        if vp is not None:
            vp[0:1].zero_()
        for i, g in enumerate(graphs):
            gn, gm = int(g.n), int(g.col.shape[0])
            if gm:
                col[e0:e0 + gm].copy_(self._h(g.col), non_blocking=True)
                col[e0:e0 + gm].add_(v0)
                if el is not None:
                    el[e0:e0 + gm].copy_(self._h(g.elabel), non_blocking=True)
            if gn:
                rp[v0 + 1:v0 + gn + 1].copy_(self._h(g.row_ptr)[1:], non_blocking=True)
                rp[v0 + 1:v0 + gn + 1].add_(e0)
            if vl is not None:
                gl = int(g.vlabel.shape[0])
                if gl:
                    vl[l0:l0 + gl].copy_(self._h(g.vlabel), non_blocking=True)
                if vp is not None and gn:
                    vp[v0 + 1:v0 + gn + 1].copy_(self._h(g.vlabel_ptr)[1:], non_blocking=True)
                    vp[v0 + 1:v0 + gn + 1].add_(l0)
                l0 += gl
            v0 += gn
            e0 += gm
            off[i + 1] = v0
        return rp, col, el, vl, vp, off

    def prepare(self, unit: Unit):
        from . import Batch, Refiner, union_of
        torch = self.torch
        s = self._stream()
        kmax = max(unit.kmax, 1)
        with torch.cuda.stream(s):
            if unit.solo:
                g = unit.jobs[0].graph
                r = Refiner(self._t(g.row_ptr), self._t(g.col), self._t(g.elabel), self._t(g.vlabel),
                            self._t(g.vlabel_ptr), kmax=kmax, stream=s, tuning=self.tuning)
                off = None
            else:
                graphs = [j.graph for j in unit.jobs]
                if _same_form(graphs):
                    rp, col, el, vl, vp, off = self._union_on_device(graphs)
                else:
                    host = [_as_numpy_graph(g) for g in graphs]
                    rp, col, el, vl, vp, off = [self._t(x) if i < 5 else x for i, x in enumerate(union_of(host))]
                r = Batch(rp, col, el, vl, vp, off, kmax=kmax, stream=s, tuning=self.tuning)
            outs = r.alloc_outputs(kmax)
        return {"r": r, "outs": outs, "off": off}

    def step_async(self, unit: Unit) -> None:
        h = unit.handle
        i = unit.step
        if unit.solo:
            h["r"].step_async(i, None if i == 0 else h["outs"][i - 1], h["outs"][i])
        else:
            h["r"].step_async(i, h["outs"][i])

    def step_result(self, unit: Unit) -> List[int]:
        h = unit.handle
        i = unit.step
        if unit.solo:
            return [h["r"].step_result(i, None if i == 0 else h["outs"][i - 1], h["outs"][i])]
        return h["r"].step_result(i, h["outs"][i])

    def run_all(self, unit: Unit) -> List[List[int]]:
        """All steps of a solo unit in one plain call (the per-graph baseline)."""
        h = unit.handle
        _, counts = h["r"].refine(unit.kmax, out=h["outs"])
        return [counts]

    def job_outputs(self, unit: Unit, member: int, k: int):
        if not self.keep_outputs:
            return None
        h = unit.handle
        if unit.solo:
            return h["outs"][:k]
        off = h["off"]
        return [o[int(off[member]):int(off[member + 1])] for o in h["outs"][:k]]

    def release(self, unit: Unit) -> None:
        h = unit.handle
        if h is None:
            return
        h["r"].close()
        unit.handle = None


def _as_numpy_graph(g):
    """A host graph with numpy arrays (pinned tensors are viewed, not copied)."""
    class G:
        pass
    out = G()
    out.n = g.n
    for a in ("row_ptr", "col", "elabel", "vlabel", "vlabel_ptr"):
        x = getattr(g, a)
        setattr(out, a, x.numpy() if hasattr(x, "numpy") else x)
    out.m = int(out.col.shape[0])
    return out


class Server:
    """Continuous-batching scheduler.

    budget_bytes bounds the summed footprint of admitted units; max_units
    bounds the number of units admitted at once (slots).  Jobs with at most
    cohort_edges edges that are admitted in the same tick share a cohort of
    up to max_cohort jobs.  With whole_edges set (and workers > 0), a job of
    at least that many edges, which runs alone anyway, is refined in one call
    on one of whole_workers threads as soon as it is prepared, overlapping the
    ticks on the device, instead of one step per tick; it still holds its
    slot and its memory until done.  ``clock`` returns seconds.
    """

    def __init__(self, backend, budget_bytes: int, max_units: int = 32, workers: int = 8,
                 cohort_edges: int = 2_000_000, max_cohort: int = 64,
                 clock: Callable[[], float] = time.perf_counter, whole_edges: Optional[int] = None,
                 whole_workers: int = 4):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_units = max_units
        self.cohort_edges = cohort_edges
        self.max_cohort = max_cohort
        self.clock = clock
        self.used = 0
        self.peak_used = 0
        self.pending: Deque[Job] = collections.deque()
        self.preparing: Dict[int, Unit] = {}
        self.running: List[Unit] = []
        self.finished: List[Job] = []
        self.rejected: List[Job] = []
        self.ticks = 0
        self.tick_sizes: List[int] = []
        self.units_made = 0
        self._jid = 0
        self._cv = threading.Condition()
        self._pool = cf.ThreadPoolExecutor(max_workers=workers) if workers > 0 else None
        self.whole_edges = whole_edges
        self._whole: Dict[int, Unit] = {}      # units refined in one call on a worker
        self._whole_pool = (cf.ThreadPoolExecutor(max_workers=whole_workers)
                            if whole_edges is not None and workers > 0 else None)
        self._ready: Deque[Unit] = collections.deque()
        self._stop = False
        self._thread: Optional[threading.Thread] = None

    # ---------------------------------------------------------------- intake
    def submit(self, graph, k: int) -> Job:
        job = Job(-1, graph, int(k), self.clock())
        job.nbytes = self.backend.footprint([graph], job.k)
        with self._cv:
            job.jid = self._jid
            self._jid += 1
            if job.nbytes > self.budget:
                job.error = MemoryError(f"job needs {job.nbytes} bytes, the budget is {self.budget}")
                job.finished = job.arrival
                self.rejected.append(job)
                job.done.set()
            elif job.k < 0:
                job.error = ValueError("k must be >= 0")
                job.finished = job.arrival
                self.rejected.append(job)
                job.done.set()
            else:
                self.pending.append(job)
            self._cv.notify_all()
        return job

    # ---------------------------------------------------------------- scheduling
    def _units_active(self) -> int:
        return len(self.running) + len(self.preparing) + len(self._ready) + len(self._whole)

    def _admit(self) -> None:
        """FIFO admission: the queue head is never overtaken, so no job starves."""
        while self.pending and self._units_active() < self.max_units:
            head = self.pending[0]
            members = [head]
            nbytes = head.nbytes
            if head.m <= self.cohort_edges and head.k > 0:
                # grow the cohort with following small jobs while the union still fits
                idx = 1
                while idx < len(self.pending) and len(members) < self.max_cohort:
                    nxt = self.pending[idx]
                    if nxt.m > self.cohort_edges or nxt.k <= 0:
                        break
                    cand = members + [nxt]
                    fp = self.backend.footprint([j.graph for j in cand], max(j.k for j in cand))
                    if self.used + fp > self.budget:
                        break
                    members, nbytes = cand, fp
                    idx += 1
            if self.used + nbytes > self.budget:
                break
            for _ in members:
                self.pending.popleft()
            now = self.clock()
            unit = Unit(self.units_made, members, max(j.k for j in members), nbytes)
            self.units_made += 1
            for i, j in enumerate(members):
                j.unit, j.member, j.admitted = unit, i, now
            self.used += nbytes
            self.peak_used = max(self.peak_used, self.used)
            self.preparing[unit.uid] = unit
            if self._pool is None:
                self._prepare(unit)
            else:
                self._pool.submit(self._prepare, unit)

    def _prepare(self, unit: Unit) -> None:
        try:
            if unit.kmax > 0:
                unit.handle = self.backend.prepare(unit)
        except BaseException as e:  # reported on the jobs, the loop goes on
            unit.error = e
        now = self.clock()
        for j in unit.jobs:
            j.ready = now
        whole = (unit.error is None and self._whole_pool is not None and unit.solo and unit.kmax > 0
                 and unit.jobs[0].m >= self.whole_edges)
        with self._cv:
            self.preparing.pop(unit.uid, None)
            if whole:
                self._whole[unit.uid] = unit
            else:
                self._ready.append(unit)
            self._cv.notify_all()
        if whole:
            self._whole_pool.submit(self._run_whole, unit)

    def _run_whole(self, unit: Unit) -> None:
        """Every step of a large solo unit in one call, then its job completes."""
        start = self.clock()
        for j in unit.jobs:
            j.started = start
        counts: List[int] = []
        try:
            counts = self.backend.run_all(unit)[0]
        except BaseException as e:  # reported on the job, the loop goes on
            unit.error = e
        with self._cv:
            now = self.clock()
            job = unit.jobs[0]
            if unit.error is None:
                job.counts = [int(x) for x in counts[: job.k]]
                unit.step = unit.kmax
                self._complete(job, now)
            self._whole.pop(unit.uid, None)
            self._retire(unit, now)
            self._admit()
            self._cv.notify_all()

    def _complete(self, job: Job, now: float) -> None:
        if job.error is None and job.unit is not None and job.unit.handle is not None and job.k > 0:
            try:
                job.outputs = self.backend.job_outputs(job.unit, job.member, job.k)
            except BaseException as e:
                job.error = e
        job.finished = now
        self.finished.append(job)
        job.done.set()

    def _retire(self, unit: Unit, now: float) -> None:
        for j in unit.jobs:
            if not j.done.is_set():
                j.error = j.error or unit.error
                self._complete(j, now)
        try:
            if unit.handle is not None:
                self.backend.release(unit)
        except BaseException as e:
            for j in unit.jobs:
                j.error = j.error or e
        self.used -= unit.nbytes

    def _take_ready(self) -> None:
        now = self.clock()
        while self._ready:
            unit = self._ready.popleft()
            for j in unit.jobs:
                j.started = now
            if unit.error is not None or unit.kmax == 0:
                for j in unit.jobs:
                    j.error = unit.error
                self._retire(unit, now)
                continue
            for j in unit.jobs:       # k = 0 members are done at once
                if j.k == 0:
                    self._complete(j, now)
            self.running.append(unit)

    def tick(self) -> int:
        """Admit what fits, then advance every running unit by one step.  Returns the number of jobs advanced."""
        with self._cv:
            self._admit()
            self._take_ready()
            batch = list(self.running)
        if not batch:
            return 0
        for u in batch:
            try:
                self.backend.step_async(u)
            except BaseException as e:
                u.error = e
        results = {}
        for u in batch:
            if u.error is None:
                try:
                    results[u.uid] = self.backend.step_result(u)
                except BaseException as e:
                    u.error = e
        with self._cv:
            now = self.clock()
            self.ticks += 1
            advanced = 0
            keep = []
            for u in batch:
                if u.error is None:
                    cnts = results[u.uid]
                    for j in u.jobs:
                        if u.step < j.k:
                            j.counts.append(int(cnts[j.member]))
                            advanced += 1
                    u.step += 1
                    for j in u.jobs:
                        if j.k == u.step:
                            self._complete(j, now)
                if u.error is not None or u.step >= u.kmax:
                    self._retire(u, now)
                else:
                    keep.append(u)
            self.running = keep
            self.tick_sizes.append(advanced)
            self._admit()
            self._cv.notify_all()
        return advanced

    def idle(self) -> bool:
        with self._cv:
            return not (self.pending or self.preparing or self._ready or self.running or self._whole)

    # ---------------------------------------------------------------- loop
    def _loop(self) -> None:
        while True:
            n = self.tick()
            if n == 0:
                with self._cv:
                    if self._stop and not (self.pending or self.preparing or self._ready or self.running
                                           or self._whole):
                        return
                    self._cv.wait(timeout=0.001)

    def start(self) -> "Server":
        self._thread = threading.Thread(target=self._loop, name="kbisim-server", daemon=True)
        self._thread.start()
        return self

    def stop(self, wait: bool = True) -> None:
        """Finish every submitted job, then stop the loop."""
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        if wait and self._thread is not None:
            self._thread.join()
        if self._pool is not None:
            self._pool.shutdown(wait=wait)
        if self._whole_pool is not None:
            self._whole_pool.shutdown(wait=wait)

    def run_until_idle(self, max_ticks: int = 1 << 30) -> None:
        """Drive the loop from the calling thread (no background thread)."""
        for _ in range(max_ticks):
            if self.idle():
                return
            if self.tick() == 0:
                with self._cv:
                    if self.preparing or self._whole:
                        self._cv.wait(timeout=0.001)
        raise RuntimeError("server did not become idle")

    # ---------------------------------------------------------------- reporting
    def stats(self) -> Dict[str, float]:
        ok = [j for j in self.finished if j.error is None]
        lat = sorted(j.latency for j in ok)

        def pct(p):
            if not lat:
                return float("nan")
            idx = min(len(lat) - 1, max(0, -(-p * len(lat) // 100) - 1))
            return lat[int(idx)]
        prep = sorted(j.ready - j.arrival for j in ok)
        return {"jobs": len(self.finished), "errors": len(self.finished) - len(ok),
                "p50_admit_prepare_s": prep[len(prep) // 2] if prep else float("nan"),
                "rejected": len(self.rejected), "p50_s": pct(50), "p99_s": pct(99),
                "mean_jobs_per_tick": (sum(self.tick_sizes) / len(self.tick_sizes)) if self.tick_sizes else 0.0,
                "ticks": self.ticks, "units": self.units_made, "peak_bytes": self.peak_used}


class FifoServer(Server):
    """Baseline: one job at a time, each refined by one plain per-graph call (no batching, no overlap)."""

    def __init__(self, backend, budget_bytes: int, clock=time.perf_counter):
        super().__init__(backend, budget_bytes, max_units=1, workers=0, cohort_edges=-1, clock=clock)

    def tick(self) -> int:
        with self._cv:
            self._admit()
            self._take_ready()
            batch = list(self.running)
        for u in batch:
            try:
                counts = self.backend.run_all(u)[0]
            except BaseException as e:
                u.error = e
                counts = []
            with self._cv:
                now = self.clock()
                j = u.jobs[0]
                if u.error is None:
                    j.counts = list(counts[: j.k])
                    u.step = u.kmax
                    self._complete(j, now)
                self._retire(u, now)
                self.running.remove(u)
                self.ticks += 1
                self.tick_sizes.append(1)
                self._cv.notify_all()
        return len(batch)
