#!/usr/bin/env python3
"""Benchmark of k-bisimulation refinement on one MI355X.

A step is one call of kbisim_refine(k=10) on the whole graph: ten full
refinement iterations (signature gather and dedupe, key hashing, grouping,
exact check, first-vertex numbering), inputs already resident in HBM.  The
metric is edge-iterations per second: m * k * steps / time.

Default workload: RDF-like RMAT, scale 27 (134,217,728 vertices),
1,000,000,000 directed edges, (a, b, c, d) = (0.57, 0.19, 0.19, 0.05),
0-3 type labels per vertex (sizes 0/1/2/3 with probability .25/.55/.15/.05)
drawn Zipf(1.0) from 1,000 types and distinct within a vertex, 1,000 edge
labels Zipf(1.2), seed 3.  The paper's datasets are not available; this
synthetic recipe stands in for its billion-edge class (BSBM1B; the 2B-edge
run, --workload rmat_rdf_s28_m2B_k10, for BTC2B).

Prints one JSON line with the throughput, a roofline entry for the dominant
kernel (timed with HIP events inside the timed region) and the CPU reference
timed on a bounded sample of the same graph.  The sample is the rows of the
first n/8 vertices with their targets renumbered compactly; its first
refinement step equals the full graph's on those vertices (ids are numbered
by first vertex), which the run checks against the GPU.  The reference runs
in a child process forked before the GPU is touched, so it overlaps the GPU
legs.  With --mode all (the default) the line also carries the 100M-edge
plain figure, the batched form (4,096 graphs, edge counts log-uniform
1k-2M, half uniform-random and half RMAT, k = 10, autotuned launch shapes,
against per-graph plain calls) and the served form (Poisson arrivals at 200
jobs/s of RMAT jobs with 10k-50M edges and k uniform in 1..10 under a 200 GB
budget: p50/p99 latency and jobs/s, and the capacity of the
continuous-batching server against a one-job-at-a-time server).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s (published)
CPU_SAMPLE_SHIFT = 3   # the CPU reference refines the rows of the first n >> 3 vertices

WORKLOADS = {
    "rmat_s23_m100M_k10": dict(kind="rmat", scale=23, m=100_000_000, seed=2, k=10,
                               desc="RMAT s23, 100M edges, 32 vertex labels Zipf(1.0), 64 edge labels Zipf(1.1)"),
    "uniform_n10k_m50k_k10": dict(kind="tiny", seed=1, k=10,
                                  desc="uniform 10k vertices, 50k edges, 4 vertex / 8 edge labels uniform"),
    "rmat_rdf_s27_m1B_k10": dict(kind="rdf", scale=27, m=1_000_000_000, seed=3, k=10,
                                 desc="RDF-like RMAT s27, 1B edges, 0-3 type labels Zipf(1.0) over 1000, "
                                      "1000 edge labels Zipf(1.2)"),
    "rmat_rdf_s28_m2B_k10": dict(kind="rdf", scale=28, m=2_000_000_000, seed=4, k=10,
                                 desc="RDF-like RMAT s28, 2B edges, labels as the 1B recipe"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_graph(w):
    import graphgen
    if w["kind"] == "rmat":
        return graphgen.rmat(w["scale"], w["m"], seed=w["seed"])
    if w["kind"] == "tiny":
        return graphgen.tiny(seed=w["seed"])
    if w["kind"] == "rdf":
        return graphgen.rmat_rdf(w["scale"], w["m"], seed=w["seed"])
    raise KeyError(w["kind"])


def algorithmic_bytes(kernel: str, tiers, n: int, m: int) -> float:
    """Bytes a kernel must move per launch by its function (see the design notes).

    Signature kernels: per CSR entry 12 B (target 4, edge label 4, gathered
    previous block 4), per vertex 12 B (row extent 8, own previous block 4);
    each kernel is charged for the vertices and entries of its degree tier.
    k_lookup: per vertex key hash 8 + distinct count 4 + own block 4 read,
    representative 4 written.  k_scan and k_assign: representative 4 read,
    id 4 written per vertex.
    """
    t = tiers
    if kernel == "k_sig_range":
        return 12.0 * t["range"]["entries"] + 12.0 * t["range"]["vertices"]
    if kernel == "k_sig_row":
        return 12.0 * t["workgroup"]["entries"] + 12.0 * t["workgroup"]["vertices"]
    if kernel == "k_hub_stage":
        return 12.0 * (t["hub"]["entries"] + t["hub_global"]["entries"])
    if kernel == "k_hub_final":
        return 12.0 * (t["hub"]["vertices"] + t["hub_global"]["vertices"])
    if kernel == "k_lookup":
        return 20.0 * n
    if kernel in ("k_scan", "k_assign"):
        return 8.0 * n
    return 0.0


def source_digest() -> str:
    """Digest of the device-kernel source (code lines only, comments and blank lines dropped):
    counter figures taken on other kernels are not reported."""
    h = hashlib.sha256()
    for rel in ["paper_2204_05821_amd/csrc/kernels.h"]:
        with open(os.path.join(ROOT, rel)) as f:
            for line in f:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they match the current source."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
        entry = data.get(workload, {}).get(kernel)
        if not entry or entry.get("source_digest") != source_digest():
            return None
        return float(entry["bytes_per_launch"])
    except Exception:
        return None


def pair_bits(g) -> int:
    """Bits of the largest (edge label, block id) pair of a graph: label bits + block-id bits."""
    import numpy as np
    lb = int(np.max(g.elabel)).bit_length() if g.elabel is not None and g.m else 0
    return max(1, int(max(1, g.n) - 1).bit_length()) + lb


def host_info():
    """Cores this process may use, the machine's core count and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": usable, "cpu_count": os.cpu_count(), "cpu_model": model}


def _cpu_child(g, w, conn):
    try:
        import graphgen
        import oracle
        t0 = time.perf_counter()
        vs = max(1, g.n >> CPU_SAMPLE_SHIFT)
        s = graphgen.prefix_subgraph(g, vs)
        build_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        ids, counts, secs = oracle.refine(s, 1, timings=True)
        wall = time.perf_counter() - t0
        it = secs[0]
        conn.send({"value": s.m / it, "unit": "edge-iterations/s", "cores": 1, "kind": "oracle",
                   "sample": f"refinement iteration 1 of {w['k']} on the rows of the first {vs} of {g.n} vertices "
                             f"({s.m} of {g.m} entries; the {s.n - vs} other vertices they name renumbered "
                             f"compactly, labels kept), {it:.1f} s of refinement, {wall:.1f} s with P0, "
                             f"{build_s:.1f} s to cut the sample; single-threaded C++, one process",
                   "prefix_vertices": vs, "sample_entries": int(s.m), "host": host_info(),
                   "_p1_prefix": ids[0][:vs].copy()})
    except BaseException as e:  # report instead of dying silently
        conn.send({"error": repr(e)})
    finally:
        conn.close()


class CpuBaseline:
    """The CPU reference on a bounded sample, in a child forked before any GPU call."""

    def __init__(self, g, w):
        import multiprocessing as mp
        ctx = mp.get_context("fork")
        self.rx, tx = ctx.Pipe(duplex=False)
        self.proc = ctx.Process(target=_cpu_child, args=(g, w, tx), daemon=True)
        self.proc.start()
        tx.close()

    def collect(self, gpu_p1_prefix=None, gpu_count1=None):
        res = self.rx.recv()
        self.proc.join()
        if "error" in res:
            log(f"[bench] CPU reference failed: {res['error']}")
            return None
        p1 = res.pop("_p1_prefix")
        if gpu_p1_prefix is not None:
            import numpy as np
            res["agrees_with_gpu"] = bool(np.array_equal(p1, gpu_p1_prefix[:len(p1)]))
            if not res["agrees_with_gpu"]:
                log("[bench] WARNING: the CPU reference differs from the GPU on the sample's vertices")
        return res


def copy_probe(kb, torch, mib):
    nbytes = mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    kb.copy_probe(dst, src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        kb.copy_probe(dst, src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    assert torch.equal(dst, src)
    return {"copy_probe_bytes": nbytes, "ms": ms, "GBs_read_plus_write": 2 * nbytes / ms / 1e6}


def run_plain(args, kb, torch, workload, g, cpu_job=None, extras=True):
    """The plain form on one graph: timed k = 10 calls, per-kernel figures, roofline entry."""
    w = WORKLOADS[workload]
    k = w["k"]
    dev = torch.device("cuda:0")
    rp, col, el, vl, vp = kb.to_device(g, dev)
    torch.cuda.synchronize()
    best, tune_report = None, None
    if args.autotune and not args.no_autotune:
        from paper_2204_05821_amd import tune
        holder = {}

        def make(cand):   # every candidate on the first candidate's workspace
            rr = kb.Refiner(rp, col, el, vl, vp, kmax=k, tuning=kb.tuning(**cand), workspace=holder.get("ws"))
            holder["ws"] = rr.workspace
            holder["outs"] = holder.get("outs") or rr.alloc_outputs(k)
            return rr

        t0 = time.perf_counter()
        best, tune_report = tune.autotune(make, lambda rr: rr.refine(k, out=holder["outs"]),
                                          key="plain|" + tune.degree_signature(g.row_ptr), rounds=3, reps=1,
                                          knobs=tune.knobs_for(int(np.diff(g.row_ptr).max()), pair_bits(g)),
                                          cache_path=args.tune_cache)
        del holder
        log(f"[bench] autotune {time.perf_counter() - t0:.1f}s: best {best}; {tune_report['ms']}")
    t0 = time.perf_counter()
    r = kb.Refiner(rp, col, el, vl, vp, kmax=k, tuning=kb.tuning(**best) if best else None)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    tiers = r.schedule_info()
    log(f"[bench] create {create_ms:.1f} ms, workspace {r.workspace_bytes / 2**30:.2f} GiB, tiers {tiers}")
    outs = r.alloc_outputs(k)
    for i in range(args.warmup):
        _, counts = r.refine(k, out=outs)
        log(f"[bench] warmup {i + 1}/{args.warmup} counts {counts}")
    stream = r.stream
    if not args.no_profile:
        # inside the timed region only the signature kernels carry events
        r.profile(True, kinds=["k_sig_range", "k_sig_row"])
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        _, counts = r.refine(k, out=outs)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = max(gpu_ms, wall * 1e3) / args.steps
    value = g.m * k * args.steps / (ms_per_step * args.steps / 1e3)
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step ({gpu_ms:.1f} ms events, {wall * 1e3:.1f} ms wall)")
    p1_prefix = outs[0][:max(1, g.n >> CPU_SAMPLE_SHIFT)].cpu().numpy() if cpu_job is not None else None

    kernels = {}
    roofline = None
    if not args.no_profile:
        timed = {name: v for name, v in r.profile_read().items() if v[1]}
        # per-kernel breakdown from a separate pass with every launch bracketed (not the timed region)
        r.profile(True)
        for _ in range(max(1, min(args.steps, 5))):
            r.refine(k, out=outs)
        prof = r.profile_read()
        r.profile(False)
        total = sum(v[0] for v in prof.values())
        for name, (ms, cnt) in prof.items():
            if cnt:
                kernels[name] = {"ms_per_launch": ms / cnt, "launches": cnt, "share": ms / total if total else 0}
        dom = max((kk for kk in timed if algorithmic_bytes(kk, tiers, g.n, g.m) > 0),
                  key=lambda kk: timed[kk][0])
        ab = algorithmic_bytes(dom, tiers, g.n, g.m)
        avg = timed[dom][0] / timed[dom][1]
        achieved = ab / (avg / 1e3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(dom, workload),
                    "algorithmic_bytes_per_launch": ab, "avg_launch_ms": round(avg, 5)}
    b_alg = 12.0 * g.m + 16.0 * g.n
    step_gbs = b_alg * k / (ms_per_step / 1e3) / 1e9
    # the bare random gather over all entries, for the same partition: the
    # ceiling the signature kernels work against (one pass = one iteration's gathers)
    probe_ms = r.gather_probe(outs[k - 1], reps=5)
    gather = {"ms_per_pass": probe_ms, "entries": g.m, "G_gathers_per_s": g.m / (probe_ms / 1e3) / 1e9,
              "algorithmic_GBs": 8.0 * g.m / (probe_ms / 1e3) / 1e9}
    if roofline is not None:
        sig_ms = sum(kernels[kk]["ms_per_launch"] for kk in ("k_sig_range", "k_sig_row", "k_hub_stage",
                                                             "k_hub_reduce") if kk in kernels)
        gather["signature_kernels_ms_per_iteration"] = sig_ms
        gather["probe_share_of_signature_time"] = probe_ms / sig_ms if sig_ms else None
    log(f"[bench] gather probe: {probe_ms:.3f} ms per pass over {g.m} entries "
        f"({gather['G_gathers_per_s']:.1f} G gathers/s)")

    work_efficient = summary = None
    if not extras:
        r.close()
        del rp, col, el, vl, vp, outs, r
        torch.cuda.empty_cache()
        return {"workload": workload, "value": value, "unit": "edge-iterations/s", "ms_per_step": ms_per_step,
                "steps": args.steps, "n": g.n, "m": g.m, "k": k, "recipe": w["desc"], "seed": w["seed"],
                "roofline": roofline, "step_hbm": {"algorithmic_bytes_per_iteration": b_alg,
                                                   "achieved_GBs": round(step_gbs, 1),
                                                   "frac_of_peak": round(step_gbs / HBM_PEAK_GBS, 4)},
                "counts": counts, "gather_probe": gather, "create_ms": round(create_ms, 1), "kernels": kernels,
                "tiers": tiers}
    # Work-efficient mode (singleton blocks skipped, stop at the fixpoint): reported
    # separately; its outputs must equal the full-work outputs.
    full = [o.clone() for o in outs]
    r.work_efficient(True)
    _, we_counts = r.refine(k, out=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, we_counts = r.refine(k, out=outs)
    torch.cuda.synchronize()
    we_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    we_steps = r.work_efficient(None)
    we_same = we_counts == counts and all(torch.equal(a, b) for a, b in zip(outs, full))
    r.work_efficient(False)
    # Summary graph of the chain's last step: source blocks P_k, target blocks P_{k-1}.
    r.quotient(full[k - 1], full[k - 2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qs, ql, qd = r.quotient(full[k - 1], full[k - 2])
    torch.cuda.synchronize()
    summary = {"ms": (time.perf_counter() - t0) * 1e3, "edges": int(qs.numel()), "blocks": counts[k - 1],
               "note": "distinct (P_k block, label, P_(k-1) block) triples, sorted; device radix sort"}
    log(f"[bench] summary graph: {summary['edges']} edges over {summary['blocks']} blocks in {summary['ms']:.2f} ms")
    del full, qs, ql, qd
    log(f"[bench] work-efficient: {we_ms:.3f} ms per call, {we_steps} steps computed, identical {we_same}")
    work_efficient = {"ms_per_call": we_ms, "steps_computed": we_steps,
                      "equivalent_edge_iterations_per_s": g.m * k / (we_ms / 1e3),
                      "speedup_vs_full_work": ms_per_step / we_ms, "identical_outputs": bool(we_same),
                      "note": "singleton blocks skipped and the loop stopped at the fixpoint; not the headline value"}
    r.close()
    del outs, r
    torch.cuda.empty_cache()
    # after the main context is released: the leg holds a cached context, an edited copy of the
    # targets and a fresh context for the check (about 3.5 workspaces on the 2B-edge graph)
    incremental = None if args.no_incremental else incremental_leg(kb, torch, g, (rp, col, el, vl, vp), k,
                                                                   ms_per_step, we_ms)
    del rp, col, el, vl, vp
    torch.cuda.empty_cache()

    cpu = None
    if cpu_job is not None:
        log("[bench] waiting for the CPU reference ...")
        cpu = cpu_job.collect(p1_prefix)
        if cpu:
            log(f"[bench] CPU reference: {cpu['value']:.3e} edge-iterations/s ({cpu['sample']}); "
                f"agrees with the GPU: {cpu.get('agrees_with_gpu')}")

    return {
        "metric": "edge-iterations/sec at k=10 (plain)",
        "value": value,
        "unit": "edge-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": workload, "n": g.n, "m": g.m, "k": k, "recipe": w["desc"],
                   "seed": w["seed"], "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "step_hbm": {"algorithmic_bytes_per_iteration": b_alg, "achieved_GBs": round(step_gbs, 1),
                     "frac_of_peak": round(step_gbs / HBM_PEAK_GBS, 4)},
        "counts": counts,
        "gather_probe": gather,
        "work_efficient": work_efficient,
        "summary_graph": summary,
        "incremental": incremental,
        "create_ms": round(create_ms, 1),
        "tuning": best,
        "autotune_ms": tune_report["ms"] if tune_report else None,
        "kernels": kernels,
        "tiers": tiers,
    }


def incremental_leg(kb, torch, g, dev, k, full_ms, we_ms=None, sizes=(1, 1000, 100_000), reps=3):
    """Updates after edits: a context with its chain cached, then edited copies of the graph
    (the targets of `e` random entries replaced by random vertices, so the rows of their
    sources change), recomputed by kbisim_incr_update and timed against a full refine call
    and against the work-efficient refine (both stop computing at the fixpoint); each result
    is compared with a fresh context's refinement of the edited graph."""
    rp, col, el, vl, vp = dev
    r = kb.Refiner(rp, col, el, vl, vp, kmax=k)
    t0 = time.perf_counter()
    r.incremental()
    torch.cuda.synchronize()
    enable_ms = (time.perf_counter() - t0) * 1e3
    r.refine(k)
    t0 = time.perf_counter()
    base_ids, base_counts = r.refine(k)
    torch.cuda.synchronize()
    cached_ms = (time.perf_counter() - t0) * 1e3
    rng = np.random.default_rng(123)
    out = {"cached_refine_ms": cached_ms, "full_refine_ms": full_ms, "work_efficient_refine_ms": we_ms,
           "enable_ms": enable_ms, "state_GiB": r.incr_state.numel() / 2**30,
           "note": "an update stops at the fixpoint (two consecutive partitions with equal block counts) and "
                   "copies the later partitions", "edits": []}
    outs = r.alloc_outputs(k)
    for e in sizes:
        idx = np.sort(rng.choice(g.m, size=e, replace=False))
        rows = np.unique(np.searchsorted(g.row_ptr, idx, side="right") - 1).astype(np.int32)
        col2 = col.clone()
        col2[torch.from_numpy(idx).to(col.device)] = torch.from_numpy(
            rng.integers(0, g.n, size=e).astype(np.int32)).to(col.device)
        rows_d = torch.from_numpy(rows).to(col.device)
        r.update(rp, col2, el, rows_d, k, out=outs)      # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, counts = r.update(rp, col2, el, rows_d, k, out=outs)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        f = kb.Refiner(rp, col2, el, vl, vp, kmax=k)
        fids, fcounts = f.refine(k)
        same = fcounts == counts and all(torch.equal(a, b) for a, b in zip(fids, outs))
        f.close()
        del f, fids, col2
        torch.cuda.empty_cache()
        out["edits"].append({"edited_entries": e, "edited_rows": int(len(rows)), "update_ms": ms,
                             "speedup_vs_full_refine": full_ms / ms,
                             "speedup_vs_work_efficient_refine": we_ms / ms if we_ms else None,
                             "identical_to_refine_of_edited_graph": same, "counts": counts})
        log(f"[bench] incremental: {e} edited entries ({len(rows)} rows): {ms:.2f} ms per k={k} update "
            f"({full_ms / ms:.1f}x a full refine, {(we_ms or 0) / ms:.1f}x a work-efficient one), identical {same}")
    r.close()
    del r, outs, base_ids
    torch.cuda.empty_cache()
    return out


def run_batched(args, kb, torch):
    """4,096 graphs as one batch (captured k-loop, autotuned shapes) against per-graph plain calls."""
    import numpy as np
    import graphgen
    from paper_2204_05821_amd import tune
    k = 10
    t0 = time.perf_counter()
    sizes = graphgen.batch_sizes(args.batch_graphs)
    graphs = [graphgen.batch_graph(i, m) for i, m in enumerate(sizes)]
    m_total = sum(g.m for g in graphs)
    log(f"[batched] generated {len(graphs)} graphs, {m_total} edges in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    rp, col, el, vl, vp, off = kb.union_of(graphs)
    d = [None if x is None else torch.from_numpy(x).cuda() for x in (rp, col, el, vl, vp)]
    torch.cuda.synchronize()
    del rp, col, el, vl, vp
    log(f"[batched] union on device in {time.perf_counter() - t0:.1f}s")

    holder = {}

    def make(cand):   # every candidate on the first candidate's workspace
        b = kb.Batch(*d, off, kmax=k, tuning=kb.tuning(**cand), graphs=True, workspace=holder.get("ws"))
        holder["ws"] = b.workspace
        holder["outs"] = holder.get("outs") or b.alloc_outputs(k)
        return b

    def run(b):
        return b.refine(k, out=holder["outs"])

    max_deg = max(int(np.diff(gr.row_ptr).max()) if gr.m else 0 for gr in graphs)
    pbits = max(int(max(1, gr.n) - 1).bit_length() for gr in graphs) + max(
        int(gr.elabel.max()).bit_length() if gr.elabel is not None and gr.m else 0 for gr in graphs)
    t0 = time.perf_counter()
    best, report = tune.autotune(make, run, key="batch|" + tune.degree_signature(d[0].cpu().numpy()), rounds=3,
                                 reps=1, knobs=tune.knobs_for(max_deg, pbits), cache_path=args.tune_cache)
    log(f"[batched] autotune {time.perf_counter() - t0:.1f}s: best {best}; {report['ms']}")
    t0 = time.perf_counter()
    b = kb.Batch(*d, off, kmax=k, tuning=kb.tuning(**best), graphs=True, workspace=holder["ws"])
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    outs = holder["outs"]
    for _ in range(2):
        _, counts = b.refine(k, out=outs)
    reps = args.batch_steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, counts = b.refine(k, out=outs)
    torch.cuda.synchronize()
    batched_s = (time.perf_counter() - t0) / reps
    packed = [o.clone() for o in outs]
    b.close()
    del b, holder, d, outs
    torch.cuda.empty_cache()
    log(f"[batched] batched: {batched_s * 1e3:.1f} ms per k={k} pass, create {create_ms:.0f} ms")

    # per-graph plain calls: one context per graph, created before timing
    t0 = time.perf_counter()
    refs = [kb.refiner_for(g, kmax=k) for g in graphs]
    gouts = [r.alloc_outputs(k) for r in refs]
    torch.cuda.synchronize()
    log(f"[batched] {len(refs)} per-graph contexts in {time.perf_counter() - t0:.1f}s")
    for r, o in zip(refs, gouts):
        r.refine(k, out=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pg_counts = None
    for _ in range(reps):
        pg_counts = [r.refine(k, out=o)[1] for r, o in zip(refs, gouts)]
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / reps
    same = pg_counts == counts
    for gi in range(0, len(graphs), max(1, len(graphs) // 64)):
        for i in range(k):
            if not torch.equal(gouts[gi][i], packed[i][int(off[gi]):int(off[gi + 1])]):
                same = False
    for r in refs:
        r.close()
    del refs, gouts, packed
    torch.cuda.empty_cache()
    log(f"[batched] per-graph plain: {plain_s * 1e3:.1f} ms per pass; identical results: {same}")
    return {"workload": f"batch_{len(graphs)}_graphs_m1k-2M_k10", "graphs": len(graphs), "m_total": m_total,
            "k": k, "value": m_total * k / batched_s, "unit": "edge-iterations/s",
            "ms_per_pass": batched_s * 1e3, "per_graph_plain": {"value": m_total * k / plain_s,
                                                                 "ms_per_pass": plain_s * 1e3},
            "speedup_vs_per_graph": plain_s / batched_s, "identical_to_per_graph": bool(same),
            "tuning": best, "autotune_ms": report["ms"][:8], "autotune_samples": report.get("samples"),
            "create_ms": round(create_ms, 1),
            "recipe": "graph g: m_g log-uniform 1e3..2e6; even g uniform-random n=max(16,m/8), odd g RMAT "
                      "(0.57,0.19,0.19,0.05) scale ceil(log2(m/8)); 16 vertex and 32 edge labels uniform"}


def run_serve(args, kb, torch):
    """Poisson arrivals under a 200 GB budget; capacity against one-job-at-a-time."""
    import random
    import graphgen
    from paper_2204_05821_amd import serve
    t0 = time.perf_counter()
    pool = []
    for j in range(args.serve_pool):   # one host graph at a time: only the pinned copies stay
        pool.append(serve.DeviceBackend.pin(graphgen.serving_pool_graph(j)))
    pool_m = [g.m for g in pool]
    log(f"[serve] pool of {len(pool)} graphs ({sum(pool_m)} edges) pinned in {time.perf_counter() - t0:.1f}s")
    budget = 200 * 10**9
    rnd = random.Random(11)

    def draw_jobs(count):
        return [(rnd.randrange(len(pool)), rnd.randint(1, 10)) for _ in range(count)]

    whole = {"whole_edges": args.serve_whole_edges} if args.serve_whole_edges > 0 else {}

    def closed_loop(server_cls, jobs, **kw):
        be = serve.DeviceBackend(streams=4, keep_outputs=False)
        srv = server_cls(be, budget, **kw).start()
        t = time.perf_counter()
        js = [srv.submit(pool[gi], k) for gi, k in jobs]
        srv.stop()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        err = [j.error for j in js if j.error is not None]
        if err:
            raise err[0]
        return wall, [j.counts for j in js], srv.stats()

    # warm-up (library load, allocator, first contexts)
    closed_loop(serve.Server, draw_jobs(16), **whole)
    # capacity: the same job list through both servers
    jobs = draw_jobs(args.serve_capacity_jobs)
    ek = sum(pool_m[gi] * k for gi, k in jobs)
    cont_s, cont_counts, cont_st = closed_loop(serve.Server, jobs, **whole)
    fifo_s, fifo_counts, _ = closed_loop(serve.FifoServer, jobs)
    log(f"[serve] capacity on {len(jobs)} jobs: continuous {cont_s:.2f}s, one-at-a-time {fifo_s:.2f}s, "
        f"identical counts {cont_counts == fifo_counts}")

    # open loop: Poisson arrivals at the offered rate
    be = serve.DeviceBackend(streams=4, keep_outputs=False)
    srv = serve.Server(be, budget, **whole).start()
    t_end = time.perf_counter() + args.serve_seconds
    submitted = []
    nxt = time.perf_counter()
    while True:
        nxt += rnd.expovariate(args.serve_rate)
        if nxt > t_end:
            break
        dt = nxt - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        gi, k = rnd.randrange(len(pool)), rnd.randint(1, 10)
        submitted.append((srv.submit(pool[gi], k), pool_m[gi]))
    srv.stop()
    torch.cuda.synchronize()
    st = srv.stats()
    js = [j for j, _ in submitted]
    first = min(j.arrival for j in js)
    last = max(j.finished for j in js)
    ek_open = sum(m * j.k for j, m in submitted)
    # where the slowest 1% of jobs spend their time
    slow = sorted(submitted, key=lambda jm: -jm[0].latency)[:max(1, len(submitted) // 100)]
    tail = {"jobs": len(slow),
            "mean_edges": sum(m for _, m in slow) / len(slow),
            "mean_k": sum(j.k for j, _ in slow) / len(slow),
            "mean_queue_ms": 1e3 * sum(j.admitted - j.arrival for j, _ in slow) / len(slow),
            "mean_prepare_ms": 1e3 * sum(j.ready - j.admitted for j, _ in slow) / len(slow),
            "mean_run_ms": 1e3 * sum(j.finished - j.ready for j, _ in slow) / len(slow)}
    log(f"[serve] Poisson {args.serve_rate}/s for {args.serve_seconds}s: {st}; slowest 1%: {tail}")
    return {"workload": "serve_poisson200_rmat_m10k-50M_k1-10", "rate_per_s": args.serve_rate,
            "seconds": args.serve_seconds, "jobs": len(js), "errors": st["errors"] + st["rejected"],
            "p50_ms": st["p50_s"] * 1e3, "p99_ms": st["p99_s"] * 1e3,
            "p50_admit_prepare_ms": st["p50_admit_prepare_s"] * 1e3,
            "jobs_per_s": len(js) / (last - first), "edge_iterations_per_s": ek_open / (last - first),
            "mean_jobs_per_tick": st["mean_jobs_per_tick"], "units": st["units"], "slowest_1pct": tail,
            "peak_budget_bytes": st["peak_bytes"], "budget_bytes": budget,
            "capacity": {"jobs": len(jobs), "continuous_jobs_per_s": len(jobs) / cont_s,
                         "one_at_a_time_jobs_per_s": len(jobs) / fifo_s,
                         "continuous_edge_iterations_per_s": ek / cont_s,
                         "one_at_a_time_edge_iterations_per_s": ek / fifo_s,
                         "speedup": fifo_s / cont_s, "identical_counts": cont_counts == fifo_counts,
                         "mean_jobs_per_tick": cont_st["mean_jobs_per_tick"]},
            "pool": {"graphs": len(pool), "edges": sum(pool_m)},
            "whole_edges": args.serve_whole_edges or None,
            "shape": ("as configured: 256 pool graphs, 60 s of arrivals" if len(pool) == 256 and
                      args.serve_seconds == 60 else f"reduced: {len(pool)} pool graphs, {args.serve_seconds:g} s "
                                                     "of arrivals (configured: 256 graphs, 60 s)"),
            "latency": "arrival to counts on the host and ids on the device, H2D of the CSR included"}


def main():
    wall0 = time.perf_counter()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="all", choices=["all", "plain", "batched", "serve"])
    ap.add_argument("--workload", default="rmat_rdf_s27_m1B_k10", choices=sorted(WORKLOADS))
    ap.add_argument("--extra-workload", default="rmat_s23_m100M_k10",
                    help="a second plain workload reported beside the headline in --mode all ('' = none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip per-kernel event timing")
    ap.add_argument("--no-incremental", action="store_true", help="skip the incremental-update leg")
    ap.add_argument("--autotune", action="store_true",
                    help="plain form: search the launch shapes first (default: the library defaults, which the "
                         "search picks within noise on this workload)")
    ap.add_argument("--no-autotune", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--batch-graphs", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--tune-cache", default=None, help="JSON file for autotuner choices (default: none kept)")
    ap.add_argument("--serve-pool", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-capacity-jobs", type=int, default=200)
    ap.add_argument("--serve-whole-edges", type=int, default=2_000_001,
                    help="jobs of at least this many edges (solo units) are refined in one call on a worker "
                         "instead of one step per tick (0 = every unit steps per tick)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run the library's streaming copy kernel on this many MiB (bandwidth and counter "
                         "calibration) and print its rate")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the refinement of one graph runs on one GPU; no multi-GPU figure is produced "
              "(the sharding design is described in the design notes).", file=sys.stderr)
        sys.exit(2)

    # Host inputs first: the CPU reference is forked before anything touches the GPU.
    g = cpu_job = None
    if args.mode in ("all", "plain") and not args.copy_probe_mib:
        t0 = time.perf_counter()
        g = make_graph(WORKLOADS[args.workload])
        log(f"[bench] generated {args.workload}: n={g.n} m={g.m} in {time.perf_counter() - t0:.1f}s")
        if not args.no_cpu_baseline:
            cpu_job = CpuBaseline(g, WORKLOADS[args.workload])

    import torch
    import paper_2204_05821_amd as kb
    torch.cuda.set_device(torch.device("cuda:0"))

    if args.copy_probe_mib:
        print(json.dumps(copy_probe(kb, torch, args.copy_probe_mib)), flush=True)
        return
    res = None
    if args.mode in ("all", "plain"):
        res = run_plain(args, kb, torch, args.workload, g, cpu_job)
        del g
        if args.mode == "all" and args.extra_workload and args.extra_workload != args.workload:
            t0 = time.perf_counter()
            g2 = make_graph(WORKLOADS[args.extra_workload])
            log(f"[bench] generated {args.extra_workload}: n={g2.n} m={g2.m} in {time.perf_counter() - t0:.1f}s")
            res["plain_extra"] = run_plain(args, kb, torch, args.extra_workload, g2, None, extras=False)
            del g2
    if args.mode in ("all", "batched"):
        bres = run_batched(args, kb, torch)
        res = bres if res is None else dict(res, batched=bres)
    if args.mode in ("all", "serve"):
        sres = run_serve(args, kb, torch)
        res = sres if res is None else dict(res, served=sres)
    res["bench_wall_s"] = round(time.perf_counter() - wall0, 1)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
