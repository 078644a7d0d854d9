#!/usr/bin/env python3
"""Benchmark of k-bisimulation refinement on one MI355X.

A step is one call of kbisim_refine(k=10) on the whole graph: ten full
refinement iterations (signature gather and dedupe, key hashing, grouping,
exact check, first-vertex numbering), inputs already resident in HBM.  The
metric is edge-iterations per second: m * k * steps / time.

Default workload: RMAT scale 23 (8,388,608 vertices), 100,000,000 directed
edges, (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), one vertex label per vertex
drawn Zipf(1.0) over 32 labels, edge labels Zipf(1.1) over 64, seed 2.
The paper's datasets are not available; this synthetic recipe stands in for
its 100M-edge class.

Prints one JSON line with the throughput, a roofline entry for the dominant
kernel (timed with HIP events inside the timed region) and the CPU reference
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s (published)

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
    if kernel == "k_sig_block":
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
    h = hashlib.sha256()
    for rel in ["paper_2204_05821_amd/csrc/kernels.h", "paper_2204_05821_amd/csrc/kbisim.hip"]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
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


def cpu_baseline(g, w, max_iters: int = 1):
    """The CPU reference, as it stands, on a bounded sample: the first refinement iteration(s)."""
    import oracle
    t0 = time.perf_counter()
    ids, counts, secs = oracle.refine(g, max_iters, timings=True)
    wall = time.perf_counter() - t0
    it = sum(secs)
    value = g.m * max_iters / it
    return {"value": value, "unit": "edge-iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"iteration 1..{max_iters} of {w['k']} on the full graph (n={g.n}, m={g.m}), "
                      f"{it:.1f} s of refinement, {wall:.1f} s wall, single-threaded C++",
            "counts": counts}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat_s23_m100M_k10", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip per-kernel event timing")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run the library's streaming copy kernel on this many MiB (bandwidth and counter "
                         "calibration) and print its rate")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU; a multi-GPU figure is not produced "
              "(the sharding design is described in the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2204_05821_amd as kb

    if args.copy_probe_mib:
        nbytes = args.copy_probe_mib << 20
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
        print(json.dumps({"copy_probe_bytes": nbytes, "ms": ms, "GBs_read_plus_write": 2 * nbytes / ms / 1e6}),
              flush=True)
        return

    w = WORKLOADS[args.workload]
    k = w["k"]
    t0 = time.perf_counter()
    g = make_graph(w)
    log(f"[bench] generated {args.workload}: n={g.n} m={g.m} in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rp, col, el, vl, vp = kb.to_device(g, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = kb.Refiner(rp, col, el, vl, vp, kmax=k)
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
        r.profile(True)
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

    kernels = {}
    roofline = None
    if not args.no_profile:
        prof = r.profile_read()
        r.profile(False)
        total = sum(v[0] for v in prof.values())
        for name, (ms, cnt) in prof.items():
            if cnt:
                kernels[name] = {"ms_per_launch": ms / cnt, "launches": cnt, "share": ms / total if total else 0}
        dom = max((kk for kk in kernels if algorithmic_bytes(kk, tiers, g.n, g.m) > 0),
                  key=lambda kk: kernels[kk]["ms_per_launch"] * kernels[kk]["launches"])
        ab = algorithmic_bytes(dom, tiers, g.n, g.m)
        avg = kernels[dom]["ms_per_launch"]
        achieved = ab / (avg / 1e3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(dom, args.workload),
                    "algorithmic_bytes_per_launch": ab, "avg_launch_ms": round(avg, 5)}
    b_alg = 12.0 * g.m + 16.0 * g.n
    step_gbs = b_alg * k / (ms_per_step / 1e3) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU reference on iteration 1 ...")
        cpu = cpu_baseline(g, w)
        log(f"[bench] CPU reference: {cpu['value']:.3e} edge-iterations/s ({cpu['sample']})")
        if cpu.pop("counts")[0] != counts[0]:
            log("[bench] WARNING: CPU reference count differs from the GPU count at iteration 1")

    res = {
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
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "k": k, "recipe": w["desc"],
                   "seed": w["seed"], "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "step_hbm": {"algorithmic_bytes_per_iteration": b_alg, "achieved_GBs": round(step_gbs, 1),
                     "frac_of_peak": round(step_gbs / HBM_PEAK_GBS, 4)},
        "counts": counts,
        "create_ms": round(create_ms, 1),
        "kernels": kernels,
        "tiers": tiers,
    }
    r.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
