"""Autotuner for launch shapes.

Knobs (all in ``kbisim_tuning``; results never depend on them): set-key form
(``key_bits``: 32-bit exact-or-hashed, hashed, 64-bit), range capacity (the
row-tier threshold, ``range_edges``), hub chunk and hub partition size (only
when the graph has hub rows) and the numbering scan's items per thread
(``scan_items``).

The search is coordinate-wise: starting from the defaults, one knob at a
time takes each of its values, keeping the others at the best found so far.
For one knob every value is timed in ``rounds`` interleaved rounds, the order
of the values rotating from round to round, and the median decides, so a
value is not favoured by where it falls in the sequence.  The value in place
(the default, or the start) is kept unless another one's median is lower by
more than ``margin`` (a fraction of the kept value's median): differences
within timing noise do not move the choice, so it does not depend on the
order in which knobs or values are tried.  Every runner is
built on the same workspace (the caller's ``make`` passes one buffer, sized
for the input, to every candidate), so no candidate pays for allocator churn
left by another.  Every candidate's partitions and counts must be
bit-identical to the first one's.  Choices are cached in a JSON file keyed by
the GPU architecture and a coarse degree histogram of the input.
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

DEFAULTS = dict(key_bits=0, range_edges=0, hub_chunk=2048, hub_part_target=2048, scan_items=16)
# range_edges 0 = by key width (2048 entries with 32-bit keys, 1024 with 64-bit keys)
KNOBS = [("key_bits", [0, 32, 64]), ("range_edges", [0, 1024, 2048]), ("hub_chunk", [2048, 4096]),
         ("hub_part_target", [1024, 2048]), ("scan_items", [8, 16])]
HUB_KNOBS = ("hub_chunk", "hub_part_target")

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "kbisim", "tune.json")


def degree_signature(row_ptr: np.ndarray) -> str:
    """Coarse shape of an input: n, m and the share of entries per power-of-two degree class."""
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64))
    n, m = int(deg.shape[0]), int(deg.sum())
    if m == 0:
        return f"n{n}_m0"
    cls = np.zeros(deg.shape, dtype=np.int64)
    nz = deg > 0
    cls[nz] = np.floor(np.log2(deg[nz])).astype(np.int64) + 1
    share = np.bincount(cls, weights=deg, minlength=32)[:32] / m
    coarse = ",".join(f"{x:.2f}" for x in share)
    return f"n{n.bit_length()}_m{m.bit_length()}_{hashlib.sha1(coarse.encode()).hexdigest()[:12]}"


def knobs_for(max_degree: int, pair_bits: int) -> List[Tuple[str, List[int]]]:
    """The knobs that can change the work split of an input.

    max_degree: longest row.  pair_bits: bits of the largest (edge label, block
    id) pair, i.e. bit width of the largest label plus that of the largest
    graph's vertex count.  Hub knobs matter only with rows beyond the row tiers
    (8,192 entries, or 19,456 with 32-bit keys); exact 32-bit keys exist only
    when pairs fit 31 bits (otherwise the default already hashes them)."""
    out = []
    for name, vals in KNOBS:
        if name in HUB_KNOBS and max_degree <= 8192:
            continue
        if name == "key_bits" and pair_bits > 31:
            vals = [0, 64]
        out.append((name, list(vals)))
    return out


def _arch() -> str:
    try:
        import torch
        return getattr(torch.cuda.get_device_properties(0), "gcnArchName", "gpu").split(":")[0]
    except Exception:
        return "unknown"


def load_cache(path: str = DEFAULT_CACHE) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except Exception:
        return {}


def save_cache(data: Dict, path: str = DEFAULT_CACHE) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(make: Callable[[Dict], object], run: Callable[[object], Tuple[list, list]], key: str,
             rounds: int = 3, reps: int = 1, knobs: Optional[Sequence[Tuple[str, List[int]]]] = None,
             start: Optional[Dict] = None, cache_path: Optional[str] = DEFAULT_CACHE,
             close: Callable[[object], None] = lambda r: r.close(), sync: Optional[Callable[[], None]] = None,
             margin: float = 0.01) -> Tuple[Dict, Dict]:
    """Pick the fastest tuning for `key`.

    make(tuning_dict) builds a runner (on the caller's shared workspace),
    run(runner) performs one refinement call and returns (device outputs,
    counts), close(runner) releases it.  Each timed sample is one warm-up
    call followed by `reps` timed calls on a freshly made runner.  Returns
    (best tuning dict, report with every sample).  Raises if two candidates
    disagree.
    """
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    cache = load_cache(cache_path) if cache_path else {}
    full_key = f"{_arch()}|{key}"
    if full_key in cache:
        return cache[full_key]["best"], cache[full_key]
    best = dict(DEFAULTS, **(start or {}))
    knobs = list(knobs if knobs is not None else KNOBS)
    ref = {}
    samples: Dict[str, List[float]] = {}

    def sample(cand: Dict) -> float:
        r = make(cand)
        try:
            outs, counts = run(r)                 # warm-up (and capture), also the result to compare
            sync()
            if not ref:
                ref["outs"] = [o.clone() for o in outs]
                ref["counts"] = counts
            elif counts != ref["counts"] or any(not bool((a == b).all()) for a, b in zip(outs, ref["outs"])):
                raise AssertionError(f"tuning {cand} changed the result")
            t0 = time.perf_counter()
            for _ in range(reps):
                run(r)
            sync()
            return (time.perf_counter() - t0) * 1e3 / reps
        finally:
            close(r)

    for name, values in knobs:
        values = list(values)
        if len(values) < 2:
            continue
        times: Dict[int, List[float]] = {v: [] for v in values}
        for rd in range(rounds):
            order = values[rd % len(values):] + values[:rd % len(values)]
            if rd % 2:
                order = order[::-1]
            for v in order:
                cand = dict(best, **{name: v})
                ms = sample(cand)
                times[v].append(ms)
                samples.setdefault(json.dumps(cand, sort_keys=True), []).append(round(ms, 3))
        med = {v: statistics.median(t) for v, t in times.items()}
        cur = best[name] if best[name] in med else min(values, key=lambda v: (med[v], values.index(v)))
        fastest = min(values, key=lambda v: (med[v], v))
        if med[fastest] < med[cur] * (1.0 - margin):
            cur = fastest
        best[name] = cur
    ranked = sorted(((statistics.median(t), json.loads(c)) for c, t in samples.items()), key=lambda x: x[0])
    report = {"best": best, "ms": [[round(ms, 3), c] for ms, c in ranked], "samples": samples,
              "rounds": rounds, "reps": reps, "margin": margin,
              "search": "coordinate, interleaved rounds, median; the value in place kept within the margin"}
    if cache_path:
        cache[full_key] = report
        save_cache(cache, cache_path)
    return best, report
