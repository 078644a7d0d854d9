"""Autotuner for launch shapes (range capacity, hub chunk, hub partition size).

For a given graph or batch it runs every candidate tuning, times a few
refinement calls after a warm-up, checks that every candidate's partitions
and counts are bit-identical to the first candidate's (launch shape must
never change results), and returns the fastest.  Choices are cached in a
JSON file keyed by the GPU architecture and a coarse degree histogram of the
input, so a later run on a similar input skips the search.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

CANDIDATES = [dict(range_edges=re, hub_chunk=hc, hub_part_target=hp)
              for re, hc, hp in itertools.product([1024, 2048], [2048, 4096], [1024, 2048])]

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
             reps: int = 2, candidates: Optional[List[Dict]] = None, cache_path: Optional[str] = DEFAULT_CACHE,
             close: Callable[[object], None] = lambda r: r.close()) -> Tuple[Dict, Dict]:
    """Pick the fastest candidate for `key`.

    make(tuning_dict) builds a runner, run(runner) performs one refinement call
    and returns (device outputs, counts); close(runner) releases it.  Returns
    (best tuning dict, report).  Raises if two candidates disagree.
    """
    import torch
    cache = load_cache(cache_path) if cache_path else {}
    full_key = f"{_arch()}|{key}"
    if full_key in cache:
        return cache[full_key]["best"], cache[full_key]
    cands = candidates or CANDIDATES
    ref_outs, ref_counts = None, None
    timings = []
    for cand in cands:
        r = make(cand)
        outs, counts = run(r)                 # warm-up (and capture), also the result to compare
        run(r)
        torch.cuda.synchronize()
        if ref_outs is None:
            ref_outs = [o.clone() for o in outs]
            ref_counts = counts
        else:
            if counts != ref_counts or any(not torch.equal(a, b) for a, b in zip(outs, ref_outs)):
                close(r)
                raise AssertionError(f"tuning {cand} changed the result")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            run(r)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        timings.append((ms, cand))
        close(r)
    timings.sort(key=lambda x: x[0])
    report = {"best": timings[0][1], "ms": [[round(ms, 3), c] for ms, c in timings]}
    if cache_path:
        cache[full_key] = report
        save_cache(cache, cache_path)
    return timings[0][1], report
