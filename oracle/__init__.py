"""CPU reference for k-bisimulation partition refinement — TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it and shares no code with
it (the only common dependency is the seeded input generator ``graphgen``).

Three independent references live here:

* ``refine`` / ``initial`` — the plain definition (``oracle.cpp``): per vertex
  a sorted, duplicate-free vector of (edge label, previous block) pairs, and a
  ``std::map`` from (previous block, that vector) to dense ids numbered by
  first vertex.  Def. edge-labeled-fw-bisimulation for the step, the base case
  of Def. vertex-labeled-bw-bisimulation for P0, Def. signature for the pair
  set, Alg. schaetzle-alg for the loop structure.
* ``brute.brute_force`` — pairwise relations straight from the definitions
  (tiny graphs only).
* ``splitter.splitter_refine`` — a splitter-based refinement in the style of
  Alg. kaushik-alg, adapted to (edge label, block) splitters.

``check_initial`` / ``check_step`` (``stepcheck.cpp``) check a given
partition chain against the definition at sizes the plain reference cannot
reach in test time: canonical ids, and each partition exactly the partition
by (previous block, signature).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# KBISIM_SANITIZE=1 selects copies built with AddressSanitizer and
# UndefinedBehaviorSanitizer (host code only; the process must preload libasan).
SANITIZE = os.environ.get("KBISIM_SANITIZE", "") == "1"
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
_SUFFIX = "_san.so" if SANITIZE else ".so"
_LIB_PATH = os.path.join(_HERE, "liboracle" + _SUFFIX)
_lib = None


_CHECK_PATH = os.path.join(_HERE, "libstepcheck" + _SUFFIX)
_check_lib = None


def build(force: bool = True, sanitize: Optional[bool] = None) -> str:
    """Compile liboracle.so and libstepcheck.so (or their sanitizer copies, *_san.so) in place."""
    san = SANITIZE if sanitize is None else sanitize
    suffix = "_san.so" if san else ".so"
    for src, lib, extra in [("oracle.cpp", "liboracle" + suffix, []),
                            ("stepcheck.cpp", "libstepcheck" + suffix, ["-fopenmp"])]:
        src = os.path.join(_HERE, src)
        lib = os.path.join(_HERE, lib)
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
            tmp = lib + ".tmp"
            flags = ["-O1"] + SAN_FLAGS if san else ["-O2"]
            subprocess.check_call(["g++"] + flags + ["-std=c++17", "-fPIC", "-shared", "-Wall"] + extra +
                                  ["-o", tmp, src])
            os.replace(tmp, lib)
    return os.path.join(_HERE, "liboracle" + suffix)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    lib.oracle_initial.argtypes = [ctypes.c_int64, vp, vp, vp, vp]
    lib.oracle_initial.restype = ctypes.c_int
    lib.oracle_refine.argtypes = [ctypes.c_int64, ctypes.c_int64, vp, vp, vp, vp, vp, vp, ctypes.c_int, vp, vp, vp]
    lib.oracle_refine.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def initial(g) -> Tuple[np.ndarray, int]:
    """P0: blocks of equal vertex label sets, ids numbered by first vertex."""
    lib = _load()
    out = np.empty(g.n, dtype=np.int32)
    cnt = np.zeros(1, dtype=np.int64)
    vp, vl = _c(g.vlabel_ptr, np.int64), _c(g.vlabel, np.int32)
    rc = lib.oracle_initial(g.n, _p(vp), _p(vl), _p(out), _p(cnt))
    if rc != 0:
        raise ValueError(f"oracle_initial failed: {rc}")
    return out, int(cnt[0])


def refine(g, k: int, start: Optional[np.ndarray] = None, timings: bool = False):
    """Partitions P_1..P_k (list of int32 arrays) and their block counts.

    ``start`` replaces P0 by a given partition (resume from P_i).  With
    ``timings`` the per-iteration wall times (seconds) are returned as well.
    """
    lib = _load()
    n = g.n
    out = np.empty((k, n), dtype=np.int32)
    counts = np.zeros(max(k, 1), dtype=np.int64)
    secs = np.zeros(max(k, 1), dtype=np.float64)
    rp, col, el = _c(g.row_ptr, np.int64), _c(g.col, np.int32), _c(g.elabel, np.int32)
    vp, vl = _c(g.vlabel_ptr, np.int64), _c(g.vlabel, np.int32)
    st = _c(start, np.int32)
    rc = lib.oracle_refine(n, g.m, _p(rp), _p(col), _p(el), _p(vp), _p(vl), _p(st), k, _p(out), _p(counts), _p(secs))
    if rc != 0:
        raise ValueError(f"oracle_refine failed: {rc}")
    ids: List[np.ndarray] = [out[i] for i in range(k)]
    cl = [int(c) for c in counts[:k]]
    if timings:
        return ids, cl, [float(s) for s in secs[:k]]
    return ids, cl


MUTATIONS = {
    "multiset": 1, "no_old_block": 2, "no_edge_label": 3, "source_block": 4,
    "key_order_ids": 5, "drop_last_edge": 6, "p0_no_labels": 7, "p0_first_label": 8,
}


class planted_mistake:
    """Context manager: run the reference with one planted mistake (mutation tests only)."""

    def __init__(self, name: str):
        self.code = MUTATIONS[name]

    def __enter__(self):
        lib = _load()
        lib.oracle_set_mutation.argtypes = [ctypes.c_int]
        lib.oracle_set_mutation.restype = ctypes.c_int
        self.old = lib.oracle_set_mutation(self.code)
        return self

    def __exit__(self, *exc):
        _load().oracle_set_mutation(self.old)
        return False


# ---------------------------------------------------------------- property checks

CHECK_CODES = {-1: "ids not numbered by first vertex", -2: "not a refinement of the previous partition",
               -3: "a block holds two different signatures", -4: "two blocks share one key",
               -5: "bad input"}


def _check():
    global _check_lib
    if _check_lib is not None:
        return _check_lib
    if not os.path.exists(_CHECK_PATH):
        build(force=False)
    lib = ctypes.CDLL(_CHECK_PATH)
    vp = ctypes.c_void_p
    lib.stepcheck_threads.argtypes = [ctypes.c_int]
    lib.stepcheck_threads.restype = ctypes.c_int
    lib.stepcheck_initial.argtypes = [ctypes.c_int64, vp, vp, vp, vp]
    lib.stepcheck_initial.restype = ctypes.c_int64
    lib.stepcheck_step.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, vp]
    lib.stepcheck_step.restype = ctypes.c_int64
    _check_lib = lib
    return lib


def check_threads(threads: int = 0) -> int:
    """Set (threads > 0) and return the number of threads the property checks use."""
    return int(_check().stepcheck_threads(threads))


def _raise(code, bad, what):
    raise AssertionError(f"{what}: {CHECK_CODES.get(code, code)} (vertex {bad})")


def check_initial(g, p0) -> int:
    """Block count of P0 if ``p0`` is the canonical label-set partition, else AssertionError."""
    lib = _check()
    bad = np.zeros(1, dtype=np.int64)
    p0 = _c(p0, np.int32)
    rc = lib.stepcheck_initial(g.n, _p(_c(g.vlabel_ptr, np.int64)), _p(_c(g.vlabel, np.int32)), _p(p0), _p(bad))
    if rc < 0:
        _raise(int(rc), int(bad[0]), "P0")
    return int(rc)


def check_step(g, prev, cur) -> int:
    """Block count of ``cur`` if it is the canonical refinement step of ``prev``, else AssertionError."""
    lib = _check()
    bad = np.zeros(1, dtype=np.int64)
    prev, cur = _c(prev, np.int32), _c(cur, np.int32)
    rc = lib.stepcheck_step(g.n, _p(_c(g.row_ptr, np.int64)), _p(_c(g.col, np.int32)), _p(_c(g.elabel, np.int32)),
                            _p(prev), _p(cur), _p(bad))
    if rc < 0:
        _raise(int(rc), int(bad[0]), "step")
    return int(rc)
