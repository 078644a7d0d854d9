"""Python binding of libkbisim (k-bisimulation partition refinement on MI355X).

Argument marshalling only: every step of the refinement runs in the HIP
kernels of ``libkbisim.so`` behind the C ABI of ``include/kbisim.h``.  PyTorch
provides device memory and the stream.  There is no CPU fallback: importing
the package without the built library raises.

Quick use::

    import paper_2204_05821_amd as kb
    ids, counts = kb.refine(row_ptr, col, elabel=elabel, vlabel=vlabel, k=10)

All tensors are device tensors: row_ptr int64 [n+1], col int32 [m], elabel
int32 [m] or None, vlabel int32 [n] (one label per vertex) or the label-set
form vlabel_ptr int64 [n+1] + vlabel int32 [nlabels], or None for P0 = {V}.
The graph is read as out-edges; transpose it first for backward bisimulation.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkbisim.so")

OK, EINVAL, EGRAPH, ENOSPACE, EHIP, ERANGE, EINTERNAL = 0, -1, -2, -3, -4, -5, -6


class KbisimError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {_lib().kbisim_strerror(code).decode()} ({code})")


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("nlabels", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("elabel", ctypes.c_void_p),
                ("vlabel_ptr", ctypes.c_void_p), ("vlabel", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    """Launch-shape parameters (0 = default); results never depend on them."""
    _fields_ = [("range_edges", ctypes.c_int), ("hub_chunk", ctypes.c_int), ("hub_part_target", ctypes.c_int),
                ("key_bits", ctypes.c_int), ("scan_items", ctypes.c_int), ("reserved", ctypes.c_int * 3)]

    def as_dict(self):
        return {"range_edges": self.range_edges, "hub_chunk": self.hub_chunk,
                "hub_part_target": self.hub_part_target, "key_bits": self.key_bits, "scan_items": self.scan_items}


def tuning(range_edges: int = 0, hub_chunk: int = 0, hub_part_target: int = 0, key_bits: int = 0,
           scan_items: int = 0) -> Tuning:
    return Tuning(range_edges, hub_chunk, hub_part_target, key_bits, scan_items)


_LIB = None


def _lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2204_05821_amd/build.py (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    lib.kbisim_workspace_bytes.argtypes = [ctypes.POINTER(_Graph), i32, ctypes.POINTER(sz)]
    lib.kbisim_create.argtypes = [ctypes.POINTER(_Graph), i32, vp, sz, vp, ctypes.POINTER(vp)]
    lib.kbisim_create_tuned.argtypes = [ctypes.POINTER(_Graph), i32, ctypes.POINTER(Tuning), vp, sz, vp,
                                        ctypes.POINTER(vp)]
    lib.kbisim_use_graphs.argtypes = [vp, i32]
    lib.kbisim_set_stream.argtypes = [vp, vp]
    lib.kbisim_step_async.argtypes = [vp, i32, vp, vp]
    lib.kbisim_step_result.argtypes = [vp, i32, vp, vp, ctypes.POINTER(i64)]
    lib.kbisim_batch_workspace_bytes.argtypes = [ctypes.POINTER(_Graph), i64, i32, ctypes.POINTER(sz)]
    lib.kbisim_batch_create.argtypes = [ctypes.POINTER(_Graph), i64, vp, i32, ctypes.POINTER(Tuning), vp, sz, vp,
                                        ctypes.POINTER(vp)]
    lib.kbisim_batch_refine.argtypes = [vp, i32, ctypes.POINTER(vp), vp]
    lib.kbisim_transpose_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(sz)]
    lib.kbisim_transpose_workspace_bytes.restype = i32
    lib.kbisim_transpose.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.kbisim_transpose.restype = i32
    lib.kbisim_quotient_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    lib.kbisim_quotient_workspace_bytes.restype = i32
    lib.kbisim_quotient.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(i64), vp, sz]
    lib.kbisim_quotient.restype = i32
    lib.kbisim_incr_state_bytes.argtypes = [ctypes.POINTER(_Graph), i32, ctypes.POINTER(sz)]
    lib.kbisim_incr_state_bytes.restype = i32
    lib.kbisim_incr_enable.argtypes = [vp, vp, sz]
    lib.kbisim_incr_enable.restype = i32
    lib.kbisim_incr_update.argtypes = [vp, ctypes.POINTER(_Graph), vp, i64, i32, ctypes.POINTER(vp),
                                       ctypes.POINTER(i64)]
    lib.kbisim_incr_update.restype = i32
    lib.kbisim_gather_probe.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_double)]
    lib.kbisim_gather_probe.restype = i32
    lib.kbisim_work_efficient.argtypes = [vp, i32, ctypes.POINTER(i32)]
    lib.kbisim_work_efficient.restype = i32
    lib.kbisim_profile_select.argtypes = [vp, ctypes.c_uint32]
    lib.kbisim_profile_select.restype = i32
    lib.kbisim_batch_step_async.argtypes = [vp, i32, vp]
    lib.kbisim_batch_step_result.argtypes = [vp, i32, vp, vp]
    lib.kbisim_batch_context.argtypes = [vp, ctypes.POINTER(vp)]
    lib.kbisim_batch_destroy.argtypes = [vp]
    lib.kbisim_initial.argtypes = [vp, vp, ctypes.POINTER(i64)]
    lib.kbisim_refine.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(i64)]
    lib.kbisim_refine_from.argtypes = [vp, vp, i32, ctypes.POINTER(vp), ctypes.POINTER(i64)]
    lib.kbisim_destroy.argtypes = [vp]
    lib.kbisim_profile_enable.argtypes = [vp, i32]
    lib.kbisim_profile_read.argtypes = [vp, vp, vp]
    lib.kbisim_kernel_name.argtypes = [i32]
    lib.kbisim_kernel_name.restype = ctypes.c_char_p
    lib.kbisim_schedule_info.argtypes = [vp, vp]
    lib.kbisim_copy_probe.argtypes = [vp, vp, sz, vp]
    lib.kbisim_strerror.argtypes = [i32]
    lib.kbisim_strerror.restype = ctypes.c_char_p
    lib.kbisim_version.restype = ctypes.c_char_p
    for f in ("kbisim_workspace_bytes", "kbisim_create", "kbisim_initial", "kbisim_refine", "kbisim_refine_from",
              "kbisim_destroy", "kbisim_profile_enable", "kbisim_profile_read", "kbisim_schedule_info",
              "kbisim_copy_probe", "kbisim_create_tuned", "kbisim_use_graphs", "kbisim_batch_workspace_bytes",
              "kbisim_batch_create", "kbisim_batch_refine", "kbisim_batch_context", "kbisim_batch_destroy",
              "kbisim_step_async", "kbisim_step_result", "kbisim_batch_step_async", "kbisim_batch_step_result"):
        getattr(lib, f).restype = i32
    _LIB = lib
    return lib


def version() -> str:
    return _lib().kbisim_version().decode()


NKERNELS = 11


def kernel_names() -> List[str]:
    return [_lib().kbisim_kernel_name(i).decode() for i in range(NKERNELS)]


def copy_probe(dst: torch.Tensor, src: torch.Tensor, stream=None) -> None:
    """Copy src to dst (same byte size, multiple of 16) with the library's streaming copy kernel."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    rc = _lib().kbisim_copy_probe(_ptr(dst), _ptr(src), nbytes, _stream_handle(stream))
    if rc:
        raise KbisimError(rc, "kbisim_copy_probe")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(t: Optional[torch.Tensor], dtype, name: str, device):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} device tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t


def _stream_handle(stream) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(given: Optional[torch.Tensor], nbytes: int, device) -> torch.Tensor:
    """The caller's workspace (a uint8 device tensor of at least nbytes), or a new one."""
    if given is None:
        return torch.empty(nbytes, dtype=torch.uint8, device=device)
    _check(given, torch.uint8, "workspace", device)
    if given.numel() < nbytes:
        raise ValueError(f"workspace holds {given.numel()} bytes, {nbytes} needed")
    return given


class Refiner:
    """A context bound to one graph: P0 and the degree schedule are computed once.

    ``refine(k)`` may then be called repeatedly; each call restarts from P0.
    """

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, elabel: Optional[torch.Tensor] = None,
                 vlabel: Optional[torch.Tensor] = None, vlabel_ptr: Optional[torch.Tensor] = None,
                 kmax: int = 10, stream=None, tuning: Optional[Tuning] = None, graphs: bool = False,
                 workspace: Optional[torch.Tensor] = None):
        lib = _lib()
        self.device = row_ptr.device
        self.row_ptr = _check(row_ptr, torch.int64, "row_ptr", self.device)
        self.col = _check(col, torch.int32, "col", self.device)
        self.elabel = _check(elabel, torch.int32, "elabel", self.device)
        self.vlabel = _check(vlabel, torch.int32, "vlabel", self.device)
        self.vlabel_ptr = _check(vlabel_ptr, torch.int64, "vlabel_ptr", self.device)
        self.n = int(row_ptr.numel()) - 1
        self.m = int(col.numel())
        self.kmax = int(kmax)
        nl = int(vlabel.numel()) if (vlabel is not None and vlabel_ptr is not None) else 0
        self._g = _Graph(self.n, self.m, nl, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.elabel),
                         _ptr(self.vlabel_ptr), _ptr(self.vlabel))
        nbytes = ctypes.c_size_t(0)
        rc = lib.kbisim_workspace_bytes(ctypes.byref(self._g), self.kmax, ctypes.byref(nbytes))
        if rc:
            raise KbisimError(rc, "kbisim_workspace_bytes")
        self.workspace_bytes = int(nbytes.value)
        with torch.cuda.device(self.device):
            self.workspace = _workspace(workspace, self.workspace_bytes, self.device)
            if stream is None:
                # graph capture needs a stream of its own (default priority)
                stream = torch.cuda.Stream(device=self.device) if graphs else torch.cuda.current_stream()
            self.stream = stream
            self.tuning = tuning
            ctx = ctypes.c_void_p(0)
            torch.cuda.current_stream().synchronize()
            rc = lib.kbisim_create_tuned(ctypes.byref(self._g), self.kmax,
                                         ctypes.byref(tuning) if tuning is not None else None,
                                         _ptr(self.workspace), self.workspace_bytes, _stream_handle(self.stream),
                                         ctypes.byref(ctx))
        if rc:
            raise KbisimError(rc, "kbisim_create")
        self._ctx = ctx
        if graphs:
            rc = lib.kbisim_use_graphs(self._ctx, 1)
            if rc:
                raise KbisimError(rc, "kbisim_use_graphs")

    def set_stream(self, stream) -> None:
        """Run later calls on `stream`, after everything enqueued so far on the current one."""
        rc = _lib().kbisim_set_stream(self._ctx, _stream_handle(stream))
        if rc:
            raise KbisimError(rc, "kbisim_set_stream")
        self.stream = stream

    def close(self):
        if getattr(self, "_ctx", None):
            _lib().kbisim_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def initial(self) -> Tuple[torch.Tensor, int]:
        out = torch.empty(self.n, dtype=torch.int32, device=self.device)
        cnt = ctypes.c_int64(0)
        rc = _lib().kbisim_initial(self._ctx, _ptr(out), ctypes.byref(cnt))
        if rc:
            raise KbisimError(rc, "kbisim_initial")
        return out, int(cnt.value)

    def work_efficient(self, enable: Optional[bool] = True) -> int:
        """Turn the work-efficient mode on/off (None: leave it); returns the steps the last call computed."""
        steps = ctypes.c_int(0)
        rc = _lib().kbisim_work_efficient(self._ctx, -1 if enable is None else int(bool(enable)), ctypes.byref(steps))
        if rc:
            raise KbisimError(rc, "kbisim_work_efficient")
        return int(steps.value)

    def incremental(self, state: Optional[torch.Tensor] = None) -> None:
        """Cache the chain of later refine calls (from P0) so that update() can recompute it after edits.

        The state buffer (device uint8, kbisim_incr_state_bytes) is allocated unless given.
        """
        lib = _lib()
        nbytes = ctypes.c_size_t(0)
        rc = lib.kbisim_incr_state_bytes(ctypes.byref(self._g), self.kmax, ctypes.byref(nbytes))
        if rc:
            raise KbisimError(rc, "kbisim_incr_state_bytes")
        with torch.cuda.device(self.device):
            self.incr_state = _workspace(state, int(nbytes.value), self.device)
        rc = lib.kbisim_incr_enable(self._ctx, _ptr(self.incr_state), int(nbytes.value))
        if rc:
            raise KbisimError(rc, "kbisim_incr_enable")

    def update(self, row_ptr: torch.Tensor, col: torch.Tensor, elabel: Optional[torch.Tensor],
               rows: torch.Tensor, k: int, out: Optional[Sequence[torch.Tensor]] = None):
        """P'_1..P'_k of the edited graph (row_ptr, col, elabel: same vertices and vertex labels)
        whose rows differ from the cached graph's only at the vertices in ``rows`` (int32 device
        tensor).  The cached chain (the last refine call) is left as it is."""
        if out is None:
            out = self.alloc_outputs(k)
        row_ptr = _check(row_ptr, torch.int64, "row_ptr", self.device)
        col = _check(col, torch.int32, "col", self.device)
        elabel = _check(elabel, torch.int32, "elabel", self.device)
        rows = _check(rows, torch.int32, "rows", self.device)
        g = _Graph(int(row_ptr.numel()) - 1, int(col.numel()), self._g.nlabels, _ptr(row_ptr), _ptr(col),
                   _ptr(elabel), self._g.vlabel_ptr, self._g.vlabel)
        for t in out[:k]:
            _check(t, torch.int32, "out", self.device)
        ptrs = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in out[:k]])
        counts = (ctypes.c_int64 * max(k, 1))()
        rc = _lib().kbisim_incr_update(self._ctx, ctypes.byref(g), _ptr(rows), int(rows.numel()), k, ptrs, counts)
        if rc:
            raise KbisimError(rc, "kbisim_incr_update")
        return list(out[:k]), [int(counts[i]) for i in range(k)]

    def gather_probe(self, pid: torch.Tensor, reps: int = 5) -> float:
        """Milliseconds of one pass of the bare random gather over all entries (the signature bound)."""
        _check(pid, torch.int32, "pid", self.device)
        ms = ctypes.c_double(0.0)
        rc = _lib().kbisim_gather_probe(self._ctx, _ptr(pid), int(reps), ctypes.byref(ms))
        if rc:
            raise KbisimError(rc, "kbisim_gather_probe")
        return float(ms.value)

    def quotient(self, src_pid: torch.Tensor, dst_pid: torch.Tensor):
        """Summary graph: distinct (source block, label, target block) triples, sorted.

        With src_pid = P_k and dst_pid = P_{k-1} this is the summary graph of the
        k-bisimulation.  Returns three device int32 tensors of equal length.
        """
        _check(src_pid, torch.int32, "src_pid", self.device)
        _check(dst_pid, torch.int32, "dst_pid", self.device)
        lib = _lib()
        nbytes = ctypes.c_size_t(0)
        rc = lib.kbisim_quotient_workspace_bytes(self._ctx, ctypes.byref(nbytes))
        if rc:
            raise KbisimError(rc, "kbisim_quotient_workspace_bytes")
        with torch.cuda.device(self.device):
            ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            cap = max(self.m, 1)
            out = [torch.empty(cap, dtype=torch.int32, device=self.device) for _ in range(3)]
            cnt = ctypes.c_int64(0)
            torch.cuda.current_stream().synchronize()
            rc = lib.kbisim_quotient(self._ctx, _ptr(src_pid), _ptr(dst_pid), _ptr(out[0]), _ptr(out[1]),
                                     _ptr(out[2]), ctypes.byref(cnt), _ptr(ws), int(nbytes.value))
        if rc:
            raise KbisimError(rc, "kbisim_quotient")
        c = int(cnt.value)
        return out[0][:c], out[1][:c], out[2][:c]

    def profile(self, enable: bool = True, kinds: Optional[Sequence[str]] = None) -> None:
        """Start (and reset) or stop per-kernel event timing of later refine calls;
        ``kinds`` limits the timing to these kernel names (default: all)."""
        names = kernel_names()
        mask = 0xFFFFFFFF if kinds is None else sum(1 << names.index(k) for k in kinds)
        rc = _lib().kbisim_profile_select(self._ctx, mask)
        if rc:
            raise KbisimError(rc, "kbisim_profile_select")
        rc = _lib().kbisim_profile_enable(self._ctx, 1 if enable else 0)
        if rc:
            raise KbisimError(rc, "kbisim_profile_enable")

    def profile_read(self):
        """{kernel name: (total ms, launches)} since profile(True)."""
        ms = (ctypes.c_double * NKERNELS)()
        cnt = (ctypes.c_int64 * NKERNELS)()
        rc = _lib().kbisim_profile_read(self._ctx, ms, cnt)
        if rc:
            raise KbisimError(rc, "kbisim_profile_read")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(kernel_names())}

    def schedule_info(self):
        """Vertices and CSR entries per degree tier (range, workgroup, staged hub, global-set hub)."""
        info = (ctypes.c_int64 * 8)()
        rc = _lib().kbisim_schedule_info(self._ctx, info)
        if rc:
            raise KbisimError(rc, "kbisim_schedule_info")
        names = ["range", "workgroup", "hub", "hub_global"]
        return {names[i]: {"vertices": int(info[2 * i]), "entries": int(info[2 * i + 1])} for i in range(4)}

    def alloc_outputs(self, k: int) -> List[torch.Tensor]:
        return [torch.empty(self.n, dtype=torch.int32, device=self.device) for _ in range(k)]

    def step_async(self, i: int, prev: Optional[torch.Tensor], out: torch.Tensor) -> None:
        """Enqueue step i (P_{i+1} from prev, None = P0) without synchronising."""
        rc = _lib().kbisim_step_async(self._ctx, i, _ptr(prev), _ptr(out))
        if rc:
            raise KbisimError(rc, "kbisim_step_async")

    def step_result(self, i: int, prev: Optional[torch.Tensor], out: torch.Tensor) -> int:
        """Finish step i (synchronises the context's stream); the block count of P_{i+1}."""
        cnt = ctypes.c_int64(0)
        rc = _lib().kbisim_step_result(self._ctx, i, _ptr(prev), _ptr(out), ctypes.byref(cnt))
        if rc:
            raise KbisimError(rc, "kbisim_step_result")
        return int(cnt.value)

    def refine(self, k: int, out: Optional[Sequence[torch.Tensor]] = None,
               start: Optional[torch.Tensor] = None) -> Tuple[List[torch.Tensor], List[int]]:
        """P_1..P_k (or P_{i+1}.. from ``start`` = P_i) and their block counts."""
        if out is None:
            out = self.alloc_outputs(k)
        if len(out) < k:
            raise ValueError("need k output tensors")
        for t in out[:k]:
            _check(t, torch.int32, "out", self.device)
            if t.numel() != self.n:
                raise ValueError("output tensors must hold n ids")
        ptrs = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in out[:k]])
        counts = (ctypes.c_int64 * max(k, 1))()
        if start is None:
            rc = _lib().kbisim_refine(self._ctx, k, ptrs, counts)
        else:
            _check(start, torch.int32, "start", self.device)
            rc = _lib().kbisim_refine_from(self._ctx, _ptr(start), k, ptrs, counts)
        if rc:
            raise KbisimError(rc, "kbisim_refine")
        return list(out[:k]), [int(counts[i]) for i in range(k)]


def refine(row_ptr, col, elabel=None, vlabel=None, vlabel_ptr=None, k: int = 10):
    """One-shot: partitions P_1..P_k and their block counts."""
    r = Refiner(row_ptr, col, elabel, vlabel, vlabel_ptr, kmax=max(k, 1))
    try:
        return r.refine(k)
    finally:
        r.close()


def to_device(g, device="cuda"):
    """Device tensors (row_ptr, col, elabel, vlabel, vlabel_ptr) of a host graph with numpy arrays."""
    def t(a):
        return None if a is None else torch.from_numpy(a).to(device)
    return t(g.row_ptr), t(g.col), t(g.elabel), t(g.vlabel), t(g.vlabel_ptr)


def transpose(row_ptr: torch.Tensor, col: torch.Tensor, elabel: Optional[torch.Tensor] = None,
              stream=None) -> Tuple[torch.Tensor, torch.Tensor, Optional[torch.Tensor]]:
    """Transposed CSR on the device (backward refinement = forward refinement of the transpose).

    Returns (row_ptr, col, elabel) device tensors; elabel is None when the input has none.
    """
    lib = _lib()
    dev = row_ptr.device
    row_ptr = _check(row_ptr, torch.int64, "row_ptr", dev)
    col = _check(col, torch.int32, "col", dev)
    elabel = _check(elabel, torch.int32, "elabel", dev)
    n, m = int(row_ptr.numel()) - 1, int(col.numel())
    nbytes = ctypes.c_size_t(0)
    rc = lib.kbisim_transpose_workspace_bytes(n, m, ctypes.byref(nbytes))
    if rc:
        raise KbisimError(rc, "kbisim_transpose_workspace_bytes")
    with torch.cuda.device(dev):
        ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=dev)
        out_rp = torch.empty(n + 1, dtype=torch.int64, device=dev)
        out_col = torch.empty(max(m, 0), dtype=torch.int32, device=dev)
        out_el = torch.empty(max(m, 0), dtype=torch.int32, device=dev) if elabel is not None else None
        torch.cuda.current_stream().synchronize()
        rc = lib.kbisim_transpose(n, m, _ptr(row_ptr), _ptr(col), _ptr(elabel), _ptr(out_rp), _ptr(out_col),
                                  _ptr(out_el), _ptr(ws), int(nbytes.value), _stream_handle(stream))
    if rc:
        raise KbisimError(rc, "kbisim_transpose")
    return out_rp, out_col, out_el


def refiner_for(g, kmax: int = 10, device="cuda") -> Refiner:
    rp, col, el, vl, vp = to_device(g, device)
    return Refiner(rp, col, el, vl, vp, kmax=kmax)


class Batch:
    """Many independent graphs refined by the same launches (their disjoint union).

    ``refine(k)`` returns the k packed id arrays (per-graph ids, union vertex
    order) and counts as a list of lists ``counts[g][i]``.
    """

    def __init__(self, row_ptr, col, elabel, vlabel, vlabel_ptr, vert_off, kmax: int = 10, stream=None,
                 tuning: Optional[Tuning] = None, graphs: bool = False, workspace: Optional[torch.Tensor] = None):
        import numpy as np
        lib = _lib()
        self.device = row_ptr.device
        self.row_ptr = _check(row_ptr, torch.int64, "row_ptr", self.device)
        self.col = _check(col, torch.int32, "col", self.device)
        self.elabel = _check(elabel, torch.int32, "elabel", self.device)
        self.vlabel = _check(vlabel, torch.int32, "vlabel", self.device)
        self.vlabel_ptr = _check(vlabel_ptr, torch.int64, "vlabel_ptr", self.device)
        self.vert_off = np.ascontiguousarray(vert_off, dtype=np.int64)
        self.num_graphs = len(self.vert_off) - 1
        self.n = int(row_ptr.numel()) - 1
        self.m = int(col.numel())
        self.kmax = int(kmax)
        nl = int(vlabel.numel()) if (vlabel is not None and vlabel_ptr is not None) else 0
        self._g = _Graph(self.n, self.m, nl, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.elabel),
                         _ptr(self.vlabel_ptr), _ptr(self.vlabel))
        nbytes = ctypes.c_size_t(0)
        rc = lib.kbisim_batch_workspace_bytes(ctypes.byref(self._g), self.num_graphs, self.kmax, ctypes.byref(nbytes))
        if rc:
            raise KbisimError(rc, "kbisim_batch_workspace_bytes")
        self.workspace_bytes = int(nbytes.value)
        with torch.cuda.device(self.device):
            self.workspace = _workspace(workspace, self.workspace_bytes, self.device)
            if stream is None:
                stream = torch.cuda.Stream(device=self.device) if graphs else torch.cuda.current_stream()
            self.stream = stream
            torch.cuda.current_stream().synchronize()
            b = ctypes.c_void_p(0)
            rc = lib.kbisim_batch_create(ctypes.byref(self._g), self.num_graphs,
                                         ctypes.c_void_p(self.vert_off.ctypes.data), self.kmax,
                                         ctypes.byref(tuning) if tuning is not None else None,
                                         _ptr(self.workspace), self.workspace_bytes, _stream_handle(self.stream),
                                         ctypes.byref(b))
        if rc:
            raise KbisimError(rc, "kbisim_batch_create")
        self._b = b
        ctx = ctypes.c_void_p(0)
        lib.kbisim_batch_context(self._b, ctypes.byref(ctx))
        self._ctx = ctx
        if graphs:
            rc = lib.kbisim_use_graphs(self._ctx, 1)
            if rc:
                raise KbisimError(rc, "kbisim_use_graphs")

    def set_stream(self, stream) -> None:
        """Run later calls on `stream`, after everything enqueued so far on the current one."""
        rc = _lib().kbisim_set_stream(self._ctx, _stream_handle(stream))
        if rc:
            raise KbisimError(rc, "kbisim_set_stream")
        self.stream = stream

    def close(self):
        if getattr(self, "_b", None):
            _lib().kbisim_batch_destroy(self._b)
            self._b = None
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc_outputs(self, k: int) -> List[torch.Tensor]:
        return [torch.empty(self.n, dtype=torch.int32, device=self.device) for _ in range(k)]

    def refine(self, k: int, out: Optional[Sequence[torch.Tensor]] = None):
        if out is None:
            out = self.alloc_outputs(k)
        for t in out[:k]:
            _check(t, torch.int32, "out", self.device)
            if t.numel() != self.n:
                raise ValueError("output tensors must hold n ids")
        ptrs = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in out[:k]])
        counts = (ctypes.c_int64 * max(self.num_graphs * k, 1))()
        rc = _lib().kbisim_batch_refine(self._b, k, ptrs, counts)
        if rc:
            raise KbisimError(rc, "kbisim_batch_refine")
        cl = [[int(counts[g * k + i]) for i in range(k)] for g in range(self.num_graphs)]
        return list(out[:k]), cl

    def work_efficient(self, enable: Optional[bool] = True) -> int:
        """Turn the work-efficient mode on/off (None: leave it); returns the steps the last call computed."""
        steps = ctypes.c_int(0)
        rc = _lib().kbisim_work_efficient(self._ctx, -1 if enable is None else int(bool(enable)), ctypes.byref(steps))
        if rc:
            raise KbisimError(rc, "kbisim_work_efficient")
        return int(steps.value)

    def step_async(self, i: int, out: torch.Tensor) -> None:
        """Enqueue step i (per-graph ids of P_{i+1} into out) without synchronising."""
        rc = _lib().kbisim_batch_step_async(self._b, i, _ptr(out))
        if rc:
            raise KbisimError(rc, "kbisim_batch_step_async")

    def step_result(self, i: int, out: torch.Tensor) -> List[int]:
        """Finish step i; per-graph block counts of P_{i+1}."""
        counts = (ctypes.c_int64 * max(self.num_graphs, 1))()
        rc = _lib().kbisim_batch_step_result(self._b, i, _ptr(out), counts)
        if rc:
            raise KbisimError(rc, "kbisim_batch_step_result")
        return [int(counts[g]) for g in range(self.num_graphs)]

    def profile(self, enable: bool = True) -> None:
        rc = _lib().kbisim_profile_enable(self._ctx, 1 if enable else 0)
        if rc:
            raise KbisimError(rc, "kbisim_profile_enable")

    def profile_read(self):
        ms = (ctypes.c_double * NKERNELS)()
        cnt = (ctypes.c_int64 * NKERNELS)()
        rc = _lib().kbisim_profile_read(self._ctx, ms, cnt)
        if rc:
            raise KbisimError(rc, "kbisim_profile_read")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(kernel_names())}


def union_of(graphs):
    """Disjoint union of host graphs (numpy CSR): global column ids and vertex offsets.

    Returns (row_ptr, col, elabel, vlabel, vlabel_ptr, vert_off) as numpy arrays.
    All graphs must use the same label form (edge labels or none; one label per
    vertex, label sets, or none).
    """
    import numpy as np
    vert_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vert_off[i + 1] = vert_off[i] + g.n
    edge_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        edge_off[i + 1] = edge_off[i] + g.m
    row_ptr = np.concatenate([g.row_ptr[:-1] + edge_off[i] for i, g in enumerate(graphs)] + [edge_off[-1:]])
    col = np.concatenate([g.col + np.int32(vert_off[i]) for i, g in enumerate(graphs)]).astype(np.int32)
    # A graph without edge labels is the same as one whose edges all carry
    # label 0; a graph without vertex labels is the same as one whose
    # vertices all carry one label (or all the empty set): P0 = {V} either way.
    if any(g.elabel is not None for g in graphs):
        elabel = np.concatenate([g.elabel if g.elabel is not None else np.zeros(g.m, dtype=np.int32)
                                 for g in graphs]).astype(np.int32)
    else:
        elabel = None
    kinds = {("sets" if g.vlabel_ptr is not None else ("one" if g.vlabel is not None else "none")) for g in graphs}
    vlabel = vlabel_ptr = None
    if "sets" in kinds:
        ptrs, labs, base = [], [], 0
        for g in graphs:
            if g.vlabel_ptr is not None:
                p, l = g.vlabel_ptr, g.vlabel
            elif g.vlabel is not None:
                p, l = np.arange(g.n + 1, dtype=np.int64), g.vlabel
            else:
                p, l = np.zeros(g.n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32)
            ptrs.append(p[:-1] + base)
            labs.append(np.asarray(l, dtype=np.int32))
            base += int(p[-1])
        vlabel_ptr = np.concatenate(ptrs + [np.array([base], dtype=np.int64)])
        vlabel = np.concatenate(labs).astype(np.int32)
    elif "one" in kinds:
        vlabel = np.concatenate([g.vlabel if g.vlabel is not None else np.zeros(g.n, dtype=np.int32)
                                 for g in graphs]).astype(np.int32)
    return (row_ptr.astype(np.int64), col, elabel, vlabel,
            None if vlabel_ptr is None else vlabel_ptr.astype(np.int64), vert_off)


def batch_for(graphs, kmax: int = 10, device="cuda", tuning: Optional[Tuning] = None, graphs_mode: bool = False):
    rp, col, el, vl, vp, off = union_of(graphs)

    def t(a):
        return None if a is None else torch.from_numpy(a).to(device)
    return Batch(t(rp), t(col), t(el), t(vl), t(vp), off, kmax=kmax, tuning=tuning, graphs=graphs_mode)
