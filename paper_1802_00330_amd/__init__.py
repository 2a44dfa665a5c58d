"""Python binding of the MI355X interval branch-and-bound library (libibb.so).

Argument marshalling only: every step of the search runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream for ``solve``; the
names ``ibb_*`` mirror the C entry points of ``include/ibb.h``.

There is no fallback: if ``libibb.so`` has not been built, or no GPU is
visible, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# IBB_LIBRARY may name another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("IBB_LIBRARY") or os.path.join(_HERE, "libibb.so")

OK = 0
SCHEDULE_QUEUE, SCHEDULE_LEVELS, SCHEDULE_AUTO = 0, 1, 2
ERR_INVALID_ARG, ERR_BUDGET, ERR_OUTPUT_CAPACITY, ERR_QUEUE_OVERFLOW = -1, -2, -3, -4
ERR_NO_MEMORY, ERR_DEVICE, ERR_UNSUPPORTED, ERR_TIMEOUT = -5, -6, -7, -8
ERR_WORKSPACE_LIMIT = -9
NOALLOC_WORKSPACE_BYTES = 64 << 20
SPLIT_WIDEST, SPLIT_ALL = 0, 1
CONTRACT_HS, CONTRACT_KRAWCZYK = 0, 1
INCLUDE_NATURAL, INCLUDE_MEAN_VALUE = 0, 1
UNDECIDED, UNIQUE = 0, 1
MAX_N = 16

STATS_FIELDS = ("processed", "excluded_eval", "excluded_hs", "hs_skipped", "recontracted",
                "bisected", "emitted_unique", "emitted_undecided")

EXPORTS = ("ibb_ctx_create", "ibb_ctx_destroy", "ibb_strerror", "ibb_params_default", "ibb_solve",
           "ibb_workspace_size", "ibb_solve_async", "ibb_last_level_sizes", "ibb_last_kernel_ms",
           "ibb_selftest_ops", "ibb_debug_step", "ibb_solve_batch", "ibb_server_config_default",
           "ibb_server_create", "ibb_server_destroy", "ibb_server_submit", "ibb_server_step", "ibb_server_poll",
           "ibb_server_cancel", "ibb_server_pending", "ibb_round", "ibb_batch_plan_create", "ibb_batch_plan_run",
           "ibb_batch_plan_destroy", "ibb_batch_get_config", "ibb_batch_set_config", "ibb_batch_tune",
           "ibb_solve_noalloc", "ibb_server_finished", "ibb_backtrack", "ibb_batch_set_memory")


class IbbSystem(C.Structure):
    _fields_ = [("n", C.c_int32), ("term_off", C.c_void_p), ("expo", C.c_void_p), ("coef", C.c_void_p)]


class IbbParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_boxes", C.c_int64), ("split_mode", C.c_int32),
                ("max_recontract", C.c_int32), ("recontract_ratio", C.c_double),
                ("hs_max_width", C.c_double), ("schedule", C.c_int32), ("contractor", C.c_int32),
                ("inclusion", C.c_int32), ("reserved", C.c_int32)]


class IbbServerConfig(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("frontier_cap", C.c_int64), ("reserve_per_solve", C.c_int64),
                ("levels_per_quantum", C.c_int32), ("out_cap_per_solve", C.c_int32), ("pool_bytes", C.c_int64)]


class IbbBatchConfig(C.Structure):
    """Launch configuration of one lane-count class of batch members (ibb_batch_config)."""
    _fields_ = [("lanes", C.c_int32), ("tiles_per_claim", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("tuned", C.c_int32), ("ms", C.c_double), ("front_per_member", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class IbbStats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in STATS_FIELDS] + [("levels", C.c_int64), ("max_frontier", C.c_int64),
                                                        ("kernel_ms", C.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libibb.so and declare the C signatures (raises if missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_1802_00330_amd/build.py (hipcc, gfx950)")
    # PyTorch bundles its own HIP runtime and loads it under a name that does
    # not match an already loaded system copy.  Importing torch first makes the
    # library bind to torch's runtime, so one HIP runtime serves both.
    import torch  # noqa: F401
    L = C.CDLL(path)
    p, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.ibb_ctx_create.restype, L.ibb_ctx_create.argtypes = C.c_int, [C.c_int, C.POINTER(C.c_void_p)]
    L.ibb_ctx_destroy.restype, L.ibb_ctx_destroy.argtypes = None, [p]
    L.ibb_strerror.restype, L.ibb_strerror.argtypes = C.c_char_p, [C.c_int]
    L.ibb_params_default.restype, L.ibb_params_default.argtypes = None, [C.POINTER(IbbParams)]
    L.ibb_solve.restype = C.c_int
    L.ibb_solve.argtypes = [p, C.POINTER(IbbSystem), p, p, C.POINTER(IbbParams), p, p, p, i64,
                            C.POINTER(C.c_int64), C.POINTER(IbbStats)]
    L.ibb_workspace_size.restype, L.ibb_workspace_size.argtypes = C.c_size_t, [i32, i64, i64]
    L.ibb_solve_async.restype = C.c_int
    L.ibb_solve_async.argtypes = [p, C.POINTER(IbbSystem), p, p, C.POINTER(IbbParams), p, C.c_size_t, i64, i64,
                                  p, p, p, p, p]
    L.ibb_solve_noalloc.restype = C.c_int
    L.ibb_solve_noalloc.argtypes = [p, C.POINTER(IbbSystem), p, p, C.POINTER(IbbParams), i64, i64, p, p, p, p, p]
    L.ibb_last_level_sizes.restype, L.ibb_last_level_sizes.argtypes = i64, [p, p, i64]
    L.ibb_selftest_ops.restype, L.ibb_selftest_ops.argtypes = C.c_int, [p, i32, i64, p, p, p]
    L.ibb_last_kernel_ms.restype, L.ibb_last_kernel_ms.argtypes = C.c_double, [p]
    L.ibb_solve_batch.restype = C.c_int
    L.ibb_solve_batch.argtypes = [p, i32, p, p, p, p, p, p, p, i64, p, p, p]
    L.ibb_server_config_default.restype = None
    L.ibb_server_config_default.argtypes = [C.POINTER(IbbServerConfig)]
    L.ibb_server_create.restype = C.c_int
    L.ibb_server_create.argtypes = [p, C.POINTER(IbbServerConfig), C.POINTER(C.c_void_p)]
    L.ibb_server_destroy.restype, L.ibb_server_destroy.argtypes = None, [p]
    L.ibb_server_submit.restype = i64
    L.ibb_server_submit.argtypes = [p, C.POINTER(IbbSystem), p, p, C.POINTER(IbbParams)]
    L.ibb_server_step.restype, L.ibb_server_step.argtypes = C.c_int, [p]
    L.ibb_server_poll.restype = C.c_int
    L.ibb_server_poll.argtypes = [p, i64, p, p, p, i64, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                  C.POINTER(IbbStats)]
    L.ibb_server_cancel.restype, L.ibb_server_cancel.argtypes = C.c_int, [p, i64]
    L.ibb_server_finished.restype, L.ibb_server_finished.argtypes = i64, [p, p, i64]
    L.ibb_backtrack.restype = C.c_int
    L.ibb_backtrack.argtypes = [i32, p, p, i64, p, p, i32, p, i32, p, i64, C.POINTER(C.c_int64)]
    L.ibb_server_pending.restype = C.c_int
    L.ibb_server_pending.argtypes = [p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.ibb_debug_step.restype = C.c_int
    L.ibb_debug_step.argtypes = [p, C.POINTER(IbbSystem), p, p, C.POINTER(IbbParams), p, i64]
    L.ibb_batch_plan_create.restype = C.c_int
    L.ibb_batch_plan_create.argtypes = [p, i32, p, p, p, p, C.POINTER(C.c_void_p)]
    L.ibb_batch_plan_run.restype = C.c_int
    L.ibb_batch_plan_run.argtypes = [p, p, p, p, i64, p, p, p]
    L.ibb_batch_plan_destroy.restype, L.ibb_batch_plan_destroy.argtypes = None, [p]
    L.ibb_batch_get_config.restype = C.c_int
    L.ibb_batch_get_config.argtypes = [p, i32, C.POINTER(IbbBatchConfig)]
    L.ibb_batch_set_config.restype = C.c_int
    L.ibb_batch_set_config.argtypes = [p, i32, C.POINTER(IbbBatchConfig)]
    L.ibb_batch_tune.restype, L.ibb_batch_tune.argtypes = C.c_int, [p, i32, p, p, p, p, i32]
    L.ibb_batch_set_memory.restype, L.ibb_batch_set_memory.argtypes = C.c_int, [p, i64]
    L.ibb_round.restype = C.c_int
    L.ibb_round.argtypes = [p, C.POINTER(IbbSystem), C.POINTER(IbbParams), i64, p, p, p, p, p, p, i64,
                            C.POINTER(C.c_int64), p, p, p, i64, C.POINTER(C.c_int64), C.POINTER(IbbStats)]
    _lib = L
    return L


def ibb_strerror(status: int) -> str:
    return load_library().ibb_strerror(int(status)).decode()


class Context:
    """An ibb_ctx on one HIP device."""

    def __init__(self, device: int = 0):
        L = load_library()
        h = C.c_void_p()
        st = L.ibb_ctx_create(int(device), C.byref(h))
        if st != OK:
            raise RuntimeError(f"ibb_ctx_create({device}) failed: {ibb_strerror(st)}")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            load_library().ibb_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ibb_ctx_create(device: int = 0) -> Context:
    return Context(device)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class _SysRef:
    """Keeps the numpy arrays of a system alive for the duration of a call."""

    def __init__(self, s):
        self.term_off = np.ascontiguousarray(s.term_off, dtype=np.int32)
        self.expo = np.ascontiguousarray(s.expo, dtype=np.uint8)
        self.coef = np.ascontiguousarray(s.coef, dtype=np.float64)
        self.c = IbbSystem(int(s.n), self.term_off.ctypes.data, self.expo.ctypes.data, self.coef.ctypes.data)


def make_params(tol: float, max_boxes: int = 100_000_000, split_mode: int = SPLIT_WIDEST,
                max_recontract: int = 16, recontract_ratio: float = 0.5,
                hs_max_width: float = float("inf"), schedule: int = 2, contractor: int = CONTRACT_HS,
                inclusion: int = INCLUDE_NATURAL) -> IbbParams:
    return IbbParams(float(tol), int(max_boxes), int(split_mode), int(max_recontract),
                     float(recontract_ratio), float(hs_max_width), int(schedule), int(contractor), int(inclusion), 0)


@dataclass
class Result:
    status: int
    lo: np.ndarray   # [m, n]
    hi: np.ndarray   # [m, n]
    tag: np.ndarray  # [m] uint8
    stats: dict
    levels: int = 0
    max_frontier: int = 0
    kernel_ms: float = 0.0


def ibb_solve(ctx: Context, s, params: IbbParams, lo=None, hi=None, cap: int = 1 << 14) -> Result:
    """Host-pointer entry point (the library allocates device memory)."""
    L = load_library()
    ref = _SysRef(s)
    lo = np.ascontiguousarray(s.lo if lo is None else lo, dtype=np.float64)
    hi = np.ascontiguousarray(s.hi if hi is None else hi, dtype=np.float64)
    while True:
        olo = np.zeros((cap, s.n))
        ohi = np.zeros((cap, s.n))
        otag = np.zeros(cap, dtype=np.uint8)
        nout = C.c_int64(0)
        st_ = IbbStats()
        st = L.ibb_solve(ctx.handle, C.byref(ref.c), _ptr(lo), _ptr(hi), C.byref(params), _ptr(olo), _ptr(ohi),
                         _ptr(otag), int(cap), C.byref(nout), C.byref(st_))
        if st == ERR_OUTPUT_CAPACITY and nout.value > cap:
            cap = int(nout.value)
            continue
        m = int(nout.value) if st == OK else 0
        stats = {f: int(getattr(st_, f)) for f in STATS_FIELDS}
        return Result(st, olo[:m].copy(), ohi[:m].copy(), otag[:m].copy(), stats, int(st_.levels),
                      int(st_.max_frontier), float(st_.kernel_ms))


def ibb_last_level_sizes(ctx: Context, cap: int = 1 << 16) -> np.ndarray:
    buf = np.zeros(cap, dtype=np.int64)
    m = load_library().ibb_last_level_sizes(ctx.handle, _ptr(buf), int(cap))
    return buf[:min(m, cap)].copy()


def ibb_last_kernel_ms(ctx: Context) -> float:
    return float(load_library().ibb_last_kernel_ms(ctx.handle))


def ibb_workspace_size(n: int, frontier_cap: int, out_cap: int) -> int:
    return int(load_library().ibb_workspace_size(int(n), int(frontier_cap), int(out_cap)))


def ibb_solve_async(ctx: Context, s, params: IbbParams, ws, frontier_cap: int, out_cap: int,
                    out_lo, out_hi, out_tag, info, stream=None, lo=None, hi=None) -> int:
    """Device-pointer entry point: ws/out_*/info are torch CUDA tensors (or
    integer device addresses); the solve is enqueued on `stream`."""
    import torch

    def addr(t):
        return t.data_ptr() if isinstance(t, torch.Tensor) else int(t)

    ref = _SysRef(s)
    lo = np.ascontiguousarray(s.lo if lo is None else lo, dtype=np.float64)
    hi = np.ascontiguousarray(s.hi if hi is None else hi, dtype=np.float64)
    if stream is None:
        stream = torch.cuda.current_stream()
    sh = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    nbytes = ws.numel() * ws.element_size() if isinstance(ws, torch.Tensor) else ibb_workspace_size(
        s.n, frontier_cap, out_cap)
    return load_library().ibb_solve_async(ctx.handle, C.byref(ref.c), _ptr(lo), _ptr(hi), C.byref(params),
                                          C.c_void_p(addr(ws)), C.c_size_t(nbytes), int(frontier_cap),
                                          int(out_cap), C.c_void_p(addr(out_lo)), C.c_void_p(addr(out_hi)),
                                          C.c_void_p(addr(out_tag)), C.c_void_p(addr(info)),
                                          C.c_void_p(sh))


def ibb_solve_noalloc(ctx: Context, s, params: IbbParams, frontier_cap: int, out_cap: int,
                      out_lo, out_hi, out_tag, info, stream=None, lo=None, hi=None) -> int:
    """ibb_solve_async on the library's own per-device workspace array (no
    device allocation): out_*/info are torch CUDA tensors or device addresses."""
    import torch

    def addr(t):
        return t.data_ptr() if isinstance(t, torch.Tensor) else int(t)

    ref = _SysRef(s)
    lo = np.ascontiguousarray(s.lo if lo is None else lo, dtype=np.float64)
    hi = np.ascontiguousarray(s.hi if hi is None else hi, dtype=np.float64)
    if stream is None:
        stream = torch.cuda.current_stream()
    sh = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    return load_library().ibb_solve_noalloc(ctx.handle, C.byref(ref.c), _ptr(lo), _ptr(hi), C.byref(params),
                                            int(frontier_cap), int(out_cap), C.c_void_p(addr(out_lo)),
                                            C.c_void_p(addr(out_hi)), C.c_void_p(addr(out_tag)),
                                            C.c_void_p(addr(info)), C.c_void_p(sh))


def solve(ctx: Context, s, tol: Optional[float] = None, frontier_cap: int = 1 << 20, out_cap: int = 1 << 12,
          device: str = "cuda", stream=None, **kw) -> Result:
    """Solve one system with torch-allocated device memory on a torch stream;
    grows the frontier / output buffers and retries on capacity errors."""
    import torch

    lo = kw.pop("lo", None)
    hi = kw.pop("hi", None)
    params = make_params(s.tol if tol is None else tol, **kw)
    while True:
        nbytes = ibb_workspace_size(s.n, frontier_cap, out_cap)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        olo = torch.empty(max(out_cap, 1) * s.n, dtype=torch.float64, device=device)
        ohi = torch.empty_like(olo)
        otag = torch.empty(max(out_cap, 1), dtype=torch.uint8, device=device)
        info = torch.zeros(16, dtype=torch.int64, device=device)
        st = ibb_solve_async(ctx, s, params, ws, frontier_cap, out_cap, olo, ohi, otag, info, stream=stream,
                             lo=lo, hi=hi)
        if st != OK:
            return Result(st, np.zeros((0, s.n)), np.zeros((0, s.n)), np.zeros(0, np.uint8), {})
        (stream or torch.cuda.current_stream()).synchronize()
        inf = info.cpu().numpy()
        status = int(inf[0])
        if status == ERR_QUEUE_OVERFLOW:
            frontier_cap *= 4
            continue
        if status == ERR_OUTPUT_CAPACITY:
            out_cap = int(inf[1])
            continue
        stats = dict(zip(STATS_FIELDS, (int(v) for v in inf[2:10])))
        m = int(inf[1]) if status == OK else 0
        lo = olo[: m * s.n].view(m, s.n).cpu().numpy() if m else np.zeros((0, s.n))
        hi = ohi[: m * s.n].view(m, s.n).cpu().numpy() if m else np.zeros((0, s.n))
        tag = otag[:m].cpu().numpy() if m else np.zeros(0, np.uint8)
        return Result(status, lo, hi, tag, stats, int(inf[10]), int(inf[11]))


def ibb_selftest_ops(ctx: Context, op: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    out = np.zeros_like(a)
    st = load_library().ibb_selftest_ops(ctx.handle, int(op), int(a.size), _ptr(a), _ptr(b), _ptr(out))
    if st != OK:
        raise RuntimeError(f"ibb_selftest_ops: {ibb_strerror(st)}")
    return out


def dbg_len(n: int) -> int:
    return 6 * n * n + 8 * n + 4


def ibb_debug_step(ctx: Context, s, lo, hi, params: Optional[IbbParams] = None) -> np.ndarray:
    """Intermediates of the device step on one box (see include/ibb.h)."""
    ref = _SysRef(s)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    params = params or make_params(s.tol)
    dump = np.zeros(dbg_len(s.n))
    st = load_library().ibb_debug_step(ctx.handle, C.byref(ref.c), _ptr(lo), _ptr(hi), C.byref(params),
                                       _ptr(dump), int(dump.size))
    if st != OK:
        raise RuntimeError(f"ibb_debug_step: {ibb_strerror(st)}")
    return dump


def ibb_backtrack(lo, hi, x0_lo, x0_hi, level: int, out_level: Optional[int] = None):
    """Backtracking merge (Alg. 5) of boxes lo/hi [m, n] inside the initial box
    x0: returns (counts [level + 1], cells of round out_level [c, n] int64)."""
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    x0_lo = np.ascontiguousarray(x0_lo, dtype=np.float64)
    x0_hi = np.ascontiguousarray(x0_hi, dtype=np.float64)
    n = int(x0_lo.size)
    m = int(lo.size // n) if n else 0
    out_level = level if out_level is None else out_level
    counts = np.zeros(level + 1, dtype=np.int64)
    cap = 1024
    while True:
        cells = np.zeros((cap, n), dtype=np.int64)
        nout = C.c_int64(0)
        st = load_library().ibb_backtrack(n, _ptr(x0_lo), _ptr(x0_hi), m, _ptr(lo), _ptr(hi), int(level),
                                          _ptr(counts), int(out_level), _ptr(cells), int(cap), C.byref(nout))
        if st == ERR_OUTPUT_CAPACITY:
            cap = int(nout.value)
            continue
        if st != OK:
            raise RuntimeError(f"ibb_backtrack: {ibb_strerror(st)}")
        return counts.copy(), cells[: int(nout.value)].copy()


@dataclass
class Round:
    child_lo: np.ndarray   # [c, n]
    child_hi: np.ndarray
    child_rec: np.ndarray  # [c] uint32: bit 0 proven, bits 8-15 recontraction count
    emit_lo: np.ndarray    # [e, n]
    emit_hi: np.ndarray
    emit_tag: np.ndarray   # [e] uint8
    stats: dict


def ibb_round(ctx: Context, s, lo, hi, rec=None, params: Optional[IbbParams] = None) -> Round:
    """One round of the search on the boxes lo[b], hi[b] (see include/ibb.h);
    children and emitted boxes in unspecified order."""
    ref = _SysRef(s)
    lo = np.ascontiguousarray(np.asarray(lo, dtype=np.float64).reshape(-1, s.n))
    hi = np.ascontiguousarray(np.asarray(hi, dtype=np.float64).reshape(-1, s.n))
    m = lo.shape[0]
    rec = np.zeros(m, dtype=np.uint32) if rec is None else np.ascontiguousarray(rec, dtype=np.uint32)
    params = params or make_params(s.tol)
    ccap, ecap = max(4 * m, 16), max(m, 16)
    L = load_library()
    while True:
        clo, chi = np.zeros((ccap, s.n)), np.zeros((ccap, s.n))
        crec = np.zeros(ccap, dtype=np.uint32)
        elo, ehi = np.zeros((ecap, s.n)), np.zeros((ecap, s.n))
        etag = np.zeros(ecap, dtype=np.uint8)
        nc, ne = C.c_int64(0), C.c_int64(0)
        st_ = IbbStats()
        st = L.ibb_round(ctx.handle, C.byref(ref.c), C.byref(params), m, _ptr(lo), _ptr(hi), _ptr(rec), _ptr(clo),
                         _ptr(chi), _ptr(crec), ccap, C.byref(nc), _ptr(elo), _ptr(ehi), _ptr(etag), ecap,
                         C.byref(ne), C.byref(st_))
        if st == ERR_OUTPUT_CAPACITY:
            ccap, ecap = max(ccap, int(nc.value)), max(ecap, int(ne.value))
            continue
        if st != OK:
            raise RuntimeError(f"ibb_round: {ibb_strerror(st)}")
        c, e = int(nc.value), int(ne.value)
        return Round(clo[:c].copy(), chi[:c].copy(), crec[:c].copy(), elo[:e].copy(), ehi[:e].copy(),
                     etag[:e].copy(), {f: int(getattr(st_, f)) for f in STATS_FIELDS})


def _batch_inputs(systems, params):
    B = len(systems)
    refs = [_SysRef(s) for s in systems]
    arr = (IbbSystem * B)(*[r.c for r in refs])
    lo = np.zeros((B, MAX_N))
    hi = np.zeros((B, MAX_N))
    for b, s in enumerate(systems):
        lo[b, :s.n] = s.lo
        hi[b, :s.n] = s.hi
    if params is None:
        params = [make_params(s.tol) for s in systems]
    parr = (IbbParams * B)(*params)
    return refs, arr, lo, hi, parr


def _batch_results(call, systems, cap, name):
    B = len(systems)
    while True:
        olo = np.zeros((max(cap, 1), MAX_N))
        ohi = np.zeros((max(cap, 1), MAX_N))
        otag = np.zeros(max(cap, 1), dtype=np.uint8)
        off = np.zeros(B + 1, dtype=np.int64)
        status = np.zeros(B, dtype=np.int32)
        stats = (IbbStats * B)()
        st = call(_ptr(olo), _ptr(ohi), _ptr(otag), int(cap), _ptr(off), _ptr(status), stats)
        if st == ERR_OUTPUT_CAPACITY:
            cap = int(off[-1])
            continue
        if st != OK:
            raise RuntimeError(f"{name}: {ibb_strerror(st)}")
        out = []
        for b, s in enumerate(systems):
            a, e = int(off[b]), int(off[b + 1])
            sd = {f: int(getattr(stats[b], f)) for f in STATS_FIELDS}
            out.append(Result(int(status[b]), olo[a:e, :s.n].copy(), ohi[a:e, :s.n].copy(), otag[a:e].copy(), sd))
        return out


def ibb_solve_batch(ctx: Context, systems, params=None, cap: int = 1 << 16):
    """Solve many systems in one pass; returns a list of Result (one per system)."""
    L = load_library()
    refs, arr, lo, hi, parr = _batch_inputs(systems, params)

    def call(*outs):
        return L.ibb_solve_batch(ctx.handle, int(len(systems)), arr, _ptr(lo), _ptr(hi), parr, *outs)

    return _batch_results(call, systems, cap, "ibb_solve_batch")


def ibb_batch_get_config(ctx: Context, cls: int) -> IbbBatchConfig:
    """The context's launch configuration of lane-count class cls (0..3)."""
    c = IbbBatchConfig()
    st = load_library().ibb_batch_get_config(ctx.handle, int(cls), C.byref(c))
    if st != OK:
        raise RuntimeError(f"ibb_batch_get_config: {ibb_strerror(st)}")
    return c


def ibb_batch_set_config(ctx: Context, cls: int, lanes: int, tiles_per_claim: int = 1, blocks_per_cu: int = 0):
    """Force the launch configuration of lane-count class cls."""
    c = IbbBatchConfig(int(lanes), int(tiles_per_claim), int(blocks_per_cu), 0, 0.0)
    st = load_library().ibb_batch_set_config(ctx.handle, int(cls), C.byref(c))
    if st != OK:
        raise RuntimeError(f"ibb_batch_set_config: {ibb_strerror(st)}")


def ibb_batch_set_memory(ctx: Context, nbytes: int):
    """Bound the device workspace of batch solves (0: the free device memory);
    a batch whose frontier needs more is solved in parts."""
    st = load_library().ibb_batch_set_memory(ctx.handle, int(nbytes))
    if st != OK:
        raise RuntimeError(f"ibb_batch_set_memory: {ibb_strerror(st)}")


def ibb_batch_tune(ctx: Context, systems, params=None, sample: int = 256):
    """Autotune the batch launch configuration of each class present among the
    systems (ibb_batch_tune); returns the four class configurations as dicts."""
    refs, arr, lo, hi, parr = _batch_inputs(systems, params)
    st = load_library().ibb_batch_tune(ctx.handle, int(len(systems)), arr, _ptr(lo), _ptr(hi), parr, int(sample))
    if st != OK:
        raise RuntimeError(f"ibb_batch_tune: {ibb_strerror(st)}")
    return [ibb_batch_get_config(ctx, q).as_dict() for q in range(4)]


class BatchPlan:
    """A batch recorded once (ibb_batch_plan_create) and replayed by run()."""

    def __init__(self, ctx: Context, systems, params=None):
        self._L = load_library()
        self.systems = list(systems)
        refs, arr, lo, hi, parr = _batch_inputs(self.systems, params)
        h = C.c_void_p()
        st = self._L.ibb_batch_plan_create(ctx.handle, int(len(self.systems)), arr, _ptr(lo), _ptr(hi), parr,
                                           C.byref(h))
        if st != OK:
            raise RuntimeError(f"ibb_batch_plan_create: {ibb_strerror(st)}")
        self.handle = h

    def run(self, cap: int = 1 << 16):
        def call(*outs):
            return self._L.ibb_batch_plan_run(self.handle, *outs)

        return _batch_results(call, self.systems, cap, "ibb_batch_plan_run")

    def close(self):
        if self.handle:
            self._L.ibb_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server (ibb_server_*): submit, step, poll."""

    def __init__(self, ctx: Context, **cfg):
        L = load_library()
        c = IbbServerConfig()
        L.ibb_server_config_default(C.byref(c))
        for k, v in cfg.items():
            setattr(c, k, v)
        h = C.c_void_p()
        st = L.ibb_server_create(ctx.handle, C.byref(c), C.byref(h))
        if st != OK:
            raise RuntimeError(f"ibb_server_create: {ibb_strerror(st)}")
        self.handle = h
        self.ctx = ctx
        self.n = {}

    def submit(self, s, params: Optional[IbbParams] = None) -> int:
        ref = _SysRef(s)
        lo = np.ascontiguousarray(s.lo, dtype=np.float64)
        hi = np.ascontiguousarray(s.hi, dtype=np.float64)
        params = params or make_params(s.tol)
        rid = load_library().ibb_server_submit(self.handle, C.byref(ref.c), _ptr(lo), _ptr(hi), C.byref(params))
        if rid < 0:
            raise RuntimeError(f"ibb_server_submit: {ibb_strerror(int(rid))}")
        self.n[rid] = s.n
        return int(rid)

    def step(self) -> int:
        k = load_library().ibb_server_step(self.handle)
        if k < 0:
            raise RuntimeError(f"ibb_server_step: {ibb_strerror(k)}")
        return int(k)

    def poll(self, rid: int, cap: int = 1 << 12) -> Optional[Result]:
        n = self.n[rid]
        olo = np.zeros((cap, n))
        ohi = np.zeros((cap, n))
        otag = np.zeros(cap, dtype=np.uint8)
        m = C.c_int64(0)
        status = C.c_int32(0)
        st_ = IbbStats()
        st = load_library().ibb_server_poll(self.handle, int(rid), _ptr(olo), _ptr(ohi), _ptr(otag), int(cap),
                                            C.byref(m), C.byref(status), C.byref(st_))
        if st == 1:
            return None
        if st != OK:
            raise RuntimeError(f"ibb_server_poll: {ibb_strerror(st)}")
        del self.n[rid]
        k = int(m.value) if status.value == OK else 0
        stats = {f: int(getattr(st_, f)) for f in STATS_FIELDS}
        return Result(int(status.value), olo[:k].copy(), ohi[:k].copy(), otag[:k].copy(), stats)

    def finished(self, cap: int = 4096) -> list:
        """Ids harvested since the previous call (ibb_server_finished)."""
        out = []
        buf = np.zeros(cap, dtype=np.int64)
        while True:
            m = int(load_library().ibb_server_finished(self.handle, _ptr(buf), int(cap)))
            if m < 0:
                raise RuntimeError(f"ibb_server_finished: {ibb_strerror(m)}")
            out.extend(int(v) for v in buf[:m])
            if m < cap:
                return out

    def cancel(self, rid: int) -> bool:
        """Removes a request not admitted yet; False once it is on the device."""
        st = load_library().ibb_server_cancel(self.handle, int(rid))
        if st == OK:
            del self.n[rid]
            return True
        if st == ERR_UNSUPPORTED:
            return False
        raise RuntimeError(f"ibb_server_cancel: {ibb_strerror(st)}")

    def pending(self):
        q, a = C.c_int64(0), C.c_int64(0)
        load_library().ibb_server_pending(self.handle, C.byref(q), C.byref(a))
        return int(q.value), int(a.value)

    def close(self):
        if self.handle:
            load_library().ibb_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
