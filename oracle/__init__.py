"""ctypes binding of the CPU oracle (``oracle/ibb_oracle.c``).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library never
links, loads or calls it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ibb_oracle.c")
_LIB = os.path.join(_HERE, "libibb_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-frounding-math", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas", "-Wno-maybe-uninitialized", "-Wno-stringop-overflow"]

STATS_FIELDS = ("processed", "excluded_eval", "excluded_hs", "hs_skipped", "recontracted",
                "bisected", "emitted_unique", "emitted_undecided")

OK, ERR_INVALID_ARG, ERR_BUDGET, ERR_OUTPUT_CAPACITY = 0, -1, -2, -3
SPLIT_WIDEST, SPLIT_ALL = 0, 1
CONTRACT_HS, CONTRACT_KRAWCZYK = 0, 1
INCLUDE_NATURAL, INCLUDE_MEAN_VALUE = 0, 1
HS_EMPTY, HS_SKIPPED, HS_DONE = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (always when ``force``)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        d, i32, i64, p = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        for nm in ("rd_add", "ru_add", "rd_sub", "ru_sub", "rd_mul", "ru_mul", "rd_div", "ru_div"):
            f = getattr(L, "oracle_" + nm)
            f.restype, f.argtypes = d, [d, d]
        L.oracle_i_mul.restype, L.oracle_i_mul.argtypes = None, [d, d, d, d, p]
        L.oracle_i_pow.restype, L.oracle_i_pow.argtypes = None, [d, d, C.c_int, p]
        L.oracle_i_div_ext.restype, L.oracle_i_div_ext.argtypes = C.c_int, [d, d, d, d, p]
        L.oracle_eval_F.restype, L.oracle_eval_F.argtypes = None, [C.c_int, p, p, p, p, p, p, p]
        L.oracle_eval_J.restype, L.oracle_eval_J.argtypes = None, [C.c_int, p, p, p, p, p, p, p]
        L.oracle_fp32_inverse.restype, L.oracle_fp32_inverse.argtypes = C.c_int, [C.c_int, p, p]
        L.oracle_hs.restype, L.oracle_hs.argtypes = C.c_int, [C.c_int, p, p, p, p, p, p, p, p, C.c_int]
        L.oracle_exclusion_keep.restype = None
        L.oracle_exclusion_keep.argtypes = [C.c_int, p, p, p, i64, p, p, p]
        L.oracle_set_chain.restype, L.oracle_set_chain.argtypes = None, [p, i64]
        L.oracle_chain_len.restype, L.oracle_chain_len.argtypes = i64, []
        L.oracle_hs_trace.restype = C.c_int
        L.oracle_hs_trace.argtypes = [C.c_int, p, p, p, p, p, p, C.c_int]
        L.oracle_solve.restype = C.c_int
        L.oracle_solve.argtypes = [C.c_int, p, p, p, p, p, d, i64, i32, i32, d, d,
                                   p, p, p, i64, p, p, C.c_int, C.c_uint64, i32, i32]
        L.oracle_round.restype = C.c_int
        L.oracle_round.argtypes = [C.c_int, p, p, p, i64, p, p, p, d, i32, i32, d, d,
                                   p, p, p, i64, p, p, p, p, i64, p, p, i32, i32]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# --- primitives -------------------------------------------------------------
def rd_add(a, b): return lib().oracle_rd_add(a, b)
def ru_add(a, b): return lib().oracle_ru_add(a, b)
def rd_sub(a, b): return lib().oracle_rd_sub(a, b)
def ru_sub(a, b): return lib().oracle_ru_sub(a, b)
def rd_mul(a, b): return lib().oracle_rd_mul(a, b)
def ru_mul(a, b): return lib().oracle_ru_mul(a, b)
def rd_div(a, b): return lib().oracle_rd_div(a, b)
def ru_div(a, b): return lib().oracle_ru_div(a, b)


def i_mul(x, y):
    out = np.zeros(2)
    lib().oracle_i_mul(float(x[0]), float(x[1]), float(y[0]), float(y[1]), _ptr(out))
    return float(out[0]), float(out[1])


def i_pow(x, p):
    out = np.zeros(2)
    lib().oracle_i_pow(float(x[0]), float(x[1]), int(p), _ptr(out))
    return float(out[0]), float(out[1])


def i_div_ext(x, y):
    out = np.zeros(4)
    k = lib().oracle_i_div_ext(float(x[0]), float(x[1]), float(y[0]), float(y[1]), _ptr(out))
    return [(float(out[2 * i]), float(out[2 * i + 1])) for i in range(k)]


def _sys_arrays(s):
    return (np.ascontiguousarray(s.term_off, dtype=np.int32),
            np.ascontiguousarray(s.expo, dtype=np.uint8),
            np.ascontiguousarray(s.coef, dtype=np.float64))


def eval_F(s, lo, hi):
    to, ex, co = _sys_arrays(s)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    olo, ohi = np.zeros(s.n), np.zeros(s.n)
    lib().oracle_eval_F(s.n, _ptr(to), _ptr(ex), _ptr(co), _ptr(lo), _ptr(hi), _ptr(olo), _ptr(ohi))
    return olo, ohi


def eval_J(s, lo, hi):
    to, ex, co = _sys_arrays(s)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    olo, ohi = np.zeros((s.n, s.n)), np.zeros((s.n, s.n))
    lib().oracle_eval_J(s.n, _ptr(to), _ptr(ex), _ptr(co), _ptr(lo), _ptr(hi), _ptr(olo), _ptr(ohi))
    return olo, ohi


def exclusion_keep(s, lo, hi):
    """The exclusion test on many boxes (rows of lo/hi): True where the box is kept."""
    to, ex, co = _sys_arrays(s)
    lo = np.ascontiguousarray(lo, dtype=np.float64).reshape(-1, s.n)
    hi = np.ascontiguousarray(hi, dtype=np.float64).reshape(-1, s.n)
    keep = np.zeros(lo.shape[0], dtype=np.uint8)
    lib().oracle_exclusion_keep(s.n, _ptr(to), _ptr(ex), _ptr(co), int(lo.shape[0]), _ptr(lo), _ptr(hi), _ptr(keep))
    return keep.astype(bool)


def fp32_inverse(M):
    M = np.ascontiguousarray(M, dtype=np.float32)
    n = M.shape[0]
    Y = np.zeros((n, n), dtype=np.float32)
    st = lib().oracle_fp32_inverse(n, _ptr(M), _ptr(Y))
    return (Y if st == 0 else None)


def hs(s, lo, hi, contractor: int = CONTRACT_HS):
    """One contraction step (Hansen-Sengupta, or Krawczyk with
    contractor=CONTRACT_KRAWCZYK): (status, lo', hi', unique)."""
    to, ex, co = _sys_arrays(s)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    olo, ohi = lo.copy(), hi.copy()
    u = C.c_int(0)
    st = lib().oracle_hs(s.n, _ptr(to), _ptr(ex), _ptr(co), _ptr(lo), _ptr(hi), _ptr(olo), _ptr(ohi),
                         C.byref(u), int(contractor))
    return st, olo, ohi, bool(u.value)


def hs_trace(s, lo, hi, contractor: int = CONTRACT_HS):
    """Intermediates of one contraction step (layout: see oracle_hs_trace)."""
    to, ex, co = _sys_arrays(s)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    tr = np.zeros(6 * s.n * s.n + 8 * s.n + 4)
    st = lib().oracle_hs_trace(s.n, _ptr(to), _ptr(ex), _ptr(co), _ptr(lo), _ptr(hi), _ptr(tr), int(contractor))
    return st, tr


def proof_chains(s, cap=4096, **kw):
    """Boxes stepped while proven (or when proven) during a solve: list of
    (lo, hi, lo', hi')."""
    buf = np.zeros(cap * 4 * s.n)
    lib().oracle_set_chain(_ptr(buf), cap)
    try:
        solve(s, **kw)
        m = int(lib().oracle_chain_len())
    finally:
        lib().oracle_set_chain(None, 0)
    d = buf[: m * 4 * s.n].reshape(m, 4, s.n)
    return [(d[i, 0], d[i, 1], d[i, 2], d[i, 3]) for i in range(m)]


@dataclass
class Result:
    status: int
    lo: np.ndarray   # [m, n]
    hi: np.ndarray   # [m, n]
    tag: np.ndarray  # [m] uint8, 1 = unique root proven, 0 = undecided
    stats: dict


def solve(s, tol: Optional[float] = None, max_boxes: int = 10_000_000, split_mode: int = SPLIT_WIDEST,
          max_recontract: int = 16, recontract_ratio: float = 0.5, hs_max_width: float = float("inf"),
          cap: int = 1 << 16, order: int = 0, seed: int = 0, lo=None, hi=None,
          contractor: int = CONTRACT_HS, inclusion: int = INCLUDE_NATURAL) -> Result:
    to, ex, co = _sys_arrays(s)
    lo = np.ascontiguousarray(s.lo if lo is None else lo, dtype=np.float64)
    hi = np.ascontiguousarray(s.hi if hi is None else hi, dtype=np.float64)
    tol = s.tol if tol is None else tol
    while True:
        olo = np.zeros((cap, s.n))
        ohi = np.zeros((cap, s.n))
        otag = np.zeros(cap, dtype=np.uint8)
        nout = C.c_int64(0)
        stats = np.zeros(8, dtype=np.int64)
        st = lib().oracle_solve(s.n, _ptr(to), _ptr(ex), _ptr(co), _ptr(lo), _ptr(hi), float(tol),
                                int(max_boxes), int(split_mode), int(max_recontract),
                                float(recontract_ratio), float(hs_max_width), _ptr(olo), _ptr(ohi),
                                _ptr(otag), int(cap), C.byref(nout), _ptr(stats), int(order), int(seed),
                                int(contractor), int(inclusion))
        if st == ERR_OUTPUT_CAPACITY:
            cap = int(nout.value)
            continue
        m = int(nout.value) if st == OK else 0
        return Result(st, olo[:m].copy(), ohi[:m].copy(), otag[:m].copy(),
                      dict(zip(STATS_FIELDS, (int(v) for v in stats))))


@dataclass
class Round:
    status: int
    child_lo: np.ndarray   # [c, n], in push order
    child_hi: np.ndarray
    child_rec: np.ndarray  # [c] uint32: bit 0 proven, bits 8-15 recontraction count
    emit_lo: np.ndarray    # [e, n], in emission order
    emit_hi: np.ndarray
    emit_tag: np.ndarray   # [e] uint8
    stats: dict


def round_step(s, lo, hi, rec=None, tol: Optional[float] = None, split_mode: int = SPLIT_WIDEST,
               max_recontract: int = 16, recontract_ratio: float = 0.5,
               hs_max_width: float = float("inf"), contractor: int = CONTRACT_HS,
               inclusion: int = INCLUDE_NATURAL) -> Round:
    """One round of the search on the boxes lo[b], hi[b] (see oracle_round)."""
    to, ex, co = _sys_arrays(s)
    lo = np.ascontiguousarray(np.asarray(lo, dtype=np.float64).reshape(-1, s.n))
    hi = np.ascontiguousarray(np.asarray(hi, dtype=np.float64).reshape(-1, s.n))
    m = lo.shape[0]
    rec = np.zeros(m, dtype=np.uint32) if rec is None else np.ascontiguousarray(rec, dtype=np.uint32)
    tol = s.tol if tol is None else tol
    ccap, ecap = max(4 * m, 16), max(m, 16)
    while True:
        clo, chi = np.zeros((ccap, s.n)), np.zeros((ccap, s.n))
        crec = np.zeros(ccap, dtype=np.uint32)
        elo, ehi = np.zeros((ecap, s.n)), np.zeros((ecap, s.n))
        etag = np.zeros(ecap, dtype=np.uint8)
        nc, ne = C.c_int64(0), C.c_int64(0)
        stats = np.zeros(8, dtype=np.int64)
        st = lib().oracle_round(s.n, _ptr(to), _ptr(ex), _ptr(co), int(m), _ptr(lo), _ptr(hi), _ptr(rec),
                                float(tol), int(split_mode), int(max_recontract), float(recontract_ratio),
                                float(hs_max_width), _ptr(clo), _ptr(chi), _ptr(crec), int(ccap), C.byref(nc),
                                _ptr(elo), _ptr(ehi), _ptr(etag), int(ecap), C.byref(ne), _ptr(stats),
                                int(contractor), int(inclusion))
        if st == ERR_OUTPUT_CAPACITY:
            ccap, ecap = max(ccap, int(nc.value)), max(ecap, int(ne.value))
            continue
        c, e = (int(nc.value), int(ne.value)) if st == OK else (0, 0)
        return Round(st, clo[:c].copy(), chi[:c].copy(), crec[:c].copy(), elo[:e].copy(), ehi[:e].copy(),
                     etag[:e].copy(), dict(zip(STATS_FIELDS, (int(v) for v in stats))))
