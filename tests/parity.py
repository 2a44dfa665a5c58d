"""Comparison helpers for GPU-vs-oracle parity (bit-exact box lists)."""
import numpy as np


def assert_same(gpu, ref, what=""):
    assert gpu.status == ref.status, (what, gpu.status, ref.status)
    if ref.status != 0:
        return
    assert gpu.stats == ref.stats, (what, gpu.stats, ref.stats)
    assert gpu.lo.shape == ref.lo.shape, (what, gpu.lo.shape, ref.lo.shape)
    # bit-exact, with -0 written as +0 on both sides
    assert np.array_equal(gpu.lo.view(np.uint64), ref.lo.view(np.uint64)), what
    assert np.array_equal(gpu.hi.view(np.uint64), ref.hi.view(np.uint64)), what
    assert np.array_equal(gpu.tag, ref.tag), what


def box_rows(lo, hi, rec):
    """Rows (lo bits..., hi bits..., record) with -0 made +0, sorted: a
    multiset of boxes that compares bit for bit."""
    lo = np.where(lo == 0, 0.0, lo).view(np.uint64)
    hi = np.where(hi == 0, 0.0, hi).view(np.uint64)
    rows = np.concatenate([lo, hi, np.asarray(rec, dtype=np.uint64).reshape(-1, 1)], axis=1)
    if rows.shape[0] == 0:
        return rows
    order = np.lexsort(rows.T[::-1])
    return rows[order]


def first_row_difference(a, b):
    """Index of the first differing row of two sorted row sets, or None."""
    m = min(a.shape[0], b.shape[0])
    if a.shape[0] == b.shape[0] and np.array_equal(a, b):
        return None
    neq = np.nonzero((a[:m] != b[:m]).any(axis=1))[0]
    return int(neq[0]) if neq.size else m
