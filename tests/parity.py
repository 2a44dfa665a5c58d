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
