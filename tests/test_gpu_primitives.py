"""Device rounding primitives (eq 25-27, single-precision preconditioner
arithmetic) against the oracle and exact rationals, bit for bit."""
import math
import random

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SUB = 5e-324


def _pairs(seed, n, nonzero_b=False):
    rnd = random.Random(seed)
    edge = [0.0, -0.0, 1.0, -1.0, 0.5, 3.0, 0.1, -0.1, 1e308, -1e308, 1.7976931348623157e308, SUB, -SUB,
            2.2250738585072014e-308, 1e-310, -1e-310, 2.0 ** -969, 2.0 ** -1000, 1.0 + 2.0 ** -52,
            1.0 - 2.0 ** -53, 2.0 ** 52, 1e16, 7.0, -3.0, 1e-300, 3e-320, 1e200, -2.5e-310]
    a, b = [], []
    for x in edge:
        for y in edge:
            a.append(x)
            b.append(y)
    for _ in range(n):
        e1, e2 = rnd.randint(-1074, 1023), rnd.randint(-1074, 1023)
        a.append(rnd.uniform(-2, 2) * 2.0 ** max(e1, -1022) * (2.0 ** (e1 + 1022) if e1 < -1022 else 1.0))
        b.append(rnd.uniform(-2, 2) * 2.0 ** max(e2, -1022) * (2.0 ** (e2 + 1022) if e2 < -1022 else 1.0))
        a.append(rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-60, 60))
        b.append(rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-60, 60))
    a, b = np.array(a), np.array(b)
    ok = np.isfinite(a) & np.isfinite(b)
    if nonzero_b:
        ok &= b != 0
    return a[ok], b[ok]


@pytest.mark.parametrize("op,name", [(0, "rd_add"), (1, "ru_add"), (2, "rd_sub"), (3, "ru_sub"),
                                     (4, "rd_mul"), (5, "ru_mul"), (6, "rd_div"), (7, "ru_div")])
def test_directed_ops_match_oracle(gpu_ctx, oracle_lib, op, name):
    import paper_1802_00330_amd as P
    a, b = _pairs(100 + op, 20000, nonzero_b=op >= 6)
    got = P.ibb_selftest_ops(gpu_ctx, op, a, b)
    ref = getattr(oracle_lib, name)
    exp = np.array([ref(x, y) for x, y in zip(a, b)])
    bad = np.nonzero(~((got == exp) | (np.isnan(got) & np.isnan(exp))))[0]
    assert bad.size == 0, [(a[i], b[i], got[i], exp[i]) for i in bad[:5]]


def test_midpoint_and_narrowing(gpu_ctx, oracle_lib):
    import paper_1802_00330_amd as P
    rnd = np.random.default_rng(0)
    lo = rnd.uniform(-4, 4, 20000) * 10.0 ** rnd.integers(-30, 30, 20000)
    hi = lo + np.abs(rnd.uniform(0, 1, 20000)) * 10.0 ** rnd.integers(-40, 5, 20000)
    mid = P.ibb_selftest_ops(gpu_ctx, 9, lo, hi)
    exp = np.array([oracle_lib.rd_mul(oracle_lib.rd_add(x, y), 0.5) for x, y in zip(lo, hi)])
    assert np.array_equal(mid, exp)
    assert np.all((lo <= mid) & (mid <= hi))
    x = np.concatenate([lo, [3.4028235677973366e38, 3.4028234663852886e38 * 1.0000001, 1e-45, 7e-46, 1.5e-45,
                             -2.5e-45, 1.0 + 2.0 ** -24, 1.0 + 3 * 2.0 ** -24, 1e39, -1e39]])
    nar = P.ibb_selftest_ops(gpu_ctx, 8, x, x)
    exp = x.astype(np.float32).astype(np.float64)  # IEEE round to nearest even
    assert np.array_equal(nar, exp)


def test_single_precision_ops_round_to_nearest(gpu_ctx):
    import paper_1802_00330_amd as P
    rnd = np.random.default_rng(1)
    a = rnd.uniform(-1, 1, 50000).astype(np.float32) * np.float32(2.0) ** rnd.integers(-140, 100, 50000).astype(np.float32)
    b = rnd.uniform(-1, 1, 50000).astype(np.float32) * np.float32(2.0) ** rnd.integers(-20, 20, 50000).astype(np.float32)
    b[b == 0] = 1.0
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    with np.errstate(all="ignore"):
        assert np.array_equal(P.ibb_selftest_ops(gpu_ctx, 10, a64, b64), (a * b).astype(np.float64))
        assert np.array_equal(P.ibb_selftest_ops(gpu_ctx, 11, a64, b64), (a / b).astype(np.float64))
