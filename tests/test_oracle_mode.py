"""Every oracle entry point leaves the caller's floating-point rounding mode
unchanged (its interval operations switch the mode per bound); a leaked
directed mode would silently change what the caller computes next, e.g. the
coefficients of the next generated system."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as W

LIBC = ctypes.CDLL(None)
FE_TONEAREST, FE_DOWNWARD, FE_UPWARD = 0, 0x400, 0x800


def _calls():
    s = W.circle_line()
    b = W.banded(0, n=4)
    yield "rd_add", lambda: oracle.rd_add(1.0, 1e-30)
    yield "i_mul", lambda: oracle.i_mul((-1.0, 2.0), (3.0, 4.0))
    yield "i_pow", lambda: oracle.i_pow((-1.5, 2.0), 3)
    yield "i_div_ext", lambda: oracle.i_div_ext((1.0, 2.0), (-1.0, 3.0))
    yield "eval_F", lambda: oracle.eval_F(s, s.lo, s.hi)
    yield "eval_J", lambda: oracle.eval_J(s, s.lo, s.hi)
    yield "fp32_inverse", lambda: oracle.fp32_inverse(np.array([[2.0, 1.0], [1.0, 3.0]], dtype=np.float32))
    yield "hs", lambda: oracle.hs(b, b.lo, b.hi)
    yield "hs_trace", lambda: oracle.hs_trace(b, b.lo, b.hi)
    yield "solve", lambda: oracle.solve(s)
    yield "round", lambda: oracle.round_step(s, s.lo, s.hi)


@pytest.mark.parametrize("caller_mode", [FE_TONEAREST, FE_UPWARD, FE_DOWNWARD])
def test_entry_points_keep_caller_mode(oracle_lib, caller_mode):
    calls = list(_calls())
    try:
        for name, f in calls:
            LIBC.fesetround(caller_mode)
            f()
            assert LIBC.fegetround() == caller_mode, name
    finally:
        LIBC.fesetround(FE_TONEAREST)


def test_generators_refuse_directed_mode():
    LIBC.fesetround(FE_UPWARD)
    try:
        with pytest.raises(RuntimeError):
            W.banded(0)
    finally:
        LIBC.fesetround(FE_TONEAREST)
    W.banded(0)
