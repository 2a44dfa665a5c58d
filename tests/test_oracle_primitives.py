"""Pins for the oracle's directed rounding (eq 25-27) and interval operations
(eq 5-10), against exact rational arithmetic."""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

from tests.exact import F, round_down, round_up

SUB = 5e-324  # smallest subnormal


def _operands(seed, count):
    rnd = random.Random(seed)
    vals = [0.0, -0.0, 1.0, -1.0, 0.5, 3.0, 0.1, -0.1, 1e308, -1e308, 1.7976931348623157e308,
            SUB, -SUB, 2.2250738585072014e-308, 1e-310, -1e-310, 2.0 ** -969, 2.0 ** -1000,
            1.0 + 2.0 ** -52, 1.0 - 2.0 ** -53, 2.0 ** 52, 2.0 ** 53 + 2.0, 1e16, 7.0, -3.0]
    pairs = [(a, b) for a in vals for b in vals]
    for _ in range(count):
        e1, e2 = rnd.randint(-60, 60), rnd.randint(-60, 60)
        pairs.append((rnd.uniform(-1, 1) * 2.0 ** e1, rnd.uniform(-1, 1) * 2.0 ** e2))
        pairs.append((rnd.uniform(-1, 1), rnd.uniform(-1, 1)))
    return pairs


@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_directed_rounding_exact(oracle_lib, op):
    O = oracle_lib
    fns = {"add": (O.rd_add, O.ru_add, lambda a, b: a + b),
           "sub": (O.rd_sub, O.ru_sub, lambda a, b: a - b),
           "mul": (O.rd_mul, O.ru_mul, lambda a, b: a * b),
           "div": (O.rd_div, O.ru_div, lambda a, b: a / b)}[op]
    rd, ru, exact = fns
    n = 0
    for a, b in _operands(1234 + len(op), 3000):
        if op == "div" and b == 0:
            continue
        q = exact(F(a), F(b))
        lo, hi = rd(a, b), ru(a, b)
        if q == 0:
            assert lo == 0 and hi == 0
        else:
            assert lo == round_down(q), (op, a, b)
            assert hi == round_up(q), (op, a, b)
        assert lo <= hi
        n += 1
    assert n > 3000


def test_directed_rounding_brackets_nearest(oracle_lib):
    O = oracle_lib
    rnd = random.Random(7)
    for _ in range(2000):
        a, b = rnd.uniform(-10, 10), rnd.uniform(-10, 10)
        for rd, ru, f in ((O.rd_add, O.ru_add, a + b), (O.rd_mul, O.ru_mul, a * b)):
            lo, hi = rd(a, b), ru(a, b)
            assert lo <= f <= hi
            assert hi == lo or math.nextafter(lo, math.inf) == hi


def test_interval_product_is_rounded_exact_hull(oracle_lib):
    """eq (27): the product interval is the exact range of x*y (extremes over the
    four endpoint products), lower end rounded down, upper end rounded up."""
    rnd = random.Random(3)
    edge = [-2.0, -1.0, -0.5, -0.0, 0.0, 0.3, 1.0, 3.0]
    cases = [((a, b), (c, d)) for a in edge for b in edge for c in edge for d in edge if a <= b and c <= d]
    for _ in range(3000):
        a, b = sorted((rnd.uniform(-5, 5), rnd.uniform(-5, 5)))
        c, d = sorted((rnd.uniform(-5, 5), rnd.uniform(-5, 5)))
        cases.append(((a, b), (c, d)))
    for x, y in cases:
        prods = [F(u) * F(v) for u in x for v in y]
        lo, hi = oracle_lib.i_mul(x, y)
        assert lo == round_down(min(prods)) or (min(prods) == 0 and lo == 0)
        assert hi == round_up(max(prods)) or (max(prods) == 0 and hi == 0)


def _exact_pow_range(a, b, p):
    """Exact min and max of x^p over [a,b] (rationals)."""
    A, B = F(a), F(b)
    vals = [A ** p, B ** p]
    if p % 2 == 0 and A < 0 < B:
        vals.append(Fraction(0))
    return min(vals), max(vals)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 8])
def test_power_encloses_exact_range_tightly(oracle_lib, p):
    rnd = random.Random(p)
    cases = [(-1.0, 2.0), (-3.0, -2.0), (0.5, 3.0), (-2.0, 0.0), (0.0, 0.0), (-0.1, 0.1), (1.0, 1.0)]
    for _ in range(500):
        a, b = sorted((rnd.uniform(-3, 3), rnd.uniform(-3, 3)))
        cases.append((a, b))
    for a, b in cases:
        lo, hi = oracle_lib.i_pow((a, b), p)
        emin, emax = _exact_pow_range(a, b, p)
        assert F(lo) <= emin and emax <= F(hi)
        # chained rounding: at most p-1 roundings in each direction
        tol = Fraction(p) * Fraction(2) ** -51
        assert emin - F(lo) <= tol * abs(emin) + Fraction(SUB)
        assert F(hi) - emax <= tol * abs(emax) + Fraction(SUB)


def test_power_closed_forms(oracle_lib):
    # even powers are tight over intervals containing zero (not the product [-2,4])
    assert oracle_lib.i_pow((-1.0, 2.0), 2) == (0.0, 4.0)
    assert oracle_lib.i_pow((-3.0, -2.0), 3) == (-27.0, -8.0)
    assert oracle_lib.i_pow((-3.0, -2.0), 2) == (4.0, 9.0)
    assert oracle_lib.i_pow((0.5, 3.0), 4) == (0.0625, 81.0)


def _sample_quotients(x, y, rnd, k=400):
    a, b = x
    c, d = y
    pts = []
    for _ in range(k):
        u = F(a) + (F(b) - F(a)) * Fraction(rnd.randint(0, 1000), 1000)
        v = F(c) + (F(d) - F(c)) * Fraction(rnd.randint(0, 1000), 1000)
        if v != 0:
            pts.append(u / v)
    for u in (F(a), F(b)):
        for v in (F(c), F(d)):
            if v != 0:
                pts.append(u / v)
    return pts


def test_extended_division_sign_classes(oracle_lib):
    """eq (10): every quotient x/y (y != 0) lies in the result; bounded ends are
    attained by endpoint quotients up to one rounding; no quotient falls in the
    gap between two pieces; y = [0,0] with 0 not in x gives the empty set."""
    rnd = random.Random(11)
    xs = [(-3.0, -1.0), (-2.0, 0.0), (-1.0, 2.0), (0.0, 3.0), (1.0, 4.0), (0.0, 0.0)]
    ys = [(-4.0, -2.0), (-3.0, 0.0), (-1.0, 2.0), (0.0, 5.0), (2.0, 3.0), (0.0, 0.0)]
    seen_two = 0
    for x in xs:
        for y in ys:
            pieces = oracle_lib.i_div_ext(x, y)
            zx = x[0] <= 0 <= x[1]
            if y == (0.0, 0.0):
                assert pieces == ([] if not zx else [(-math.inf, math.inf)])
                continue
            if y[0] <= 0 <= y[1] and zx:
                assert pieces == [(-math.inf, math.inf)]
                continue
            assert 1 <= len(pieces) <= 2
            qs = _sample_quotients(x, y, rnd)
            for q in qs:
                assert any(F(lo) <= q <= F(hi) if math.isfinite(lo) and math.isfinite(hi) else
                           ((lo == -math.inf or F(lo) <= q) and (hi == math.inf or q <= F(hi)))
                           for lo, hi in pieces), (x, y, q)
            ends = [F(u) / F(v) for u in x for v in y if v != 0]
            for lo, hi in pieces:
                if math.isfinite(lo):
                    assert any(lo == round_down(e) for e in ends), (x, y, lo)
                if math.isfinite(hi):
                    assert any(hi == round_up(e) for e in ends), (x, y, hi)
            if len(pieces) == 2:
                seen_two += 1
                (l1, h1), (l2, h2) = pieces
                assert l1 == -math.inf and h2 == math.inf and h1 < l2
                # the gap holds no quotient
                assert not any(F(h1) < q < F(l2) for q in qs)
    assert seen_two >= 2


def test_extended_division_random_containment(oracle_lib):
    rnd = random.Random(5)
    for _ in range(400):
        a, b = sorted((rnd.uniform(-4, 4), rnd.uniform(-4, 4)))
        c, d = sorted((rnd.uniform(-4, 4), rnd.uniform(-4, 4)))
        if rnd.random() < 0.3:
            c = -abs(c)
            d = abs(d)
        pieces = oracle_lib.i_div_ext((a, b), (c, d))
        for q in _sample_quotients((a, b), (c, d), rnd, 100):
            ok = False
            for lo, hi in pieces:
                if (lo == -math.inf or F(lo) <= q) and (hi == math.inf or q <= F(hi)):
                    ok = True
            assert ok


def test_ordinary_division_is_rounded_exact_hull(oracle_lib):
    rnd = random.Random(9)
    for _ in range(1000):
        a, b = sorted((rnd.uniform(-4, 4), rnd.uniform(-4, 4)))
        c, d = sorted((rnd.uniform(0.1, 4), rnd.uniform(0.1, 4)))
        if rnd.random() < 0.5:
            c, d = -d, -c
        (lo, hi), = oracle_lib.i_div_ext((a, b), (c, d))
        qs = [F(u) / F(v) for u in (a, b) for v in (c, d)]
        assert lo == round_down(min(qs)) and hi == round_up(max(qs))
