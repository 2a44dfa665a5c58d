"""Whole-solve pins for the oracle (Alg. 1-3): closed-form roots, brute force on
tiny systems, planted roots, order independence, error handling."""
import math
from fractions import Fraction

import numpy as np
import pytest
import sympy

import workloads as W
from tests.exact import F


def _contains(lo, hi, r, slack=0.0):
    return bool(np.all(lo - slack <= r) and np.all(r <= hi + slack))


def test_circle_line_two_unique_boxes(oracle_lib):
    """x^2+y^2=1, x=y on [-2,2]^2: exactly two proven boxes, around
    +-(1/sqrt2, 1/sqrt2), each no wider than the tolerance."""
    s = W.circle_line()
    r = oracle_lib.solve(s)
    assert r.status == 0
    assert r.tag.tolist() == [1, 1]
    assert np.all(r.hi - r.lo <= 1e-6)
    for b, sign in ((0, -1), (1, 1)):
        for k in range(2):
            lo, hi = F(r.lo[b, k]), F(r.hi[b, k])
            # sign * t encloses 1/sqrt2  <=>  the squares bracket 1/2
            if sign > 0:
                assert lo > 0 and lo * lo <= Fraction(1, 2) <= hi * hi
            else:
                assert hi < 0 and hi * hi <= Fraction(1, 2) <= lo * lo
    # the same in the paper's split-everything mode
    r2 = oracle_lib.solve(s, split_mode=oracle_lib.SPLIT_ALL)
    assert r2.status == 0 and r2.tag.tolist() == [1, 1]


def _poly_from_roots(roots):
    c = [Fraction(1)]
    for r in roots:
        r = Fraction(r)
        nc = [Fraction(0)] * (len(c) + 1)
        for i, v in enumerate(c):
            nc[i + 1] += v
            nc[i] -= r * v
        c = nc
    return c


@pytest.mark.parametrize("seed", range(8))
def test_univariate_brute_force(oracle_lib, seed):
    """n = 1, exact: the stored polynomial (its double coefficients taken as
    rationals) has no real root in [-2,2] outside the emitted boxes (Sturm
    counts on every gap), every proven box holds exactly one root, and for
    simple roots away from split points each root gets a proven box; a sign
    change count on a fine grid agrees."""
    rng = np.random.default_rng(seed)
    deg = int(rng.integers(2, 7))
    roots = sorted({Fraction(int(v), 61) for v in rng.integers(-110, 110, size=deg)})
    cf = _poly_from_roots(roots)
    s = W.univariate([float(c) for c in cf], -2.0, 2.0, tol=1e-9)
    r = oracle_lib.solve(s)
    assert r.status == 0
    x = sympy.Symbol("x")
    P = sympy.Poly(sum(sympy.Rational(F(c)) * x ** k for k, c in enumerate(s.coef)), x)
    total = P.count_roots(-2, 2)
    assert total == len(roots)
    boxes = sorted((F(r.lo[b, 0]), F(r.hi[b, 0])) for b in range(len(r.tag)))
    # gaps between the union of boxes hold no root
    edges = [Fraction(-2)]
    for lo, hi in boxes:
        edges.extend([lo, hi])
    edges.append(Fraction(2))
    for u, v in zip(edges[0::2], edges[1::2]):
        if u < v:
            inner = P.count_roots(sympy.Rational(u), sympy.Rational(v))
            inner -= int(P.eval(sympy.Rational(u)) == 0) + int(P.eval(sympy.Rational(v)) == 0)
            assert inner == 0, (u, v)
    for b in range(len(r.tag)):
        if r.tag[b]:
            assert P.count_roots(sympy.Rational(F(r.lo[b, 0])), sympy.Rational(F(r.hi[b, 0]))) == 1
    grid = np.linspace(-2, 2, 40001)
    vals = np.polyval(s.coef[::-1], grid)
    assert int(np.sum(np.sign(vals[1:]) * np.sign(vals[:-1]) < 0)) == total
    assert int(r.tag.sum()) == total


def test_product_system_n2_all_roots(oracle_lib):
    """(x-a)(x-b) = 0, (y-c) + (x-a)(x-b) = 0 type systems: all 2x1 roots known."""
    a, b, c = 0.25, -0.75, 0.5
    eqs = [
        [(1.0, (2, 0)), (-(a + b), (1, 0)), (a * b, (0, 0))],
        [(1.0, (0, 1)), (1.0, (2, 0)), (-(a + b), (1, 0)), (a * b - c, (0, 0))],
    ]
    s = W.systems._pack(2, eqs, -2.0, 2.0, 1e-9, "prod2")
    r = oracle_lib.solve(s)
    assert r.status == 0
    for root in ([a, c], [b, c]):
        assert any(_contains(r.lo[i], r.hi[i], np.array(root)) for i in range(len(r.tag)))
    assert int(r.tag.sum()) == 2


@pytest.mark.parametrize("seed", range(6))
def test_product_systems_all_roots_enclosed(oracle_lib, seed):
    s = W.product_linear(seed=[1, seed], n=3)
    r = oracle_lib.solve(s)
    assert r.status == 0
    for root in s.roots:
        assert any(_contains(r.lo[i], r.hi[i], root, 1e-12) for i in range(len(r.tag))), root
    for i in range(len(r.tag)):
        if r.tag[i]:
            assert sum(_contains(r.lo[i], r.hi[i], root, 1e-12) for root in s.roots) == 1


@pytest.mark.parametrize("seed", range(6))
def test_planted_root_enclosed_small_dense(oracle_lib, seed):
    s = W.dense_planted(seed, n=3, n_terms=6, max_deg=2)
    r = oracle_lib.solve(s)
    assert r.status == 0
    root = s.roots[0]
    assert any(_contains(r.lo[i], r.hi[i], root, 1e-12) for i in range(len(r.tag)))


def _same(r1, r2):
    return (r1.status == r2.status and np.array_equal(r1.lo, r2.lo) and np.array_equal(r1.hi, r2.hi)
            and np.array_equal(r1.tag, r2.tag) and r1.stats == r2.stats)


@pytest.mark.parametrize("maker", [lambda: W.circle_line(),
                                   lambda: W.dense_planted(0, n=3, n_terms=6, max_deg=2),
                                   lambda: W.product_linear(seed=[2, 0], n=3)])
def test_order_independence(oracle_lib, maker):
    """Each box's fate depends only on the box, so LIFO, FIFO and random
    processing orders give identical sorted lists and identical counters."""
    s = maker()
    base = oracle_lib.solve(s, order=0)
    assert base.status == 0
    assert _same(base, oracle_lib.solve(s, order=1))
    for seed in (1, 2):
        assert _same(base, oracle_lib.solve(s, order=2, seed=seed))


def test_budget_is_on_tree_nodes(oracle_lib):
    s = W.circle_line()
    full = oracle_lib.solve(s)
    n = full.stats["processed"]
    assert oracle_lib.solve(s, max_boxes=n).status == 0
    assert oracle_lib.solve(s, max_boxes=n - 1).status == oracle_lib.ERR_BUDGET


def test_invalid_arguments(oracle_lib):
    s = W.circle_line()
    assert oracle_lib.solve(s, tol=0.0).status == oracle_lib.ERR_INVALID_ARG
    assert oracle_lib.solve(s, tol=float("nan")).status == oracle_lib.ERR_INVALID_ARG
    assert oracle_lib.solve(s, lo=[1.0, 0.0], hi=[0.0, 1.0]).status == oracle_lib.ERR_INVALID_ARG
    assert oracle_lib.solve(s, max_boxes=0).status == oracle_lib.ERR_INVALID_ARG
    bad = W.circle_line()
    bad.coef[0] = float("inf")
    assert oracle_lib.solve(bad).status == oracle_lib.ERR_INVALID_ARG


def test_output_is_sorted_and_canonical(oracle_lib):
    s = W.product_linear(seed=[3, 1], n=4)
    r = oracle_lib.solve(s)
    keys = [tuple(r.lo[i]) + tuple(r.hi[i]) + (int(r.tag[i]),) for i in range(len(r.tag))]
    assert keys == sorted(keys)
    assert not np.any(np.signbit(r.lo) & (r.lo == 0)) and not np.any(np.signbit(r.hi) & (r.hi == 0))
