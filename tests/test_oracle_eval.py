"""Pins for the oracle's interval evaluation F(X) (Def. 1) and interval
Jacobian J(X) (Alg. 3, first step): closed forms, exact point values,
containment of exact values, and symbolic derivatives from sympy."""
import random
from fractions import Fraction

import numpy as np
import pytest
import sympy

import workloads as W
from tests.exact import F, poly_value


def _sys(n, eqs, lo=-1.0, hi=1.0):
    return W.systems._pack(n, eqs, lo, hi, 1e-6, "t")


def test_closed_forms(oracle_lib):
    s = W.univariate([-2.0, 0.0, 1.0], 1.0, 2.0)  # x^2 - 2
    lo, hi = oracle_lib.eval_F(s, [1.0], [2.0])
    assert (lo[0], hi[0]) == (-1.0, 2.0)
    lo, hi = oracle_lib.eval_F(s, [-2.0], [2.0])
    assert (lo[0], hi[0]) == (-2.0, 2.0)  # tight square: [0,4] - 2
    # circle/line at a corner box
    c = W.circle_line()
    lo, hi = oracle_lib.eval_F(c, [0.5, -1.0], [1.0, 0.25])
    assert (lo[0], hi[0]) == (-0.75, 1.0)  # [0.25,1]+[0,1]-1
    assert (lo[1], hi[1]) == (0.25, 2.0)   # [0.5,1]-[-1,0.25]


def _random_system(rng, n, deg, terms):
    allexp = W.systems._exponents(n, deg)
    eqs = []
    for _ in range(n):
        idx = rng.choice(len(allexp), size=min(terms, len(allexp)), replace=False)
        eq = [(float(rng.uniform(-2, 2)), allexp[int(j)]) for j in idx]
        eq.append((float(rng.uniform(-1, 1)), (0,) * n))
        eqs.append(eq)
    return _sys(n, eqs)


def test_point_boxes_exact_on_dyadics(oracle_lib):
    """At a dyadic point with short mantissas every operation is exact, so the
    degenerate box evaluates to exactly f(x): a dropped, duplicated or
    misindexed term changes the value."""
    rng = np.random.default_rng(0)
    for trial in range(30):
        n = int(rng.integers(1, 6))
        s = _random_system(rng, n, 3, 6)
        # dyadic coefficients and point
        s.coef[:] = np.round(s.coef * 8) / 8
        x = np.round(rng.uniform(-2, 2, size=n) * 4) / 4
        lo, hi = oracle_lib.eval_F(s, x, x)
        for i, (c, e) in enumerate(s.equations()):
            v = poly_value(c, e, [F(t) for t in x])
            assert F(lo[i]) == v == F(hi[i]), (trial, i)


def test_point_boxes_enclose_exact_value(oracle_lib):
    rng = np.random.default_rng(1)
    for trial in range(30):
        n = int(rng.integers(1, 7))
        s = _random_system(rng, n, 4, 8)
        x = rng.uniform(-2, 2, size=n)
        lo, hi = oracle_lib.eval_F(s, x, x)
        for i, (c, e) in enumerate(s.equations()):
            v = poly_value(c, e, [F(t) for t in x])
            assert F(lo[i]) <= v <= F(hi[i])
            assert hi[i] - lo[i] <= 1e-12 * (1 + abs(float(v))) * len(c)


def test_box_encloses_sampled_exact_values(oracle_lib):
    rng = np.random.default_rng(2)
    for trial in range(20):
        n = int(rng.integers(1, 6))
        s = _random_system(rng, n, 3, 6)
        a = rng.uniform(-2, 1, size=n)
        b = a + rng.uniform(0, 1, size=n)
        lo, hi = oracle_lib.eval_F(s, a, b)
        for _ in range(20):
            t = [F(a[k]) + (F(b[k]) - F(a[k])) * Fraction(int(rng.integers(0, 65)), 64) for k in range(n)]
            for i, (c, e) in enumerate(s.equations()):
                v = poly_value(c, e, t)
                assert F(lo[i]) <= v <= F(hi[i])


def _sympy_jacobian(s):
    xs = sympy.symbols(f"x0:{s.n}")
    J = []
    for c, e in s.equations():
        f = sum(sympy.Rational(F(ci)) * sympy.Mul(*[xs[k] ** int(e_t[k]) for k in range(s.n)])
                for ci, e_t in zip(c, e))
        J.append([sympy.diff(f, xs[k]) for k in range(s.n)])
    return xs, J


def test_jacobian_matches_symbolic_derivative(oracle_lib):
    rng = np.random.default_rng(3)
    for trial in range(12):
        n = int(rng.integers(2, 5))
        s = _random_system(rng, n, 3, 5)
        s.coef[:] = np.round(s.coef * 8) / 8
        xs, J = _sympy_jacobian(s)
        # exact at dyadic points
        x = np.round(rng.uniform(-2, 2, size=n) * 4) / 4
        lo, hi = oracle_lib.eval_J(s, x, x)
        sub = {xs[k]: sympy.Rational(F(x[k])) for k in range(n)}
        for i in range(n):
            for k in range(n):
                v = Fraction(str(J[i][k].subs(sub)))
                assert F(lo[i, k]) == v == F(hi[i, k]), (trial, i, k)
                if J[i][k] == 0:
                    assert lo[i, k] == 0 and hi[i, k] == 0
        # containment over a box
        a = rng.uniform(-2, 1, size=n)
        b = a + rng.uniform(0, 1, size=n)
        lo, hi = oracle_lib.eval_J(s, a, b)
        for _ in range(10):
            t = [F(a[k]) + (F(b[k]) - F(a[k])) * Fraction(int(rng.integers(0, 17)), 16) for k in range(n)]
            sub = {xs[k]: sympy.Rational(t[k]) for k in range(n)}
            for i in range(n):
                for k in range(n):
                    v = Fraction(str(J[i][k].subs(sub)))
                    assert F(lo[i, k]) <= v <= F(hi[i, k])


def test_jacobian_orientation(oracle_lib):
    """J[i][k] = d f_i / d x_k (not its transpose): f0 = x1^3, f1 = x0."""
    s = _sys(2, [[(1.0, (0, 3))], [(1.0, (1, 0))]])
    lo, hi = oracle_lib.eval_J(s, [2.0, 2.0], [2.0, 2.0])
    assert lo.tolist() == [[0.0, 12.0], [1.0, 0.0]]
    assert hi.tolist() == [[0.0, 12.0], [1.0, 0.0]]


def test_jacobian_coefficient_rounding_is_outward(oracle_lib):
    """d(c x^3)/dx = 3c x^2 with 3c inexact: the coefficient is enclosed."""
    c = 0.1
    s = W.univariate([0.0, 0.0, 0.0, c], -1.0, 1.0)
    lo, hi = oracle_lib.eval_J(s, [1.0], [1.0])
    exact = 3 * F(c)
    assert F(lo[0, 0]) < exact < F(hi[0, 0])
