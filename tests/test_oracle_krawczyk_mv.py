"""Pins of the oracle's Krawczyk step (eq 15-16) and of its mean-value
exclusion test (the centred inclusion of Sec. 2.2): worked examples whose
operator values are derived in exact rationals, boxes without roots that only
these tests discard, and whole solves with known roots."""
from fractions import Fraction

import numpy as np

import workloads as W
from workloads.systems import _pack
from tests.exact import F, round_down, round_up

KRAW = 1


def _kraw_trace(oracle_lib, s, lo, hi):
    """(status, K as [n][2], X' as [n][2], unique flag) from the step trace."""
    st, tr = oracle_lib.hs_trace(s, np.asarray(lo, float), np.asarray(hi, float), contractor=KRAW)
    n = s.n
    K = tr[6 * n * n + 4 * n: 6 * n * n + 6 * n].reshape(n, 2)
    X = tr[6 * n * n + 6 * n: 6 * n * n + 8 * n].reshape(n, 2)
    return st, K, X, tr[6 * n * n + 8 * n + 2] == 1.0


def _encloses_tightly(lo, hi, exact_lo, exact_hi, ulps=4):
    """[lo, hi] contains [exact_lo, exact_hi] and overshoots by at most a few
    units in the last place on each side."""
    if not (F(lo) <= exact_lo and exact_hi <= F(hi)):
        return False
    a, b = round_down(exact_lo), round_up(exact_hi)
    for _ in range(ulps):
        a, b = np.nextafter(a, -np.inf), np.nextafter(b, np.inf)
    return lo >= a and hi <= b


def test_krawczyk_sqrt2_exact():
    """f = x^2 - 2 on X = [1, 2]: x = 1.5, f(x) = 1/4, J(X) = [2, 4], mid J = 3,
    Y = fl32(1/3).  K(X) = x - Y/4 + (1 - Y [2, 4]) [-1/2, 1/2] is
    [3/2 - Y/4 - (4Y - 1)/2, 3/2 - Y/4 + (4Y - 1)/2] in exact arithmetic
    (|1 - 2Y| < |1 - 4Y|); it lies inside (1, 2), so the step proves one root."""
    import oracle
    s = W.univariate([-2.0, 0.0, 1.0], 1.0, 2.0)
    st, K, X, unique = _kraw_trace(oracle, s, [1.0], [2.0])
    assert st == oracle.HS_DONE and unique
    Y = Fraction(float(np.float32(1.0 / 3.0)))
    c = Fraction(3, 2) - Y / 4
    r = (4 * Y - 1) / 2
    assert _encloses_tightly(K[0, 0], K[0, 1], c - r, c + r)
    assert K[0, 0] * K[0, 0] < 2 < K[0, 1] * K[0, 1]
    assert (X == K).all()


def test_krawczyk_linear_system_exact():
    """f = A x - b, A = [[2, 1], [1, 3]], b = A x*: J = A exactly, Y = the
    single-precision inverse of A; K(X) = x - Y(Ax - b) + (I - YA)(X - x) in
    exact arithmetic from that Y, enclosed to a few ulps; it holds x* and is
    far narrower than X."""
    import oracle
    xs = [Fraction(3, 10), Fraction(-7, 10)]
    A = [[2, 1], [1, 3]]
    b = [sum(A[i][j] * xs[j] for j in range(2)) for i in range(2)]
    terms = []
    for i in range(2):
        terms.append([(float(A[i][0]), (1, 0)), (float(A[i][1]), (0, 1)), (-float(b[i]), (0, 0))])
    s = _pack(2, terms, [-1.0, -1.0], [1.0, 1.0], 1e-8, "linear2")
    lo = np.array([0.25, -0.75])
    hi = np.array([0.375, -0.625])
    st, K, X, unique = _kraw_trace(oracle, s, lo, hi)
    assert st == oracle.HS_DONE and unique
    Yf = oracle.fp32_inverse(np.array(A, dtype=np.float32))
    Y = [[Fraction(float(Yf[i, j])) for j in range(2)] for i in range(2)]
    xc = [(F(lo[k]) + F(hi[k])) / 2 for k in range(2)]
    cb = [F(v) for v in (-float(b[0]), -float(b[1]))]
    fx = [sum(A[i][j] * xc[j] for j in range(2)) + cb[i] for i in range(2)]
    for i in range(2):
        center = xc[i] - sum(Y[i][k] * fx[k] for k in range(2))
        rad = Fraction(0)
        for j in range(2):
            m = (1 if i == j else 0) - sum(Y[i][k] * A[k][j] for k in range(2))
            rad += abs(m) * (F(hi[j]) - F(lo[j])) / 2
        assert _encloses_tightly(K[i, 0], K[i, 1], center - rad, center + rad), i
        assert F(K[i, 0]) <= xs[i] <= F(K[i, 1])
        assert K[i, 1] - K[i, 0] < 1e-5


def test_krawczyk_empty_where_the_natural_extension_keeps_the_box():
    """f = x^2 - 2x + 0.9 has no root in [0.95, 1.15] (f <= -0.0775 there), but
    the natural extension gives [-0.4975, 0.3225].  x = 1.05, f(x) = -0.0975,
    J(X) = [-0.1, 0.3], Y ~ 10: K(X) ~ [1.825, 2.225] misses X."""
    import oracle
    s = W.univariate([0.9, -2.0, 1.0], 0.95, 1.15)
    flo, fhi = oracle.eval_F(s, [0.95], [1.15])
    assert flo[0] < 0 < fhi[0]
    st, K, _, _ = _kraw_trace(oracle, s, [0.95], [1.15])
    assert st == oracle.HS_EMPTY
    assert 1.8 < K[0, 0] < 1.85 and 2.2 < K[0, 1] < 2.25


def test_mean_value_form_excludes_where_natural_keeps():
    """f = x^2 - 2x + 1.001 = (x - 1)^2 + 0.001 on [0.99, 1.01]: the natural
    extension gives about [-0.0389, 0.0411] (keeps the box); the mean-value form
    f(1) + J(X)(X - 1) = 0.001 + [-0.02, 0.02][-0.01, 0.01] = [0.0008, 0.0012]
    excludes 0, so one round discards the box by evaluation."""
    import oracle
    s = W.univariate([1.001, -2.0, 1.0], 0.99, 1.01, tol=1e-12)
    flo, fhi = oracle.eval_F(s, [0.99], [1.01])
    assert flo[0] < 0 < fhi[0]
    nat = oracle.round_step(s, [0.99], [1.01], hs_max_width=0.0)
    mv = oracle.round_step(s, [0.99], [1.01], hs_max_width=0.0, inclusion=oracle.INCLUDE_MEAN_VALUE)
    assert nat.stats["excluded_eval"] == 0 and len(nat.child_lo) == 2
    assert mv.stats["excluded_eval"] == 1 and len(mv.child_lo) == 0 and len(mv.emit_lo) == 0


def _check_known_roots(r, roots, n):
    """Every known root lies in an output box; every proven box holds exactly one."""
    assert r.status == 0
    for x in roots:
        assert any(np.all(r.lo[b] <= x) and np.all(x <= r.hi[b]) for b in range(len(r.tag))), x
    for b in np.nonzero(r.tag == 1)[0]:
        inside = [x for x in roots if np.all(r.lo[b] <= x) and np.all(x <= r.hi[b])]
        assert len(inside) == 1, (b, inside)


def test_whole_solves_with_krawczyk_and_mean_value():
    import oracle
    s = W.circle_line()
    for kw in ({"contractor": KRAW}, {"inclusion": 1}, {"contractor": KRAW, "inclusion": 1}):
        r = oracle.solve(s, **kw)
        assert r.status == 0 and r.tag.tolist() == [1, 1], kw
        c = 2 ** -0.5
        assert np.all(r.lo[1] <= c) and np.all(c <= r.hi[1]) and np.all(r.lo[0] <= -c) and np.all(-c <= r.hi[0])
    for n in (3, 4):
        s = W.product_linear([4, n], n=n)
        for kw in ({"contractor": KRAW}, {"inclusion": 1}):
            r = oracle.solve(s, **kw)
            _check_known_roots(r, s.roots, n)
            assert int(r.tag.sum()) == len(s.roots), kw
    # planted roots of the dense workload stay enclosed
    s = W.dense_planted(0, n=4, n_terms=6, max_deg=2)
    for kw in ({"contractor": KRAW}, {"inclusion": 1}):
        r = oracle.solve(s, **kw)
        assert r.status == 0
        for x in s.roots:
            assert any(np.all(r.lo[b] <= x) and np.all(x <= r.hi[b]) for b in range(len(r.tag))), kw


def test_invalid_variant_codes_are_rejected():
    import oracle
    s = W.circle_line()
    assert oracle.solve(s, contractor=2).status == oracle.ERR_INVALID_ARG
    assert oracle.solve(s, inclusion=3).status == oracle.ERR_INVALID_ARG
