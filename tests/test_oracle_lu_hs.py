"""Pins for the single-precision approximate inverse (Sec. 2.3's B ~ inv(J_c),
Alg. 3 second step) and for the Hansen-Sengupta step (eq 17-22, Alg. 3)."""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from tests.exact import F, poly_value


# ---------------------------------------------------------------- inverse
def test_inverse_is_inverse(oracle_lib):
    rng = np.random.default_rng(0)
    for n in range(1, 17):
        for _ in range(5):
            M = rng.uniform(-1, 1, size=(n, n)) + np.diag(rng.uniform(1, 2, size=n) * rng.choice([-1, 1], n))
            Mf = M.astype(np.float32)
            Y = oracle_lib.fp32_inverse(Mf)
            assert Y is not None
            E = Y.astype(np.float64) @ Mf.astype(np.float64) - np.eye(n)
            E2 = Mf.astype(np.float64) @ Y.astype(np.float64) - np.eye(n)
            assert np.abs(E).max() < 1e-4 and np.abs(E2).max() < 1e-4


def test_inverse_exact_for_scaled_permutations(oracle_lib):
    """M = P D with power-of-two D: every operation is exact, so Y = D^-1 P^T."""
    rng = np.random.default_rng(1)
    for n in range(1, 13):
        perm = rng.permutation(n)
        d = 2.0 ** rng.integers(-4, 5, size=n) * rng.choice([-1, 1], n)
        M = np.zeros((n, n), dtype=np.float32)
        for i in range(n):
            M[i, perm[i]] = d[i]
        Y = oracle_lib.fp32_inverse(M)
        expect = np.linalg.inv(M.astype(np.float64))
        assert np.array_equal(Y.astype(np.float64), expect)


def test_inverse_exact_for_unit_triangular_dyadic(oracle_lib):
    """Unit lower-triangular with small dyadic entries: the inverse is integral
    times dyadics and every step is exact in single precision."""
    L = np.array([[1, 0, 0], [0.5, 1, 0], [-0.25, 2, 1]], dtype=np.float32)
    Y = oracle_lib.fp32_inverse(L)
    assert np.array_equal(Y.astype(np.float64), np.linalg.inv(L.astype(np.float64)))
    U = L.T.copy()
    Y = oracle_lib.fp32_inverse(U)
    assert np.array_equal(Y.astype(np.float64), np.linalg.inv(U.astype(np.float64)))


def test_inverse_pivoting_handles_zero_leading_entry(oracle_lib):
    M = np.array([[0, 1], [1, 0]], dtype=np.float32)
    assert np.array_equal(oracle_lib.fp32_inverse(M), M)
    M = np.array([[0, 2, 0], [0, 0, 4], [8, 0, 0]], dtype=np.float32)
    assert np.array_equal(oracle_lib.fp32_inverse(M).astype(np.float64), np.linalg.inv(M.astype(np.float64)))


def test_inverse_rejects_singular_and_nonfinite(oracle_lib):
    assert oracle_lib.fp32_inverse(np.zeros((3, 3), np.float32)) is None
    assert oracle_lib.fp32_inverse(np.array([[1, 2], [2, 4]], np.float32)) is None
    M = np.eye(3, dtype=np.float32)
    M[1, 2] = np.inf
    assert oracle_lib.fp32_inverse(M) is None
    M = np.eye(2, dtype=np.float32) * 1e30
    M[0, 1] = 3e38
    assert oracle_lib.fp32_inverse(M) is None or np.all(np.isfinite(oracle_lib.fp32_inverse(M)))


# ---------------------------------------------------------------- HS step
def _linear(A, b, lo, hi):
    """System A x - b = 0 as monomials."""
    n = len(b)
    eqs = []
    for i in range(n):
        eq = [(float(A[i][k]), tuple(1 if m == k else 0 for m in range(n))) for k in range(n) if A[i][k] != 0]
        eq.append((float(-b[i]), (0,) * n))
        eqs.append(eq)
    return W.systems._pack(n, eqs, lo, hi, 1e-9, "linear")


def test_hs_diagonal_linear_is_tight_and_unique(oracle_lib):
    A = [[4.0, 0.0], [0.0, -2.0]]
    b = [1.0, 3.0]  # x = 0.25, y = -1.5 exactly
    s = _linear(A, b, -2.0, 2.0)
    st, lo, hi, u = oracle_lib.hs(s, s.lo, s.hi)
    assert st == oracle_lib.HS_DONE and u
    assert lo.tolist() == [0.25, -1.5] and hi.tolist() == [0.25, -1.5]


def test_hs_linear_contains_solution_and_proves_uniqueness(oracle_lib):
    rng = np.random.default_rng(2)
    for trial in range(40):
        n = int(rng.integers(1, 9))
        A = np.round((rng.uniform(-1, 1, size=(n, n)) + np.diag(rng.uniform(3, 4, n))) * 16) / 16
        xs = np.round(rng.uniform(-1, 1, size=n) * 64) / 64
        b = A @ xs  # exact: short dyadics
        s = _linear(A, b, -2.0, 2.0)
        st, lo, hi, u = oracle_lib.hs(s, s.lo, s.hi)
        assert st == oracle_lib.HS_DONE
        assert np.all(lo <= xs) and np.all(xs <= hi)
        assert u  # diagonally dominant: the contraction lands strictly inside
        assert np.all(hi - lo < 1e-3)


def test_hs_sqrt2(oracle_lib):
    s = W.univariate([-2.0, 0.0, 1.0], 1.0, 2.0)
    lo, hi = np.array([1.0]), np.array([2.0])
    proven = False
    for _ in range(6):
        st, lo, hi, u = oracle_lib.hs(s, lo, hi)
        assert st == oracle_lib.HS_DONE
        assert F(lo[0]) ** 2 <= 2 <= F(hi[0]) ** 2
        proven = proven or u
    # proven on an early step (strictly inside); at machine resolution the
    # enclosure can no longer land strictly inside, so later steps do not prove
    assert proven and hi[0] - lo[0] < 1e-14


def test_hs_excludes_rootless_box(oracle_lib):
    s = _linear([[1.0]], [5.0], 0.0, 1.0)
    st, *_ = oracle_lib.hs(s, s.lo, s.hi)
    assert st == oracle_lib.HS_EMPTY


def test_hs_zero_derivative_uses_extended_division(oracle_lib):
    """x^2 - 1/4 on [-1,1]: mid J = 0 -> preconditioner unusable -> skipped;
    on [-1, 0.75] the point x = -0.125 gives J(X) containing 0."""
    s = W.univariate([-0.25, 0.0, 1.0], -1.0, 1.0)
    st, *_ = oracle_lib.hs(s, np.array([-1.0]), np.array([1.0]))
    assert st == oracle_lib.HS_SKIPPED
    st, lo, hi, u = oracle_lib.hs(s, np.array([-1.0]), np.array([0.75]))
    assert st == oracle_lib.HS_DONE and not u
    # both roots are kept
    assert lo[0] <= -0.5 and 0.5 <= hi[0]


def test_hs_keeps_all_roots_of_product_systems(oracle_lib):
    """Soundness: every root inside X is inside HS(X); a box proven unique holds
    exactly one root."""
    rng = np.random.default_rng(4)
    checked = 0
    for trial in range(25):
        s = W.product_linear(seed=[9, trial], n=int(rng.integers(2, 5)))
        for _ in range(8):
            c = rng.uniform(-1.5, 1.5, size=s.n)
            w = rng.uniform(0.05, 1.0, size=s.n)
            lo, hi = c - w, c + w
            st, nlo, nhi, u = oracle_lib.hs(s, lo, hi)
            inside = [r for r in s.roots if np.all(lo <= r) and np.all(r <= hi)]
            if st == oracle_lib.HS_EMPTY:
                assert not any(np.all(lo + 1e-9 <= r) and np.all(r <= hi - 1e-9) for r in inside)
                continue
            if st == oracle_lib.HS_SKIPPED:
                continue
            for r in inside:
                # planted roots are exact only up to coefficient rounding
                assert np.all(nlo <= r + 1e-9) and np.all(r - 1e-9 <= nhi)
            if u:
                assert len([r for r in s.roots if np.all(nlo - 1e-9 <= r) and np.all(r <= nhi + 1e-9)]) == 1
            checked += 1
    assert checked > 50


def test_hs_gauss_seidel_uses_updated_components(oracle_lib):
    """x0 - 1/2 = 0, x1 - x0 = 0 on [-4,4]^2: the sweep first narrows X0 to
    {1/2}; with that update X1 narrows to {1/2} in the same step (a Jacobi
    sweep would give X1 = [-4,4] - ...)."""
    A = [[1.0, 0.0], [-1.0, 1.0]]
    s = _linear(A, [0.5, 0.0], -4.0, 4.0)
    st, lo, hi, u = oracle_lib.hs(s, s.lo, s.hi)
    assert st == oracle_lib.HS_DONE
    assert lo.tolist() == [0.5, 0.5] and hi.tolist() == [0.5, 0.5]
