"""Generators for the polynomial systems used throughout the repository.

A system is stored in sparse monomial form:

* ``n``         number of variables = number of equations;
* ``term_off``  int32[n+1], equation ``i`` owns terms ``term_off[i]:term_off[i+1]``;
* ``expo``      uint8[T, n], exponent vector of each term;
* ``coef``      float64[T], coefficient of each term;
* ``lo, hi``    float64[n], the initial box;
* ``tol``       the box-width tolerance.

Workload recipes (all seeded, PCG64 via ``numpy.random.default_rng``):

* circle/line, n=2: x^2+y^2-1, x-y on [-2,2]^2, tol 1e-6 (two known roots).
* dense planted, n=6: per equation 20 distinct monomials of total degree 1..3
  drawn without replacement, coefficients U[-1,1], plus a constant term that
  makes a planted root r ~ U[-1,1]^6 exact up to one rounding; redrawn while
  cond(J(r)) > 1e8; box [-2,2]^6, tol 1e-8.
* banded, n=12: f_i = a_i x_i + b_i x_i^3 + 1 - sum_{1<=|j-i|<=2} c_ij (x_j + x_j^2),
  a~U[2,3], b~U[4,6], c~U[0.5,1.5]; box [-1,1]^12, tol 1e-10.
* batch: n~U{2..12}, degree D~U{2,3,4}, m~U{5..30} monomials of total degree
  1..D per equation (capped at the number that exist), coefficients U[-1,1],
  one planted root; box [-2,2]^n, tol 1e-8.  System k of a batch draws from
  ``default_rng([seed, k])``.
* product of quadratics, n~U{4..8}: q_k=(x_k-r_k)(x_k-s_k) for k<min(n,6),
  q_k = x_k - r_k otherwise, mixed as f = A q with cond(A) <= 10, so the system
  has 2^min(n,6) planted roots; box [-2,2]^n.
* served stream: Poisson arrivals mixing banded systems (tol 1e-8) and
  product systems.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from fractions import Fraction
from typing import List, Optional, Sequence

import numpy as np


@dataclass
class System:
    n: int
    term_off: np.ndarray  # int32 [n+1]
    expo: np.ndarray      # uint8 [T, n]
    coef: np.ndarray      # float64 [T]
    lo: np.ndarray        # float64 [n]
    hi: np.ndarray        # float64 [n]
    tol: float
    name: str = ""
    roots: List[np.ndarray] = field(default_factory=list)  # planted roots (approximate)

    @property
    def n_terms(self) -> int:
        return int(self.coef.shape[0])

    def equations(self):
        """Yield (coef, expo) arrays per equation."""
        for i in range(self.n):
            a, b = int(self.term_off[i]), int(self.term_off[i + 1])
            yield self.coef[a:b], self.expo[a:b]


_LIBC = None


def _require_nearest():
    """The generators round with the floating-point unit's current mode; a
    mode other than round-to-nearest (left behind by some native library)
    would change the coefficients, so it is refused."""
    global _LIBC
    if _LIBC is None:
        import ctypes
        _LIBC = ctypes.CDLL(None)
    if _LIBC.fegetround() != 0:  # FE_TONEAREST
        raise RuntimeError("workloads: the floating-point rounding mode is not round-to-nearest")


def _pack(n: int, eqs: Sequence[Sequence[tuple]], lo, hi, tol, name, roots=()) -> System:
    """eqs[i] is a list of (coef, exponent tuple) in stored order."""
    _require_nearest()
    term_off = np.zeros(n + 1, dtype=np.int32)
    coefs, expos = [], []
    for i, terms in enumerate(eqs):
        term_off[i + 1] = term_off[i] + len(terms)
        for c, a in terms:
            coefs.append(float(c))
            expos.append(tuple(int(x) for x in a))
    return System(
        n=n,
        term_off=term_off,
        expo=np.array(expos, dtype=np.uint8).reshape(len(expos), n),
        coef=np.array(coefs, dtype=np.float64),
        lo=np.full(n, float(lo)) if np.isscalar(lo) else np.asarray(lo, dtype=np.float64),
        hi=np.full(n, float(hi)) if np.isscalar(hi) else np.asarray(hi, dtype=np.float64),
        tol=float(tol),
        name=name,
        roots=[np.asarray(r, dtype=np.float64) for r in roots],
    )


def _exponents(n: int, max_deg: int) -> List[tuple]:
    """All exponent vectors of total degree 1..max_deg (graded, then lexicographic)."""
    out = []
    for d in range(1, max_deg + 1):
        for combo in itertools.combinations_with_replacement(range(n), d):
            a = [0] * n
            for k in combo:
                a[k] += 1
            out.append(tuple(a))
    return out


def _planted_constant(coefs, expos, r) -> float:
    """-(sum_t c_t r^alpha_t), exact in rationals, rounded once to nearest."""
    rf = [Fraction(float(x)) for x in r]
    maxp = max((max(a) for a in expos), default=0)
    pw = [[Fraction(1)] for _ in rf]
    for k, x in enumerate(rf):
        for _ in range(maxp):
            pw[k].append(pw[k][-1] * x)
    s = Fraction(0)
    for c, a in zip(coefs, expos):
        t = Fraction(float(c))
        for k, p in enumerate(a):
            if p:
                t *= pw[k][p]
        s += t
    return float(-s)


def _jacobian_at(n, eqs, r) -> np.ndarray:
    """Point Jacobian in float64 (used only to reject ill-conditioned draws)."""
    J = np.zeros((n, n))
    for i, terms in enumerate(eqs):
        for c, a in terms:
            for k in range(n):
                if a[k] == 0:
                    continue
                v = c * a[k]
                for m in range(n):
                    e = a[m] - (1 if m == k else 0)
                    if e:
                        v *= r[m] ** e
                J[i, k] += v
    return J


def circle_line() -> System:
    """x^2 + y^2 - 1 = 0, x - y = 0 on [-2,2]^2; roots +-(1/sqrt2, 1/sqrt2)."""
    eqs = [
        [(1.0, (2, 0)), (1.0, (0, 2)), (-1.0, (0, 0))],
        [(1.0, (1, 0)), (-1.0, (0, 1))],
    ]
    s = 0.5 ** 0.5
    return _pack(2, eqs, -2.0, 2.0, 1e-6, "circle_line", roots=[[s, s], [-s, -s]])


def _random_planted(rng, n, max_deg, n_terms_fn, box, tol, name, max_cond=1e8, tries=64):
    allexp = _exponents(n, max_deg)
    for _ in range(tries):
        eqs = []
        for _i in range(n):
            m = min(n_terms_fn(), len(allexp))
            idx = rng.choice(len(allexp), size=m, replace=False)
            c = rng.uniform(-1.0, 1.0, size=m)
            eqs.append([(float(c[j]), allexp[int(idx[j])]) for j in range(m)])
        r = rng.uniform(-1.0, 1.0, size=n)
        J = _jacobian_at(n, eqs, r)
        if not np.all(np.isfinite(J)) or np.linalg.cond(J) > max_cond:
            continue
        for i in range(n):
            c0 = _planted_constant([t[0] for t in eqs[i]], [t[1] for t in eqs[i]], r)
            eqs[i].append((c0, (0,) * n))
        return _pack(n, eqs, -box, box, tol, name, roots=[r])
    raise RuntimeError("could not draw a well-conditioned planted system")


def dense_planted(seed: int, n: int = 6, n_terms: int = 20, max_deg: int = 3,
                  box: float = 2.0, tol: float = 1e-8) -> System:
    rng = np.random.default_rng(seed)
    return _random_planted(rng, n, max_deg, lambda: n_terms, box, tol,
                           f"dense_planted(n={n},seed={seed})")


def banded(seed: int, n: int = 12, tol: float = 1e-10, half_band: int = 2) -> System:
    rng = np.random.default_rng(seed)
    a = rng.uniform(2.0, 3.0, size=n)
    b = rng.uniform(4.0, 6.0, size=n)
    c = rng.uniform(0.5, 1.5, size=(n, n))
    eqs = []
    for i in range(n):
        e = lambda k, p: tuple(p if m == k else 0 for m in range(n))  # noqa: E731
        terms = [(a[i], e(i, 1)), (b[i], e(i, 3)), (1.0, (0,) * n)]
        for j in range(max(0, i - half_band), min(n, i + half_band + 1)):
            if j == i:
                continue
            terms.append((-c[i, j], e(j, 1)))
            terms.append((-c[i, j], e(j, 2)))
        eqs.append(terms)
    return _pack(n, eqs, -1.0, 1.0, tol, f"banded(n={n},seed={seed})")


def batch_planted(seed: int = 0, count: int = 4096, n_range=(2, 12), deg_range=(2, 4),
                  terms_range=(5, 30), box: float = 2.0, tol: float = 1e-8,
                  indices: Optional[Sequence[int]] = None) -> List[System]:
    out = []
    ks = range(count) if indices is None else indices
    for k in ks:
        rng = np.random.default_rng([seed, int(k)])
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        D = int(rng.integers(deg_range[0], deg_range[1] + 1))
        s = _random_planted(rng, n, D, lambda: int(rng.integers(terms_range[0], terms_range[1] + 1)),
                            box, tol, f"batch(seed={seed},k={k},n={n},D={D})")
        out.append(s)
    return out


def product_linear(seed, n: Optional[int] = None, tol: float = 1e-8, box: float = 2.0,
                   n_quad_max: int = 6) -> System:
    """f = A q with q_k = (x_k - r_k)(x_k - s_k) (k < min(n,6)) or x_k - r_k."""
    rng = np.random.default_rng(seed)
    if n is None:
        n = int(rng.integers(4, 9))
    nq = min(n, n_quad_max)
    r = rng.uniform(-1.5, 1.5, size=n)
    s = np.empty(n)
    for k in range(n):
        while True:
            s[k] = rng.uniform(-1.5, 1.5)
            if abs(s[k] - r[k]) >= 0.1:
                break
    while True:
        A = rng.uniform(-1.0, 1.0, size=(n, n)) + np.diag(rng.choice([-3.0, 3.0], size=n))
        if np.linalg.cond(A) <= 10.0:
            break
    F = Fraction
    eqs = []
    for i in range(n):
        terms = []
        const = F(0)
        for k in range(n):
            aik = F(float(A[i, k]))
            e1 = tuple(1 if m == k else 0 for m in range(n))
            if k < nq:
                e2 = tuple(2 if m == k else 0 for m in range(n))
                terms.append((float(aik), e2))
                terms.append((float(-aik * (F(float(r[k])) + F(float(s[k])))), e1))
                const += aik * F(float(r[k])) * F(float(s[k]))
            else:
                terms.append((float(aik), e1))
                const -= aik * F(float(r[k]))
        terms.append((float(const), (0,) * n))
        eqs.append(terms)
    roots = []
    for bits in itertools.product((0, 1), repeat=nq):
        x = r.copy()
        for k in range(nq):
            if bits[k]:
                x[k] = s[k]
        roots.append(x)
    return _pack(n, eqs, -box, box, tol, f"product(n={n},seed={seed})", roots=roots)


def univariate(coefs_low_to_high, lo, hi, tol=1e-9, name="univariate") -> System:
    """p(x) = sum_k c_k x^k as a 1-variable system."""
    terms = [(float(c), (k,)) for k, c in enumerate(coefs_low_to_high) if c != 0 or k == 0]
    return _pack(1, [terms], lo, hi, tol, name)


def served_stream(seed: int = 0, rate: float = 2000.0, duration: float = 10.0,
                  tol: float = 1e-8, max_requests: Optional[int] = None):
    """Poisson request stream: list of (arrival_seconds, System)."""
    rng = np.random.default_rng([seed, 0x5E5])
    t = 0.0
    out = []
    k = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration or (max_requests is not None and k >= max_requests):
            break
        if rng.random() < 0.5:
            s = banded(seed=int(1_000_000 + seed * 100_003 + k), tol=tol)
        else:
            s = product_linear(seed=[seed, 7, k], tol=tol)
        out.append((t, s))
        k += 1
    return out
