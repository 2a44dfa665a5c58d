"""Exact-rational helpers for the CPU pins (independent of the oracle's code).

``round_down(q)``/``round_up(q)`` give the largest/smallest double below/above a
rational, i.e. the IEEE-754 roundTowardNegative/Positive of an exact value.
"""
import math
from fractions import Fraction

DBL_MAX = Fraction(1.7976931348623157e308)


def round_down(q: Fraction) -> float:
    if q > DBL_MAX:
        return 1.7976931348623157e308
    if q < -DBL_MAX:
        return -math.inf
    d = float(q)  # nearest
    if Fraction(d) > q:
        d = math.nextafter(d, -math.inf)
    return d


def round_up(q: Fraction) -> float:
    return -round_down(-q)


def F(x) -> Fraction:
    return Fraction(float(x))


def poly_value(coefs, expos, point):
    """Exact value of sum_t c_t prod_k x_k^e_tk at a rational point."""
    s = Fraction(0)
    for c, e in zip(coefs, expos):
        t = F(c)
        for k, p in enumerate(e):
            if p:
                t *= point[k] ** int(p)
        s += t
    return s
