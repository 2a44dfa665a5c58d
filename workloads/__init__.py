"""Seeded synthetic polynomial systems shared by the oracle tests, the GPU
parity tests and the benchmark.

This module only *builds inputs*: sparse monomial systems (exponent vectors and
FP64 coefficients), initial boxes and tolerances.  It contains none of the
interval method's arithmetic.  Where a root is planted, the constant term is
computed exactly with rationals and rounded once to the nearest double.
"""
from .systems import (  # noqa: F401
    System,
    circle_line,
    dense_planted,
    banded,
    batch_planted,
    product_linear,
    univariate,
    served_stream,
)
