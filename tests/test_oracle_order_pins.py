"""Pins of the oracle's operation orders that rounding makes visible.

Each case below has an expected result derived by hand in exact arithmetic,
step by step, with every single-precision or double-precision rounding stated.
The inputs are chosen so that the plausible alternative order gives different
bits; each docstring names that alternative and what it would give.

* The approximate inverse of mid J (Sec. 2.3, the matrix B; Alg. 3, second
  step): LU with partial pivoting that takes the FIRST row of largest
  magnitude, forward substitution over j ascending, back substitution
  subtracting the terms for j from n-1 down.
* Powers (Def. 1, evaluated with eq 27's directed products): each bound of X^p
  is a left-to-right chain t <- R(t * x) of p-1 products, not a chain of
  squarings.

fl() below is single-precision round-to-nearest-even; 2^k is a power of two.
"""
import numpy as np


def _bits32(a):
    return np.asarray(a, dtype=np.float32).view(np.uint32)


# ------------------------------------------------------------ pivot tie-break
def test_inverse_pivot_tie_takes_first_row(oracle_lib):
    """M = [[1, 1], [-1, 2]]: column 0 has |1| = |-1|, a tie.

    First row (the reading): no exchange.  l = -1/1 = -1 exactly and
    U = [[1, 1], [0, 2 - (-1)(1)]] = [[1, 1], [0, 3]] exactly.
      column 0: z = (1, 0 - (-1)(1)) = (1, 1); x1 = fl(1/3).
        1/3 = 1.0101...b x 2^-2; 24 significant bits round up (the bits
        after the 23rd fraction bit are 1010..., above one half):
        fl(1/3) = 11184811 x 2^-25.
        x0 = fl(1 - 11184811 x 2^-25) = fl(22369621 x 2^-25); 22369621 has 25
        bits, halfway between 22369620 and 22369622: ties to even,
        22369620 x 2^-25 = 11184810 x 2^-24.
      column 1: z = (0, 1); x1 = 11184811 x 2^-25; x0 = -x1.
      Y = [[11184810 x 2^-24, -11184811 x 2^-25],
           [11184811 x 2^-25,  11184811 x 2^-25]].
    Last row (the alternative): rows exchanged, [[-1, 2], [1, 1]], l = -1,
    U22 = 1 - (-1)(2) = 3; column 0 then has z = (0, 1), x1 = fl(1/3) and
    x0 = fl((0 - 2 x1) / -1) = 11184811 x 2^-24, one unit above.
    """
    M = np.array([[1, 1], [-1, 2]], dtype=np.float32)
    Y = oracle_lib.fp32_inverse(M)
    expect = np.array([[11184810 * 2.0 ** -24, -11184811 * 2.0 ** -25],
                       [11184811 * 2.0 ** -25, 11184811 * 2.0 ** -25]], dtype=np.float32)
    assert np.array_equal(_bits32(Y), _bits32(expect))
    # the other tie-break's value differs in the last bit
    assert np.float32(11184811 * 2.0 ** -24) != Y[0, 0]


# ------------------------------------------------------ substitution orders
def test_inverse_back_substitution_runs_j_descending(oracle_lib):
    """U = [[1, a, b, 1], [0, 1, 0, d], [0, 0, 1, e], [0, 0, 0, 1]] with
    a = e = 2^-13, b = d = 2^-12 (upper triangular: the LU is U itself, every
    multiplier 0, and forward substitution gives z = e_c exactly).

    Column 3: x3 = 1; x2 = (0 - e x3)/1 = -2^-13; x1 = (0 - d x3)/1 = -2^-12.
    x0 = 0 - b x2 - a x1 - 1 x3 with a x1 = b x2 = -2^-25 (exact products).
    Descending j (the reading): t = 0 - 1 = -1; t = fl(-1 + 2^-25): halfway
    between -1 and -(1 - 2^-24), ties to the even -1; t = fl(-1 + 2^-25) = -1
    again, so Y[0][3] = -1.
    Ascending j (the alternative): t = 2^-25; t = 2^-25 + 2^-25 = 2^-24;
    t = 2^-24 - 1 = -(1 - 2^-24) exactly, a different value.
    """
    a = e = 2.0 ** -13
    b = d = 2.0 ** -12
    U = np.array([[1, a, b, 1], [0, 1, 0, d], [0, 0, 1, e], [0, 0, 0, 1]], dtype=np.float32)
    Y = oracle_lib.fp32_inverse(U)
    assert Y[0, 3] == np.float32(-1.0)
    assert np.float32(-(1 - 2.0 ** -24)) != np.float32(-1.0)
    # the other entries are exact: column 3 rows 1..3 as derived above
    assert Y[1, 3] == np.float32(-2.0 ** -12) and Y[2, 3] == np.float32(-2.0 ** -13) and Y[3, 3] == 1


def test_inverse_forward_substitution_runs_j_ascending(oracle_lib):
    """L = [[1, 0, 0, 0], [a, 1, 0, 0], [b, 0, 1, 0], [1, d, e, 1]] with
    a = e = 2^-13, b = d = 2^-12.  Column 0 holds 1, a, b, 1: a tie between
    rows 0 and 3, resolved to row 0 (no exchange); every later pivot is the
    unit diagonal, and elimination leaves the entries unchanged (the row
    subtracted has zeros there), so the factors are L and U = I.

    Column 0 of L z = e_0: z0 = 1, z1 = 0 - a = -2^-13, z2 = 0 - b = -2^-12,
    z3 = 0 - 1 z0 - d z1 - e z2 with d z1 = e z2 = -2^-25.
    Ascending j (the reading): t = -1, then fl(-1 + 2^-25) = -1 twice (ties
    to even), z3 = -1.  Descending j (the alternative): t = 2^-25, 2^-24,
    then 2^-24 - 1 = -(1 - 2^-24).  Back substitution with U = I only
    subtracts zero products, so Y[3][0] = z3 = -1.
    """
    a = e = 2.0 ** -13
    b = d = 2.0 ** -12
    L = np.array([[1, 0, 0, 0], [a, 1, 0, 0], [b, 0, 1, 0], [1, d, e, 1]], dtype=np.float32)
    Y = oracle_lib.fp32_inverse(L)
    assert Y[3, 0] == np.float32(-1.0)
    assert Y[1, 0] == np.float32(-2.0 ** -13) and Y[2, 0] == np.float32(-2.0 ** -12) and Y[0, 0] == 1


# ---------------------------------------------------------------- power chain
def test_power_is_a_left_to_right_chain(oracle_lib):
    """x = 2^27 + 1, X = [x, x], p = 4.  A double has 53 significant bits.

    Lower bound, t <- R(t x) rounded down:
      x^2 = 2^54 + 2^28 + 1 (unit in the last place 4 at 2^54): 2^54 + 2^28
      t x = 2^81 + 3 2^54 + 2^28 (ulp 2^29):                2^81 + 3 2^54
      t x = 2^108 + 2^83 + 3 2^54 (ulp 2^56):               2^108 + 2^83
    Upper bound, rounded up:
      x^2 -> 2^54 + 2^28 + 4
      t x = 2^81 + 3 2^54 + 3 2^28 + 4 -> 2^81 + 3 2^54 + 2^30
      t x = 2^108 + 2^83 + 2^57 + 3 2^54 + 2^30 -> 2^108 + 2^83 + 3 2^56
    Squaring (the alternative), s = x^2 rounded, then s^2 rounded:
      lower (2^54 + 2^28)^2 = 2^108 + 2^83 + 2^56 (exact), one unit higher;
      upper (2^54 + 2^28 + 4)^2 = 2^108 + 2^83 + 3 2^56 + 2^31 + 16
            -> 2^108 + 2^83 + 4 2^56, one unit higher.
    Both enclose x^4 = 2^108 + 2^83 + 6 2^54 + 2^29 + 1.
    """
    x = 2.0 ** 27 + 1
    lo, hi = oracle_lib.i_pow((x, x), 4)
    assert lo == 2.0 ** 108 + 2.0 ** 83
    assert hi == 2.0 ** 108 + 2.0 ** 83 + 3 * 2.0 ** 56
    # odd power of a negative point: the same chain on |x|, negated and swapped
    lo3, hi3 = oracle_lib.i_pow((-x, -x), 3)
    # |x|^3 rounded down: 2^81 + 3 2^54; rounded up: 2^81 + 3 2^54 + 2^30
    assert lo3 == -(2.0 ** 81 + 3 * 2.0 ** 54 + 2.0 ** 30)
    assert hi3 == -(2.0 ** 81 + 3 * 2.0 ** 54)
