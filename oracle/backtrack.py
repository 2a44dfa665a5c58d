"""Backtracking merge of output boxes into cells of the bisection grid (Alg. 5).

TEST INFRASTRUCTURE (part of the oracle): only ``tests/`` and the CPU legs of
``bench.py`` may import this module; the library never calls it.

Alg. 5 maps a box of round k of the all-coordinate bisection (Alg. 2) to the
box of round k-1 it was split from, coordinate by coordinate, and drops the
duplicates; repeating it merges the tiny output boxes into a few "readable"
cells, one per isolated root once the count stops changing (Tab. 3, 6, 8).
The printed case split of Alg. 5 is garbled; the reading taken here: a
round-k interval of width w lies in the round-(k-1) grid of width 2w either as
the lower half (its lower end is a multiple of 2w from the grid origin) or as
the upper half, and its parent is [lo, lo + 2w] or [hi - 2w, hi] accordingly.
On integer cell indices (cell j of round k covers
[a + j (b-a)/2^k, a + (j+1) (b-a)/2^k] in a coordinate whose initial range is
[a, b]) that is j -> floor(j / 2).

Output boxes of a contracting solver are not grid cells, so each box first
becomes the set of round-`level` cells it meets: per coordinate the cells
whose interior meets the box's interior (a degenerate coordinate: the cell
[B_j, B_{j+1}) holding the point, the last cell closed).  Every computation
is exact (rationals); the reference for the library's ibb_backtrack.
"""
from fractions import Fraction
from itertools import product
from typing import Dict, List, Sequence, Tuple


def _index(x: Fraction, a: Fraction, w: Fraction, level: int) -> int:
    """The j with B_j <= x < B_{j+1}, B_j = a + j w / 2^level, clamped to the
    grid (x = b falls in the last cell)."""
    j = (x - a) * (1 << level) // w  # floor of an exact rational
    return max(0, min((1 << level) - 1, int(j)))


def coordinate_cells(lo: float, hi: float, a: float, b: float, level: int) -> range:
    """Indices of the round-`level` cells of [a, b] that the interval [lo, hi] meets."""
    A, B, L, H = Fraction(a), Fraction(b), Fraction(lo), Fraction(hi)
    w = B - A
    j0 = _index(L, A, w, level)
    if L == H:
        return range(j0, j0 + 1)
    j1 = _index(H, A, w, level)
    # an upper end on a grid line touches the next cell only in a face point
    if A + j1 * w / (1 << level) == H and j1 > j0:
        j1 -= 1
    return range(j0, j1 + 1)


def box_cells(box_lo: Sequence[float], box_hi: Sequence[float], x0_lo: Sequence[float],
              x0_hi: Sequence[float], level: int) -> List[Tuple[int, ...]]:
    """All round-`level` cells (index tuples) that the box meets."""
    ranges = [coordinate_cells(l, h, a, b, level) for l, h, a, b in zip(box_lo, box_hi, x0_lo, x0_hi)]
    return [tuple(c) for c in product(*ranges)]


def parent(cell: Tuple[int, ...]) -> Tuple[int, ...]:
    """Alg. 5 on cell indices: the round-(k-1) cell a round-k cell came from."""
    return tuple(j // 2 for j in cell)


def backtrack(boxes_lo, boxes_hi, x0_lo, x0_hi, level: int) -> Dict[int, List[Tuple[int, ...]]]:
    """Distinct cells at every round k = level, level-1, ..., 0: the boxes'
    round-`level` cells, then Alg. 5 applied round after round with the
    duplicates removed.  Returns {k: sorted cells}."""
    cells = set()
    for lo, hi in zip(boxes_lo, boxes_hi):
        for c in box_cells(lo, hi, x0_lo, x0_hi, level):
            cells.add(c)
    out = {level: sorted(cells)}
    for k in range(level, 0, -1):
        cells = {parent(c) for c in cells}
        out[k - 1] = sorted(cells)
    return out


def cluster_level(counts: Sequence[int]) -> int:
    """The round at which the paper stops merging: scanning from the finest
    round toward the root, the first round k whose count equals that of round
    k-1 (the count has stopped changing); 0 if none.  counts[k] is the number
    of cells at round k."""
    for k in range(len(counts) - 1, 0, -1):
        if counts[k] == counts[k - 1]:
            return k
    return 0
