"""Pins of the oracle's backtracking merge (Alg. 5, oracle/backtrack.py)."""
import os
import random
from fractions import Fraction

import pytest

from oracle import backtrack as B

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "backtrack_tables.txt")


def _paper_parent(lo: Fraction, hi: Fraction):
    """Alg. 5 for one interval of a grid cell, as read (the printed case split
    swapped): with the parent width w = 2 (hi - lo), the interval is the lower
    half of its parent when lo / w is an integer, else the upper half."""
    w = 2 * (hi - lo)
    if (lo / w).denominator == 1:
        return lo, lo + w
    assert (hi / w).denominator == 1
    return hi - w, hi


@pytest.mark.parametrize("c,level", [(1, 2), (1, 5), (8, 3), (32, 7), (2, 30)])
def test_parent_index_equals_the_papers_interval_formula(c, level):
    """On the grids of the paper's symmetric initial boxes [-c, c] (Tab. 1-8),
    the index map j -> j // 2 gives the parent interval of Alg. 5."""
    rng = random.Random(level * 1000 + c)
    a, b = Fraction(-c), Fraction(c)
    w = (b - a) / (1 << level)
    for _ in range(200):
        j = rng.randrange(1 << level)
        lo, hi = a + j * w, a + (j + 1) * w
        plo, phi = _paper_parent(lo, hi)
        p = B.parent((j,))[0]
        assert (plo, phi) == (a + p * 2 * w, a + (p + 1) * 2 * w), (j, lo, hi)


def test_worked_example():
    """X0 = [-2, 2]^2, round 3 (cells 0.5 wide): the box [0.1, 0.2] x [-0.3, 0.6]
    meets cells 4 (x) and 3, 4, 5 (y); merging gives 3, 2, 2, 1 cells at
    rounds 3, 2, 1, 0."""
    out = B.backtrack([[0.1, -0.3]], [[0.2, 0.6]], [-2.0, -2.0], [2.0, 2.0], 3)
    assert out[3] == [(4, 3), (4, 4), (4, 5)]
    assert out[2] == [(2, 1), (2, 2)]
    assert out[1] == [(1, 0), (1, 1)]
    assert out[0] == [(0, 0)]


def test_grid_cells_map_to_themselves():
    x0lo, x0hi = [-1.0, -8.0, 0.0], [1.0, 8.0, 3.0]
    level = 4
    for j in ((0, 0, 0), (15, 15, 15), (7, 8, 3), (8, 7, 12)):
        lo = [a + k * (b - a) / 16 for k, a, b in zip(j, x0lo, x0hi)]
        hi = [a + (k + 1) * (b - a) / 16 for k, a, b in zip(j, x0lo, x0hi)]
        assert B.box_cells(lo, hi, x0lo, x0hi, level) == [j]
    # a point on a grid line belongs to the cell above it; the upper end of X0
    # to the last cell
    assert list(B.coordinate_cells(0.0, 0.0, -1.0, 1.0, 3)) == [4]
    assert list(B.coordinate_cells(1.0, 1.0, -1.0, 1.0, 3)) == [7]
    assert list(B.coordinate_cells(-1.0, -1.0, -1.0, 1.0, 3)) == [0]


def test_coordinate_cells_by_brute_force():
    """Against the definition, cell by cell in exact arithmetic: a
    non-degenerate interval meets cell j when the open interiors meet; a point
    lies in the half-open cell [B_j, B_{j+1}) (the last cell closed)."""
    rng = random.Random(7)
    for _ in range(400):
        a = rng.choice([-2.0, -1.0, -0.75, 0.0, -3.3])
        b = a + rng.choice([4.0, 2.0, 1.5, 0.1, 3.7])
        level = rng.randrange(0, 6)
        m = 1 << level
        w = (Fraction(b) - Fraction(a)) / m
        grid = [Fraction(a) + k * w for k in range(m + 1)]

        def pick():
            if rng.random() < 0.4:  # a grid line, as far as a double can hold it
                return float(grid[rng.randrange(m + 1)])
            return a + (b - a) * rng.random()

        x, y = sorted((pick(), pick()))
        if rng.random() < 0.15:
            y = x
        X, Y = Fraction(x), Fraction(y)
        if X == Y:
            want = [j for j in range(m) if grid[j] <= X < grid[j + 1] or (j == m - 1 and X == grid[m])]
        else:
            want = [j for j in range(m) if grid[j] < Y and X < grid[j + 1]]
        assert list(B.coordinate_cells(x, y, a, b, level)) == want, (x, y, a, b, level)


def test_merge_invariants():
    rng = random.Random(3)
    n, level = 3, 9
    x0lo, x0hi = [-2.0] * n, [2.0] * n
    boxes_lo, boxes_hi = [], []
    for _ in range(30):
        c = [rng.uniform(-1.9, 1.9) for _ in range(n)]
        r = [rng.uniform(0.0, 0.01) for _ in range(n)]
        boxes_lo.append([u - v for u, v in zip(c, r)])
        boxes_hi.append([u + v for u, v in zip(c, r)])
    out = B.backtrack(boxes_lo, boxes_hi, x0lo, x0hi, level)
    counts = [len(out[k]) for k in range(level + 1)]
    assert counts[0] == 1
    assert all(counts[k - 1] <= counts[k] for k in range(1, level + 1))
    # every box lies inside the union of its cells, at every round
    for k in range(level + 1):
        cells = set(out[k])
        w = [Fraction(b - a) / (1 << k) for a, b in zip(x0lo, x0hi)]
        for lo, hi in zip(boxes_lo, boxes_hi):
            mine = B.box_cells(lo, hi, x0lo, x0hi, k)
            assert set(mine) <= cells
            for i in range(n):
                js = sorted({c[i] for c in mine})
                assert Fraction(x0lo[i]) + js[0] * w[i] <= Fraction(lo[i])
                assert Fraction(hi[i]) <= Fraction(x0lo[i]) + (js[-1] + 1) * w[i]


def test_cluster_level_reads_the_papers_tables():
    """Tab. 3, 6, 8: the count at the round where it stops changing is the
    number of isolated roots the text states."""
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        name, roots, *seq = line.split()
        counts = [int(v) for v in seq][::-1]  # index = round, coarsest first
        k = B.cluster_level(counts)
        assert counts[k] == counts[k - 1] == int(roots), name
        # every finer round still had more boxes
        assert all(counts[j] > counts[j - 1] for j in range(k + 1, len(counts))), name
