"""The library's backtracking merge (ibb_backtrack, host code of libibb.so)
against the oracle's (oracle/backtrack.py): identical cell counts at every
round and identical cells, on the stored output lists of the dense n=6 and
banded n=12 workloads, the circle/line system, and random boxes with ends on
grid lines.  Host-only: runs without a GPU."""
import glob
import json
import math
import os
import random
import re

import numpy as np
import pytest

import workloads as W
from oracle import backtrack as OB

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lib():
    import paper_1802_00330_amd as P
    try:
        P.load_library()
    except (RuntimeError, OSError) as e:
        pytest.skip(f"libibb.so not loadable here: {e}")
    return P


def start_level(lo, hi, x0lo, x0hi):
    """The finest round whose cells are at least as wide as every box in every
    coordinate (each box then meets at most two cells per coordinate)."""
    k = 50
    for l, h, a, b in zip(np.ravel(lo), np.ravel(hi), np.tile(x0lo, len(lo)), np.tile(x0hi, len(lo))):
        w = h - l
        if w > 0:
            k = min(k, int(math.floor(math.log2((b - a) / w))))
    return max(0, k)


def _compare(P, lo, hi, x0lo, x0hi, level, what):
    counts, cells = P.ibb_backtrack(lo, hi, x0lo, x0hi, level)
    ref = OB.backtrack(lo.tolist(), hi.tolist(), list(x0lo), list(x0hi), level)
    assert counts.tolist() == [len(ref[k]) for k in range(level + 1)], what
    assert [tuple(c) for c in cells.tolist()] == ref[level], what
    k = max(0, level // 2)
    _, mid = P.ibb_backtrack(lo, hi, x0lo, x0hi, level, out_level=k)
    assert [tuple(c) for c in mid.tolist()] == ref[k], what
    return counts


CASES = sorted(p for p in glob.glob(os.path.join(GOLD, "expected_*_s*.json")) if "served" not in p)


@pytest.mark.parametrize("path", CASES, ids=[os.path.basename(p) for p in CASES])
def test_stored_outputs(path):
    P = _lib()
    g = json.load(open(path))
    seed = int(re.search(r"_s(\d+)", g["case"]).group(1))
    s = (W.dense_planted if g["case"].startswith("dense") else W.banded)(seed)
    lo = np.array([[float.fromhex(v) for v in row] for row in g["lo"]]).reshape(-1, s.n)
    hi = np.array([[float.fromhex(v) for v in row] for row in g["hi"]]).reshape(-1, s.n)
    level = start_level(lo, hi, s.lo, s.hi)
    counts = _compare(P, lo, hi, s.lo, s.hi, level, g["case"])
    assert counts[0] == 1 and all(counts[k - 1] <= counts[k] for k in range(1, level + 1))


def test_circle_line_paper_mode(oracle_lib):
    """The paper's setting: every coordinate bisected (Alg. 2) and no
    contraction, so the output boxes are grid cells; merging them stops
    changing at the two roots +-(1/sqrt 2, 1/sqrt 2)."""
    P = _lib()
    s = W.circle_line()
    r = oracle_lib.solve(s, split_mode=oracle_lib.SPLIT_ALL, hs_max_width=0.0)
    level = start_level(r.lo, r.hi, s.lo, s.hi)
    counts = _compare(P, r.lo, r.hi, s.lo, s.hi, level, "circle_line")
    k = OB.cluster_level(counts.tolist())
    assert counts[k] == 2 and k > 10, counts.tolist()


def test_random_boxes_on_grid_lines():
    P = _lib()
    rng = random.Random(11)
    for trial in range(60):
        n = rng.randrange(1, 5)
        x0lo = np.array([rng.choice([-2.0, -1.0, -0.3, 0.0]) for _ in range(n)])
        x0hi = x0lo + np.array([rng.choice([4.0, 2.0, 1.7, 0.5]) for _ in range(n)])
        level = rng.randrange(0, 9)
        m = rng.randrange(0, 12)
        lo = np.zeros((m, n))
        hi = np.zeros((m, n))
        for b in range(m):
            for i in range(n):
                a, c = x0lo[i], x0hi[i]
                grid = [a + (c - a) * j / (1 << level) for j in range((1 << level) + 1)]

                def pick():
                    return rng.choice(grid) if rng.random() < 0.4 else a + (c - a) * rng.random()

                # a box at most about three cells wide, ends often on grid lines
                u = pick()
                j = rng.randrange(len(grid))
                v = grid[j] if rng.random() < 0.4 and grid[j] >= u else u + (c - a) / (1 << level) * rng.choice(
                    [0.0, 0.3, 1.0, 2.5])
                if v - u > 3.0 * (c - a) / (1 << level):
                    v = u
                lo[b, i], hi[b, i] = max(a, u), min(c, v)
        _compare(P, lo, hi, x0lo, x0hi, level, f"trial {trial}")


def test_invalid_arguments():
    P = _lib()
    x0lo, x0hi = np.array([-1.0, -1.0]), np.array([1.0, 1.0])
    with pytest.raises(RuntimeError):  # box outside X0
        P.ibb_backtrack(np.array([[-2.0, 0.0]]), np.array([[0.0, 0.5]]), x0lo, x0hi, 3)
    with pytest.raises(RuntimeError):  # level above the maximum
        P.ibb_backtrack(np.zeros((1, 2)), np.zeros((1, 2)), x0lo, x0hi, 51)
    with pytest.raises(RuntimeError):  # empty initial range
        P.ibb_backtrack(np.zeros((1, 2)), np.zeros((1, 2)), x0lo, x0lo, 3)
    counts, cells = P.ibb_backtrack(np.zeros((0, 2)), np.zeros((0, 2)), x0lo, x0hi, 4)
    assert counts.tolist() == [0] * 5 and cells.shape == (0, 2)
