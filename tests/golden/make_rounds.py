"""Writes the oracle's per-round kept-box counts for the paper's worked examples
(all coordinates bisected, no contraction) to tests/golden/oracle_rounds.json.
Calls only the CPU oracle.   python tests/golden/make_rounds.py [last_round]"""
import itertools
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from tests.golden_systems import load  # noqa: E402


def rounds(name, last):
    s, _ = load(name)
    level = [(s.lo.copy(), s.hi.copy())]
    out = {1: 1}
    for rnd in range(2, last + 1):
        nxt = []
        for lo, hi in level:
            mid = (lo + hi) / 2  # exact: dyadic boxes
            for bits in itertools.product((0, 1), repeat=s.n):
                b = np.array(bits, dtype=bool)
                clo, chi = np.where(b, mid, lo), np.where(b, hi, mid)
                flo, fhi = oracle.eval_F(s, clo, chi)
                if np.all(flo <= 0) and np.all(fhi >= 0):
                    nxt.append((clo, chi))
        level = nxt
        out[rnd] = len(level)
        print(name, rnd, len(level), flush=True)
    return out


if __name__ == "__main__":
    last = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    res = {name: rounds(name, last) for name in ("katsura8", "noon9", "kinema")}
    with open(os.path.join(HERE, "oracle_rounds.json"), "w") as fh:
        json.dump(res, fh, indent=1)
