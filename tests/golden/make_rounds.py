"""Writes the oracle's per-round kept-box counts for the paper's worked examples
(all coordinates bisected, no contraction) to tests/golden/oracle_rounds.json.
Calls only the CPU oracle: the kept boxes of round r are the children of the
kept boxes of round r-1 (each bisected in every coordinate, Alg. 2) that pass
the exclusion test (Def. 2), tested in C by oracle.exclusion_keep; the last
round is only counted.   python tests/golden/make_rounds.py [last_round]"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from tests.golden_systems import load  # noqa: E402


def children(lo, hi):
    """All 2^n children of each box (exact midpoints: the boxes are dyadic)."""
    m, n = lo.shape
    mid = (lo + hi) / 2
    bits = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(bool)  # [2^n, n]
    clo = np.where(bits[None], mid[:, None], lo[:, None]).reshape(-1, n)
    chi = np.where(bits[None], hi[:, None], mid[:, None]).reshape(-1, n)
    return clo, chi


def rounds(name, last, chunk=256):
    s, _ = load(name)
    lo, hi = s.lo[None].copy(), s.hi[None].copy()
    out = {1: 1}
    for rnd in range(2, last + 1):
        kept_lo, kept_hi, count = [], [], 0
        for a in range(0, lo.shape[0], chunk):
            clo, chi = children(lo[a:a + chunk], hi[a:a + chunk])
            keep = oracle.exclusion_keep(s, clo, chi)
            count += int(keep.sum())
            if rnd < last:
                kept_lo.append(clo[keep])
                kept_hi.append(chi[keep])
        out[rnd] = count
        print(name, rnd, count, flush=True)
        if rnd < last:
            lo, hi = np.concatenate(kept_lo), np.concatenate(kept_hi)
    return out


if __name__ == "__main__":
    last = int(sys.argv[1]) if len(sys.argv) > 1 else 5
    res = {name: rounds(name, last) for name in ("katsura8", "noon9", "kinema")}
    with open(os.path.join(HERE, "oracle_rounds.json"), "w") as fh:
        json.dump(res, fh, indent=1)
