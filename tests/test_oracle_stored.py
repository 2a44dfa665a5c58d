"""The stored oracle results are reproducible: re-running the oracle's single
contraction step on the stored proof-chain boxes gives the stored boxes (a
check that the oracle computes the same on any host)."""
import json
import os

import numpy as np
import pytest

import workloads as W

MAKERS = {"dense6_s0": lambda: W.dense_planted(0), "dense6_s1": lambda: W.dense_planted(1),
          "banded12_s0": lambda: W.banded(0), "banded12_s1": lambda: W.banded(1)}


# the stored results that carry proof chains (make_expected.py stores them for
# the cases of MAKERS only)
PATHS = [os.path.join(os.path.dirname(__file__), "golden", f"expected_{k}.json") for k in sorted(MAKERS)]


@pytest.mark.parametrize("path", PATHS)
def test_stored_chains_reproduce(oracle_lib, path):
    g = json.load(open(path))
    assert "chains" in g, path
    s = MAKERS[g["case"]]()
    for k, c in enumerate(g["chains"]):
        lo, hi, elo, ehi = (np.array([float.fromhex(v) for v in a]) for a in c)
        st, nlo, nhi, u = oracle_lib.hs(s, lo, hi)
        bad = np.nonzero((nlo != elo) | (nhi != ehi))[0]
        assert bad.size == 0, (g["case"], k, [(int(i), float(nlo[i]).hex(), float(elo[i]).hex(),
                                               float(nhi[i]).hex(), float(ehi[i]).hex()) for i in bad[:4]])
