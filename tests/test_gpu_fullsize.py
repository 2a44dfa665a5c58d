"""Full-size workloads on the device against the oracle's stored results
(written by tests/golden/make_expected.py, which calls only the oracle):
bit-identical sorted box lists and tree counters."""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# the dense n=6 and banded n=12 workloads, seeds 0..4 (up to 16.8 million
# tree nodes per solve); seed 0 also with the Krawczyk contractor and with the
# mean-value exclusion test
CASES = {}
for _k in range(5):
    CASES[f"dense6_s{_k}"] = ((lambda k: lambda: W.dense_planted(k))(_k), {})
    CASES[f"banded12_s{_k}"] = ((lambda k: lambda: W.banded(k))(_k), {})
for _name, _mk in (("dense6", W.dense_planted), ("banded12", W.banded)):
    CASES[f"{_name}_s0_krawczyk"] = ((lambda mk: lambda: mk(0))(_mk), {"contractor": 1})
    CASES[f"{_name}_s0_meanvalue"] = ((lambda mk: lambda: mk(0))(_mk), {"inclusion": 1})


def _load(name):
    path = os.path.join(GOLD, f"expected_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle result {path}")
    return json.load(open(path))


@pytest.mark.parametrize("name", sorted(CASES))
def test_full_size_matches_stored_oracle(gpu_ctx, name):
    import paper_1802_00330_amd as P
    g = _load(name)
    make, kw = CASES[name]
    s = make()
    print(f"[fullsize] {name}: {g['stats']['processed']} nodes", flush=True)
    r = P.solve(gpu_ctx, s, **kw)
    assert r.status == g["status"] == 0
    assert r.stats == g["stats"]
    lo = np.array([[float.fromhex(v) for v in row] for row in g["lo"]]).reshape(-1, s.n)
    hi = np.array([[float.fromhex(v) for v in row] for row in g["hi"]]).reshape(-1, s.n)
    assert np.array_equal(r.lo.view(np.uint64), lo.view(np.uint64))
    assert np.array_equal(r.hi.view(np.uint64), hi.view(np.uint64))
    assert r.tag.tolist() == g["tag"]
