"""Writes the oracle's results for full-size workloads to tests/golden/expected_*.json.

Calls only the CPU oracle (oracle/) and the input generators (workloads/); the
GPU tests compare the device search against these files bit for bit.  Floats
are stored as hex strings (float.hex) so that they round-trip exactly.

    python tests/golden/make_expected.py dense6_s0 banded12_s0 ...
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

CASES = {
    # dense planted, n=6, 20 monomials of degree 1..3 + constant, [-2,2]^6, tol 1e-8
    "dense6_s0": lambda: (W.dense_planted(0), {}),
    # 16.8 million tree nodes: above the oracle's default budget
    "dense6_s1": lambda: (W.dense_planted(1), {"max_boxes": 50_000_000}),
    # banded, n=12, [-1,1]^12, tol 1e-10
    "banded12_s0": lambda: (W.banded(0), {}),
    "banded12_s1": lambda: (W.banded(1), {}),
}


def run(name):
    s, kw = CASES[name]()
    t = time.time()
    r = oracle.solve(s, **kw)
    dt = time.time() - t
    out = {
        "case": name, "system": s.name, "status": r.status, "stats": r.stats, "oracle_seconds": round(dt, 2),
        "lo": [[float(v).hex() for v in row] for row in r.lo],
        "hi": [[float(v).hex() for v in row] for row in r.hi],
        "tag": [int(v) for v in r.tag],
    }
    # boxes stepped while (or when becoming) proven: the proof chains
    out["chains"] = [[[float(v).hex() for v in a] for a in c] for c in oracle.proof_chains(s, **kw)]
    with open(os.path.join(HERE, f"expected_{name}.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(name, r.status, r.stats, f"{dt:.1f}s", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        run(name)
