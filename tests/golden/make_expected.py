"""Writes the oracle's results for full-size workloads to tests/golden/expected_*.json.

Calls only the CPU oracle (oracle/) and the input generators (workloads/); the
GPU tests compare the device search against these files bit for bit.  Floats
are stored as hex strings (float.hex) so that they round-trip exactly.

    python tests/golden/make_expected.py dense6_s0 banded12_s0 ...
    python tests/golden/make_expected.py served_s0
    python tests/golden/make_expected.py dense6_s0_krawczyk dense6_s0_meanvalue ...

Cases other than the first four store no proof chains (computing them solves
the system a second time).  ``served_s0`` stores the first SERVED_PICK banded
(n=12, tol 1e-8) and the first SERVED_PICK product requests of the served
stream with seed 0, each solved alone.
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
# further seeds of the same two workloads (no proof chains)
for _k in (2, 3, 4):
    CASES[f"dense6_s{_k}"] = (lambda k: lambda: (W.dense_planted(k), {"max_boxes": 50_000_000}))(_k)
    CASES[f"banded12_s{_k}"] = (lambda k: lambda: (W.banded(k), {"max_boxes": 50_000_000}))(_k)
# the Krawczyk contractor and the mean-value exclusion test on seed 0
for _k in ("dense6", "banded12"):
    _mk = W.dense_planted if _k == "dense6" else W.banded
    CASES[f"{_k}_s0_krawczyk"] = (lambda mk: lambda: (mk(0), {"contractor": 1, "max_boxes": 50_000_000}))(_mk)
    CASES[f"{_k}_s0_meanvalue"] = (lambda mk: lambda: (mk(0), {"inclusion": 1, "max_boxes": 50_000_000}))(_mk)
WITH_CHAINS = {"dense6_s0", "dense6_s1", "banded12_s0", "banded12_s1"}
SERVED_PICK = 6
SERVED_SCAN = 40


def _pack(r):
    return {"status": r.status, "stats": r.stats,
            "lo": [[float(v).hex() for v in row] for row in r.lo],
            "hi": [[float(v).hex() for v in row] for row in r.hi],
            "tag": [int(v) for v in r.tag]}


def served_picks(seed=0):
    """Indices into served_stream(seed, max_requests=SERVED_SCAN): the first
    SERVED_PICK banded and the first SERVED_PICK product requests."""
    st = W.served_stream(seed, max_requests=SERVED_SCAN)
    banded = [k for k, (_, s) in enumerate(st) if s.name.startswith("banded")][:SERVED_PICK]
    prod = [k for k, (_, s) in enumerate(st) if not s.name.startswith("banded")][:SERVED_PICK]
    return st, sorted(banded + prod)


def _served_one(args):
    seed, k = args
    st = W.served_stream(seed, max_requests=SERVED_SCAN)
    s = st[k][1]
    t = time.time()
    r = oracle.solve(s)
    return k, s.name, time.time() - t, _pack(r)


def run_served(seed=0):
    from multiprocessing import Pool
    _, picks = served_picks(seed)
    with Pool(min(len(picks), max(1, (os.cpu_count() or 2) - 1))) as pool:
        res = pool.map(_served_one, [(seed, k) for k in picks])
    out = {"case": f"served_s{seed}", "scan": SERVED_SCAN, "requests": []}
    for k, name, dt, rec in res:
        rec.update({"index": k, "system": name, "oracle_seconds": round(dt, 2)})
        out["requests"].append(rec)
        print(k, name, rec["status"], rec["stats"]["processed"], f"{dt:.1f}s", flush=True)
    with open(os.path.join(HERE, f"expected_served_s{seed}.json"), "w") as fh:
        json.dump(out, fh, indent=1)


def run(name):
    s, kw = CASES[name]()
    t = time.time()
    r = oracle.solve(s, **kw)
    dt = time.time() - t
    out = {"case": name, "system": s.name, "oracle_seconds": round(dt, 2), **_pack(r)}
    if name in WITH_CHAINS:
        # boxes stepped while (or when becoming) proven: the proof chains
        out["chains"] = [[[float(v).hex() for v in a] for a in c] for c in oracle.proof_chains(s, **kw)]
    with open(os.path.join(HERE, f"expected_{name}.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(name, r.status, r.stats, f"{dt:.1f}s", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        if name.startswith("served_s"):
            run_served(int(name[len("served_s"):]))
        else:
            run(name)
