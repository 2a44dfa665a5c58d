"""Serving the mixed request stream: banded n=12 systems (16 lanes per box,
tol 1e-8) and product systems (n 4..8) of the served stream with seed 0,
submitted in arrival order a few per scheduling round so that they run
together on the device.  Each result must equal the oracle's result for that
request solved alone (tests/golden/expected_served_s0.json, written by
tests/golden/make_expected.py, which calls only the oracle)."""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "expected_served_s0.json")


def _stored():
    if not os.path.exists(GOLD):
        pytest.skip("no stored served results")
    g = json.load(open(GOLD))
    stream = W.served_stream(0, max_requests=g["scan"])
    return [(stream[r["index"]][1], r) for r in g["requests"]]


def _check(res, s, g):
    assert res.status == g["status"] == 0, (s.name, res.status)
    assert res.stats == g["stats"], (s.name, res.stats, g["stats"])
    lo = np.array([[float.fromhex(v) for v in row] for row in g["lo"]]).reshape(-1, s.n)
    hi = np.array([[float.fromhex(v) for v in row] for row in g["hi"]]).reshape(-1, s.n)
    assert np.array_equal(res.lo.view(np.uint64), lo.view(np.uint64)), s.name
    assert np.array_equal(res.hi.view(np.uint64), hi.view(np.uint64)), s.name
    assert res.tag.tolist() == g["tag"], s.name


def _serve(srv, systems, per_round=2, params=None):
    ids, out, pending, rounds = {}, {}, list(range(len(systems))), 0
    while pending or ids:
        for _ in range(per_round):
            if pending:
                k = pending.pop(0)
                ids[srv.submit(systems[k], None if params is None else params[k])] = k
        srv.step()
        rounds += 1
        for rid, k in list(ids.items()):
            r = srv.poll(rid)
            if r is not None:
                out[k] = r
                del ids[rid]
        assert rounds < 100000
    return out, rounds


def test_served_stream_banded12_and_products_equal_alone():
    import paper_1802_00330_amd as P
    cases = _stored()
    ctx = P.Context(0)
    srv = P.Server(ctx, max_slots=16, levels_per_quantum=4)
    systems = [s for s, _ in cases]
    print(f"[serve-stream] {len(systems)} requests: " + ", ".join(s.name for s in systems), flush=True)
    out, rounds = _serve(srv, systems)
    print(f"[serve-stream] done in {rounds} rounds", flush=True)
    for k, (s, g) in enumerate(cases):
        _check(out[k], s, g)
    srv.close()
    ctx.close()


def test_served_request_over_budget_fails_alone():
    """One request of the mix gets a node budget below its tree size: it ends
    with ERR_BUDGET, and its neighbours still equal their solves alone."""
    import paper_1802_00330_amd as P
    cases = _stored()
    # a banded request (16-lane bucket) and a product request (8-lane bucket)
    # share their buckets with the one that fails
    pick = [k for k, (s, g) in enumerate(cases) if g["stats"]["processed"] < 1_000_000][:6]
    systems = [cases[k][0] for k in pick]
    victim = 0
    budget = cases[pick[victim]][1]["stats"]["processed"] // 3
    params = [P.make_params(s.tol) for s in systems]
    params[victim] = P.make_params(systems[victim].tol, max_boxes=budget)
    ctx = P.Context(0)
    srv = P.Server(ctx, max_slots=16, levels_per_quantum=4)
    out, _ = _serve(srv, systems, per_round=3, params=params)
    assert out[victim].status == P.ERR_BUDGET
    for j, k in enumerate(pick):
        if j != victim:
            _check(out[j], *cases[k])
    srv.close()
    ctx.close()
