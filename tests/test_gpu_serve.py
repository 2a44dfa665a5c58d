"""Serving: requests arriving while others run share the device (continuous
batching); each result equals the oracle's on that request alone."""
import numpy as np
import pytest

import workloads as W
from tests.parity import assert_same

pytestmark = pytest.mark.gpu


def _requests():
    out = []
    for k in range(12):
        if k % 3 == 0:
            out.append(W.product_linear([8, k], n=3 + (k % 4)))
        elif k % 3 == 1:
            out.append(W.banded(100 + k, n=4 + (k % 5), tol=1e-8))
        else:
            out.append(W.dense_planted(k, n=4, n_terms=6, max_deg=2))
    return out


def test_served_mix_equals_alone(gpu_ctx, oracle_lib):
    import paper_1802_00330_amd as P
    reqs = _requests()
    srv = P.Server(gpu_ctx, max_slots=8, frontier_cap=1 << 16, reserve_per_solve=1 << 12, levels_per_quantum=3)
    ids = {}
    results = {}
    pending = list(range(len(reqs)))
    rounds = 0
    while pending or len(results) < len(reqs):
        # a few arrivals per round, while earlier requests are still running
        for _ in range(3):
            if pending:
                k = pending.pop(0)
                ids[srv.submit(reqs[k])] = k
        srv.step()
        rounds += 1
        for rid, k in list(ids.items()):
            r = srv.poll(rid)
            if r is not None:
                results[k] = r
                del ids[rid]
        assert rounds < 10000
    print(f"[serve] {len(reqs)} requests in {rounds} rounds", flush=True)
    for k, s in enumerate(reqs):
        assert_same(results[k], oracle_lib.solve(s), s.name)
    srv.close()


def test_admission_waits_for_memory(gpu_ctx, oracle_lib):
    """With room for one reservation per bucket, requests are admitted one at a
    time and still finish with the right results."""
    import paper_1802_00330_amd as P
    reqs = [W.product_linear([9, k], n=3) for k in range(3)]
    srv = P.Server(gpu_ctx, max_slots=4, frontier_cap=1 << 12, reserve_per_solve=1 << 12, levels_per_quantum=4)
    ids = [srv.submit(s) for s in reqs]
    srv.step()
    q, a = srv.pending()
    assert a == 1 and q == 2
    done = {}
    for _ in range(10000):
        srv.step()
        for rid in ids:
            if rid not in done:
                r = srv.poll(rid)
                if r is not None:
                    done[rid] = r
        if len(done) == len(ids):
            break
    for rid, s in zip(ids, reqs):
        assert_same(done[rid], oracle_lib.solve(s), s.name)
    srv.close()
