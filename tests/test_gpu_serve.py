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


def _run(srv, ids, rounds=10000):
    done = {}
    for _ in range(rounds):
        srv.step()
        for rid in srv.finished():
            done[rid] = srv.poll(rid)
        if len(done) == len(ids):
            break
    return done


def _bucket_bytes(G, cap):
    """Device bytes of a bucket frontier of cap boxes (two levels of boxes,
    records and system indices), as the server counts them."""
    return cap * 2 * (16 * G + 8) + 4096


def test_admission_waits_for_memory(gpu_ctx, oracle_lib):
    """With a device pool that holds one request's reservation, requests are
    admitted one at a time and still finish with the right results.  A
    product system of n=3 on [-2,2]^3 at tol 1e-8 needs at least
    3 * ceil(log2(4 / 1e-8)) = 87 bisections, so it reserves 2 * 4096 boxes of
    four lanes: two levels of 16,384 boxes."""
    import paper_1802_00330_amd as P
    reqs = [W.product_linear([9, k], n=3) for k in range(3)]
    initial = sum(_bucket_bytes(G, 1 << 12) for G in (2, 4, 8, 16))
    one = _bucket_bytes(4, 2 * 2 * 4096) - 4096
    pool = max(initial, one + one // 2)
    assert pool < 2 * one
    srv = P.Server(gpu_ctx, max_slots=4, frontier_cap=1 << 12, reserve_per_solve=1 << 12, levels_per_quantum=4,
                   pool_bytes=pool)
    ids = [srv.submit(s) for s in reqs]
    srv.step()
    q, a = srv.pending()
    assert a == 1 and q == 2
    done = _run(srv, ids)
    for rid, s in zip(ids, reqs):
        assert_same(done[rid], oracle_lib.solve(s), s.name)
    srv.close()


def test_request_outgrowing_the_pool_fails_alone(gpu_ctx, oracle_lib):
    """A banded n=12 request whose levels (up to 35,564 boxes) cannot fit the
    device pool fails alone with IBB_ERR_QUEUE_OVERFLOW; the product requests
    served beside it equal their solves alone."""
    import paper_1802_00330_amd as P
    big = W.banded(1)
    small = [W.product_linear([9, k], n=3 + k % 2) for k in range(4)]
    initial = sum(_bucket_bytes(G, 1 << 12) for G in (2, 4, 8, 16))
    pool = initial + (3 << 20)
    assert _bucket_bytes(16, 2 * 35564) > pool
    srv = P.Server(gpu_ctx, max_slots=8, frontier_cap=1 << 12, reserve_per_solve=1 << 8, levels_per_quantum=4,
                   pool_bytes=pool)
    ids = [srv.submit(big)] + [srv.submit(s) for s in small]
    done = _run(srv, ids)
    assert done[ids[0]].status == P.ERR_QUEUE_OVERFLOW
    for rid, s in zip(ids[1:], small):
        assert_same(done[rid], oracle_lib.solve(s), s.name)
    # the server goes on: the pool is free again for a request that fits
    rid = srv.submit(small[0])
    assert_same(_run(srv, [rid])[rid], oracle_lib.solve(small[0]), "after the failure")
    srv.close()
