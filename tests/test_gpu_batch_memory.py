"""Batched solves under a bound on device memory: a batch whose frontier does
not fit is solved in parts with the same results member by member; a member
whose widest level alone exceeds the bound fails alone; a plan (never split)
reports the shortage."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

# any bound below what 2^16 frontier boxes need leaves the floor of 2^16 boxes
TINY = 1 << 20
FLOOR = 1 << 16


def _same(a, b, what):
    assert a.status == b.status, f"{what}: status {a.status} != {b.status}"
    assert a.lo.shape == b.lo.shape, f"{what}: {a.lo.shape} != {b.lo.shape}"
    assert np.array_equal(a.lo.view(np.uint64), b.lo.view(np.uint64)), what
    assert np.array_equal(a.hi.view(np.uint64), b.hi.view(np.uint64)), what
    assert np.array_equal(a.tag, b.tag), what
    assert a.stats == b.stats, f"{what}: {a.stats} != {b.stats}"


def _wide_members(P, ctx, want=2):
    """Complete members of the mixed batch workload whose widest tree level
    holds between 2^12 and 2^16 boxes (from single solves)."""
    found = []
    widths = []
    for s in W.batch_planted(0, indices=range(64)):
        if not 3 <= s.n <= 8:
            continue
        p = P.make_params(s.tol, max_boxes=300_000)
        r = P.ibb_solve(ctx, s, p)
        widths.append((s.n, r.status, r.max_frontier))
        if r.status == P.OK and 4096 <= r.max_frontier < FLOOR:
            found.append((s, p, r.max_frontier))
            if len(found) == want:
                return found
    pytest.fail(f"no member with a widest level in [2^12, 2^16): {widths}")


@pytest.fixture()
def ctx():
    import paper_1802_00330_amd as P
    c = P.Context(0)  # its own context: the bound and learned capacities stay here
    yield c
    c.close()


def test_batch_split_equals_unbounded(ctx):
    import paper_1802_00330_amd as P
    wide = _wide_members(P, ctx)
    small = [W.circle_line(), W.product_linear([5, 1], n=3), W.banded(0, n=6, tol=1e-8)]
    systems, params = [], []
    for s, p, w in wide:
        copies = FLOOR // w + 2  # together wider than the floor at their widest level
        print(f"[batch-mem] {s.name}: widest {w}, {copies} copies", flush=True)
        for _ in range(copies):
            systems.append(s)
            params.append(p)
            k = len(systems) % len(small)
            systems.append(small[k])
            params.append(P.make_params(small[k].tol))
    # a member wider than the floor on its own: the dense n=6 system (widest
    # level 669,077 boxes)
    big = W.dense_planted(0)
    systems.insert(3, big)
    params.insert(3, P.make_params(big.tol))
    free = P.ibb_solve_batch(ctx, systems, params)
    assert all(r.status == P.OK for r in free)
    P.ibb_batch_set_memory(ctx, TINY)
    try:
        # cap 1: the first part overflows the output, the second only sizes its
        # own; the binding retries with the total
        bounded = P.ibb_solve_batch(ctx, systems, params, cap=1)
        for k, (a, b) in enumerate(zip(bounded, free)):
            if k == 3:
                assert a.status == P.ERR_QUEUE_OVERFLOW and len(a.tag) == 0
            else:
                _same(a, b, f"bounded[{k}] {systems[k].name}")
        # the same under measured queue sizes (parts chosen before the run)
        P.ibb_batch_tune(ctx, systems, params, sample=4)
        tuned = P.ibb_solve_batch(ctx, systems, params)
        for k, (a, b) in enumerate(zip(tuned, bounded)):
            _same(a, b, f"tuned[{k}] {systems[k].name}")
        # a plan is one batch: the shortage is reported, not split
        rest = systems[:3] + systems[4:]
        rest_p = params[:3] + params[4:]
        with pytest.raises(RuntimeError, match="out of memory"):
            P.BatchPlan(ctx, rest, rest_p).run()
    finally:
        P.ibb_batch_set_memory(ctx, 0)
    again = P.ibb_solve_batch(ctx, systems, params)
    for k, (a, b) in enumerate(zip(again, free)):
        _same(a, b, f"unbounded again[{k}]")


def test_batch_set_memory_rejects_negative(ctx):
    import paper_1802_00330_amd as P
    with pytest.raises(RuntimeError, match="invalid"):
        P.ibb_batch_set_memory(ctx, -1)
    P.ibb_batch_set_memory(ctx, 0)
