"""The 4096-system batch at full size (n 2..12, degree 2..4, 5..30 monomials per
equation, box [-2,2]^n, tol 1e-8, 100,000 tree nodes per member) in the
configuration the bench times: autotuned launch configuration, replayed from a
recorded graph.  Sampled members equal the oracle one by one; every member that
completes encloses its planted root; the eager call equals the replay."""
import numpy as np
import pytest

import workloads as W
from tests.parity import assert_same

pytestmark = pytest.mark.gpu

BUDGET = 100_000


@pytest.fixture(scope="module")
def full_batch(gpu_ctx):
    import paper_1802_00330_amd as P
    systems = W.batch_planted(0, count=4096)
    params = [P.make_params(s.tol, max_boxes=BUDGET) for s in systems]
    try:
        print(f"[fullsize-batch] tuning", flush=True)
        P.ibb_batch_tune(gpu_ctx, systems, params, sample=128)
        print(f"[fullsize-batch] eager", flush=True)
        eager = P.ibb_solve_batch(gpu_ctx, systems, params)
        print(f"[fullsize-batch] plan", flush=True)
        plan = P.BatchPlan(gpu_ctx, systems, params)
        try:
            plan.run()
            replay = plan.run()
        finally:
            plan.close()
    finally:
        for q in range(4):
            P.ibb_batch_set_config(gpu_ctx, q, 2 << q)
    return systems, eager, replay


def test_replay_equals_eager(full_batch):
    systems, eager, replay = full_batch
    for k, (a, b) in enumerate(zip(eager, replay)):
        assert a.status == b.status and a.stats == b.stats, k
        assert np.array_equal(a.lo.view(np.uint64), b.lo.view(np.uint64)), k
        assert np.array_equal(a.hi.view(np.uint64), b.hi.view(np.uint64)), k
        assert np.array_equal(a.tag, b.tag), k


def test_completed_members_enclose_their_planted_root(full_batch):
    import paper_1802_00330_amd as P
    systems, _, replay = full_batch
    done = 0
    for s, r in zip(systems, replay):
        assert r.status in (P.OK, P.ERR_BUDGET), (s.name, r.status)
        if r.status != P.OK:
            assert len(r.tag) == 0
            continue
        done += 1
        assert r.stats["processed"] <= BUDGET
        for root in s.roots:
            # the planted root is exact up to the rounding of the constant terms
            inside = np.all((r.lo <= root + 1e-12) & (root - 1e-12 <= r.hi), axis=1)
            assert inside.any(), (s.name, root)
    print(f"[fullsize-batch] {done} of {len(systems)} members completed within the budget", flush=True)
    assert done > 0


def _sample(systems, replay, rng):
    """A few completed members per lane-count class (trees the oracle walks in
    seconds) and one member over the budget."""
    import paper_1802_00330_amd as P
    picks = []
    for lo_n, hi_n in ((2, 2), (3, 4), (5, 8), (9, 12)):
        ok = [k for k, (s, r) in enumerate(zip(systems, replay))
              if lo_n <= s.n <= hi_n and r.status == P.OK and r.stats["processed"] <= 30_000]
        if ok:
            picks += [int(k) for k in rng.choice(ok, size=min(3, len(ok)), replace=False)]
    over = [k for k, (s, r) in enumerate(zip(systems, replay)) if r.status == P.ERR_BUDGET and s.n <= 4]
    if over:
        picks.append(int(rng.choice(over)))
    return picks


def test_sampled_members_equal_oracle(full_batch, oracle_lib):
    import paper_1802_00330_amd as P
    systems, _, replay = full_batch
    picks = _sample(systems, replay, np.random.default_rng(2024))
    assert len(picks) >= 4
    for k in picks:
        s = systems[k]
        print(f"[fullsize-batch] oracle on member {k} ({s.name})", flush=True)
        ref = oracle_lib.solve(s, max_boxes=BUDGET)
        if ref.status != 0:
            assert replay[k].status == P.ERR_BUDGET and ref.status == P.ERR_BUDGET, k
            continue
        assert_same(replay[k], ref, f"member {k}")
