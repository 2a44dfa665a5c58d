"""Batched solves: many systems of different sizes in one pass; each system's
result (box list, tags, counters, status) equals the oracle's on it alone."""
import numpy as np
import pytest

import workloads as W
from tests.parity import assert_same

pytestmark = pytest.mark.gpu


def _mixed_systems():
    out = [W.circle_line()]
    out += [W.product_linear([5, k], n=n) for k, n in enumerate([2, 3, 4, 5, 6, 2, 3])]
    out += [W.dense_planted(k, n=4, n_terms=6, max_deg=2) for k in range(4)]
    out += [W.dense_planted(0, n=5, n_terms=8, max_deg=3)]
    out += [W.banded(k, n=n, tol=1e-8) for k, n in enumerate([4, 6, 8, 9, 12])]
    out += W.batch_planted(0, indices=[9, 11])
    out += [W.univariate(np.poly([0.3, -1.1, 1.7])[::-1], -2.0, 2.0, tol=1e-10)]
    return out


def test_batch_equals_oracle_per_system(gpu_ctx, oracle_lib):
    import paper_1802_00330_amd as P
    systems = _mixed_systems()
    print(f"[batch] {len(systems)} systems", flush=True)
    res = P.ibb_solve_batch(gpu_ctx, systems)
    for s, r in zip(systems, res):
        assert_same(r, oracle_lib.solve(s), s.name)


def test_batch_budget_is_per_system(gpu_ctx, oracle_lib):
    """One system over its budget fails alone; the others are unaffected."""
    import paper_1802_00330_amd as P
    systems = [W.circle_line(), W.product_linear([5, 1], n=3), W.banded(0, n=6, tol=1e-8)]
    ref = [oracle_lib.solve(s) for s in systems]
    params = [P.make_params(s.tol) for s in systems]
    params[1] = P.make_params(systems[1].tol, max_boxes=ref[1].stats["processed"] - 1)
    res = P.ibb_solve_batch(gpu_ctx, systems, params)
    assert res[1].status == P.ERR_BUDGET and len(res[1].tag) == 0
    assert_same(res[0], ref[0], "batch[0]")
    assert_same(res[2], ref[2], "batch[2]")


def test_batch_of_one_equals_plain(gpu_ctx):
    import paper_1802_00330_amd as P
    s = W.dense_planted(0, n=5, n_terms=8, max_deg=3)
    (r,) = P.ibb_solve_batch(gpu_ctx, [s])
    assert_same(r, P.solve(gpu_ctx, s), "batch of one")


def test_batch_invalid_member(gpu_ctx, oracle_lib):
    import paper_1802_00330_amd as P
    good = W.circle_line()
    bad = W.circle_line()
    bad.coef[0] = float("inf")
    res = P.ibb_solve_batch(gpu_ctx, [bad, good])
    assert res[0].status == P.ERR_INVALID_ARG
    assert_same(res[1], oracle_lib.solve(good), "after invalid")


def test_batch_plan_replays_equal_eager_and_oracle(gpu_ctx, oracle_lib):
    """A recorded batch plan replayed three times, with other device work and
    synchronisations in between: every replay equals the eager batch solve and
    the oracle, member by member (an invalid member keeps its status)."""
    import torch

    import paper_1802_00330_amd as P
    systems = _mixed_systems()
    bad = W.circle_line()
    bad.coef[0] = float("inf")
    systems = systems[:5] + [bad] + systems[5:]
    eager = P.ibb_solve_batch(gpu_ctx, systems)
    ref = [oracle_lib.solve(s) if k != 5 else None for k, s in enumerate(systems)]
    plan = P.BatchPlan(gpu_ctx, systems)
    try:
        for rep in range(3):
            print(f"[batch-plan] replay {rep}", flush=True)
            res = plan.run()
            assert res[5].status == P.ERR_INVALID_ARG and len(res[5].tag) == 0
            for k, (r, e) in enumerate(zip(res, eager)):
                assert_same(r, e, f"replay {rep} member {k} vs eager")
                if ref[k] is not None:
                    assert_same(r, ref[k], f"replay {rep} member {k} vs oracle")
            # the program's own work between replays
            P.solve(gpu_ctx, systems[0])
            x = torch.arange(1 << 16, dtype=torch.float64, device="cuda")
            assert float(x.sum().item()) == float((1 << 16) * ((1 << 16) - 1) // 2)
            torch.cuda.synchronize()
    finally:
        plan.close()
