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


def _defaults(P, ctx):
    for q in range(4):
        P.ibb_batch_set_config(ctx, q, 2 << q)


# forced launch configurations: (class, lanes, tiles per claim, workgroups per CU)
_CONFIGS = {
    "wider lanes, 4 tiles per claim, 1 workgroup per CU": [(0, 4, 4, 1), (1, 8, 4, 1), (2, 16, 4, 1), (3, 16, 4, 1)],
    "16 lanes for all, 2 tiles per claim": [(0, 16, 2, 0), (1, 16, 2, 0), (2, 16, 2, 0), (3, 16, 2, 0)],
    "natural lanes, 3 tiles per claim, 2 workgroups per CU": [(0, 2, 3, 2), (1, 4, 3, 2), (2, 8, 3, 2), (3, 16, 3, 2)],
}


@pytest.mark.parametrize("name", list(_CONFIGS))
def test_batch_results_independent_of_launch_config(gpu_ctx, oracle_lib, name):
    """Lanes per box, tiles per claim and workgroups per CU change how the
    device schedules the boxes, never a box's fate: every member's boxes,
    tags, counters and status equal the oracle's under each configuration."""
    import paper_1802_00330_amd as P
    systems = _mixed_systems()
    bad = W.circle_line()
    bad.coef[0] = float("inf")
    systems = systems[:3] + [bad] + systems[3:]
    ref = [oracle_lib.solve(s) if k != 3 else None for k, s in enumerate(systems)]
    try:
        for q, lanes, pop, pc in _CONFIGS[name]:
            P.ibb_batch_set_config(gpu_ctx, q, lanes, pop, pc)
        print(f"[batch-config] {name}", flush=True)
        res = P.ibb_solve_batch(gpu_ctx, systems)
        plan = P.BatchPlan(gpu_ctx, systems)
        try:
            replay = plan.run()
        finally:
            plan.close()
    finally:
        _defaults(P, gpu_ctx)
    for k, (s, r, g) in enumerate(zip(systems, res, replay)):
        if k == 3:
            assert r.status == P.ERR_INVALID_ARG and g.status == P.ERR_INVALID_ARG
            continue
        assert_same(r, ref[k], f"{name}: {s.name}")
        assert_same(g, ref[k], f"{name} (plan): {s.name}")


def test_batch_tune_keeps_results(gpu_ctx, oracle_lib):
    """The autotuner times candidate configurations on a sample of each class,
    keeps a valid one per class present, and the tuned batch still equals the
    oracle member by member."""
    import paper_1802_00330_amd as P
    systems = _mixed_systems()
    ref = [oracle_lib.solve(s) for s in systems]
    try:
        cfgs = P.ibb_batch_tune(gpu_ctx, systems, sample=6)
        print(f"[batch-tune] {cfgs}", flush=True)
        present = {min(q for q in range(4) if s.n <= 2 << q) for s in systems}
        for q, c in enumerate(cfgs):
            if q in present:
                # the class's queue size per member, measured on its sample
                assert c["tuned"] == 1 and c["ms"] > 0.0 and c["front_per_member"] >= 1.0
                assert c["lanes"] in (2 << q, 4 << q) and c["lanes"] <= 16
                assert c["tiles_per_claim"] in (1, 4) and c["blocks_per_cu"] >= 0
            else:
                assert c["tuned"] == 0 and c["lanes"] == 2 << q and c["front_per_member"] == 0.0
        # a batch of the present classes only: its frontier comes from the
        # measured widths (and grows if they fall short); results unchanged
        res = P.ibb_solve_batch(gpu_ctx, systems)
    finally:
        _defaults(P, gpu_ctx)
    for s, r, o in zip(systems, res, ref):
        assert_same(r, o, f"tuned: {s.name}")


def test_batch_set_config_rejects_invalid(gpu_ctx):
    import paper_1802_00330_amd as P
    bad = [(0, 3, 1, 0), (1, 2, 1, 0), (2, 32, 1, 0), (3, 8, 1, 0), (0, 2, 0, 0), (0, 2, 17, 0), (0, 2, 1, -1),
           (4, 16, 1, 0), (-1, 2, 1, 0)]
    try:
        for q, lanes, pop, pc in bad:
            with pytest.raises(RuntimeError, match="invalid"):
                P.ibb_batch_set_config(gpu_ctx, q, lanes, pop, pc)
        P.ibb_batch_set_config(gpu_ctx, 1, 16, 16, 3)
        c = P.ibb_batch_get_config(gpu_ctx, 1)
        assert (c.lanes, c.tiles_per_claim, c.blocks_per_cu, c.tuned) == (16, 16, 3, 0)
        with pytest.raises(RuntimeError, match="invalid"):
            P.ibb_batch_tune(gpu_ctx, [W.circle_line()], sample=0)
        with pytest.raises(RuntimeError, match="invalid"):
            P.ibb_batch_get_config(gpu_ctx, 4)
    finally:
        _defaults(P, gpu_ctx)
    assert P.ibb_batch_get_config(gpu_ctx, 1).lanes == 4
