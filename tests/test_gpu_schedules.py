"""Both device schedules (work queue, level by level) and the autotuner give the
same results: bit-identical sorted boxes and counters against the oracle, the
same budget errors at the same node counts, the same per-depth box counts, and
the same output under a ring or frontier too small to start with."""
import numpy as np
import pytest

import workloads as W
from tests.parity import assert_same

pytestmark = pytest.mark.gpu

CASES = {
    "circle_line": lambda: W.circle_line(),
    "product4": lambda: W.product_linear([7, 3], n=4),
    "dense5": lambda: W.dense_planted(2, n=5, n_terms=8, max_deg=3),
    "dense6_sub": lambda: W.dense_planted(0),
    "banded8": lambda: W.banded(3, n=8, tol=1e-8),
    "banded10": lambda: W.banded(2, n=10, tol=1e-6),
    "banded9": lambda: W.banded(2, n=9, tol=1e-6),
    "univariate": lambda: W.univariate(np.poly([0.3, -1.1, 1.7, 0.9])[::-1], -2.0, 2.0, tol=1e-10),
}


def _box(s, name):
    if name == "dense6_sub":  # a sub-box around the planted root keeps the oracle fast
        r = s.roots[0]
        return r - 0.15, r + 0.15
    return s.lo, s.hi


@pytest.mark.parametrize("name", sorted(CASES))
def test_schedules_equal_oracle(gpu_ctx, oracle_lib, name):
    import paper_1802_00330_amd as P
    s = CASES[name]()
    lo, hi = _box(s, name)
    ref = oracle_lib.solve(s, lo=lo, hi=hi)
    print(f"[schedules] {name}: {ref.stats['processed']} nodes", flush=True)
    for sched in (P.SCHEDULE_QUEUE, P.SCHEDULE_LEVELS, P.SCHEDULE_AUTO, P.SCHEDULE_AUTO):
        gpu = P.solve(gpu_ctx, s, lo=lo, hi=hi, schedule=sched)
        assert_same(gpu, ref, f"{name} schedule {sched}")


@pytest.mark.parametrize("sched", [0, 1])
def test_budget_is_the_node_count_in_both_schedules(gpu_ctx, oracle_lib, sched):
    import paper_1802_00330_amd as P
    s = W.banded(3, n=8, tol=1e-8)
    n = oracle_lib.solve(s).stats["processed"]
    assert P.solve(gpu_ctx, s, max_boxes=n, schedule=sched).status == P.OK
    assert P.solve(gpu_ctx, s, max_boxes=n - 1, schedule=sched).status == P.ERR_BUDGET


def test_depth_counts_equal_level_sizes(gpu_ctx, oracle_lib):
    """Boxes per depth counted by the work queue = the level-by-level frontier
    sizes = the oracle's round sizes."""
    import paper_1802_00330_amd as P
    s = W.dense_planted(3, n=4, n_terms=8, max_deg=3)
    sizes = {}
    for sched in (P.SCHEDULE_QUEUE, P.SCHEDULE_LEVELS):
        r = P.ibb_solve(gpu_ctx, s, P.make_params(s.tol, schedule=sched))
        assert r.status == P.OK
        sizes[sched] = P.ibb_last_level_sizes(gpu_ctx).tolist()
        assert r.levels == len(sizes[sched]) and r.max_frontier == max(sizes[sched])
    assert sizes[P.SCHEDULE_QUEUE] == sizes[P.SCHEDULE_LEVELS]
    # the oracle's rounds, one after another from the initial box
    lo, hi = s.lo.reshape(1, -1), s.hi.reshape(1, -1)
    rec = np.zeros(1, dtype=np.uint32)
    rounds = []
    while lo.shape[0]:
        rounds.append(lo.shape[0])
        o = oracle_lib.round_step(s, lo, hi, rec)
        lo, hi, rec = o.child_lo, o.child_hi, o.child_rec
    assert sizes[P.SCHEDULE_LEVELS] == rounds


@pytest.mark.parametrize("sched", [0, 1])
def test_small_ring_or_frontier_retries(gpu_ctx, oracle_lib, sched):
    import paper_1802_00330_amd as P
    s = W.product_linear([4, 4], n=4)
    ref = oracle_lib.solve(s)
    gpu = P.solve(gpu_ctx, s, frontier_cap=8, out_cap=2, schedule=sched)
    assert_same(gpu, ref, f"small capacity, schedule {sched}")
