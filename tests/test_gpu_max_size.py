"""Systems of 13 to 16 unknowns (16 is the largest the library takes): every lane
of a 16-lane group holds a row, factor indices reach 15, and the LDS scratch
and tables take their largest per-box sizes.  Single solves (both schedules),
a budget failure, and a batch of them are compared with the oracle: sorted
box lists bit for bit, identical tree counters."""
import copy

import numpy as np
import pytest

import workloads as W
from tests.parity import assert_same

pytestmark = pytest.mark.gpu

# (n, seed): dense planted systems (8 monomials of degree <= 2 per equation)
# on a sub-box of width 0.05 around the planted root, of 4.5e3 to 6.4e4 nodes
MAX_SIZE = [(13, 1), (14, 1), (16, 0)]
WIDTH = 0.05


def _case(n, seed):
    s = W.dense_planted(seed, n=n, n_terms=8, max_deg=2)
    r = s.roots[0]
    t = copy.copy(s)
    t.lo = np.ascontiguousarray(r - 0.6 * WIDTH)
    t.hi = np.ascontiguousarray(r + 1.4 * WIDTH)
    t.name = f"{s.name} sub-box {WIDTH}"
    return t


@pytest.fixture(scope="module")
def cases(oracle_lib):
    out = []
    for n, seed in MAX_SIZE:
        s = _case(n, seed)
        print(f"[max-size] oracle n={n} seed={seed}", flush=True)
        ref = oracle_lib.solve(s)
        assert ref.status == 0
        out.append((s, ref))
    return out


@pytest.mark.parametrize("sched", [0, 1])
def test_max_size_single_solves(gpu_ctx, cases, sched):
    import paper_1802_00330_amd as P
    for s, ref in cases:
        print(f"[max-size] {s.name} n={s.n} schedule {sched}", flush=True)
        assert_same(P.solve(gpu_ctx, s, schedule=sched), ref, f"{s.name} schedule {sched}")


@pytest.mark.parametrize("variant", [{"contractor": 1}, {"inclusion": 1}, {"contractor": 1, "inclusion": 1}],
                         ids=["krawczyk", "mean_value", "krawczyk_mean_value"])
def test_max_size_variants(gpu_ctx, oracle_lib, variant):
    """The Krawczyk contractor and the mean-value exclusion test at 13 and 16
    unknowns (their kernel instances with 16-lane groups fully used)."""
    import paper_1802_00330_amd as P
    for n, seed in (MAX_SIZE[0], MAX_SIZE[-1]):
        s = _case(n, seed)
        print(f"[max-size] {s.name} n={s.n} {variant}", flush=True)
        ref = oracle_lib.solve(s, **variant)
        assert ref.status == 0
        assert_same(P.solve(gpu_ctx, s, **variant), ref, f"{s.name} {variant}")


def test_max_size_budget(gpu_ctx, cases):
    import paper_1802_00330_amd as P
    s, ref = cases[-1]
    n = ref.stats["processed"]
    assert P.solve(gpu_ctx, s, max_boxes=n).status == P.OK
    assert P.solve(gpu_ctx, s, max_boxes=n - 1).status == P.ERR_BUDGET


def test_max_size_batch(gpu_ctx, oracle_lib, cases):
    """The three systems and small ones in one batch (the 16-lane launch holds
    members of 13 to 16 unknowns); each member equals the oracle alone."""
    import paper_1802_00330_amd as P
    small = [W.circle_line(), W.banded(0, n=6, tol=1e-8)]
    systems = [c[0] for c in cases] + small
    refs = [c[1] for c in cases] + [oracle_lib.solve(s) for s in small]
    res = P.ibb_solve_batch(gpu_ctx, systems)
    for s, r, o in zip(systems, res, refs):
        assert_same(r, o, f"batch: {s.name}")
