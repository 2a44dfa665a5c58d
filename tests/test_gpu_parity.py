"""GPU search vs the CPU oracle on the same seeded systems: sorted box lists
bit-exact, identical tree counters.  Sizes are chosen so the oracle finishes in
seconds while the device levels still span many tiles with ragged tails."""
import numpy as np
import pytest

import workloads as W
from tests.parity import assert_same

pytestmark = pytest.mark.gpu


def _both(ctx, oracle_lib, s, **kw):
    import paper_1802_00330_amd as P
    print(f"[parity] {s.name} n={s.n} T={s.n_terms} {kw}", flush=True)
    ref = oracle_lib.solve(s, **kw)
    gpu = P.solve(ctx, s, **kw)
    return gpu, ref


def test_circle_line(gpu_ctx, oracle_lib):
    gpu, ref = _both(gpu_ctx, oracle_lib, W.circle_line())
    assert_same(gpu, ref, "circle_line")
    assert gpu.tag.tolist() == [1, 1]


def test_circle_line_split_all(gpu_ctx, oracle_lib):
    gpu, ref = _both(gpu_ctx, oracle_lib, W.circle_line(), split_mode=1)
    assert_same(gpu, ref, "circle_line ALL")


# the paper's all-coordinate split (Alg. 2: 2^n children) with the
# contraction on, at n = 3 and 4 (8 and 16 children per split)
SPLIT_ALL_CASES = {
    "product3": lambda: W.product_linear([4, 3], n=3),
    "product4": lambda: W.product_linear([4, 4], n=4),
    "dense4": lambda: W.dense_planted(0, n=4, n_terms=6, max_deg=2),
    "dense3_cubic": lambda: W.dense_planted(1, n=3, n_terms=6, max_deg=3),
    "banded4": lambda: W.banded(0, n=4, tol=1e-8),
}


@pytest.mark.parametrize("threshold", [0.5, 0.125])
@pytest.mark.parametrize("name", ["product3", "product4", "dense4"])
def test_paper_mode_contraction_after_a_width(gpu_ctx, oracle_lib, name, threshold):
    """The paper's driver: every coordinate bisected, the contraction only on
    boxes no wider than a threshold (branch and bound alone in the first
    rounds, Tab. 1 then Tab. 2)."""
    s = SPLIT_ALL_CASES[name]()
    gpu, ref = _both(gpu_ctx, oracle_lib, s, split_mode=1, hs_max_width=threshold)
    assert ref.stats["hs_skipped"] > 0
    assert_same(gpu, ref, f"{name} ALL, contraction below {threshold}")


@pytest.mark.parametrize("name", sorted(SPLIT_ALL_CASES))
def test_split_all_with_contraction(gpu_ctx, oracle_lib, name):
    s = SPLIT_ALL_CASES[name]()
    gpu, ref = _both(gpu_ctx, oracle_lib, s, split_mode=1)
    assert ref.stats["excluded_hs"] + ref.stats["recontracted"] > 0  # the contraction acted
    assert_same(gpu, ref, f"{name} ALL")


# the Krawczyk contractor (eq 15-16) and the mean-value exclusion test, alone
# and together, on the whole search
VARIANTS = {"krawczyk": {"contractor": 1}, "mean_value": {"inclusion": 1},
            "krawczyk_mean_value": {"contractor": 1, "inclusion": 1}}
VARIANT_SYSTEMS = {
    "circle_line": lambda: W.circle_line(),
    "product3": lambda: W.product_linear([4, 3], n=3),
    "product5": lambda: W.product_linear([4, 5], n=5),
    "dense4": lambda: W.dense_planted(0, n=4, n_terms=6, max_deg=2),
    "dense5_cubic": lambda: W.dense_planted(0, n=5, n_terms=8, max_deg=3),
    "banded8": lambda: W.banded(0, n=8, tol=1e-8),
    "batch_member11": lambda: W.batch_planted(0, indices=[11])[0],
}


@pytest.mark.parametrize("variant", sorted(VARIANTS))
@pytest.mark.parametrize("name", sorted(VARIANT_SYSTEMS))
def test_contractor_and_inclusion_variants(gpu_ctx, oracle_lib, name, variant):
    s = VARIANT_SYSTEMS[name]()
    gpu, ref = _both(gpu_ctx, oracle_lib, s, **VARIANTS[variant])
    assert_same(gpu, ref, f"{name} {variant}")


def test_dense_n6_subbox_variants(gpu_ctx, oracle_lib):
    s = W.dense_planted(0)
    r = s.roots[0]
    for kw in VARIANTS.values():
        gpu, ref = _both(gpu_ctx, oracle_lib, s, lo=r - 0.14, hi=r + 0.26, **kw)
        assert_same(gpu, ref, f"dense n=6 sub-box {kw}")


def test_batch_members_with_different_variants(gpu_ctx, oracle_lib):
    """A batch whose members use different contractors and inclusions: each
    member equals its oracle solve."""
    import paper_1802_00330_amd as P
    systems = [W.product_linear([4, 3], n=3), W.dense_planted(0, n=4, n_terms=6, max_deg=2),
               W.banded(0, n=8, tol=1e-8), W.circle_line(), W.product_linear([4, 5], n=5),
               W.batch_planted(0, indices=[11])[0]]
    kws = [{}, {"contractor": 1}, {"inclusion": 1}, {"contractor": 1, "inclusion": 1}, {"contractor": 1},
           {"inclusion": 1}]
    params = [P.make_params(s.tol, **kw) for s, kw in zip(systems, kws)]
    res = P.ibb_solve_batch(gpu_ctx, systems, params)
    for s, kw, r in zip(systems, kws, res):
        assert_same(r, oracle_lib.solve(s, **kw), f"{s.name} {kw}")


def test_host_pointer_entry_point(gpu_ctx, oracle_lib):
    import paper_1802_00330_amd as P
    s = W.circle_line()
    gpu = P.ibb_solve(gpu_ctx, s, P.make_params(s.tol))
    assert_same(gpu, oracle_lib.solve(s), "ibb_solve")


@pytest.mark.parametrize("seed", range(4))
def test_univariate(gpu_ctx, oracle_lib, seed):
    rng = np.random.default_rng(seed)
    roots = np.sort(rng.uniform(-1.9, 1.9, size=int(rng.integers(2, 7))))
    c = np.poly(roots)[::-1]
    s = W.univariate(c, -2.0, 2.0, tol=1e-10)
    gpu, ref = _both(gpu_ctx, oracle_lib, s)
    assert_same(gpu, ref, s.name)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_product_systems(gpu_ctx, oracle_lib, n):
    s = W.product_linear([4, n], n=n)
    gpu, ref = _both(gpu_ctx, oracle_lib, s)
    assert_same(gpu, ref, s.name)


@pytest.mark.parametrize("seed", range(3))
def test_dense_small(gpu_ctx, oracle_lib, seed):
    s = W.dense_planted(seed, n=4, n_terms=6, max_deg=2)
    gpu, ref = _both(gpu_ctx, oracle_lib, s)
    assert_same(gpu, ref, s.name)


def test_dense_n5_cubic(gpu_ctx, oracle_lib):
    s = W.dense_planted(0, n=5, n_terms=8, max_deg=3)
    gpu, ref = _both(gpu_ctx, oracle_lib, s)
    assert_same(gpu, ref, s.name)


@pytest.mark.parametrize("n", [4, 6, 8])
def test_banded(gpu_ctx, oracle_lib, n):
    s = W.banded(0, n=n, tol=1e-8)
    gpu, ref = _both(gpu_ctx, oracle_lib, s)
    assert_same(gpu, ref, s.name)


@pytest.mark.parametrize("w", [0.05, 0.2])
def test_dense_n6_subbox(gpu_ctx, oracle_lib, w):
    s = W.dense_planted(0)
    r = s.roots[0]
    gpu, ref = _both(gpu_ctx, oracle_lib, s, lo=r - 0.7 * w, hi=r + 1.3 * w)
    assert_same(gpu, ref, f"dense n=6 sub-box {w}")


@pytest.mark.parametrize("k", [9, 11])
def test_batch_members(gpu_ctx, oracle_lib, k):
    s = W.batch_planted(0, indices=[k])[0]
    gpu, ref = _both(gpu_ctx, oracle_lib, s)
    assert_same(gpu, ref, s.name)


def test_budget_error(gpu_ctx, oracle_lib):
    s = W.circle_line()
    full = oracle_lib.solve(s)
    n = full.stats["processed"]
    import paper_1802_00330_amd as P
    assert P.solve(gpu_ctx, s, max_boxes=n).status == 0
    assert P.solve(gpu_ctx, s, max_boxes=n - 1).status == P.ERR_BUDGET


def test_rootless_box_and_point_box(gpu_ctx, oracle_lib):
    s = W.circle_line()
    gpu, ref = _both(gpu_ctx, oracle_lib, s, lo=[1.0, -2.0], hi=[2.0, -1.0])
    assert_same(gpu, ref, "rootless")
    assert len(gpu.tag) == 0
    x = 0.5 ** 0.5
    gpu, ref = _both(gpu_ctx, oracle_lib, s, lo=[x, x], hi=[x, x])
    assert_same(gpu, ref, "point box")


def test_invalid_arguments(gpu_ctx):
    import paper_1802_00330_amd as P
    s = W.circle_line()
    assert P.solve(gpu_ctx, s, tol=0.0).status == P.ERR_INVALID_ARG
    bad = W.circle_line()
    bad.coef[0] = float("nan")
    assert P.solve(gpu_ctx, bad).status == P.ERR_INVALID_ARG


def test_frontier_overflow_retry(gpu_ctx, oracle_lib):
    """A tiny frontier forces QUEUE_OVERFLOW; the binding grows it and the
    result is unchanged."""
    import paper_1802_00330_amd as P
    s = W.product_linear([4, 4], n=4)
    ref = oracle_lib.solve(s)
    gpu = P.solve(gpu_ctx, s, frontier_cap=4, out_cap=2)
    assert_same(gpu, ref, "overflow retry")
