"""The oracle's one-round function against its whole solve: running the
rounds of Alg. 1 one after another from the initial box (each round on the
children of the previous one) visits the same tree as the first-in-first-out
solve: the same counters and the same sorted output."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import box_rows

CASES = {
    "circle_line": lambda: W.circle_line(),
    "product3": lambda: W.product_linear([1, 2], n=3),
    "dense3": lambda: W.dense_planted(3, n=3, n_terms=8),
    "banded4": lambda: W.banded(2, n=4),
}


def run_rounds(s, **kw):
    lo, hi = s.lo.reshape(1, -1), s.hi.reshape(1, -1)
    rec = np.zeros(1, dtype=np.uint32)
    stats = dict.fromkeys(oracle.STATS_FIELDS, 0)
    elo, ehi, etag = [], [], []
    levels = 0
    while lo.shape[0]:
        r = oracle.round_step(s, lo, hi, rec, **kw)
        assert r.status == oracle.OK
        for k, v in r.stats.items():
            stats[k] += v
        elo.append(r.emit_lo)
        ehi.append(r.emit_hi)
        etag.append(r.emit_tag)
        lo, hi, rec = r.child_lo, r.child_hi, r.child_rec
        levels += 1
    return stats, np.concatenate(elo), np.concatenate(ehi), np.concatenate(etag), levels


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("split_mode", [oracle.SPLIT_WIDEST, oracle.SPLIT_ALL])
def test_rounds_equal_fifo_solve(oracle_lib, name, split_mode):
    s = CASES[name]()
    if split_mode == oracle.SPLIT_ALL and s.n > 3:
        pytest.skip("2^n children per split")
    stats, elo, ehi, etag, levels = run_rounds(s, split_mode=split_mode)
    ref = oracle.solve(s, split_mode=split_mode, order=1)
    assert ref.status == oracle.OK
    assert stats == ref.stats
    assert np.array_equal(box_rows(elo, ehi, etag), box_rows(ref.lo, ref.hi, ref.tag))
    assert levels > 3


def test_round_records_and_capacity(oracle_lib):
    """A proven box is stepped without the exclusion test and its record
    carries over; an empty list is a valid round."""
    s = W.circle_line()
    r0 = oracle.round_step(s, np.zeros((0, s.n)), np.zeros((0, s.n)))
    assert r0.status == oracle.OK and r0.child_lo.shape == (0, s.n) and r0.stats["processed"] == 0
    # drive one root's box until it is proven, then step it with its record
    lo, hi, rec = s.lo.reshape(1, -1), s.hi.reshape(1, -1), np.zeros(1, dtype=np.uint32)
    for _ in range(200):
        r = oracle.round_step(s, lo, hi, rec)
        if (r.child_rec & 1).any():
            k = int(np.nonzero(r.child_rec & 1)[0][0])
            assert (r.child_rec[k] >> 8) >= 1
            r2 = oracle.round_step(s, r.child_lo[k:k + 1], r.child_hi[k:k + 1], r.child_rec[k:k + 1])
            assert r2.stats["excluded_eval"] == 0
            assert r2.stats["emitted_unique"] + int((r2.child_rec & 1).sum()) == 1
            return
        lo, hi, rec = r.child_lo, r.child_hi, r.child_rec
    pytest.fail("no proven box")


def test_round_rejects_invalid_box(oracle_lib):
    s = W.circle_line()
    r = oracle.round_step(s, np.array([[1.0, 0.0]]), np.array([[0.0, 1.0]]))
    assert r.status == oracle.ERR_INVALID_ARG
