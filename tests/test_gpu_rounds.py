"""Round-by-round parity: each round set of the search tree (Alg. 1), as the
oracle produces it, is stepped once by the device (ibb_round) and once by the
oracle; children and emitted boxes must agree bit for bit as multisets, with
identical counters.  Feeding the oracle's round to both sides at every level
pins a difference to its level and, through a box-by-box search, to the one
box whose step differs."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import box_rows, first_row_difference

pytestmark = pytest.mark.gpu

CASES = {
    # name: (system, node budget over the levels compared)
    "banded12_s1": (lambda: W.banded(1), 700_000),
    "banded12_s0": (lambda: W.banded(0), 400_000),
    "dense6_s0": (lambda: W.dense_planted(0), 300_000),
    "product5": (lambda: W.product_linear([4, 5], n=5), 200_000),
}


def _rows(r, emitted):
    if emitted:
        return box_rows(r.emit_lo, r.emit_hi, r.emit_tag)
    return box_rows(r.child_lo, r.child_hi, r.child_rec)


def _hex(a):
    return [float(v).hex() for v in np.asarray(a).ravel()]


def _find_box(ctx, s, lo, hi, rec, limit=20000):
    import paper_1802_00330_amd as P
    for b in range(min(lo.shape[0], limit)):
        d = P.ibb_round(ctx, s, lo[b:b + 1], hi[b:b + 1], rec[b:b + 1])
        o = oracle.round_step(s, lo[b:b + 1], hi[b:b + 1], rec[b:b + 1])
        if (first_row_difference(_rows(d, False), _rows(o, False)) is not None
                or first_row_difference(_rows(d, True), _rows(o, True)) is not None or d.stats != o.stats):
            return b, d, o
    return None


@pytest.mark.parametrize("name", sorted(CASES))
def test_rounds_match_oracle(gpu_ctx, oracle_lib, name):
    import paper_1802_00330_amd as P
    make, budget = CASES[name]
    s = make()
    lo, hi = s.lo.reshape(1, -1), s.hi.reshape(1, -1)
    rec = np.zeros(1, dtype=np.uint32)
    nodes = level = 0
    while lo.shape[0] and nodes + lo.shape[0] <= budget:
        o = oracle.round_step(s, lo, hi, rec)
        assert o.status == oracle.OK
        d = P.ibb_round(gpu_ctx, s, lo, hi, rec)
        bad = (d.stats != o.stats
               or first_row_difference(_rows(d, False), _rows(o, False)) is not None
               or first_row_difference(_rows(d, True), _rows(o, True)) is not None)
        if bad:
            hit = _find_box(gpu_ctx, s, lo, hi, rec)
            msg = f"[rounds] {name}: level {level} ({lo.shape[0]} boxes) differs"
            if hit is not None:
                b, db, ob = hit
                msg += (f"; box #{b} rec {int(rec[b]):#x}\n  lo={_hex(lo[b])}\n  hi={_hex(hi[b])}\n"
                        f"  device children {_hex(db.child_lo)} / {_hex(db.child_hi)} rec {db.child_rec.tolist()}"
                        f" emitted {_hex(db.emit_lo)} / {_hex(db.emit_hi)}\n"
                        f"  oracle children {_hex(ob.child_lo)} / {_hex(ob.child_hi)} rec {ob.child_rec.tolist()}"
                        f" emitted {_hex(ob.emit_lo)} / {_hex(ob.emit_hi)}\n"
                        f"  stats device {db.stats} oracle {ob.stats}")
            print(msg, flush=True)
            pytest.fail(msg)
        nodes += lo.shape[0]
        level += 1
        lo, hi, rec = o.child_lo, o.child_hi, o.child_rec
    print(f"[rounds] {name}: {level} levels, {nodes} nodes equal", flush=True)
    assert level >= 5


def test_round_edge_cases(gpu_ctx, oracle_lib):
    """Empty list; boxes around a root, proven or not, one at the last
    recontraction allowed."""
    import paper_1802_00330_amd as P
    s = W.circle_line()
    d = P.ibb_round(gpu_ctx, s, np.zeros((0, s.n)), np.zeros((0, s.n)))
    assert d.child_lo.shape == (0, s.n) and d.emit_lo.shape == (0, s.n) and d.stats["processed"] == 0
    boxes_lo = np.stack([s.roots[0] - 1e-3, s.roots[0] - 1e-9, s.roots[1] - 0.3])
    boxes_hi = np.stack([s.roots[0] + 1e-3, s.roots[0] + 1e-9, s.roots[1] + 0.2])
    for rec in (np.zeros(3, dtype=np.uint32), np.array([1, 0x101, 0x0F00], dtype=np.uint32)):
        d = P.ibb_round(gpu_ctx, s, boxes_lo, boxes_hi, rec)
        o = oracle.round_step(s, boxes_lo, boxes_hi, rec)
        assert d.stats == o.stats
        assert first_row_difference(_rows(d, False), _rows(o, False)) is None
        assert first_row_difference(_rows(d, True), _rows(o, True)) is None
