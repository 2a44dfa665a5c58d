"""One search step on single boxes, device vs oracle, intermediate by
intermediate: J(X), F(mid X), single-precision mid J, Y, g, P, the bracket N_i
of eq 21 and the contracted box -- bit for bit."""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _fields(n):
    o = lambda k: [0, 2 * n * n, 2 * n * n + 2 * n, 3 * n * n + 2 * n, 4 * n * n + 2 * n,  # noqa: E731
                   4 * n * n + 4 * n, 6 * n * n + 4 * n, 6 * n * n + 6 * n, 6 * n * n + 8 * n][k]
    names = ["J", "F", "M", "Y", "g", "P", "N", "X", "flags"]
    lens = [2 * n * n, 2 * n, n * n, n * n, 2 * n, 2 * n * n, 2 * n, 2 * n, 4]
    return [(names[k], o(k), lens[k]) for k in range(9)]


def _compare(dev, ref, n):
    """First differing field, or None (fields after a skip/empty are ignored)."""
    ran = ref[6 * n * n + 8 * n + 3] == 1.0
    for name, off, ln in _fields(n):
        if not ran and name in ("g", "P", "N", "X"):
            continue
        a, b = dev[off:off + ln], ref[off:off + ln]
        bad = np.nonzero(a.view(np.uint64) != b.view(np.uint64))[0]
        # signed zeros may differ
        bad = [i for i in bad if not (a[i] == 0 and b[i] == 0)]
        if bad:
            return name, bad[:6], a[bad[:6]], b[bad[:6]]
    return None


def _boxes_around(center, rng, count, wmin=1e-12, wmax=1e-1):
    for _ in range(count):
        w = 10.0 ** rng.uniform(np.log10(wmin), np.log10(wmax))
        u1 = rng.uniform(0.2, 1.0, size=center.size)
        u2 = rng.uniform(0.2, 1.0, size=center.size)
        yield center - w * u1, center + w * u2


def _center_from_gold(name):
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", f"expected_{name}.json")))
    lo = np.array([float.fromhex(v) for v in g["lo"][0]])
    hi = np.array([float.fromhex(v) for v in g["hi"][0]])
    return (lo + hi) / 2


CASES = [
    ("banded12_s1", lambda: W.banded(1), lambda: _center_from_gold("banded12_s1")),
    ("banded12_s0", lambda: W.banded(0), lambda: _center_from_gold("banded12_s0")),
    ("dense6_s0", lambda: W.dense_planted(0), lambda: W.dense_planted(0).roots[0]),
    ("product5", lambda: W.product_linear([4, 5], n=5), lambda: W.product_linear([4, 5], n=5).roots[3]),
]


@pytest.mark.parametrize("contractor", [0, 1], ids=["hansen_sengupta", "krawczyk"])
@pytest.mark.parametrize("name,make,center", CASES)
def test_single_steps_match_oracle(gpu_ctx, oracle_lib, name, make, center, contractor):
    """Hansen-Sengupta (eq 17-22) and Krawczyk (eq 15-16; the trace's N holds
    K(X)) steps on 150 boxes around a root."""
    import paper_1802_00330_amd as P
    s = make()
    c = center()
    rng = np.random.default_rng(7)
    first = None
    nbad = 0
    params = P.make_params(s.tol, contractor=contractor)
    for k, (lo, hi) in enumerate(_boxes_around(c, rng, 150)):
        dev = P.ibb_debug_step(gpu_ctx, s, lo, hi, params)
        st, ref = oracle_lib.hs_trace(s, lo, hi, contractor=contractor)
        if dev[6 * s.n * s.n + 8 * s.n + 3] != 1.0 and st != oracle_lib.HS_SKIPPED:
            # the device excluded the box before contracting it: nothing to compare
            continue
        d = _compare(dev, ref, s.n)
        if d is not None:
            nbad += 1
            if first is None:
                first = (k, lo.tolist(), hi.tolist(), d)
    if first is not None:
        k, lo, hi, (field, idx, a, b) = first
        print(f"[hs-steps] {name}: {nbad} differing boxes; first #{k} field {field} idx {list(idx)}\n"
              f"  device {[float(v).hex() for v in a]}\n  oracle {[float(v).hex() for v in b]}\n"
              f"  lo={[float(v).hex() for v in lo]}\n  hi={[float(v).hex() for v in hi]}", flush=True)
    assert first is None


@pytest.mark.parametrize("name,make", [("banded12_s1", lambda: W.banded(1)), ("banded12_s0", lambda: W.banded(0)),
                                       ("dense6_s0", lambda: W.dense_planted(0))])
def test_proof_chain_steps_match_oracle(gpu_ctx, oracle_lib, name, make):
    """Replays the oracle's proof-chain boxes of a full-size solve one step at a
    time on the device: every contracted box bit-identical."""
    import paper_1802_00330_amd as P
    path = os.path.join(os.path.dirname(__file__), "golden", f"expected_{name}.json")
    g = json.load(open(path))
    if "chains" not in g:
        pytest.skip("no stored chain")
    s = make()
    for k, c in enumerate(g["chains"]):
        lo, hi, elo, ehi = (np.array([float.fromhex(v) for v in a]) for a in c)
        dev = P.ibb_debug_step(gpu_ctx, s, lo, hi)
        st, ref = oracle_lib.hs_trace(s, lo, hi)
        n = s.n
        d = _compare(dev, ref, n)
        X = dev[6 * n * n + 6 * n: 6 * n * n + 8 * n].reshape(n, 2)
        R = ref[6 * n * n + 6 * n: 6 * n * n + 8 * n].reshape(n, 2)
        same_chain = np.array_equal(X[:, 0], elo) and np.array_equal(X[:, 1], ehi)
        if d is not None or not same_chain:
            idx = np.nonzero((X[:, 0] != elo) | (X[:, 1] != ehi))[0][:4]
            print(f"[chain] {name} step {k}: first differing field {d and d[0]} idx {d and list(d[1])}\n"
                  f"  device {d and [float(v).hex() for v in d[2]]}\n  oracle {d and [float(v).hex() for v in d[3]]}\n"
                  f"  X' differs from the stored chain at {idx.tolist()}: device "
                  f"{[(float(X[i, 0]).hex(), float(X[i, 1]).hex()) for i in idx]} trace "
                  f"{[(float(R[i, 0]).hex(), float(R[i, 1]).hex()) for i in idx]} chain "
                  f"{[(float(elo[i]).hex(), float(ehi[i]).hex()) for i in idx]} flags {dev[-4:].tolist()} "
                  f"{ref[-4:].tolist()}\n"
                  f"  lo={[float(v).hex() for v in lo]}\n  hi={[float(v).hex() for v in hi]}", flush=True)
        assert d is None, (name, k, d and d[0])
        assert same_chain, (name, k)
