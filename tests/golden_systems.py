"""Parser for the paper's worked-example systems stored under tests/golden/."""
import os
import re

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

_TERM = re.compile(r"\s*([+-]?)\s*([^+-]+)")


def _parse_poly(text, n):
    terms = []
    for sign, body in _TERM.findall(text):
        coef = -1.0 if sign == "-" else 1.0
        e = [0] * n
        for f in body.strip().split("*"):
            f = f.strip()
            if f.startswith("x"):
                v, _, p = f[1:].partition("^")
                e[int(v) - 1] += int(p) if p else 1
            else:
                coef *= float(f)
        terms.append((coef, tuple(e)))
    return terms


def load(name):
    """Returns (System, {round: boxes kept})."""
    n, box, eqs, rounds = None, None, [], {}
    with open(os.path.join(GOLDEN, name + ".txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(" ")
            if key == "n":
                n = int(rest)
            elif key == "box":
                box = [float(v) for v in rest.split()]
            elif key == "eq":
                eqs.append(_parse_poly(rest, n))
            elif key == "rounds":
                for tok in rest.split():
                    r, b = tok.split(":")
                    rounds[int(r)] = int(b)
    return W.systems._pack(n, eqs, box[0], box[1], 1e-6, name), rounds
