"""Reader of the hand-worked fixtures in tests/golden/.

Each fixture is plain text: the label counts, the images and masks (or, for
the spatially weighted examples `swmi_*`, per-pixel weights), one `shift`
line per displacement of the map (dy, dx, N, the joint counts C_ab in
row-major (a, b) order, MI as a closed form in numbers, + - * / ( ) and
log2), and `argmax` lines (gamma, dy, dx) for Alg. 1's choice.  The values
were derived by hand from the paper's definitions; each file states the
derivation and the passages it follows.
"""

import math
import os
import re

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

_CLOSED_FORM = re.compile(r"^[0-9.+\-*/()]*(log2\([0-9.+\-*/]+\)[0-9.+\-*/()]*)*$")


def fixtures(kind: str = "cmif"):
    """Fixture files of one kind: "cmif" (labels and masks) or "swmi"
    (labels and weights)."""
    return sorted(f for f in os.listdir(GOLDEN)
                  if f.startswith(kind + "_") and f.endswith(".txt"))


def closed_form(s: str) -> float:
    """Value of a closed form such as (5-3*log2(3))/2."""
    if not _CLOSED_FORM.match(s):
        raise ValueError(f"not a closed form of the fixture grammar: {s!r}")
    return float(eval(s, {"__builtins__": {}}, {"log2": math.log2}))


def load(name: str) -> dict:
    path = os.path.join(GOLDEN, name)
    with open(path) as f:
        lines = [ln.split("#", 1)[0].strip() for ln in f]
    lines = [ln for ln in lines if ln]
    fx = dict(name=name, shifts=[], argmax=[])
    it = iter(lines)
    for ln in it:
        t = ln.split()
        if t[0] == "labels":
            fx["qa"], fx["qb"] = int(t[1]), int(t[2])
        elif t[0] in ("image", "mask", "weight"):
            h, w = int(t[2]), int(t[3])
            rows = [next(it).split() for _ in range(h)]
            arr = (np.array(rows, np.float64) if t[0] == "weight"
                   else np.array([[int(v) for v in r] for r in rows], np.uint8))
            assert arr.shape == (h, w), (name, ln)
            fx[{"image": "", "mask": "M", "weight": "W"}[t[0]] + t[1]] = arr
        elif t[0] == "shift":
            q = fx["qa"] * fx["qb"]
            # weighted examples list weighted counts (exact here: integer
            # weights), label examples pixel counts
            dy, dx, n = int(t[1]), int(t[2]), int(t[3])
            c = np.array([int(v) for v in t[4:4 + q]], np.int64)
            fx["shifts"].append(dict(dy=dy, dx=dx, n=n,
                                     joint=c.reshape(fx["qa"], fx["qb"]),
                                     mi=closed_form("".join(t[4 + q:]))))
        elif t[0] == "argmax":
            fx["argmax"].append(dict(gamma=float(t[1]), dy=int(t[2]), dx=int(t[3])))
        else:
            raise ValueError(f"{name}: unknown line {ln!r}")
    return fx


def mi_of_counts(joint) -> float:
    """Eq. 1 from a joint count table (0/0 and 0 log 0 taken as 0)."""
    joint = np.asarray(joint, np.float64)
    n = joint.sum()
    if n == 0:
        return 0.0
    pa = joint.sum(axis=1) / n
    pb = joint.sum(axis=0) / n
    mi = 0.0
    for a in range(joint.shape[0]):
        for b in range(joint.shape[1]):
            if joint[a, b] > 0:
                p = joint[a, b] / n
                mi += p * math.log2(p / (pa[a] * pb[b]))
    return mi
