"""GPU: the HIP path (through the C ABI) against the hand-worked examples of
tests/golden/, directly: N and the joint counts of every displacement
bit-exact, MI within 1e-12 of the closed forms derived on paper, and Alg. 1's
choice at each listed gamma (threshold, argmax, ties to the smallest
row-major index), in both precisions."""

import numpy as np
import pytest

import golden_io
from gpu_common import MI_TOL, run_compute, say

pytestmark = pytest.mark.gpu

CASES = [(name, g["gamma"], prec)
         for name in golden_io.fixtures()
         for g in golden_io.load(name)["argmax"]
         for prec in ("fp32", "fp64")]


@pytest.mark.parametrize("name,gamma,precision", CASES,
                         ids=[f"{n[:-4]}-g{g}-{p}" for n, g, p in CASES])
def test_worked_example(gpu, name, gamma, precision):
    fx = golden_io.load(name)
    c = dict(A=fx["A"], MA=fx["MA"], B=fx["B"], MB=fx["MB"], qa=fx["qa"],
             qb=fx["qb"], gamma=gamma)
    g = run_compute(gpu, c, precision, tag=f"golden {name} gamma {gamma}")
    ha, wa = fx["A"].shape
    for s in fx["shifts"]:
        i, j = s["dy"] + ha - 1, s["dx"] + wa - 1
        assert g["n"][0][i, j] == s["n"], s
        assert np.array_equal(g["counts"][0][:, :, i, j], s["joint"]), s
        assert abs(g["mi"][0][i, j] - s["mi"]) <= MI_TOL, (s, g["mi"][0][i, j])
    want = next(a for a in fx["argmax"] if a["gamma"] == gamma)
    b = g["best"]
    say(f"  best ({b['dy']},{b['dx']}) mi {b['mi']:.15f}; by hand "
        f"({want['dy']},{want['dx']})")
    assert (b["dy"], b["dx"]) == (want["dy"], want["dx"]), b
    assert g["stats"]["unresolved_pairs"] == 0 and g["stats"]["label_errors"] == 0
