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


SWMI_CASES = [(name, prec) for name in golden_io.fixtures("swmi")
              for prec in ("fp32", "fp64")]


@pytest.mark.parametrize("name,precision", SWMI_CASES,
                         ids=[f"{n[:-4]}-{p}" for n, p in SWMI_CASES])
def test_worked_swmi(gpu, name, precision):
    """Spatially weighted MI (Sec. 3.3, Eq. 13) through the soft path, the
    memberships being the weighted level sets: MI against the hand-derived
    closed forms, within 1e-9 everywhere in FP64 and 1e-5 in FP32 where the
    weighted N reaches half its maximum (the soft path's FP32 bar; below it
    the joint values approach the FP32 transform's absolute error)."""
    cm, torch = gpu
    fx = golden_io.load(name)
    qa, qb = fx["qa"], fx["qb"]
    pa = np.stack([(fx["A"] == a) * fx["WA"] for a in range(qa)]).astype(np.float32)
    pb = np.stack([(fx["B"] == b) * fx["WB"] for b in range(qb)]).astype(np.float32)
    say(f"[gpu] golden swmi {name} {precision}")
    plan = cm.Plan([(*fx["A"].shape, *fx["B"].shape)], qa, qb,
                   precision=precision, mode="soft", flags=0)
    r = plan.compute(torch.from_numpy(pa).cuda(), None,
                     torch.from_numpy(pb).cuda(), None, mi=True, n=True)
    mi = r["mi"][0][0].cpu().numpy()
    ha, wa = fx["A"].shape
    nmax = max(s["n"] for s in fx["shifts"])
    for s in fx["shifts"]:
        i, j = s["dy"] + ha - 1, s["dx"] + wa - 1
        err = abs(mi[i, j] - s["mi"])
        if precision == "fp64":
            assert err <= 1e-9, (s, mi[i, j])
        elif s["n"] >= 0.5 * nmax:
            assert err <= 1e-5, (s, mi[i, j])
        say(f"  dx {s['dx']:+d} N {s['n']}: MI {mi[i, j]:.12f} by hand "
            f"{s['mi']:.12f}")
