"""GPU: the two-stage global alignment of Sec. 3.6 (grid search, then
random search around the grid's best angle) through cmif_align_two_stage.
Its result must equal the oracle's Alg. 1 over the grid followed by the
refinement angles theta* + u_k 2 pi / |grid| (a later angle wins only with
a strictly larger MI), up to the near-tie rule; the stage results, the
angle indices and the corner error (Sec. 5.2) are checked too."""

import math

import numpy as np
import pytest

import synth
from gpu_common import MI_TOL, dev, say

pytestmark = pytest.mark.gpu


def _oracle_two_stage(oracle, c, B, MB, q, grid, u):
    """Alg. 1 over the grid, then over the refinement angles computed from
    the oracle's own grid result (same FP64 formula as the boundary)."""
    og = oracle.align(c["A"], c["MA"], B, MB, q, q, grid, 0.5)
    th0 = og["angle"] if og["angle_index"] >= 0 else 0.0
    half = 2.0 * math.pi / len(grid)
    ref = [th0 + v * half for v in u]
    o = oracle.align(c["A"], c["MA"], B, MB, q, q, grid + ref, 0.5)
    return og, ref, o


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_two_stage_matches_oracle(gpu, oracle, precision):
    cm, torch = gpu
    q = 4
    c = synth.random_case(4242, 64, 64, 64, 64, q, q, mask_density=None,
                          smooth=2.5)
    # B: A turned by -13 degrees about its centre (mask carried), so the
    # alignment angle lies between grid points 0 and 30 degrees
    B, MB = oracle.warp_nn(c["A"], c["MA"], math.radians(-13.0))
    grid = [math.radians(30.0 * k) for k in range(12)]
    u = np.random.default_rng(2106).uniform(-1.0, 1.0, 32)
    ins = [dev(torch, x) for x in (c["A"], c["MA"], B, MB)]
    say(f"[gpu] two-stage alignment {precision}")
    r = cm.align_two_stage(*ins, (64, 64, 64, 64), q, q, grid,
                           refine_offsets=u, precision=precision)
    say(f"two-stage {r['stage']} best {r['best']} grid {r['grid_best']}")
    og, ref, o = _oracle_two_stage(oracle, c, B, MB, q, grid, list(u))
    g = r["grid_best"]
    assert g["angle_index"] == og["angle_index"]
    assert abs(g["mi"] - og["mi"]) <= MI_TOL
    assert r["best"]["mi"] >= g["mi"]
    b = r["best"]
    k = b["angle_index"]
    if (k, b["dy"], b["dx"]) != (o["angle_index"], o["dy"], o["dx"]):
        # near-tie: the oracle's own value at the GPU's pick
        th = (grid + ref)[k]
        mo, _, _ = oracle.cmif_at(c["A"], c["MA"], *oracle.warp_nn(B, MB, th),
                                  q, q, b["dy"], b["dx"])
        assert abs(mo - o["mi"]) <= MI_TOL, (b, o)
    assert abs(b["mi"] - o["mi"]) <= MI_TOL and b["n"] == o["n"]
    # the refinement found the turn more closely than the 30-degree grid
    assert r["stage"] == "refine" and k >= len(grid)
    assert b["angle_rad"] == ref[k - len(grid)]
    rb = r["refine_best"]
    assert rb["angle_index"] == k - len(grid) and rb["mi"] == b["mi"]
    assert abs(math.degrees(b["angle_rad"]) - 13.0) < 6.0


def test_two_stage_batch_and_corner_error(gpu, oracle):
    """Two image pairs in one plan (each refined around its own grid angle)
    on rotated, moved, relabelled synthetic pairs with known transforms:
    per pair the oracle's two-stage result, and the corner error of the
    paper's success measure below 2 % of the width."""
    cm, torch = gpu
    n, q = 96, 6
    cases = [synth.rotated_case(5150 + k, n, q) for k in range(2)]
    grid = [-math.pi + 2.0 * math.pi * i / 36 for i in range(36)]
    u = list(np.random.default_rng(7).uniform(-1.0, 1.0, 16))
    plan = cm.Plan([(n, n, n, n)] * 2, q, q, angles=grid)
    ins = [[dev(torch, c[k]) for c in cases] for k in ("A", "MA", "B", "MB")]
    say("[gpu] two-stage alignment, two pairs in one plan")
    r = plan.align_two_stage(*ins, refine_offsets=u)
    for p, c in enumerate(cases):
        og, ref, o = _oracle_two_stage(oracle, c, c["B"], c["MB"], q, grid, u)
        b = r["best"][p]
        assert abs(b["mi"] - o["mi"]) <= MI_TOL, (p, b, o)
        assert r["grid_best"][p]["angle_index"] == og["angle_index"]
        err = cm.cmif_corner_error(b, (n, n, n, n), c["truth"])
        say(f"pair {p}: best angle {math.degrees(b['angle_rad']):.2f} deg "
            f"chi ({b['dy']},{b['dx']}) truth {c['theta_deg']:.2f} deg shift "
            f"{c['shift']}: corner error {err:.2f} px")
        assert err < 0.02 * n
