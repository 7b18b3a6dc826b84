"""GPU: the two-stage global alignment of Sec. 3.6 (grid search, then
random search around the grid's best angle).  Its result must equal the
oracle's Alg. 1 over the grid followed by the refinement angles (a later
angle wins only with a strictly larger MI), up to the near-tie rule."""

import math

import numpy as np
import pytest

import synth
from gpu_common import MI_TOL, dev, say

pytestmark = pytest.mark.gpu


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
    rng = np.random.default_rng(2106)
    ins = [dev(torch, x) for x in (c["A"], c["MA"], B, MB)]
    say(f"[gpu] two-stage alignment {precision}")
    r = cm.align_two_stage(*ins, (64, 64, 64, 64), q, q, grid, rng=rng,
                           precision=precision)
    say(f"two-stage {r['stage']} best {r['best']} grid {r['grid_best']}")
    g = r["grid_best"]
    lo = g["angle_rad"] - 2 * math.pi / 12
    hi = g["angle_rad"] + 2 * math.pi / 12
    assert len(r["refine_angles"]) == 32
    assert all(lo <= t <= hi for t in r["refine_angles"])
    assert r["best"]["mi"] >= g["mi"]
    o = oracle.align(c["A"], c["MA"], B, MB, q, q, grid + r["refine_angles"],
                     0.5)
    b = r["best"]
    k = b["angle_index"] + (12 if r["stage"] == "refine" else 0)
    if (k, b["dy"], b["dx"]) != (o["angle_index"], o["dy"], o["dx"]):
        # near-tie: the oracle's own value at the GPU's pick
        th = (grid + r["refine_angles"])[k]
        mo, _, _ = oracle.cmif_at(c["A"], c["MA"], *oracle.warp_nn(B, MB, th),
                                  q, q, b["dy"], b["dx"])
        assert abs(mo - o["mi"]) <= MI_TOL, (b, o)
    assert abs(b["mi"] - o["mi"]) <= MI_TOL and b["n"] == o["n"]
    # the refinement found the turn more closely than the 30-degree grid
    assert r["stage"] == "refine"
    assert abs(math.degrees(b["angle_rad"]) - 13.0) < 6.0
