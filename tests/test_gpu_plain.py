"""GPU: the paper-shaped plain FP64 schedule (every transform alone, separate
product and entropy kernels, materialised maps, host sync per angle) gives
the fused path's results: N exact, MI within 1e-12 of the oracle, the same
per-angle and global argmax."""

import math

import numpy as np
import pytest

import synth
from gpu_common import MI_TOL, argmax_ok, dev, say

pytestmark = pytest.mark.gpu

PLAIN = 1 << 3  # CMIF_FLAG_PLAIN_SCHEDULE


@pytest.mark.parametrize("case", [(64, 64, 64, 64, 4, 4, None),
                                  (37, 53, 29, 61, 3, 5, 0.8),
                                  (90, 17, 100, 250, 4, 7, 0.6)],
                         ids=["64-q4", "37x53-29x61-q35", "90x17-100x250-q47"])
def test_plain_matches_oracle_and_fused(gpu, oracle, case):
    cm, torch = gpu
    ha, wa, hb, wb, qa, qb, dens = case
    c = synth.random_case(3000 + ha * wa, ha, wa, hb, wb, qa, qb,
                          mask_density=dens)
    angles = [0.0, math.radians(21.0), math.pi]
    ins = [dev(torch, c[k]) for k in ("A", "MA", "B", "MB")]
    say(f"[gpu] plain schedule {case}")
    plain = cm.Plan([(ha, wa, hb, wb)], qa, qb, angles=angles,
                    precision="fp64", flags=PLAIN)
    rp = plain.compute(*ins, mi=True, n=True, best=True, per_angle=True)
    fused = cm.Plan([(ha, wa, hb, wb)], qa, qb, angles=angles, precision="fp64")
    rf = fused.compute(*ins, mi=True, n=True, best=True, per_angle=True)
    for k, th in enumerate(angles):
        bw, mw = oracle.warp_nn(c["B"], c["MB"], th)
        o = oracle.cmif_direct(c["A"], c["MA"], bw, mw, qa, qb)
        n = rp["n"][0][k].cpu().numpy()
        mi = rp["mi"][0][k].cpu().numpy()
        assert np.array_equal(n, o["n"])
        assert np.abs(mi - o["mi"]).max() <= MI_TOL
        pp, pf = rp["per_angle"][0][k], rf["per_angle"][0][k]
        ok, _ = argmax_ok(oracle, o["mi"], o["n"], 0.5,
                          (pp["dy"] + ha - 1) * o["mi"].shape[1] + pp["dx"] + wa - 1)
        assert ok
        assert abs(pp["mi"] - pf["mi"]) <= MI_TOL
    assert abs(rp["best"][0]["mi"] - rf["best"][0]["mi"]) <= MI_TOL
