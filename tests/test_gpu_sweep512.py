"""GPU parity at the full sweep workload (512x512, Q 16, 180 angles at 2
degrees, 8 angles per pass: the launch configuration bench.py times).

The oracle computes three angles' full maps (the identity, the planted
angle's neighbour and one more) with counts digests, and every angle's MI
and N at sampled displacements one by one; the GPU's per-angle argmax for
the three full angles and the global Alg. 1 result are checked against it,
and against the planted transform."""

import math

import numpy as np
import pytest

import synth
from gpu_common import MI_TOL, argmax_ok, dev, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sweep(gpu):
    cm, torch = gpu
    c = synth.config3()
    ins = [dev(torch, c[k]) for k in ("A", "MA", "B", "MB")]
    say("[gpu] sweep 512x512 q16 180 angles: compute + align")
    plan = cm.Plan([(512, 512, 512, 512)], 16, 16, angles=c["angles"],
                   gamma=c["gamma"], precision="fp32")
    assert plan.info()["angle_batch"] == 8
    res = plan.compute(*ins, mi=True, n=True, digest=True, best=True,
                       per_angle=True)
    al = plan.align(*ins, per_angle=True)
    return c, plan, res, al


def test_sweep_full_angles_vs_oracle(sweep, oracle):
    c, plan, res, al = sweep
    n_ang = len(c["angles"])
    truth = int(round(c["theta_deg"] / 2.0)) % n_ang
    for k in sorted({0, truth, 97}):
        th = c["angles"][k]
        bw, mw = oracle.warp_nn(c["B"], c["MB"], th)
        say(f"oracle full map, angle {k} ({math.degrees(th):.0f} deg)")
        o = oracle.cmif_direct(c["A"], c["MA"], bw, mw, 16, 16, digest=True)
        assert np.array_equal(res["digest"][0][k].cpu().numpy().view(np.uint64),
                              o["digest"])
        n = res["n"][0][k].cpu().numpy()
        mi = res["mi"][0][k].cpu().numpy()
        assert np.array_equal(n, o["n"])
        assert np.abs(mi - o["mi"]).max() <= MI_TOL
        pa = res["per_angle"][0][k]
        ok, near = argmax_ok(oracle, o["mi"], o["n"], c["gamma"],
                             (pa["dy"] + 511) * 1023 + pa["dx"] + 511)
        assert ok and pa["angle_index"] == k
        assert al["per_angle"][0][k] == pa


def test_sweep_sampled_shifts_all_angles(sweep, oracle):
    c, plan, res, al = sweep
    rng = np.random.default_rng(2106)
    idx = [(int(rng.integers(0, 1023)), int(rng.integers(0, 1023)))
           for _ in range(6)] + [(511, 511), (511 + c["shift"][0], 511 + c["shift"][1])]
    ii = np.array([p[0] for p in idx])
    jj = np.array([p[1] for p in idx])
    mi_s = res["mi"][0][:, ii, jj].cpu().numpy()
    n_s = res["n"][0][:, ii, jj].cpu().numpy()
    for k, th in enumerate(c["angles"]):
        bw, mw = oracle.warp_nn(c["B"], c["MB"], th)
        for s, (i, j) in enumerate(idx):
            mi, n, _ = oracle.cmif_at(c["A"], c["MA"], bw, mw, 16, 16,
                                      i - 511, j - 511)
            assert n_s[k, s] == n, (k, i, j)
            assert abs(mi_s[k, s] - mi) <= MI_TOL, (k, i, j)
    say(f"sampled {len(idx)} shifts x {len(c['angles'])} angles")


def test_sweep_alignment_result(sweep):
    c, plan, res, al = sweep
    b = al["best"][0]
    assert b == res["best"][0]
    # planted: theta 301.893 deg, shift (-82, 31); the grid has 2-degree steps
    assert b["angle_index"] == 151 and (b["dy"], b["dx"]) == tuple(c["shift"])
    assert al["stats"]["flagged_pairs"] == al["stats"]["fallback_pairs"]
    assert al["stats"]["max_residual"] < 0.25
    assert al["stats"]["unresolved_pairs"] == 0
    # the paper's success measure (Sec. 5.2): mean corner error < 2 % of
    # the width against the planted transform
    import paper_2106_14699_amd as cm
    err = cm.cmif_corner_error(b, (512, 512, 512, 512), c["truth"])
    say(f"best {b}; stats {al['stats']}; corner error {err:.3f} px")
    assert err < 0.02 * 512
