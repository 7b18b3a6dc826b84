"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar (counts are integers, MI is FP64 accumulation of exact counts):
  * joint counts, N and digests: bit-exact;
  * MI: |GPU - oracle| <= 1e-12 absolute on both precisions (the FP32 path
    rounds every count to the exact integer, after which the arithmetic is
    FP64; 1e-12 is the FP64-path bound and is kept for both);
  * argmax: equal to the oracle's, or the oracle's own MI at the GPU's pick
    is within 1e-12 of the oracle's maximum (near-ties from FP64 summation
    order), counted and printed.
"""

import math
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

from gpu_common import (MI_TOL, argmax_ok, check_map, dev, run_compute,
                        say)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config1_exact(gpu, oracle, precision):
    c = synth.config1()
    g = run_compute(gpu, c, precision, tag="64x64-q4")
    o = oracle.cmif_direct(c["A"], c["MA"], c["B"], c["MB"], 4, 4, counts=True)
    check_map(oracle, g, o)
    b = g["best"]
    assert (b["dy"], b["dx"]) == (7, -5), b
    idx, v, n = oracle.argmax(o["mi"], o["n"], 0.5)
    assert abs(b["mi"] - v) <= MI_TOL and b["n"] == n
    assert g["stats"]["flagged_pairs"] == 0
    assert g["stats"]["label_errors"] == 0


def test_config2_fp32_disc_mask(gpu, oracle):
    c = synth.config2()
    g = run_compute(gpu, c, "fp32", digest=True, tag="256x256-q8-disc")
    o = oracle.cmif_direct(c["A"], c["MA"], c["B"], c["MB"], 8, 8,
                           counts=True, digest=True)
    check_map(oracle, g, o)
    assert np.array_equal(g["digest"][0], o["digest"])
    b = g["best"]
    ok, near = argmax_ok(oracle, o["mi"], o["n"], 0.5,
                         (b["dy"] + 255) * o["mi"].shape[1] + (b["dx"] + 255))
    assert ok
    assert (b["dy"], b["dx"]) == tuple(c["shift"])
    say(f"config2 residual {g['stats']['max_residual']:.3e} near_tie={near}")
    assert g["stats"]["max_residual"] < 0.25


RAGGED = [
    # ha, wa, hb, wb, qa, qb, mask density, precision
    (37, 53, 29, 61, 3, 5, 0.8, "fp32"),
    (37, 53, 29, 61, 3, 5, 0.8, "fp64"),
    (1, 130, 7, 3, 2, 2, None, "fp32"),
    (90, 17, 100, 250, 4, 7, 0.6, "fp32"),
    (128, 128, 1, 1, 5, 3, None, "fp64"),
    (200, 199, 57, 3, 6, 6, 0.9, "fp32"),
    (64, 65, 65, 64, 16, 16, 0.7, "fp32"),
    (33, 31, 40, 44, 9, 13, 0.5, "fp64"),
    (20, 300, 300, 20, 2, 3, 0.9, "fp32"),
    # 3 * 2^k FFT sides (12-point first stages): 768 x 768, then 256 rows x
    # 1536 columns (the two-wave split row transform at 1536), then 1536
    # rows (column transforms at 1536) x 256 columns
    (300, 280, 310, 290, 5, 6, 0.8, "fp32"),
    (300, 280, 310, 290, 5, 6, 0.8, "fp64"),
    (100, 700, 90, 650, 3, 4, 0.9, "fp32"),
    (700, 60, 650, 80, 4, 3, 0.9, "fp64"),
    (700, 60, 650, 80, 4, 3, None, "fp32"),
]


@pytest.mark.parametrize("case", RAGGED, ids=[f"{r[0]}x{r[1]}-{r[2]}x{r[3]}-q{r[4]}{r[5]}-{r[7]}"
                                              for r in RAGGED])
def test_ragged_sizes_exact(gpu, oracle, case):
    ha, wa, hb, wb, qa, qb, dens, prec = case
    c = synth.random_case(1000 + ha * wa + hb, ha, wa, hb, wb, qa, qb,
                          mask_density=dens)
    g = run_compute(gpu, c, prec, digest=True, tag=str(case))
    o = oracle.cmif_direct(c["A"], c["MA"], c["B"], c["MB"], qa, qb,
                           counts=True, digest=True)
    check_map(oracle, g, o)
    assert np.array_equal(g["digest"][0], o["digest"])
    # exact without the FP64 re-run: the FP32 pass itself reads the pair
    # columns right (the column and row lengths differ in several cases)
    assert g["stats"]["flagged_pairs"] == 0, g["stats"]
    ok, near = argmax_ok(oracle, o["mi"], o["n"], 0.5,
                         (g["best"]["dy"] + ha - 1) * o["mi"].shape[1] +
                         g["best"]["dx"] + wa - 1)
    if g["best"]["angle_index"] >= 0:
        assert ok


def test_iid_labels_and_single_label(gpu, oracle):
    c = synth.random_case(77, 50, 60, 70, 40, 8, 8, mask_density=0.5,
                          smooth=None)
    g = run_compute(gpu, c, "fp32", tag="iid")
    o = oracle.cmif_direct(c["A"], c["MA"], c["B"], c["MB"], 8, 8, counts=True)
    check_map(oracle, g, o)
    # one label on either side: MI is exactly 0 everywhere (H_AB = H_A or
    # H_B term by term), in the oracle and on the GPU, so Alg. 1 keeps the
    # identity (angle index -1, chi = 0, I = 0)
    for prec in ("fp32", "fp64"):
        for side in ("a", "b"):
            c1 = (dict(c, A=np.zeros_like(c["A"]), qa=1) if side == "a"
                  else dict(c, B=np.zeros_like(c["B"]), qb=1))
            g1 = run_compute(gpu, c1, prec, counts=False,
                             tag=f"q{side}=1 {prec}")
            o1 = oracle.cmif_direct(c1["A"], c1["MA"], c1["B"], c1["MB"],
                                    c1["qa"], c1["qb"])
            assert np.all(o1["mi"] == 0.0)
            assert np.all(g1["mi"] == 0.0)
            assert np.array_equal(g1["n"][0], o1["n"])
            b = g1["best"]
            assert (b["angle_index"], b["dy"], b["dx"], b["mi"]) == (-1, 0, 0, 0.0)
    # an odd Q_B: the last row-transform pack carries one pair only, and its
    # unused half must count nothing (N equals the oracle's everywhere)
    c3 = synth.random_case(78, 61, 47, 55, 66, 5, 7, mask_density=0.7)
    g3 = run_compute(gpu, c3, "fp32", tag="qb=7 odd")
    o3 = oracle.cmif_direct(c3["A"], c3["MA"], c3["B"], c3["MB"], 5, 7,
                            counts=True)
    check_map(oracle, g3, o3)
    assert g["mi"].min() >= 0.0 and g3["mi"].min() >= 0.0


def test_label_out_of_range_reported(gpu, oracle):
    c = synth.random_case(5, 40, 40, 40, 40, 4, 4, mask_density=None)
    A = c["A"].copy()
    A[3, 5] = 9
    A[10, 11] = 4
    g = run_compute(gpu, dict(c, A=A), "fp32", tag="label-range")
    assert g["stats"]["label_errors"] == 2
    # those pixels belong to no level set: same counts as with them masked out
    MA = c["MA"].copy()
    MA[3, 5] = 0
    MA[10, 11] = 0
    o = oracle.cmif_direct(A, MA, c["B"], c["MB"], 4, 4, counts=True)
    assert np.array_equal(g["counts"][0], o["counts"])


def test_rotations_bit_exact(gpu, oracle):
    c = synth.random_case(31, 48, 56, 41, 37, 5, 4, mask_density=0.85)
    angles = [0.0, math.radians(17.0), math.pi / 2, math.pi,
              math.radians(251.0), -math.radians(33.3)]
    g = run_compute(gpu, c, "fp32", angles=angles, per_angle=True,
                    tag="rotations")
    for k, th in enumerate(angles):
        bw, mw = oracle.warp_nn(c["B"], c["MB"], th)
        o = oracle.cmif_direct(c["A"], c["MA"], bw, mw, 5, 4, counts=True)
        check_map(oracle, g, o, angle=k)
        pa = g["per_angle"][k]
        ok, _ = argmax_ok(oracle, o["mi"], o["n"], 0.5,
                          (pa["dy"] + 47) * o["mi"].shape[1] + pa["dx"] + 55)
        assert ok and pa["angle_index"] == k
        assert pa["angle_rad"] == th


def test_align_matches_oracle(gpu, oracle):
    cm, torch = gpu
    c = synth.config3(n_angles=12, size=96, q=8)
    angles = [math.radians(30.0 * i) for i in range(12)]
    n = 96
    plan = cm.Plan([(n, n, n, n)], 8, 8, angles=angles, gamma=0.5)
    say("[gpu] align 96x96 q8 12 angles")
    r = plan.align(dev(torch, c["A"]), dev(torch, c["MA"]), dev(torch, c["B"]),
                   dev(torch, c["MB"]), per_angle=True)
    ref = oracle.align(c["A"], c["MA"], c["B"], c["MB"], 8, 8, angles, 0.5,
                       per_angle=True)
    near = 0
    for k in range(12):
        gk, ok_ = r["per_angle"][0][k], ref["per_angle"][k]
        assert abs(gk["mi"] - ok_["mi"]) <= MI_TOL
        if (gk["dy"], gk["dx"]) != (ok_["dy"], ok_["dx"]):
            near += 1
    b = r["best"][0]
    assert abs(b["mi"] - ref["mi"]) <= MI_TOL
    if b["angle_index"] != ref["angle_index"]:
        near += 1
    say(f"align near-ties: {near}")


def test_determinism(gpu):
    c = synth.random_case(8, 100, 90, 80, 110, 6, 6, mask_density=0.8)
    g1 = run_compute(gpu, c, "fp32", counts=False, tag="det-1")
    g2 = run_compute(gpu, c, "fp32", counts=False, tag="det-2")
    assert np.array_equal(g1["mi"].view(np.uint64), g2["mi"].view(np.uint64))


def test_two_pairs_one_plan(gpu, oracle):
    cm, torch = gpu
    c1 = synth.random_case(41, 30, 44, 52, 25, 3, 4, mask_density=0.7)
    c2 = synth.random_case(42, 70, 20, 15, 66, 3, 4, mask_density=0.9)
    sizes = [(*c1["A"].shape, *c1["B"].shape), (*c2["A"].shape, *c2["B"].shape)]
    plan = cm.Plan(sizes, 3, 4, angles=[0.0, 0.3])
    say("[gpu] two pairs one plan")
    res = plan.compute([dev(torch, c1["A"]), dev(torch, c2["A"])],
                       [dev(torch, c1["MA"]), dev(torch, c2["MA"])],
                       [dev(torch, c1["B"]), dev(torch, c2["B"])],
                       [dev(torch, c1["MB"]), dev(torch, c2["MB"])],
                       counts=True)
    for p, c in enumerate((c1, c2)):
        for k, th in enumerate((0.0, 0.3)):
            bw, mw = oracle.warp_nn(c["B"], c["MB"], th)
            o = oracle.cmif_direct(c["A"], c["MA"], bw, mw, 3, 4, counts=True)
            assert np.array_equal(res["counts"][p][k].cpu().numpy(), o["counts"])
            assert np.abs(res["mi"][p][k].cpu().numpy() - o["mi"]).max() <= MI_TOL


def test_empty_overlap_everywhere(gpu, oracle):
    """All of A masked out: N = 0 at every displacement, MI = 0 (Eq. 12
    conventions), and Alg. 1 keeps the identity."""
    cm, torch = gpu
    c = synth.random_case(90, 33, 47, 29, 38, 4, 3, mask_density=0.7)
    c = dict(c, MA=np.zeros_like(c["MA"]))
    g = run_compute(gpu, c, "fp32", angles=[0.0, 0.7], digest=True,
                    tag="all-masked")
    assert not g["n"].any() and not g["mi"].any() and not g["counts"].any()
    assert not g["digest"].any()
    b = g["best"]
    assert (b["angle_index"], b["dy"], b["dx"], b["mi"], b["n"]) == (-1, 0, 0, 0.0, 0)
    o = oracle.cmif_direct(c["A"], c["MA"], c["B"], c["MB"], 4, 3)
    assert not o["n"].any()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_max_labels_64(gpu, oracle, prec):
    """Q_A = Q_B = 64 (the largest label count): 4096 label pairs."""
    c = synth.random_case(64, 40, 36, 44, 30, 64, 64, mask_density=0.9,
                          smooth=None)
    g = run_compute(gpu, c, prec, digest=True, tag="q64")
    o = oracle.cmif_direct(c["A"], c["MA"], c["B"], c["MB"], 64, 64,
                           counts=True, digest=True)
    check_map(oracle, g, o)
    assert np.array_equal(g["digest"][0], o["digest"])
