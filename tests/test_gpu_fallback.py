"""GPU: the FP64 re-run of flagged label pairs (Sec. 3.2: transforms whose
rounding residual is too large are recomputed in double precision) and the
precision stress case (1024x1024, Q = 16, FFT length 2048).

The re-run must leave every result exactly as the oracle has it: forced
through it (CMIF_FLAG_FORCE_FALLBACK) the counts, digests and N are
bit-exact and the MI maps are bitwise the ones of the plain FP32 pass (the
same integer counts enter the same FP64 sums in the same order)."""

import math

import numpy as np
import pytest

import synth
from gpu_common import MI_TOL, check_map, dev, run_compute, say

pytestmark = pytest.mark.gpu

FORCE = 1  # CMIF_FLAG_FORCE_FALLBACK

CASES = [
    # ha, wa, hb, wb, qa, qb, mask density, angles (degrees), batch, capacity
    (64, 64, 64, 64, 4, 4, None, [0.0, 33.0, 270.0], 0, 0),
    (37, 53, 29, 61, 3, 5, 0.8, [0.0, -12.5], 0, 64),
    (90, 17, 100, 250, 4, 7, 0.6, [0.0], 0, 28),
    (200, 199, 57, 3, 6, 6, 0.9, [0.0, 90.0, 181.0, 45.0], 2, 72),
]


def _ids(c):
    return f"{c[0]}x{c[1]}-{c[2]}x{c[3]}-q{c[4]}{c[5]}-a{len(c[7])}-cap{c[9]}"


@pytest.mark.parametrize("case", CASES, ids=[_ids(c) for c in CASES])
def test_forced_fallback_exact(gpu, oracle, case):
    ha, wa, hb, wb, qa, qb, dens, degs, batch, cap = case
    c = synth.random_case(4000 + ha * wb + qa, ha, wa, hb, wb, qa, qb,
                          mask_density=dens)
    angles = [math.radians(d) for d in degs]
    g = run_compute(gpu, c, "fp32", angles=angles, digest=True, per_angle=True,
                    flags=FORCE, fallback_capacity=cap, angle_batch=batch,
                    tag="forced " + _ids(case))
    plain = run_compute(gpu, c, "fp32", angles=angles, digest=True,
                        per_angle=True, angle_batch=batch, tag="plain")
    for k, th in enumerate(angles):
        bw, mw = oracle.warp_nn(c["B"], c["MB"], th)
        o = oracle.cmif_direct(c["A"], c["MA"], bw, mw, qa, qb, counts=True,
                               digest=True)
        check_map(oracle, g, o, angle=k)
        assert np.array_equal(g["digest"][k], o["digest"])
    assert np.array_equal(g["mi"].view(np.uint64), plain["mi"].view(np.uint64))
    assert np.array_equal(g["n"], plain["n"])
    for k in range(len(angles)):
        pg, pp = g["per_angle"][k], plain["per_angle"][k]
        assert (pg["dy"], pg["dx"], pg["mi"]) == (pp["dy"], pp["dx"], pp["mi"])
    # every pair of every angle listed, up to the per-pass capacity
    nb = batch if batch > 0 else len(angles)
    per_pass = [min(nb, len(angles) - a0) * qa * qb
                for a0 in range(0, len(angles), nb)]
    capacity = cap if cap > 0 else 64
    kept = sum(min(p, capacity) for p in per_pass)
    st = g["stats"]
    say(f"fallback_pairs={st['fallback_pairs']} overflow={st['fallback_overflow']}"
        f" expected kept={kept}")
    assert st["fallback_pairs"] == kept
    assert st["fallback_overflow"] == sum(per_pass) - kept
    assert plain["stats"]["fallback_pairs"] == plain["stats"]["flagged_pairs"]


def test_forced_fallback_align(gpu, oracle):
    cm, torch = gpu
    c = synth.config3(n_angles=12, size=96, q=8)
    angles = [math.radians(30.0 * i) for i in range(12)]
    ins = [dev(torch, c[k]) for k in ("A", "MA", "B", "MB")]
    say("[gpu] forced-fallback align 96x96 q8 12 angles, 5 per pass")
    pf = cm.Plan([(96, 96, 96, 96)], 8, 8, angles=angles, gamma=0.5,
                 flags=FORCE, angle_batch=5, fallback_capacity=320)
    rf = pf.align(*ins, per_angle=True)
    pp = cm.Plan([(96, 96, 96, 96)], 8, 8, angles=angles, gamma=0.5,
                 angle_batch=5)
    rp = pp.align(*ins, per_angle=True)
    for k in range(12):
        a, b = rf["per_angle"][0][k], rp["per_angle"][0][k]
        assert (a["dy"], a["dx"], a["mi"], a["n"]) == (b["dy"], b["dx"], b["mi"], b["n"])
    assert rf["best"][0] == rp["best"][0]
    ref = oracle.align(c["A"], c["MA"], c["B"], c["MB"], 8, 8, angles, 0.5)
    assert abs(rf["best"][0]["mi"] - ref["mi"]) <= MI_TOL
    assert rf["stats"]["fallback_pairs"] == 12 * 64


def _sampled_shifts(rng, ha, wa, hb, wb, extra):
    pts = {(0, 0), (-(ha - 1), -(wa - 1)), (hb - 1, wb - 1), (-(ha - 1), wb - 1),
           (hb - 1, -(wa - 1))}
    pts.update(extra)
    while len(pts) < 24:
        pts.add((int(rng.integers(-(ha - 1), hb)), int(rng.integers(-(wa - 1), wb))))
    return sorted(pts)


def _stress(gpu, oracle, c, tag):
    """FP32 and FP64 plans on a 1024x1024 pair: digests equal (so are the
    counts, with overwhelming probability), MI and N at sampled shifts equal
    the oracle's direct evaluation, N sums to |M_A| |M_B|."""
    ha, wa = c["A"].shape
    hb, wb = c["B"].shape
    g32 = run_compute(gpu, c, "fp32", counts=False, digest=True, best=True,
                      tag=tag + " fp32")
    g64 = run_compute(gpu, c, "fp64", counts=False, digest=True, best=True,
                      tag=tag + " fp64")
    st = g32["stats"]
    say(f"{tag}: max residual {st['max_residual']:.4f} flagged "
        f"{st['flagged_pairs']} re-run {st['fallback_pairs']} overflow "
        f"{st['fallback_overflow']}")
    assert st["fallback_overflow"] == 0 and st["unresolved_pairs"] == 0
    assert st["fallback_pairs"] == st["flagged_pairs"]
    assert np.array_equal(g32["digest"][0], g64["digest"][0])
    assert np.array_equal(g32["n"][0], g64["n"][0])
    assert np.abs(g32["mi"][0] - g64["mi"][0]).max() <= MI_TOL
    total = int(c["MA"].astype(np.int64).sum()) * int(c["MB"].astype(np.int64).sum())
    assert int(g32["n"][0].astype(np.int64).sum()) == total
    rng = np.random.default_rng(2106)
    extra = {tuple(c["shift"])} if "shift" in c else set()
    for dy, dx in _sampled_shifts(rng, ha, wa, hb, wb, extra):
        mi, n, _ = oracle.cmif_at(c["A"], c["MA"], c["B"], c["MB"], c["qa"],
                                  c["qb"], dy, dx)
        i, j = dy + ha - 1, dx + wa - 1
        assert g32["n"][0][i, j] == n, (dy, dx)
        assert abs(g32["mi"][0][i, j] - mi) <= MI_TOL, (dy, dx)
    return g32


def test_precision_stress_1024_q16(gpu, oracle):
    c = synth.config4()
    g = _stress(gpu, oracle, c, "1024x1024-q16")
    assert g["stats"]["max_residual"] < 0.25
    b = g["best"]
    assert (b["dy"], b["dx"]) == tuple(c["shift"])


def test_precision_stress_1024_q16_full_oracle_map(gpu, oracle):
    """The stress pair's FP32-rounded map against the oracle's full direct
    map (every one of the 2047 x 2047 displacements, all 256 label pairs):
    N bit-exact everywhere, all 256 count digests equal, MI within 1e-12
    everywhere.  The oracle visits (1024^2)^2 pixel pairs (about half a
    minute on 16 host threads)."""
    import time
    c = synth.config4()
    g = run_compute(gpu, c, "fp32", counts=False, digest=True, best=True,
                    tag="1024x1024-q16 full oracle map")
    st = g["stats"]
    assert st["unresolved_pairs"] == 0
    say(f"[cpu] oracle direct map 1024x1024 q16 on {oracle.max_threads()} "
        "threads")
    t0 = time.perf_counter()
    o = oracle.cmif_direct(c["A"], c["MA"], c["B"], c["MB"], 16, 16,
                           digest=True)
    say(f"[cpu] oracle done in {time.perf_counter() - t0:.1f} s")
    assert np.array_equal(g["n"][0], o["n"]), "N map differs"
    bad = np.argwhere(g["digest"][0] != o["digest"])
    assert bad.size == 0, f"{len(bad)} label pairs' digests differ: {bad[:4]}"
    err = float(np.abs(g["mi"][0] - o["mi"]).max())
    say(f"max|dMI| vs oracle over the full map {err:.3e}; max residual "
        f"{st['max_residual']:.4f}")
    assert err <= MI_TOL
    idx, v, _ = oracle.argmax(o["mi"], o["n"], 0.5)
    b = g["best"]
    assert (b["dy"], b["dx"]) == tuple(c["shift"])
    assert divmod(idx, o["mi"].shape[1]) == (b["dy"] + 1023, b["dx"] + 1023)


def test_precision_stress_1024_q2_full_overlap(gpu, oracle):
    # two labels over full masks: joint counts up to about 2^19 at small
    # shifts, the largest FP32 transform values of any supported size; any
    # pair whose residual reaches 0.25 goes through the FP64 re-run
    c = synth.random_case(2106, 1024, 1024, 1024, 1024, 2, 2, mask_density=None)
    _stress(gpu, oracle, c, "1024x1024-q2")


def test_precision_stress_1024_q1_full_overlap(gpu, oracle):
    # one label over full masks: the joint count is N itself, up to 2^20 at
    # zero displacement, the largest value any supported size produces
    c = synth.random_case(2107, 1024, 1024, 1024, 1024, 1, 1, mask_density=None)
    g = _stress(gpu, oracle, c, "1024x1024-q1")
    assert int(g["n"][0].max()) == 1 << 20
