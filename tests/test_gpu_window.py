"""GPU: displacement windows (the padded search window of Alg. 1).

A plan may restrict each image pair to a window [y0, y1] x [x0, x1] of the
full displacement set.  The maps, counts, digests and argmax then cover the
window only, and the FFT side is the alias-free size for the window.  Bar:
  * counts, N and digests (taken over the window's own map indices):
    bit-exact against the oracle's full map cut to the window;
  * MI: <= 1e-12 against the oracle, and bitwise equal to the same plan
    without a window (the same integer counts reduced in the same order);
  * argmax per angle: the oracle's argmax over the window, gamma taken
    relative to the window's max N (near-ties accepted as elsewhere).
"""

import math

import numpy as np
import pytest

import synth
from gpu_common import MI_TOL, argmax_ok, dev, say

pytestmark = pytest.mark.gpu

FORCE = 1 << 0


def _cut(o, ha, wa, w):
    y0, y1, x0, x1 = w
    rs = slice(y0 + ha - 1, y1 + ha)
    cs = slice(x0 + wa - 1, x1 + wa)
    return dict(mi=o["mi"][rs, cs], n=o["n"][rs, cs],
                counts=o["counts"][:, :, rs, cs])


def _digest(oracle, counts):
    qa, qb, sh, sw = counts.shape
    w = np.array([oracle.digest_weight(i) for i in range(sh * sw)], np.uint64)
    flat = counts.reshape(qa, qb, sh * sw).astype(np.uint64)
    return (flat * w[None, None, :]).sum(axis=2, dtype=np.uint64)


# (ha, wa, hb, wb) per pair and a window per pair: containing 0, all
# positive, all negative, one displacement, one row
SIZES = [(41, 47, 36, 52), (33, 40, 45, 38), (30, 44, 30, 44), (25, 31, 28, 27),
         (38, 35, 33, 29), (150, 140, 160, 150)]
WINDOWS = [(-12, 9, -20, 14), (3, 30, 5, 37), (-29, -6, -30, -2), (4, 4, -7, -7),
           (-5, -5, -34, 28), (-30, 30, -20, 25)]
# the last pair: FFT 256 x 256 with its window, 512 x 512 for the full set


@pytest.mark.parametrize("precision,flags", [("fp32", 0), ("fp64", 0),
                                             ("fp32", FORCE)],
                         ids=["fp32", "fp64", "fp32-forced-rerun"])
def test_windows_match_oracle_and_full_maps(gpu, oracle, precision, flags):
    cm, torch = gpu
    qa, qb = 4, 5
    angles = [0.0, math.radians(25.0), math.radians(160.0)]
    cases = [synth.random_case(900 + k, *s, qa, qb, mask_density=0.85)
             for k, s in enumerate(SIZES)]
    say(f"[gpu] windows {precision} flags={flags} pairs={len(SIZES)}")
    pw = cm.Plan(SIZES, qa, qb, angles=angles, precision=precision,
                 flags=flags, windows=WINDOWS)
    pf = cm.Plan(SIZES, qa, qb, angles=angles, precision=precision, flags=flags)
    ins = [[dev(torch, c[k]) for c in cases] for k in ("A", "MA", "B", "MB")]
    rw = pw.compute(*ins, mi=True, n=True, counts=True, digest=True,
                    per_angle=True)
    rf = pf.compute(*ins, mi=True, n=True)
    near = 0
    last = len(SIZES) - 1
    assert cm.cmif_plan_query(pw.handle)["fft_h"] == 128  # pair 0
    assert pw.map_shape(last) == (61, 46)
    for p, (s, w, c) in enumerate(zip(SIZES, WINDOWS, cases)):
        ha, wa, hb, wb = s
        assert tuple(rw["mi"][p].shape[1:]) == (w[1] - w[0] + 1, w[3] - w[2] + 1)
        for k, th in enumerate(angles):
            bw, mw = oracle.warp_nn(c["B"], c["MB"], th)
            o = _cut(oracle.cmif_direct(c["A"], c["MA"], bw, mw, qa, qb,
                                        counts=True), ha, wa, w)
            g_mi = rw["mi"][p][k].cpu().numpy()
            g_n = rw["n"][p][k].cpu().numpy()
            assert np.array_equal(g_n, o["n"]), (p, k)
            assert np.array_equal(rw["counts"][p][k].cpu().numpy(), o["counts"]), (p, k)
            assert np.abs(g_mi - o["mi"]).max() <= MI_TOL, (p, k)
            dg = rw["digest"][p][k].cpu().numpy().view(np.uint64)
            assert np.array_equal(dg, _digest(oracle, o["counts"])), (p, k)
            # the windowed map is the full map's cut, bit for bit
            y0, y1, x0, x1 = w
            full = rf["mi"][p][k].cpu().numpy()[y0 + ha - 1:y1 + ha,
                                                 x0 + wa - 1:x1 + wa]
            assert np.array_equal(g_mi.view(np.uint64), full.view(np.uint64)), (p, k)
            b = rw["per_angle"][p][k]
            g_idx = (b["dy"] - y0) * o["mi"].shape[1] + (b["dx"] - x0)
            ok, nt = argmax_ok(oracle, o["mi"], o["n"], 0.5, g_idx)
            assert ok, (p, k, b)
            near += int(nt)
    say(f"windows {precision}: near-ties {near}")


def test_window_shrinks_fft_and_aligns(gpu, oracle):
    """A window of +-40 around 0 on 200 x 200 images needs P >= 240 (256)
    instead of 512 for the full set; the alignment over angles equals the
    oracle's Alg. 1 over the window."""
    cm, torch = gpu
    n, q = 200, 6
    c = synth.random_case(1234, n, n, n, n, q, q, mask_density=None)
    # B is A moved by (11, -7): the best displacement is inside the window
    B = np.zeros_like(c["A"])
    B[11:, :n - 7] = c["A"][:n - 11, 7:]
    MB = np.zeros_like(B)
    MB[11:, :n - 7] = 1
    angles = [math.radians(a) for a in (-4.0, 0.0, 4.0)]
    win = [(-40, 40, -40, 40)]
    plan = cm.Plan([(n, n, n, n)], q, q, angles=angles, windows=win)
    info = plan.info()
    say(f"window plan fft {info['fft_h']}x{info['fft_w']}")
    assert (info["fft_h"], info["fft_w"]) == (256, 256)
    full = cm.Plan([(n, n, n, n)], q, q, angles=angles)
    assert (full.info()["fft_h"], full.info()["fft_w"]) == (512, 512)
    r = plan.align(*[dev(torch, x) for x in (c["A"], c["MA"], B, MB)],
                   per_angle=True)
    best = r["best"][0]
    assert (best["dy"], best["dx"], best["angle_index"]) == (11, -7, 1), best
    # per angle against the oracle over the window
    for k, th in enumerate(angles):
        bw, mw = oracle.warp_nn(B, MB, th)
        o = _cut(oracle.cmif_direct(c["A"], c["MA"], bw, mw, q, q, counts=True),
                 n, n, win[0])
        b = r["per_angle"][0][k]
        g_idx = (b["dy"] + 40) * 81 + (b["dx"] + 40)
        ok, _ = argmax_ok(oracle, o["mi"], o["n"], 0.5, g_idx)
        assert ok, (k, b)
        i, j = divmod(g_idx, 81)
        assert b["n"] == o["n"][i, j]
        assert abs(b["mi"] - o["mi"][i, j]) <= MI_TOL
    assert r["stats"]["label_errors"] == 0


def test_template_matching_window(gpu, oracle):
    """The paper's run-time experiment shape at a small side: a 128 x 128
    reference, the floating image half of it cut at a seeded offset, the
    map over every placement (window [-(64), 0]^2, FFT 128 instead of 256
    for the full set); map equal to the oracle's cut, offset recovered."""
    cm, torch = gpu
    c = synth.template_pair(128)
    w = c["window"]
    plan = cm.Plan([(128, 128, 64, 64)], 16, 16, windows=[w])
    assert (plan.info()["fft_h"], plan.info()["fft_w"]) == (128, 128)
    say(f"[gpu] template 128/64 offset {c['offset']}")
    r = plan.compute(dev(torch, c["A"]), None, dev(torch, c["B"]), None,
                     mi=True, n=True, counts=True, best=True)
    ones_a = np.ones_like(c["A"])
    ones_b = np.ones_like(c["B"])
    o = _cut(oracle.cmif_direct(c["A"], ones_a, c["B"], ones_b, 16, 16,
                                counts=True), 128, 128, w)
    assert np.array_equal(r["n"][0][0].cpu().numpy(), o["n"])
    assert np.all(o["n"] == 64 * 64)  # every placement overlaps fully
    assert np.array_equal(r["counts"][0][0].cpu().numpy(), o["counts"])
    assert np.abs(r["mi"][0][0].cpu().numpy() - o["mi"]).max() <= MI_TOL
    b = r["best"][0]
    assert (-b["dy"], -b["dx"]) == tuple(c["offset"]), (b, c["offset"])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_gamma_window_at_fft_768(gpu, oracle, precision):
    """Alg. 1's padded window for gamma = 0.5 on a 400 x 400 rotated pair:
    |chi| <= 200 per axis needs P >= 600, so the windowed plan runs at 768
    (3 * 2^8) where the full set needs 1024.  Counts, N and digests equal
    the oracle's full map cut to the window, MI within 1e-12 of the oracle
    and of the full plan's cut (the 1024-point plan may group the FP64
    entropy sums over other team shapes, so bitwise equality is not
    implied), argmax per angle by the oracle's rule."""
    cm, torch = gpu
    c = synth.config3(n_angles=1, size=400, q=8)
    n, q = 400, 8
    angles = [0.0, math.radians(round(c["theta_deg"] / 2.0) * 2.0),
              math.radians(90.0)]
    w = (-200, 200, -200, 200)
    pw = cm.Plan([(n, n, n, n)], q, q, angles=angles, precision=precision,
                 windows=[w])
    pf = cm.Plan([(n, n, n, n)], q, q, angles=angles, precision=precision)
    assert (pw.info()["fft_h"], pw.info()["fft_w"]) == (768, 768)
    assert (pf.info()["fft_h"], pf.info()["fft_w"]) == (1024, 1024)
    say(f"[gpu] gamma window +-200 on 400x400 q8 {precision} at FFT 768")
    ins = [dev(torch, c[k]) for k in ("A", "MA", "B", "MB")]
    rw = pw.compute(*ins, mi=True, n=True, counts=True, digest=True,
                    per_angle=True)
    rf = pf.compute(*ins, mi=True, n=True)
    for k, th in enumerate(angles):
        bw, mw = oracle.warp_nn(c["B"], c["MB"], th)
        o = _cut(oracle.cmif_direct(c["A"], c["MA"], bw, mw, q, q, counts=True),
                 n, n, w)
        g_mi = rw["mi"][0][k].cpu().numpy()
        assert np.array_equal(rw["n"][0][k].cpu().numpy(), o["n"]), k
        assert np.array_equal(rw["counts"][0][k].cpu().numpy(), o["counts"]), k
        dg = rw["digest"][0][k].cpu().numpy().view(np.uint64)
        assert np.array_equal(dg, _digest(oracle, o["counts"])), k
        err = float(np.abs(g_mi - o["mi"]).max())
        assert err <= MI_TOL, (k, err)
        full = rf["mi"][0][k].cpu().numpy()[200 + n - 1 - 400:200 + n,
                                             200 + n - 1 - 400:200 + n]
        assert float(np.abs(g_mi - full).max()) <= MI_TOL, k
        b = rw["per_angle"][0][k]
        g_idx = (b["dy"] + 200) * 401 + (b["dx"] + 200)
        ok, _ = argmax_ok(oracle, o["mi"], o["n"], 0.5, g_idx)
        assert ok, (k, b)
        say(f"  angle {math.degrees(th):.1f}: max|dMI| {err:.2e} best "
            f"({b['dy']},{b['dx']}) mi {b['mi']:.6f}")


def test_template_matching_2048_reference(gpu, oracle):
    """The paper's run-time experiment shape at a 2048 x 2048 reference and
    a 1024 x 1024 floating image cut from it: the map over every placement
    (window [-1024, 0]^2, FFT 2048 per axis; the full displacement set would
    need 4095).  N is the full overlap 1024^2 everywhere, MI equals the
    oracle's direct evaluation at sampled placements (corners, centre, the
    planted offset, random), and the planted offset is recovered."""
    cm, torch = gpu
    c = synth.template_pair(2048)
    w = c["window"]
    plan = cm.Plan([(2048, 2048, 1024, 1024)], 16, 16, windows=[w])
    assert (plan.info()["fft_h"], plan.info()["fft_w"]) == (2048, 2048)
    say(f"[gpu] template 2048/1024 offset {c['offset']}")
    r = plan.compute(dev(torch, c["A"]), None, dev(torch, c["B"]), None,
                     mi=True, n=True, best=True)
    n = r["n"][0][0].cpu().numpy()
    mi = r["mi"][0][0].cpu().numpy()
    assert n.shape == (1025, 1025) and np.all(n == 1024 * 1024)
    rng = np.random.default_rng(2048)
    off = c["offset"]
    pts = {(0, 0), (1024, 1024), (0, 1024), (1024, 0), (512, 512),
           (off[0], off[1])}
    while len(pts) < 12:
        pts.add((int(rng.integers(0, 1025)), int(rng.integers(0, 1025))))
    ones_a = np.ones_like(c["A"])
    ones_b = np.ones_like(c["B"])
    for oy, ox in sorted(pts):
        mo, no, _ = oracle.cmif_at(c["A"], ones_a, c["B"], ones_b, 16, 16,
                                   -oy, -ox)
        i, j = -oy - w[0], -ox - w[2]
        assert n[i, j] == no
        assert abs(mi[i, j] - mo) <= MI_TOL, (oy, ox, mi[i, j], mo)
    b = r["best"][0]
    say(f"best {b}; planted {off}")
    assert (-b["dy"], -b["dx"]) == tuple(off)
