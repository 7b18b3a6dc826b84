"""GPU: 4096-point transforms (image sides above 2048 with a displacement
window, as in the paper's template-matching runs with a 4096 reference,
Sec. 5.1).

At 4096 points the forward column kernel runs part of a tile per workgroup,
the pair column kernel one or two columns per workgroup, and the row pass
splits each map row's lags over two workgroups.  Bar, as for every other
length:
  * counts, N and digests bit-exact against the oracle's full map cut to
    the window, MI within 1e-12, argmax per angle by the oracle's rule;
  * the FP64 re-run (forced for every pair) gives the same exact result;
  * the 4096 x 4096 reference with a 2048 x 2048 floating image: N is the
    full overlap everywhere, MI equals the oracle's direct evaluation at
    sampled placements, and the planted offset is recovered.
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


# a tall pair (4096 points along y: the column kernels) and a wide pair
# (along x: the row kernels), each with a window of +-1000 on the long axis
CASES = {
    "y": ((2100, 40, 2090, 36), (-1000, 1000, -39, 35), (4096, 128)),
    "x": ((40, 2100, 36, 2090), (-39, 35, -1000, 1000), (128, 4096)),
}


@pytest.mark.parametrize("axis", ["y", "x"])
@pytest.mark.parametrize("flags", [0, FORCE], ids=["fp32", "fp32-forced-rerun"])
def test_fft_4096_matches_oracle(gpu, oracle, axis, flags):
    cm, torch = gpu
    size, w, fft = CASES[axis]
    ha, wa, hb, wb = size
    qa, qb = 4, 5
    angles = [0.0, math.radians(30.0)]
    c = synth.random_case(4096 + (axis == "x"), ha, wa, hb, wb, qa, qb,
                          mask_density=0.85)
    say(f"[gpu] fft 4096 along {axis} flags={flags} sizes {size} window {w}")
    plan = cm.Plan([size], qa, qb, angles=angles, flags=flags, windows=[w])
    assert (plan.info()["fft_h"], plan.info()["fft_w"]) == fft
    ins = [dev(torch, c[k]) for k in ("A", "MA", "B", "MB")]
    r = plan.compute(*ins, mi=True, n=True, counts=True, digest=True,
                     per_angle=True)
    st = r["stats"]
    if flags & FORCE:
        assert st["fallback_pairs"] == len(angles) * qa * qb, st
    else:
        # the FP32 pass is exact on its own (column length 4096, row length
        # 128, or the reverse: both read one layout of the pair columns)
        assert st["flagged_pairs"] == 0, st
    assert st["unresolved_pairs"] == 0 and st["label_errors"] == 0, st
    for k, th in enumerate(angles):
        bw, mw = oracle.warp_nn(c["B"], c["MB"], th)
        o = _cut(oracle.cmif_direct(c["A"], c["MA"], bw, mw, qa, qb,
                                    counts=True), ha, wa, w)
        g_mi = r["mi"][0][k].cpu().numpy()
        assert np.array_equal(r["n"][0][k].cpu().numpy(), o["n"]), k
        assert np.array_equal(r["counts"][0][k].cpu().numpy(), o["counts"]), k
        dg = r["digest"][0][k].cpu().numpy().view(np.uint64)
        assert np.array_equal(dg, _digest(oracle, o["counts"])), k
        err = float(np.abs(g_mi - o["mi"]).max())
        assert err <= MI_TOL, (k, err)
        b = r["per_angle"][0][k]
        g_idx = (b["dy"] - w[0]) * o["mi"].shape[1] + (b["dx"] - w[2])
        ok, _ = argmax_ok(oracle, o["mi"], o["n"], 0.5, g_idx)
        assert ok, (k, b)
        say(f"  angle {math.degrees(th):.0f}: max|dMI| {err:.2e} best "
            f"({b['dy']},{b['dx']})")


def test_template_matching_4096_reference(gpu, oracle):
    """A 4096 x 4096 reference and a 2048 x 2048 floating image cut from it,
    the map over every placement (window [-2048, 0]^2, FFT 4096 per axis),
    Q 16: N = 2048^2 everywhere, MI equal to the oracle's direct evaluation
    at sampled placements, the planted offset recovered."""
    cm, torch = gpu
    c = synth.template_pair(4096)
    w = c["window"]
    plan = cm.Plan([(4096, 4096, 2048, 2048)], 16, 16, windows=[w])
    assert (plan.info()["fft_h"], plan.info()["fft_w"]) == (4096, 4096)
    say(f"[gpu] template 4096/2048 offset {c['offset']}")
    r = plan.compute(dev(torch, c["A"]), None, dev(torch, c["B"]), None,
                     mi=True, n=True, best=True)
    assert r["stats"]["unresolved_pairs"] == 0, r["stats"]
    n = r["n"][0][0].cpu().numpy()
    mi = r["mi"][0][0].cpu().numpy()
    assert n.shape == (2049, 2049) and np.all(n == 2048 * 2048)
    rng = np.random.default_rng(4096)
    off = c["offset"]
    pts = {(0, 0), (2048, 2048), (0, 2048), (2048, 0), (1024, 1024),
           (off[0], off[1])}
    while len(pts) < 12:
        pts.add((int(rng.integers(0, 2049)), int(rng.integers(0, 2049))))
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
