"""Seeded synthetic inputs for the CMIF workloads.

This module generates label images, masks and soft memberships shaped like the
workloads of the paper's run-time and alignment experiments (Sec. 5: 300^2 to
834^2 images, k = 8..64 quantisation levels, rotation sweeps).  The paper's
datasets are not available, so blurred Gaussian random fields quantised into
equal-population levels stand in for k-means-quantised micrographs.

It holds none of the method's arithmetic: no histogram, correlation, entropy,
warp-by-fixed-point or argmax.  Both the CPU oracle and the GPU path consume
what it returns, and nothing here imports either of them.

Recipe (shared primitives):
  * seed = 2106_14699 + 10 * config + i, drawn with numpy.random.default_rng;
    draws happen in the order field, noise, shift, angle, permutation.
  * field(sigma): N(0,1) samples, Gaussian blur (wrap, truncate 4), then
    standardised to mean 0 / std 1.
  * qq(v, Q, mask): equal-population quantiser; thresholds are the masked
    values' quantiles k/Q (k = 1..Q-1) and a value's label is the number of
    thresholds <= it.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import ndimage

BASE_SEED = 2106_14699


def seed_for(config: int, i: int = 0) -> int:
    return BASE_SEED + 10 * config + i


def field(rng: np.random.Generator, sigma: float, shape) -> np.ndarray:
    z = rng.standard_normal(shape)
    f = ndimage.gaussian_filter(z, sigma, mode="wrap", truncate=4.0)
    f = f - f.mean()
    return f / f.std()


def qq(v: np.ndarray, q: int, mask: np.ndarray | None = None) -> np.ndarray:
    sel = v if mask is None else v[mask.astype(bool)]
    t = np.quantile(sel, np.arange(1, q) / q)
    return np.searchsorted(t, v, side="right").astype(np.uint8)


def disc_mask(h: int, w: int, radius: float) -> np.ndarray:
    y, x = np.mgrid[0:h, 0:w]
    cy, cx = (h - 1) / 2.0, (w - 1) / 2.0
    return (((y - cy) ** 2 + (x - cx) ** 2) <= radius * radius).astype(np.uint8)


def _shifted_pair(rng, sigma, h, w, q, shift_range, fixed_shift, g,
                  noise_sd, mask_a=None):
    """A = qq(F window), B(y) = qq(g(F(y - s)) + noise): the content of A at x
    reappears in B at x + s, so the CMIF peak sits at displacement s.
    Draw order: field, noise, shift."""
    m = shift_range
    canvas = field(rng, sigma, (h + 2 * m, w + 2 * m))
    noise = rng.standard_normal((h, w))
    if fixed_shift is None:
        s = tuple(int(v) for v in rng.integers(-m, m + 1, size=2))
    else:
        s = tuple(int(v) for v in fixed_shift)
    sy, sx = s
    fa = canvas[m:m + h, m:m + w]
    fb = canvas[m - sy:m - sy + h, m - sx:m - sx + w]
    a = qq(fa, q, mask_a)
    b = qq(g(fb) + noise_sd * noise, q)
    return a, b, s


def config1():
    """64x64, Q=4, blur sigma 3, B = quantised cos(2.5 f) + 0.2 N(0,1) moved
    by (7, -5); all-ones masks; one angle, FP64 path."""
    rng = np.random.default_rng(seed_for(1))
    a, b, s = _shifted_pair(rng, 3.0, 64, 64, 4, 16, (7, -5),
                            lambda v: np.cos(2.5 * v), 0.2)
    ones = np.ones((64, 64), np.uint8)
    return dict(name="plain-64x64-q4", A=a, MA=ones, B=b, MB=ones.copy(),
                qa=4, qb=4, angles=[0.0], gamma=0.5, shift=s)


def config2():
    """256x256, Q=8 (64 pairs), blur sigma 4, B = quantised sin(3 f) +
    0.3 N(0,1) moved by a seeded shift in [-40, 40]^2; A mask = centred disc
    of radius 120 (A's quantiles taken inside it), B mask all ones."""
    rng = np.random.default_rng(seed_for(2))
    ma = disc_mask(256, 256, 120.0)
    a, b, s = _shifted_pair(rng, 4.0, 256, 256, 8, 40, None,
                            lambda v: np.sin(3.0 * v), 0.3, mask_a=ma)
    return dict(name="single-256x256-q8-disc", A=a, MA=ma, B=b,
                MB=np.ones((256, 256), np.uint8), qa=8, qb=8, angles=[0.0],
                gamma=0.5, shift=s)


def rotated_intensities(rng, sigma, n, margin, shift_range, noise_sd):
    """Intensity images: A = F on the window, B(p) = cos(2.5 F(src(p))) +
    noise with src(p) = R(-theta)(p - c) + c - s, evaluated in FP64 and
    rounded to the nearest canvas pixel; M_B marks points whose source lies
    inside A's window.  Rotating B back by theta and moving it by -s
    recovers A's geometry.  Draw order: field, noise, shift, angle.
    Returns (A, B, M_B, s, theta) with A, B in FP64."""
    canvas = field(rng, sigma, (n + 2 * margin, n + 2 * margin))
    noise = rng.standard_normal((n, n))
    s = tuple(int(v) for v in rng.integers(-shift_range, shift_range + 1,
                                           size=2))
    theta = float(rng.uniform(0.0, 360.0))
    fa = canvas[margin:margin + n, margin:margin + n]
    c = (n - 1) / 2.0
    th = math.radians(theta)
    ct, st = math.cos(th), math.sin(th)
    py, px = np.mgrid[0:n, 0:n].astype(np.float64)
    vy, vx = py - c, px - c
    sxf = ct * vx + st * vy + c - s[1]
    syf = -st * vx + ct * vy + c - s[0]
    ix = np.floor(sxf + 0.5).astype(np.int64)
    iy = np.floor(syf + 0.5).astype(np.int64)
    inside = (ix >= 0) & (ix < n) & (iy >= 0) & (iy < n)
    cy = np.clip(iy + margin, 0, n + 2 * margin - 1)
    cx = np.clip(ix + margin, 0, n + 2 * margin - 1)
    fb = np.cos(2.5 * canvas[cy, cx]) + noise_sd * noise
    return fa, fb, inside.astype(np.uint8), s, theta


def rotated_pair(rng, sigma, n, q, margin, shift_range, noise_sd):
    """rotated_intensities quantised: A = qq(F), B = perm(qq(cos(2.5 F(src))
    + noise)) over the footprint M_B, perm a seeded relabelling drawn after
    the angle."""
    fa, fb, inside, s, theta = rotated_intensities(rng, sigma, n, margin,
                                                   shift_range, noise_sd)
    perm = rng.permutation(q)
    a = qq(fa, q)
    bl = qq(fb, q, inside.astype(bool))
    b = perm[bl].astype(np.uint8)
    return a, b, inside, s, theta


def truth_a_to_b(theta_deg: float, shift, n: int):
    """The true correspondence of the rotated generators as an affine map
    of A's pixel (x, y) to B's, 6 numbers (row-major 2 x 3): B's pixel p
    shows A's point R(p - c) + c - s with R = [[cos t, sin t], [-sin t,
    cos t]] in (x, y) and c the centre, so A's point x sits at B's pixel
    R^-1 (x - c + s) + c."""
    th = math.radians(theta_deg)
    ct, st = math.cos(th), math.sin(th)
    c = (n - 1) / 2.0
    sy, sx = float(shift[0]), float(shift[1])
    return (ct, -st, ct * (sx - c) - st * (sy - c) + c,
            st, ct, st * (sx - c) + ct * (sy - c) + c)


def rotated_case(seed: int, n: int, q: int):
    """A small rotated pair like the sweep's (blur sigma 4, rotation in
    [0, 360) deg, shift within n/10, noise 0.2, relabelled B, M_B the
    rotation footprint) with its true transform."""
    rng = np.random.default_rng(seed)
    a, b, mb, s, theta = rotated_pair(rng, 4.0, n, q, n // 2, n // 10, 0.2)
    return dict(A=a, MA=np.ones((n, n), np.uint8), B=b, MB=mb, qa=q, qb=q,
                shift=s, theta_deg=theta, truth=truth_a_to_b(theta, s, n))


def config3(n_angles: int = 180, size: int = 512, q: int = 16):
    """512x512, Q=16 (256 pairs), blur sigma 4 on a 1024^2 canvas; B is the
    field rotated by a seeded angle in [0, 360) deg and moved by a seeded
    shift in [-100, 100]^2, passed through cos(2.5 .) + 0.2 N(0,1), quantised
    and relabelled by a seeded permutation; M_B carries the rotation
    footprint, M_A is all ones; 180 angles at 2 degree steps."""
    rng = np.random.default_rng(seed_for(3))
    margin = max(size // 2, 100)
    a, b, mb, s, theta = rotated_pair(rng, 4.0, size, q, margin, 100, 0.2)
    angles = [math.radians(2.0 * i) for i in range(n_angles)]
    return dict(name=f"sweep-{size}x{size}-q{q}-{n_angles}ang", A=a,
                MA=np.ones((size, size), np.uint8), B=b, MB=mb, qa=q, qb=q,
                angles=angles, gamma=0.5, shift=s, theta_deg=theta,
                truth=truth_a_to_b(theta, s, size))


def table1_pair(n: int, q: int = 16):
    """An n x n pair shaped like the paper's alignment benchmark images
    (cytological 300 x 300, histological 834 x 834): the config-3 generator
    (blur sigma 4, rotation in [0, 360) deg, shift within n/10, noise 0.2,
    relabelled B) at side n; M_A all ones, M_B the rotation footprint."""
    rng = np.random.default_rng(seed_for(6, n))
    a, b, mb, s, theta = rotated_pair(rng, 4.0, n, q, n // 2, n // 10, 0.2)
    return dict(name=f"table1-{n}x{n}-q{q}", A=a, MA=np.ones((n, n), np.uint8),
                B=b, MB=mb, qa=q, qb=q, shift=s, theta_deg=theta)


def table1_intensities(n: int):
    """Intensity (FP32) version of table1_pair for the whole Alg. 1
    pipeline, quantisation included: A = F, B = cos(2.5 F(src)) + 0.2 N(0,1)
    on the rotation footprint M_B (0 outside), blur sigma 4, shift within
    n/10."""
    rng = np.random.default_rng(seed_for(7, n))
    fa, fb, mb, s, theta = rotated_intensities(rng, 4.0, n, n // 2, n // 10, 0.2)
    fb = np.where(mb == 1, fb, 0.0)
    return dict(name=f"table1-intensity-{n}x{n}", A=fa.astype(np.float32),
                B=fb.astype(np.float32), MB=mb, shift=s, theta_deg=theta,
                truth=truth_a_to_b(theta, s, n))


def template_pair(ref: int, q: int = 16):
    """Template matching as in the paper's run-time experiment: a ref x ref
    reference and a floating image of half the side cut from it at a seeded
    offset (every placement of the floating image inside the reference is a
    candidate), blur sigma 4, the floating image passed through
    cos(2.5 .) + 0.2 N(0,1) and relabelled.  The displacement pairing A(x)
    with B(x + chi) puts the floating image at chi = -offset."""
    rng = np.random.default_rng(seed_for(8, ref))
    f = field(rng, 4.0, (ref, ref))
    half = ref // 2
    off = tuple(int(v) for v in rng.integers(0, ref - half + 1, size=2))
    noise = rng.standard_normal((half, half))
    perm = rng.permutation(q)
    a = qq(f, q)
    crop = f[off[0]:off[0] + half, off[1]:off[1] + half]
    b = perm[qq(np.cos(2.5 * crop) + 0.2 * noise, q)].astype(np.uint8)
    return dict(name=f"template-{ref}-{half}-q{q}", A=a, B=b, qa=q, qb=q,
                offset=off, window=(-(ref - half), 0, -(ref - half), 0))


def config4():
    """1024x1024, Q=16, blur sigma 6, B = quantised cos(2.5 f) + 0.2 N(0,1)
    moved by a seeded shift in [-8, 8]^2; all-ones masks (overlap counts up
    to 2^20)."""
    rng = np.random.default_rng(seed_for(4))
    a, b, s = _shifted_pair(rng, 6.0, 1024, 1024, 16, 8, None,
                            lambda v: np.cos(2.5 * v), 0.2)
    ones = np.ones((1024, 1024), np.uint8)
    return dict(name="stress-1024x1024-q16", A=a, MA=ones, B=b,
                MB=ones.copy(), qa=16, qb=16, angles=[0.0], gamma=0.5,
                shift=s)


def softmax0(z: np.ndarray, temp: float) -> np.ndarray:
    z = z / temp
    z = z - z.max(axis=0, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=0, keepdims=True)


def config5(n_pairs: int = 16, q: int = 8, lo: int = 128, hi: int = 384,
            shift_max: int = 32):
    """Batch of soft-membership pairs: sides drawn uniformly in [lo, hi]
    independently; Q channels of blurred logits (sigma 4), memberships =
    softmax over channels at temperature 0.5 (float32); B's logits are A's
    canvas logits moved by a seeded shift, channel-permuted and perturbed by
    0.3 N(0,1); all-ones masks."""
    pairs = []
    for i in range(n_pairs):
        rng = np.random.default_rng(seed_for(5, i))
        ha, wa, hb, wb = (int(v) for v in rng.integers(lo, hi + 1, size=4))
        m = shift_max + 1
        ch = max(ha, hb) + 2 * m
        cw = max(wa, wb) + 2 * m
        logits = np.stack([field(rng, 4.0, (ch, cw)) for _ in range(q)])
        s = tuple(int(v) for v in rng.integers(-shift_max, shift_max + 1,
                                               size=2))
        perm = rng.permutation(q)
        noise = rng.standard_normal((q, hb, wb))
        za = logits[:, m:m + ha, m:m + wa]
        zb = logits[perm][:, m - s[0]:m - s[0] + hb, m - s[1]:m - s[1] + wb]
        zb = zb + 0.3 * noise
        pa = softmax0(za, 0.5).astype(np.float32)
        pb = softmax0(zb, 0.5).astype(np.float32)
        pairs.append(dict(PA=pa, PB=pb, MA=np.ones((ha, wa), np.uint8),
                          MB=np.ones((hb, wb), np.uint8), shift=s,
                          perm=perm))
    return dict(name=f"soft-batch{n_pairs}-q{q}", pairs=pairs, q=q,
                gamma=0.5, temperature=0.01)


def volume_pair(seed: int, shape_a, shape_b, q: int, shift, sigma: float = 2.0,
                noise: float = 0.2, mask_density: float | None = None):
    """Two label volumes cut from one blurred 3-D field (the 2-D recipe in
    three axes): A = qq(F) on its box, B = perm(qq(cos(2.5 F) + noise)) on
    the box moved by -shift, shift = (s_z, s_y, s_x).  A's voxel x then
    shows the field point that B shows at x + shift, so the planted
    displacement (A(x) paired with B(x + chi)) is chi = shift, returned as
    'chi'.  Masks all ones or Bernoulli(mask_density)."""
    rng = np.random.default_rng(seed)
    s = tuple(int(v) for v in shift)
    m = max(abs(v) for v in s) + 1
    big = tuple(max(a, b) + 2 * m for a, b in zip(shape_a, shape_b))
    f = field(rng, sigma, big)
    za, ya, xa = (m, m, m)
    fa = f[za:za + shape_a[0], ya:ya + shape_a[1], xa:xa + shape_a[2]]
    zb, yb, xb = za - s[0], ya - s[1], xa - s[2]
    fb = f[zb:zb + shape_b[0], yb:yb + shape_b[1], xb:xb + shape_b[2]]
    fb = np.cos(2.5 * fb) + noise * rng.standard_normal(fb.shape)
    perm = rng.permutation(q)
    a = qq(fa, q)
    b = perm[qq(fb, q)].astype(np.uint8)
    if mask_density is None:
        ma = np.ones(shape_a, np.uint8)
        mb = np.ones(shape_b, np.uint8)
    else:
        ma = (rng.random(shape_a) < mask_density).astype(np.uint8)
        mb = (rng.random(shape_b) < mask_density).astype(np.uint8)
    return dict(A=a, MA=ma, B=b, MB=mb, q=q, chi=s)


def random_case(seed: int, ha: int, wa: int, hb: int, wb: int, qa: int,
                qb: int, mask_density: float | None = 0.8,
                smooth: float | None = 1.5):
    """Small random label images and masks for property and parity tests.
    Labels come from blurred fields (so the maps have structure) or are
    i.i.d. uniform when smooth is None; masks are i.i.d. Bernoulli or all
    ones when mask_density is None."""
    rng = np.random.default_rng(seed)
    if smooth is None:
        a = rng.integers(0, qa, size=(ha, wa)).astype(np.uint8)
        b = rng.integers(0, qb, size=(hb, wb)).astype(np.uint8)
    else:
        a = qq(field(rng, smooth, (ha, wa)), qa)
        b = qq(field(rng, smooth, (hb, wb)), qb)
    if mask_density is None:
        ma = np.ones((ha, wa), np.uint8)
        mb = np.ones((hb, wb), np.uint8)
    else:
        ma = (rng.random((ha, wa)) < mask_density).astype(np.uint8)
        mb = (rng.random((hb, wb)) < mask_density).astype(np.uint8)
    return dict(A=a, MA=ma, B=b, MB=mb, qa=qa, qb=qb)


def random_soft_case(seed: int, ha: int, wa: int, hb: int, wb: int, q: int,
                     temp: float = 0.5, smooth: float = 1.5,
                     qb: int | None = None,
                     mask_density: float | None = None):
    """Soft memberships: softmax over channels (temperature temp) of blurred
    N(0,1) logits, q channels for A and qb (default q) for B; masks all ones
    or i.i.d. Bernoulli(mask_density)."""
    rng = np.random.default_rng(seed)
    qb = q if qb is None else qb
    za = np.stack([field(rng, smooth, (ha, wa)) for _ in range(q)])
    zb = np.stack([field(rng, smooth, (hb, wb)) for _ in range(qb)])
    if mask_density is None:
        ma = np.ones((ha, wa), np.uint8)
        mb = np.ones((hb, wb), np.uint8)
    else:
        ma = (rng.random((ha, wa)) < mask_density).astype(np.uint8)
        mb = (rng.random((hb, wb)) < mask_density).astype(np.uint8)
    return dict(PA=softmax0(za, temp).astype(np.float32),
                PB=softmax0(zb, temp).astype(np.float32), MA=ma, MB=mb)
