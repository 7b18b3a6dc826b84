"""CPU: pins of the oracle's 3-D direct method (the paper's method taken to
volumes, as its discussion states it works in nD), against sources other
than itself: brute-force enumeration with MI by Eq. 1, depth-1 volumes
against the 2-D oracle, scipy's n-D correlation of indicator volumes (via
count digests), numpy's n-D FFT with rounding, the closed-form N of full
masks, and MI(A, A; 0) = H(A)."""

import collections
import math

import numpy as np
import pytest
from scipy import signal


def rand_vol(rng, shape, q, density=None):
    lab = rng.integers(0, q, size=shape).astype(np.uint8)
    m = (np.ones(shape, np.uint8) if density is None
         else (rng.random(shape) < density).astype(np.uint8))
    return lab, m


def mi_eq1(pairs):
    """Eq. 1 on a list of (a, b) label pairs: sum p_ab log2 p_ab/(p_a p_b)."""
    n = len(pairs)
    if n == 0:
        return 0.0
    jab = collections.Counter(pairs)
    ja = collections.Counter(a for a, _ in pairs)
    jb = collections.Counter(b for _, b in pairs)
    return sum(c / n * math.log2((c / n) / ((ja[a] / n) * (jb[b] / n)))
               for (a, b), c in jab.items())


def test_bruteforce_tiny(oracle):
    rng = np.random.default_rng(3)
    A, MA = rand_vol(rng, (3, 4, 3), 3, 0.8)
    B, MB = rand_vol(rng, (2, 3, 4), 2, 0.8)
    r = oracle.cmif_direct3d(A, MA, B, MB, 3, 2)
    da, ha, wa = A.shape
    db, hb, wb = B.shape
    for k in range(da + db - 1):
        for i in range(ha + hb - 1):
            for j in range(wa + wb - 1):
                dz, dy, dx = k - (da - 1), i - (ha - 1), j - (wa - 1)
                pairs = []
                for z in range(da):
                    for y in range(ha):
                        for x in range(wa):
                            zb, yb, xb = z + dz, y + dy, x + dx
                            if (0 <= zb < db and 0 <= yb < hb and 0 <= xb < wb
                                    and MA[z, y, x] and MB[zb, yb, xb]):
                                pairs.append((A[z, y, x], B[zb, yb, xb]))
                assert r["n"][k, i, j] == len(pairs)
                assert abs(r["mi"][k, i, j] - mi_eq1(pairs)) < 1e-12


def test_depth_one_is_the_2d_map(oracle):
    rng = np.random.default_rng(4)
    A, MA = rand_vol(rng, (1, 17, 13), 4, 0.7)
    B, MB = rand_vol(rng, (1, 11, 19), 5, 0.7)
    r3 = oracle.cmif_direct3d(A, MA, B, MB, 4, 5, digest=True)
    r2 = oracle.cmif_direct(A[0], MA[0], B[0], MB[0], 4, 5, digest=True)
    assert np.array_equal(r3["n"][0], r2["n"])
    assert np.array_equal(r3["mi"][0], r2["mi"])
    assert np.array_equal(r3["digest"], r2["digest"])


def _digest(oracle, counts):
    w = np.array([oracle.digest_weight(i) for i in range(counts[0, 0].size)],
                 np.uint64)
    flat = counts.reshape(counts.shape[0], counts.shape[1], -1).astype(np.uint64)
    return (flat * w[None, None, :]).sum(axis=2, dtype=np.uint64)


def test_counts_vs_scipy_correlate_nd(oracle):
    rng = np.random.default_rng(5)
    A, MA = rand_vol(rng, (5, 6, 7), 3, 0.8)
    B, MB = rand_vol(rng, (4, 7, 5), 3, 0.8)
    r = oracle.cmif_direct3d(A, MA, B, MB, 3, 3, digest=True)
    counts = np.zeros((3, 3) + r["n"].shape, np.int64)
    for a in range(3):
        la = ((A == a) & (MA == 1)).astype(np.int64)
        for b in range(3):
            lb = ((B == b) & (MB == 1)).astype(np.int64)
            counts[a, b] = signal.correlate(lb, la, mode="full", method="direct")
    assert np.array_equal(_digest(oracle, counts), r["digest"])
    n = signal.correlate(MB.astype(np.int64), MA.astype(np.int64), mode="full",
                         method="direct")
    assert np.array_equal(n, r["n"])
    assert np.array_equal(counts.sum(axis=(0, 1)), r["n"])


def test_counts_vs_numpy_fftn_rint(oracle):
    rng = np.random.default_rng(6)
    A, MA = rand_vol(rng, (6, 5, 8), 2, 0.9)
    B, MB = rand_vol(rng, (7, 9, 4), 3, 0.9)
    r = oracle.cmif_direct3d(A, MA, B, MB, 2, 3, digest=True)
    s = r["n"].shape
    counts = np.zeros((2, 3) + s, np.int64)
    for a in range(2):
        fa = np.fft.rfftn(((A == a) & (MA == 1)).astype(np.float64), s=s, axes=(0, 1, 2))
        for b in range(3):
            fb = np.fft.rfftn(((B == b) & (MB == 1)).astype(np.float64), s=s,
                              axes=(0, 1, 2))
            circ = np.fft.irfftn(np.conj(fa) * fb, s=s, axes=(0, 1, 2))
            full = np.roll(circ, tuple(d - 1 for d in A.shape), axis=(0, 1, 2))
            counts[a, b] = np.rint(full).astype(np.int64)
    assert np.array_equal(_digest(oracle, counts), r["digest"])


def test_n_closed_form_full_masks(oracle):
    rng = np.random.default_rng(7)
    A, _ = rand_vol(rng, (4, 9, 6), 2)
    B, _ = rand_vol(rng, (6, 5, 7), 2)
    r = oracle.cmif_direct3d(A, None, B, None, 2, 2)

    def ov(la, lb, d):
        return min(la, lb - d) - max(0, -d)

    for k in range(r["n"].shape[0]):
        for i in range(r["n"].shape[1]):
            for j in range(r["n"].shape[2]):
                want = (ov(4, 6, k - 3) * ov(9, 5, i - 8) * ov(6, 7, j - 5))
                assert r["n"][k, i, j] == want


def test_self_mi_is_the_entropy(oracle):
    rng = np.random.default_rng(8)
    A, _ = rand_vol(rng, (5, 6, 7), 4)
    r = oracle.cmif_direct3d(A, None, A, None, 4, 4)
    _, cnt = np.unique(A, return_counts=True)
    p = cnt / cnt.sum()
    h = float(-(p * np.log2(p)).sum())
    assert abs(r["mi"][4, 5, 6] - h) < 1e-12
    # relabelling B bijectively leaves the map unchanged
    perm = np.array([2, 0, 3, 1], np.uint8)
    r2 = oracle.cmif_direct3d(A, None, perm[A], None, 4, 4)
    assert np.abs(r2["mi"] - r["mi"]).max() < 1e-12
