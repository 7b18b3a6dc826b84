"""Pins for the CPU oracle: each test checks the oracle against something that
is not the oracle itself -- brute force written another way, a textbook
library routine, a closed form, or an invariant the paper states.

A plausible slip anywhere in the oracle (a dropped term, a wrong sign of the
displacement, a transposed operand, unrestricted marginals, a wrong log base,
a wrong tie rule) fails at least one of these.
"""

import itertools
import math

import numpy as np
import pytest
from scipy import signal
from sklearn.metrics import mutual_info_score

import synth


# -- brute force written differently: iterate over all pixel pairs and bucket
#    them by displacement y - x, then MI through Eq. 1 (p log p/(pa pb)) ------

def brute_counts(A, MA, B, MB, qa, qb):
    ha, wa = A.shape
    hb, wb = B.shape
    sh, sw = ha + hb - 1, wa + wb - 1
    cnt = np.zeros((qa, qb, sh, sw), np.int64)
    for ya, xa in itertools.product(range(ha), range(wa)):
        if not MA[ya, xa]:
            continue
        for yb, xb in itertools.product(range(hb), range(wb)):
            if not MB[yb, xb]:
                continue
            dy, dx = yb - ya, xb - xa          # B(x + chi) pairs with A(x)
            cnt[A[ya, xa], B[yb, xb], dy + ha - 1, dx + wa - 1] += 1
    return cnt


def mi_eq1(joint):
    n = joint.sum()
    if n == 0:
        return 0.0
    p = joint / n
    pa = p.sum(1)
    pb = p.sum(0)
    s = 0.0
    for a in range(p.shape[0]):
        for b in range(p.shape[1]):
            if p[a, b] > 0:
                s += p[a, b] * math.log2(p[a, b] / (pa[a] * pb[b]))
    return s


def tiny_cases():
    rng = np.random.default_rng(7)
    shapes = [((2, 2), (2, 2)), ((2, 3), (2, 3)), ((2, 3), (3, 2)),
              ((1, 4), (2, 2)), ((3, 3), (1, 1)), ((4, 5), (3, 2))]
    out = []
    for k in range(60):
        (ha, wa), (hb, wb) = shapes[k % len(shapes)]
        qa = int(rng.integers(1, 4))
        qb = int(rng.integers(1, 4))
        A = rng.integers(0, qa, (ha, wa)).astype(np.uint8)
        B = rng.integers(0, qb, (hb, wb)).astype(np.uint8)
        MA = (rng.random((ha, wa)) < 0.75).astype(np.uint8)
        MB = (rng.random((hb, wb)) < 0.75).astype(np.uint8)
        # labels outside the mask may be anything below 256
        A[MA == 0] = rng.integers(0, 255, int((MA == 0).sum()))
        B[MB == 0] = rng.integers(0, 255, int((MB == 0).sum()))
        out.append((A, MA, B, MB, qa, qb))
    return out


def test_oracle_vs_bruteforce_tiny(oracle):
    for A, MA, B, MB, qa, qb in tiny_cases():
        r = oracle.cmif_direct(A, MA, B, MB, qa, qb, counts=True)
        bc = brute_counts(A, MA, B, MB, qa, qb)
        assert np.array_equal(r["counts"], bc)
        assert np.array_equal(r["n"], bc.sum((0, 1)))
        sh, sw = r["mi"].shape
        for i in range(sh):
            for j in range(sw):
                assert abs(r["mi"][i, j] - mi_eq1(bc[:, :, i, j])) < 1e-12


def test_exhaustive_2x2_q2(oracle):
    """Every 2x2 pair of binary label images (all-ones masks): 256 cases."""
    ones = np.ones((2, 2), np.uint8)
    for ka in range(16):
        A = np.array([(ka >> i) & 1 for i in range(4)], np.uint8).reshape(2, 2)
        for kb in range(16):
            B = np.array([(kb >> i) & 1 for i in range(4)],
                         np.uint8).reshape(2, 2)
            r = oracle.cmif_direct(A, ones, B, ones, 2, 2, counts=True)
            bc = brute_counts(A, ones, B, ones, 2, 2)
            assert np.array_equal(r["counts"], bc)
            for i in range(3):
                for j in range(3):
                    assert abs(r["mi"][i, j] - mi_eq1(bc[:, :, i, j])) < 1e-12


# -- textbook routine: scipy correlate2d of indicator images (Eq. 9) ---------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_counts_vs_scipy_correlate2d(oracle, seed):
    c = synth.random_case(seed, 17, 23, 13, 19, 4, 5, mask_density=0.7)
    r = oracle.cmif_direct(c["A"], c["MA"], c["B"], c["MB"], 4, 5,
                           counts=True)
    for a in range(4):
        la = ((c["A"] == a) & (c["MA"] == 1)).astype(np.int64)
        for b in range(5):
            lb = ((c["B"] == b) & (c["MB"] == 1)).astype(np.int64)
            z = signal.correlate2d(lb, la, mode="full")
            assert np.array_equal(r["counts"][a, b], z)
    # Eq. 11: N = M_A corr M_B
    z = signal.correlate2d(c["MB"].astype(np.int64), c["MA"].astype(np.int64),
                           mode="full")
    assert np.array_equal(r["n"], z)


# -- the paper's method with a library FFT in FP64, rounded (Sec. 3.2) ------

def test_counts_vs_numpy_fft_rint(oracle):
    c = synth.random_case(11, 40, 33, 29, 41, 3, 4, mask_density=0.9)
    A, MA, B, MB = c["A"], c["MA"], c["B"], c["MB"]
    ha, wa = A.shape
    hb, wb = B.shape
    sh, sw = ha + hb - 1, wa + wb - 1
    r = oracle.cmif_direct(A, MA, B, MB, 3, 4, counts=True)
    for a in range(3):
        fa = np.fft.rfft2(((A == a) & (MA == 1)).astype(np.float64), s=(sh, sw))
        for b in range(4):
            fb = np.fft.rfft2(((B == b) & (MB == 1)).astype(np.float64),
                              s=(sh, sw))
            circ = np.fft.irfft2(np.conj(fa) * fb, s=(sh, sw))
            full = np.roll(circ, (ha - 1, wa - 1), axis=(0, 1))
            assert np.array_equal(np.rint(full).astype(np.int64),
                                  r["counts"][a, b])


# -- sklearn mutual_info_score at sampled displacements (Eq. 1, nats) -------

def test_mi_vs_sklearn(oracle):
    c = synth.random_case(5, 31, 27, 25, 30, 5, 6, mask_density=0.85)
    A, MA, B, MB = c["A"], c["MA"], c["B"], c["MB"]
    r = oracle.cmif_direct(A, MA, B, MB, 5, 6)
    ha, wa = A.shape
    hb, wb = B.shape
    rng = np.random.default_rng(3)
    for _ in range(40):
        dy = int(rng.integers(-(ha - 1), hb))
        dx = int(rng.integers(-(wa - 1), wb))
        la, lb = [], []
        for y in range(ha):
            for x in range(wa):
                yy, xx = y + dy, x + dx
                if 0 <= yy < hb and 0 <= xx < wb and MA[y, x] and MB[yy, xx]:
                    la.append(int(A[y, x]))
                    lb.append(int(B[yy, xx]))
        v = r["mi"][dy + ha - 1, dx + wa - 1]
        if not la:
            assert v == 0.0
            continue
        ref = mutual_info_score(la, lb) / math.log(2.0)
        assert abs(v - ref) < 1e-9, (dy, dx)


# -- closed forms and invariants --------------------------------------------

def test_n_closed_form_all_ones(oracle):
    ha, wa, hb, wb = 9, 14, 11, 6
    c = synth.random_case(2, ha, wa, hb, wb, 3, 3, mask_density=None)
    r = oracle.cmif_direct(c["A"], c["MA"], c["B"], c["MB"], 3, 3)
    for i in range(ha + hb - 1):
        dy = i - (ha - 1)
        ny = min(ha, hb - dy) - max(0, -dy)
        for j in range(wa + wb - 1):
            dx = j - (wa - 1)
            nx = min(wa, wb - dx) - max(0, -dx)
            assert r["n"][i, j] == ny * nx


def test_invariants(oracle):
    c = synth.random_case(9, 21, 18, 16, 25, 4, 6, mask_density=0.6)
    A, MA, B, MB = c["A"], c["MA"], c["B"], c["MB"]
    r = oracle.cmif_direct(A, MA, B, MB, 4, 6, counts=True)
    cnt = r["counts"]
    n = r["n"]
    # Eq. 11: N = sum_a C_a = sum_b C_b = sum_ab C_ab
    assert np.array_equal(cnt.sum((0, 1)), n)
    assert np.array_equal(cnt.sum(1).sum(0), n)
    # sum over displacements of N = (sum M_A)(sum M_B)
    assert int(n.sum()) == int(MA.sum()) * int(MB.sum())
    # 0 <= MI <= min(H_A(chi), H_B(chi)) <= log2 min(Q_A, Q_B)
    ca = cnt.sum(1)
    cb = cnt.sum(0)
    with np.errstate(divide="ignore", invalid="ignore"):
        def ent(c):
            p = np.where(n > 0, c / np.maximum(n, 1), 0.0)
            return -np.where(p > 0, p * np.log2(np.where(p > 0, p, 1)), 0).sum(0)
        ha_ = ent(ca)
        hb_ = ent(cb)
    mi = r["mi"]
    assert (mi >= -1e-12).all()
    assert (mi <= np.minimum(ha_, hb_) + 1e-12).all()
    assert (mi <= math.log2(4) + 1e-12).all()
    assert (mi[n == 0] == 0).all()


def test_single_label_gives_zero(oracle):
    c = synth.random_case(4, 12, 10, 9, 13, 1, 5, mask_density=0.8)
    r = oracle.cmif_direct(c["A"] * 0, c["MA"], c["B"], c["MB"], 1, 5)
    assert np.abs(r["mi"]).max() < 1e-12


def test_self_mi_equals_entropy(oracle):
    """MI(A, A) at chi = 0 with equal masks is H_A on the mask (Eq. 2)."""
    c = synth.random_case(6, 20, 20, 20, 20, 5, 5, mask_density=0.7)
    A, MA = c["A"], c["MA"]
    r = oracle.cmif_direct(A, MA, A, MA, 5, 5)
    vals = A[MA == 1]
    p = np.bincount(vals, minlength=5) / vals.size
    h = -sum(pi * math.log2(pi) for pi in p if pi > 0)
    assert abs(r["mi"][19, 19] - h) < 1e-12
    # a bijective relabelling of B reaches the same value
    perm = np.array([3, 0, 4, 1, 2], np.uint8)
    r2 = oracle.cmif_direct(A, MA, perm[A], MA, 5, 5)
    assert abs(r2["mi"][19, 19] - h) < 1e-12
    assert np.allclose(r2["mi"], r["mi"], atol=1e-12)


def test_swap_symmetry(oracle):
    """CMIF(chi; A, B) = CMIF(-chi; B, A) (Eq. 7 read both ways)."""
    c = synth.random_case(8, 15, 11, 13, 17, 3, 4, mask_density=0.8)
    A, MA, B, MB = c["A"], c["MA"], c["B"], c["MB"]
    r1 = oracle.cmif_direct(A, MA, B, MB, 3, 4)
    r2 = oracle.cmif_direct(B, MB, A, MA, 4, 3)
    # map index of -chi in the swapped map: i2 = -dy + (hb - 1) = sh - 1 - i1
    assert np.allclose(r1["mi"], r2["mi"][::-1, ::-1], atol=1e-12)
    assert np.array_equal(r1["n"], r2["n"][::-1, ::-1])


def test_label_out_of_range_raises(oracle):
    c = synth.random_case(1, 8, 8, 8, 8, 3, 3, mask_density=None)
    A = c["A"].copy()
    A[2, 3] = 3
    with pytest.raises(oracle.OracleError):
        oracle.cmif_direct(A, c["MA"], c["B"], c["MB"], 3, 3)
    MA = c["MA"].copy()
    MA[2, 3] = 0          # outside the mask it is ignored
    oracle.cmif_direct(A, MA, c["B"], c["MB"], 3, 3)


def test_cmif_at_matches_map(oracle):
    c = synth.random_case(12, 19, 22, 24, 15, 4, 4, mask_density=0.7)
    r = oracle.cmif_direct(c["A"], c["MA"], c["B"], c["MB"], 4, 4,
                           counts=True)
    for dy, dx in [(0, 0), (-18, -21), (23, 14), (5, -7), (-3, 9)]:
        mi, n, joint = oracle.cmif_at(c["A"], c["MA"], c["B"], c["MB"], 4, 4,
                                      dy, dx)
        i, j = dy + 18, dx + 21
        assert mi == r["mi"][i, j]
        assert n == r["n"][i, j]
        assert np.array_equal(joint, r["counts"][:, :, i, j])


def test_planted_shift_config1(oracle):
    c = synth.config1()
    r = oracle.cmif_direct(c["A"], c["MA"], c["B"], c["MB"], 4, 4)
    idx, v, n = oracle.argmax(r["mi"], r["n"], 0.5)
    i, j = divmod(idx, r["mi"].shape[1])
    assert (i - 63, j - 63) == (7, -5)


# -- argmax rule (Alg. 1) -----------------------------------------------------

def test_argmax_rule(oracle):
    rng = np.random.default_rng(0)
    for _ in range(50):
        n = rng.integers(0, 100, size=200).astype(np.int64)
        mi = rng.integers(0, 5, size=200).astype(np.float64) / 4.0  # ties
        g = float(rng.choice([0.0, 0.3, 0.5, 1.0]))
        idx, v, nn = oracle.argmax(mi, n, g)
        thr = g * n.max()
        elig = n.astype(np.float64) >= thr
        masked = np.where(elig, mi, -np.inf)
        ref = int(np.argmax(masked))      # numpy: first occurrence
        assert idx == ref and v == mi[ref] and nn == n[ref]


def test_align_first_angle_wins_ties(oracle):
    """Alg. 1 line 6 replaces the best only on a strictly larger MI: with a
    symmetric pattern, 0 and 180 degrees tie and the first listed wins."""
    A = np.zeros((6, 6), np.uint8)
    A[1:5, 2:4] = 1
    ones = np.ones((6, 6), np.uint8)
    r = oracle.align(A, ones, A, ones, 2, 2, [0.0, math.pi], 0.5)
    assert r["angle_index"] == 0
    r = oracle.align(A, ones, A, ones, 2, 2, [math.pi, 0.0], 0.5)
    assert r["angle_index"] == 0


def test_align_starts_from_identity(oracle):
    """Alg. 1 initialises the best transform to the identity with I = 0 and
    replaces it only on a strictly larger MI: when no angle reaches a
    positive MI (one label in A, so MI is 0 at every displacement), the
    result is the identity (angle index -1, chi = 0, I = 0), not the first
    angle's pick."""
    rng = np.random.default_rng(3)
    A = np.zeros((9, 11), np.uint8)
    B = rng.integers(0, 3, size=(10, 8)).astype(np.uint8)
    ones_a = np.ones_like(A)
    ones_b = np.ones_like(B)
    r = oracle.align(A, ones_a, B, ones_b, 1, 3, [0.0, 0.4, math.pi], 0.5,
                     per_angle=True)
    assert (r["angle_index"], r["dy"], r["dx"], r["mi"]) == (-1, 0, 0, 0.0)
    # every angle had an eligible pick, with MI exactly 0
    assert all(p["mi"] == 0.0 and p["n"] > 0 for p in r["per_angle"])
    # one positive angle among non-positive ones is taken
    A2 = rng.integers(0, 2, size=(9, 11)).astype(np.uint8)
    r2 = oracle.align(A2, ones_a, B, ones_b, 2, 3, [0.0, 0.4], 0.5)
    assert r2["angle_index"] in (0, 1) and r2["mi"] > 0.0


def test_mi_of_joint_vs_sklearn_contingency(oracle):
    """Eq. 2 / Eq. 12 on an explicit joint table against scikit-learn's MI
    of the same contingency table (nats, divided by ln 2), including empty
    rows and columns (0 log 0 = 0) and the all-zero table (MI = 0)."""
    rng = np.random.default_rng(17)
    for qa, qb in ((2, 2), (3, 5), (7, 4), (16, 16)):
        for _ in range(5):
            t = rng.integers(0, 40, size=(qa, qb)).astype(np.int64)
            t[rng.integers(0, qa)] = 0          # an empty row of A
            ref = mutual_info_score(None, None, contingency=t) / math.log(2.0)
            assert abs(oracle.mi_of_joint(t.astype(np.float64)) - ref) <= 1e-12
    assert oracle.mi_of_joint(np.zeros((3, 3))) == 0.0
    # independent table: p_ab = p_a p_b exactly gives MI = 0
    ind = np.outer([1, 2, 3], [4, 4, 8]).astype(np.float64)
    assert abs(oracle.mi_of_joint(ind)) <= 1e-15


# -- digest: Vigna's splitmix64 reference outputs ------------------------------

def test_digest_weight_reference_values(oracle):
    # first two outputs of splitmix64 seeded with 0 (state advances by the
    # golden-ratio increment before each mix)
    assert oracle.digest_weight(0) == 0xE220A8397B1DCDAF
    assert oracle.digest_weight(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4
    assert oracle.digest_weight(2 * 0x9E3779B97F4A7C15 % 2**64) == \
        0x06C45D188009454F


def test_digest_matches_counts(oracle):
    c = synth.random_case(3, 14, 9, 10, 12, 3, 2, mask_density=0.8)
    r = oracle.cmif_direct(c["A"], c["MA"], c["B"], c["MB"], 3, 2,
                           counts=True, digest=True)
    cnt = r["counts"]
    sh, sw = cnt.shape[2:]
    w = [oracle.digest_weight(i) for i in range(sh * sw)]
    for a in range(3):
        for b in range(2):
            s = 0
            flat = cnt[a, b].ravel()
            for i in range(sh * sw):
                s = (s + int(flat[i]) * w[i]) % 2**64
            assert int(r["digest"][a, b]) == s


# -- nearest-neighbour rotation ----------------------------------------------

@pytest.mark.parametrize("h,w", [(6, 6), (7, 7), (8, 6), (5, 9)])
def test_warp_identity_and_quarter_turns(oracle, h, w):
    rng = np.random.default_rng(h * 10 + w)
    B = rng.integers(0, 7, (h, w)).astype(np.uint8)
    MB = (rng.random((h, w)) < 0.8).astype(np.uint8)
    wb, wm = oracle.warp_nn(B, MB, 0.0)
    assert np.array_equal(wm, MB) and np.array_equal(wb[MB == 1], B[MB == 1])
    if h == w:
        # output (y, x) reads source R(theta) applied to centred coordinates:
        # theta = 90 deg maps (X, Y) -> (-Y, X), i.e. B'(y, x) = B(x, h-1-y)
        for k, th in [(1, math.pi / 2), (2, math.pi), (3, 3 * math.pi / 2)]:
            wb, wm = oracle.warp_nn(B, MB, th)
            ref_b = np.rot90(B, k=k)
            ref_m = np.rot90(MB, k=k)
            assert np.array_equal(wm, ref_m)
            assert np.array_equal(wb[wm == 1], ref_b[ref_m == 1])


def test_warp_outside_is_masked(oracle):
    B = np.full((9, 15), 3, np.uint8)
    wb, wm = oracle.warp_nn(B, None, math.radians(37.0))
    # corners of a non-square image rotate out of the canvas
    assert wm[0, 0] == 0 and wm.sum() < wm.size
    assert (wb[wm == 0] == 0).all() and (wb[wm == 1] == 3).all()


def test_rot_coeffs(oracle):
    assert oracle.rot_coeffs(0.0) == (65536, 0)
    assert oracle.rot_coeffs(math.pi / 2) == (0, 65536)
    c, s = oracle.rot_coeffs(math.radians(30.0))
    assert c == round(math.cos(math.radians(30)) * 65536) and s == 32768


# -- soft (real-weight) variant ------------------------------------------------

def test_soft_one_hot_equals_hard(oracle):
    c = synth.random_case(21, 13, 11, 12, 14, 3, 4, mask_density=0.8)
    A, MA, B, MB = c["A"], c["MA"], c["B"], c["MB"]
    pa = np.stack([(A == a) for a in range(3)]).astype(np.float32)
    pb = np.stack([(B == b) for b in range(4)]).astype(np.float32)
    hard = oracle.cmif_direct(A, MA, B, MB, 3, 4, counts=True)
    soft = oracle.soft_direct(pa, MA, pb, MB, joint=True)
    assert np.array_equal(soft["joint"], hard["counts"].astype(np.float64))
    assert np.allclose(soft["mi"], hard["mi"], atol=1e-13)


@pytest.mark.parametrize("case", [(4, 11, 9, 10, 13, 3), (6, 37, 41, 29, 33, 4),
                                  (8, 64, 20, 50, 70, 5)],
                         ids=["11x9-10x13", "37x41-29x33", "64x20-50x70"])
def test_soft_torch_matches_c_direct(oracle, case):
    """The soft reference's FFT formulation (Eq. 7 through the library FFT)
    equals the C direct soft sums, joint and MI, at sizes whose transforms
    wrap (padding, odd sides, unequal images)."""
    import torch
    seed, ha, wa, hb, wb, q = case
    c = synth.random_soft_case(seed, ha, wa, hb, wb, q)
    ref = oracle.soft_direct(c["PA"], c["MA"], c["PB"], c["MB"], joint=True)
    pa = torch.tensor(c["PA"], dtype=torch.float64)
    pb = torch.tensor(c["PB"], dtype=torch.float64)
    ma = torch.tensor(c["MA"], dtype=torch.float64)
    mb = torch.tensor(c["MB"], dtype=torch.float64)
    j = oracle.soft_joint_torch(pa, ma, pb, mb)
    assert np.allclose(j.numpy(), ref["joint"], rtol=0, atol=1e-11)
    mi, n = oracle.soft_mi_torch(j)
    assert np.allclose(mi.numpy(), ref["mi"], atol=1e-10)


@pytest.mark.parametrize("case", [(5, 6, 5, 5, 6, 3), (7, 14, 11, 12, 15, 4)],
                         ids=["6x5-5x6", "14x11-12x15"])
def test_soft_autograd_vs_finite_differences(oracle, case):
    import torch
    seed, ha, wa, hb, wb, q = case
    c = synth.random_soft_case(seed, ha, wa, hb, wb, q)
    ma = torch.tensor(c["MA"], dtype=torch.float64)
    mb = torch.tensor(c["MB"], dtype=torch.float64)
    pa0 = torch.tensor(c["PA"], dtype=torch.float64)
    pb0 = torch.tensor(c["PB"], dtype=torch.float64)

    def loss(pa, pb):
        l, _, _ = oracle.soft_loss_torch([(pa, ma, pb, mb)], 0.5, 0.05)
        return l

    pa = pa0.clone().requires_grad_(True)
    pb = pb0.clone().requires_grad_(True)
    l = loss(pa, pb)
    ga, gb = torch.autograd.grad(l, (pa, pb))
    h = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(12):
        which = int(rng.integers(0, 2))
        base = pa0 if which == 0 else pb0
        idx = tuple(int(rng.integers(0, s)) for s in base.shape)
        p = base.clone()
        m = base.clone()
        p[idx] += h
        m[idx] -= h
        if which == 0:
            fd = (loss(p, pb0) - loss(m, pb0)) / (2 * h)
            g = ga[idx]
        else:
            fd = (loss(pa0, p) - loss(pa0, m)) / (2 * h)
            g = gb[idx]
        assert abs(float(fd) - float(g)) <= 1e-6 * max(1.0, abs(float(g))), \
            (which, idx, float(fd), float(g))
