"""CPU oracle for the CMIF hot path -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product path (the HIP library and its binding) never does.

Two parts:
  * cmif_oracle.c, plain C + OpenMP: the direct histogram method of Sec. 2.2
    (per displacement, count label pairs over the overlap, Eq. 12 entropies,
    Eq. 2), the Alg. 1 argmax, the integer nearest-neighbour rotation, the
    soft (real-weight) direct method, and the direct method on 3-D volumes
    (the nD case of the paper's discussion);
  * soft_* below, plain PyTorch CPU ops in FP64: the soft CMIF written as
    Eq. 7 correlations evaluated with a library FFT (torch.fft) followed by the
    Eq. 12 entropies, differentiated by autograd.  It is pinned against the C
    direct method and against central finite differences in the tests.

  * kmeans_* below, plain numpy in FP64: the mini-batch k-means quantiser
    (the QUANTIZE step of Alg. 1, Sec. 3.6; Sculley 2010) written as its
    per-sample steps.

Every function states the passage it follows.  All parts are pinned by
tests/test_oracle_pins.py, tests/test_oracle3d_pins.py and
tests/test_kmeans_oracle.py; none is "parity unpinned".
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cmif_oracle.c")
_LIB = os.path.join(_HERE, "libcmif_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc -O3 -fopenmp).  Portable x86-64 code: the
    library may run on another host than the one that built it."""
    if force or not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I = ctypes.c_int
    lib.or_cmif_direct.argtypes = [P, P, I, I, P, P, I, I, I, I, P, P, P, P, I]
    lib.or_cmif_direct.restype = I
    lib.or_cmif_at.argtypes = [P, P, I, I, P, P, I, I, I, I, I, I, P, P, P]
    lib.or_cmif_at.restype = I
    lib.or_argmax.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, P, P]
    lib.or_argmax.restype = ctypes.c_int64
    lib.or_rot_coeffs.argtypes = [ctypes.c_double, P, P]
    lib.or_rot_coeffs.restype = None
    lib.or_warp_nn.argtypes = [P, P, I, I, ctypes.c_int64, ctypes.c_int64, P,
                               P]
    lib.or_warp_nn.restype = None
    lib.or_soft_direct.argtypes = [P, P, I, I, P, P, I, I, I, I, P, P, P, I]
    lib.or_soft_direct.restype = I
    lib.or_mi_of_joint.argtypes = [P, I, I]
    lib.or_mi_of_joint.restype = ctypes.c_double
    lib.or_digest_weight.argtypes = [ctypes.c_uint64]
    lib.or_digest_weight.restype = ctypes.c_uint64
    lib.or_cmif_direct3d.argtypes = [P, P, I, I, I, P, P, I, I, I, I, I, P, P,
                                     P, I]
    lib.or_cmif_direct3d.restype = I
    lib.or_max_threads.argtypes = []
    lib.or_max_threads.restype = I
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _u8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def max_threads() -> int:
    return int(_load().or_max_threads())


def cmif_direct(A, MA, B, MB, qa, qb, counts=False, digest=False,
                nthreads=0):
    """Full CMIF map by the direct method (Sec. 2.2; Eq. 1-5, 11, 12).
    Returns dict(mi [SH,SW] f64, n [SH,SW] i64, counts [qa,qb,SH,SW] i64 or
    None, digest [qa,qb] u64 or None).  Map index [i, j] <-> displacement
    (i - (H_A - 1), j - (W_A - 1)); B is read at x + chi (Eq. 5, Eq. 7)."""
    lib = _load()
    A, B, MA, MB = _u8(A), _u8(B), _u8(MA), _u8(MB)
    ha, wa = A.shape
    hb, wb = B.shape
    sh, sw = ha + hb - 1, wa + wb - 1
    mi = np.empty((sh, sw), np.float64)
    n = np.empty((sh, sw), np.int64)
    cnt = np.empty((qa, qb, sh, sw), np.int64) if counts else None
    dig = np.empty((qa, qb), np.uint64) if digest else None
    rc = lib.or_cmif_direct(_ptr(A), _ptr(MA), ha, wa, _ptr(B), _ptr(MB), hb,
                            wb, qa, qb, _ptr(mi), _ptr(n), _ptr(cnt),
                            _ptr(dig), int(nthreads))
    if rc != 0:
        raise OracleError(f"or_cmif_direct failed with code {rc}")
    return dict(mi=mi, n=n, counts=cnt, digest=dig)


def cmif_direct3d(A, MA, B, MB, qa, qb, digest=False, nthreads=0):
    """3-D CMIF map by the direct method (Sec. 2.2 taken to volumes, as
    the paper's discussion states the method works in nD): A [da, ha, wa],
    B [db, hb, wb] uint8 labels, masks or None.  Returns dict(mi, n
    [SD, SH, SW], digest [qa, qb] u64 or None); map index [k, i, j] <->
    chi = (k - (da-1), i - (ha-1), j - (wa-1)), B read at x + chi."""
    lib = _load()
    A, B, MA, MB = _u8(A), _u8(B), _u8(MA), _u8(MB)
    da, ha, wa = A.shape
    db, hb, wb = B.shape
    sd, sh, sw = da + db - 1, ha + hb - 1, wa + wb - 1
    mi = np.empty((sd, sh, sw), np.float64)
    n = np.empty((sd, sh, sw), np.int64)
    dig = np.empty((qa, qb), np.uint64) if digest else None
    rc = lib.or_cmif_direct3d(_ptr(A), _ptr(MA), da, ha, wa, _ptr(B), _ptr(MB),
                              db, hb, wb, qa, qb, _ptr(mi), _ptr(n), _ptr(dig),
                              int(nthreads))
    if rc != 0:
        raise OracleError(f"or_cmif_direct3d failed with code {rc}")
    return dict(mi=mi, n=n, digest=dig)


def cmif_at(A, MA, B, MB, qa, qb, dy, dx):
    """CMIF at one displacement (dy, dx) by the direct method.
    Returns (mi, n, joint [qa, qb] i64)."""
    lib = _load()
    A, B, MA, MB = _u8(A), _u8(B), _u8(MA), _u8(MB)
    ha, wa = A.shape
    hb, wb = B.shape
    mi = ctypes.c_double()
    n = ctypes.c_int64()
    joint = np.empty((qa, qb), np.int64)
    rc = lib.or_cmif_at(_ptr(A), _ptr(MA), ha, wa, _ptr(B), _ptr(MB), hb, wb,
                        qa, qb, int(dy), int(dx), ctypes.byref(mi),
                        ctypes.byref(n), _ptr(joint))
    if rc != 0:
        raise OracleError(f"or_cmif_at failed with code {rc}")
    return mi.value, n.value, joint


def argmax(mi, n, gamma):
    """Alg. 1 for one transform: eligible iff N >= gamma * max N (FP64
    compare), argmax of MI over them, ties to the smallest row-major index.
    Returns (flat index, mi, n)."""
    lib = _load()
    mi = np.ascontiguousarray(mi, np.float64)
    n = np.ascontiguousarray(n, np.int64)
    bm = ctypes.c_double()
    bn = ctypes.c_int64()
    idx = lib.or_argmax(_ptr(mi), _ptr(n), mi.size, float(gamma),
                        ctypes.byref(bm), ctypes.byref(bn))
    return int(idx), bm.value, bn.value


def rot_coeffs(theta):
    """Fixed-point rotation coefficients round(cos, sin(theta) * 2^16)."""
    lib = _load()
    c = ctypes.c_int64()
    s = ctypes.c_int64()
    lib.or_rot_coeffs(float(theta), ctypes.byref(c), ctypes.byref(s))
    return c.value, s.value


def warp_nn(B, MB, theta):
    """Nearest-neighbour rotation of B and M_B about B's centre (Sec. 3.6).
    Returns (B', M') uint8."""
    lib = _load()
    B = _u8(B)
    MB = _u8(MB)
    h, w = B.shape
    c, s = rot_coeffs(theta)
    ob = np.empty_like(B)
    om = np.empty_like(B)
    lib.or_warp_nn(_ptr(B), _ptr(MB), h, w, c, s, _ptr(ob), _ptr(om))
    return ob, om


def align(A, MA, B, MB, qa, qb, angles, gamma, nthreads=0, per_angle=False):
    """Alg. 1 (lines 3-9) over the given angles, labels already quantised
    and no zero padding (the full displacement range already contains every
    displacement the padding would admit).  Per angle: warp B and M_B, full
    direct CMIF map, gamma-constrained argmax; the best starts as the identity
    with I = 0 (angle_index -1) and a strictly larger MI replaces it, so the
    first angle wins ties.
    Returns dict(angle_index, angle, dy, dx, mi, n[, per_angle list])."""
    A = _u8(A)
    ha, wa = A.shape
    # I <- 0, T <- IDENTITY (reported as angle_index -1, displacement 0)
    best = dict(angle_index=-1, angle=0.0, dy=0, dx=0, mi=0.0, n=0)
    rows = []
    for k, th in enumerate(angles):
        bw, mw = warp_nn(B, MB, th)
        mp = cmif_direct(A, MA, bw, mw, qa, qb, nthreads=nthreads)
        idx, v, nn = argmax(mp["mi"], mp["n"], gamma)
        sw = mp["mi"].shape[1]
        i, j = divmod(idx, sw)
        rec = dict(angle_index=k, angle=float(th), dy=i - (ha - 1),
                   dx=j - (wa - 1), mi=v, n=nn)
        rows.append(rec)
        if v > best["mi"]:
            best = dict(rec)
    if per_angle:
        best["per_angle"] = rows
    return best


def soft_direct(pa, MA, pb, MB, joint=False, nthreads=0):
    """Soft CMIF by the direct method in FP64 (real-weight generalisation of
    Sec. 3.3): J_ab(chi) = sum_x M_A p_a(x) M_B q_b(x + chi); marginals and N
    are sums of J; MI by Eq. 2 / Eq. 12.  pa [qa,ha,wa], pb [qb,hb,wb]
    float32.  Returns dict(mi, n, joint or None)."""
    lib = _load()
    pa = np.ascontiguousarray(pa, np.float32)
    pb = np.ascontiguousarray(pb, np.float32)
    qa, ha, wa = pa.shape
    qb, hb, wb = pb.shape
    MA, MB = _u8(MA), _u8(MB)
    sh, sw = ha + hb - 1, wa + wb - 1
    mi = np.empty((sh, sw), np.float64)
    n = np.empty((sh, sw), np.float64)
    jo = np.empty((qa, qb, sh, sw), np.float64) if joint else None
    rc = lib.or_soft_direct(_ptr(pa), _ptr(MA), ha, wa, _ptr(pb), _ptr(MB),
                            hb, wb, qa, qb, _ptr(mi), _ptr(n), _ptr(jo),
                            int(nthreads))
    if rc != 0:
        raise OracleError(f"or_soft_direct failed with code {rc}")
    return dict(mi=mi, n=n, joint=jo)


def mi_of_joint(joint):
    """Eq. 2 / Eq. 12 for one explicit [qa, qb] joint table."""
    lib = _load()
    j = np.ascontiguousarray(joint, np.float64)
    return float(lib.or_mi_of_joint(_ptr(j), j.shape[0], j.shape[1]))


def digest_weight(idx: int) -> int:
    return int(_load().or_digest_weight(int(idx)))


# ---------------------------------------------------------------------------
# Soft CMIF in FP64 PyTorch (CPU), differentiable by autograd.
# ---------------------------------------------------------------------------

def soft_joint_torch(pa, ma, pb, mb):
    """Eq. 7 correlations of the weighted level sets, all label pairs:
    J[a, b, i, j] = sum_x wa_a(x) wb_b(x + chi), chi = (i-(H_A-1), j-(W_A-1)),
    with wa = M_A p_a, wb = M_B q_b, evaluated by a library FFT on a grid
    large enough that the circular correlation does not wrap.  pa, pb are
    float64 torch tensors [q, h, w]; ma, mb float64 [h, w]."""
    import torch
    qa, ha, wa = pa.shape
    qb, hb, wb = pb.shape
    sh, sw = ha + hb - 1, wa + wb - 1
    fa = torch.fft.fft2(pa * ma, s=(sh, sw))
    fb = torch.fft.fft2(pb * mb, s=(sh, sw))
    # sum_x f(x) g(x + k)  <->  conj(F) * G
    prod = torch.conj(fa)[:, None] * fb[None, :]
    circ = torch.fft.ifft2(prod).real  # index k = chi mod (sh, sw)
    # reorder circular index k to map index i = chi + (H_A - 1)
    return torch.roll(circ, shifts=(ha - 1, wa - 1), dims=(2, 3))


def soft_mi_torch(joint):
    """Eq. 2 / Eq. 12 on real joint weights J[a, b, ...] (FP64, autograd):
    N = sum J, C_a = sum_b J, C_b = sum_a J; terms with weight <= 0 count 0
    (0 log 0 = 0); MI = 0 where N = 0."""
    import torch
    n = joint.sum(dim=(0, 1))
    ca = joint.sum(dim=1)
    cb = joint.sum(dim=0)
    safe_n = torch.where(n > 0, n, torch.ones_like(n))

    def h(c):
        p = c / safe_n
        pos = p > 0
        ps = torch.where(pos, p, torch.ones_like(p))
        return -torch.where(pos, ps * torch.log2(ps), torch.zeros_like(p)).sum(0)

    ha = h(ca)
    hb = h(cb)
    hab = h(joint.reshape(-1, *joint.shape[2:]))
    return torch.where(n > 0, ha + hb - hab, torch.zeros_like(n)), n


def soft_loss_torch(pairs, gamma=0.5, temperature=0.01):
    """Loss of the soft batch: sum over pairs of logsumexp over the eligible
    displacements (N >= gamma * max N, N = M_A corr M_B, which does not
    depend on the memberships) of MI / temperature.  pairs is a list of
    (pa, ma, pb, mb) float64 torch tensors with pa/pb requiring grad.
    Returns (loss, [mi maps], [eligibility masks])."""
    import torch
    total = 0.0
    maps, elig = [], []
    for pa, ma, pb, mb in pairs:
        j = soft_joint_torch(pa, ma, pb, mb)
        mi, _ = soft_mi_torch(j)
        nmask = soft_joint_torch(ma[None], ma, mb[None], mb)[0, 0].detach()
        nr = torch.round(nmask)
        e = nr >= gamma * nr.max()
        total = total + torch.logsumexp(mi[e] / temperature, dim=0)
        maps.append(mi)
        elig.append(e)
    return total, maps, elig


# ---------------------------------------------------------------------------
# Mini-batch k-means (the QUANTIZE step of Alg. 1, Sec. 3.6).
# ---------------------------------------------------------------------------

def _as_pixels(img):
    x = np.asarray(img)
    return x.reshape(x.shape[0] * x.shape[1], -1) if x.ndim == 3 else x.reshape(-1, 1)


def kmeans_nearest(x, centers):
    """Index of the nearest centre for each row of x (FP64 squared
    Euclidean distance, channels accumulated in order; ties to the lowest
    index, as np.argmin returns the first minimum)."""
    x = np.asarray(x, np.float64)
    c = np.asarray(centers, np.float64)
    d = np.zeros((x.shape[0], c.shape[0]), np.float64)
    for ch in range(x.shape[1]):
        e = x[:, ch][:, None] - c[:, ch][None, :]
        d = d + e * e
    return np.argmin(d, axis=1)


def kmeans_minibatch(img, k, init_idx=None, batches=None, centers=None):
    """Sculley's mini-batch k-means, the quantiser the paper uses (Sec. 3.6):
    centres start at the pixels init_idx (or at `centers`); per batch, every
    sample is assigned to its nearest centre under the centres at the start
    of the batch, then the samples are applied in batch order: the centre's
    count v grows by one and the centre becomes (1 - 1/v) c + (1/v) x.
    Indices outside the image are skipped.  Pixels are rows of channels
    (img [H, W] or [H, W, m], or already [n, m]).  Returns the centres
    [k, m] (FP64)."""
    x = _as_pixels(img)
    n, m = x.shape
    if centers is not None:
        c = np.array(centers, np.float64).reshape(k, m)
    else:
        c = np.zeros((k, m), np.float64)
        for j, idx in enumerate(np.asarray(init_idx).ravel()[:k]):
            if 0 <= idx < n:
                c[j] = x[idx].astype(np.float64)
    v = np.zeros(k, np.int64)
    for mb in ([] if batches is None else np.asarray(batches)):
        mb = np.asarray(mb).ravel()
        mb = mb[(mb >= 0) & (mb < n)]
        pts = x[mb].astype(np.float64)
        lab = kmeans_nearest(pts, c)
        for p, j in zip(pts, lab):
            v[j] += 1
            eta = 1.0 / float(v[j])
            c[j] = (1.0 - eta) * c[j] + eta * p
    return c


def kmeans_labels(img, centers, mask=None):
    """Nearest-centre label of every pixel, 0 outside the mask (uint8,
    image shape)."""
    x = _as_pixels(img)
    lab = kmeans_nearest(x, centers).astype(np.uint8)
    if mask is not None:
        lab[np.asarray(mask).reshape(-1) == 0] = 0
    shape = np.asarray(img).shape[:2]
    return lab.reshape(shape)

