"""GPU: soft-membership CMIF forward and adjoint against the FP64 oracles.

Bars:
  * forward, FP32 transforms: |MI - oracle| <= 1e-5 on eligible
    displacements (N >= gamma max N).  At displacements with a few pixels of
    overlap the joint values are below the FP32 transform's absolute error
    (about 1e-7 of the largest joint value), so the full map is only
    checked to a looser bound there;
  * forward, FP64 transforms: <= 1e-9 on eligible displacements;
  * N output (mask overlap count): exact;
  * gradients: relative L2 error <= 1e-3 (FP32) and <= 2e-7 (FP64) against
    FP64 autograd of the torch oracle with the same upstream weights (the
    gradients leave the library as float32, whose rounding alone is about
    6e-8 relative).
"""

import numpy as np
import pytest

import synth
from gpu_common import dev, say

pytestmark = pytest.mark.gpu

SAVE = 1 << 2  # CMIF_FLAG_SAVE_FOR_BACKWARD


def fdev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def eligible(n, gamma=0.5):
    return n >= gamma * n.max()


def soft_plan(cm, shape_a, shape_b, qa, qb, precision, flags=SAVE, angles=None):
    return cm.Plan([(*shape_a, *shape_b)], qa, qb, angles=angles,
                   precision=precision, mode="soft", flags=flags)


def one_hot(lab, q):
    return np.stack([(lab == k).astype(np.float32) for k in range(q)])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_soft_one_hot_equals_hard(gpu, oracle, precision):
    cm, torch = gpu
    c = synth.random_case(606, 45, 52, 38, 41, 4, 5, mask_density=0.8)
    say(f"[gpu] soft one-hot vs hard 45x52/38x41 q4,5 {precision}")
    hard = cm.Plan([(45, 52, 38, 41)], 4, 5, precision="fp64")
    rh = hard.compute(dev(torch, c["A"]), dev(torch, c["MA"]),
                      dev(torch, c["B"]), dev(torch, c["MB"]), mi=True, n=True)
    sp = soft_plan(cm, (45, 52), (38, 41), 4, 5, precision, flags=0)
    rs = sp.compute(fdev(torch, one_hot(c["A"], 4)), dev(torch, c["MA"]),
                    fdev(torch, one_hot(c["B"], 5)), dev(torch, c["MB"]),
                    mi=True, n=True, best=True)
    mh, nh = rh["mi"][0][0].cpu().numpy(), rh["n"][0][0].cpu().numpy()
    ms, ns = rs["mi"][0][0].cpu().numpy(), rs["n"][0][0].cpu().numpy()
    assert np.array_equal(ns, nh), "overlap count differs from the hard N"
    e = eligible(nh)
    err = np.abs(ms - mh)[e].max()
    say(f"one-hot {precision}: eligible max|dMI| {err:.3e}, "
        f"full-map max {np.abs(ms - mh).max():.3e}")
    assert err <= (1e-5 if precision == "fp32" else 1e-9)
    assert rs["stats"]["nonfinite_inputs"] == 0


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", [(40, 36, 33, 45, 3, 4, 0.8),
                                  (64, 64, 64, 64, 8, 8, None),
                                  (17, 90, 70, 20, 2, 5, 0.9),
                                  # column and row lengths on either side of
                                  # 1024 (1536 x 128 and 128 x 1536)
                                  (600, 30, 560, 40, 3, 4, 0.9),
                                  (30, 600, 40, 560, 3, 4, 0.9)],
                         ids=["40x36-33x45-q34", "64-q8", "17x90-70x20-q25",
                              "600x30-560x40-q34", "30x600-40x560-q34"])
def test_soft_forward_vs_oracle(gpu, oracle, precision, case):
    cm, torch = gpu
    ha, wa, hb, wb, qa, qb, dens = case
    c = synth.random_soft_case(700 + ha + wb, ha, wa, hb, wb, qa, qb=qb,
                               mask_density=dens)
    say(f"[gpu] soft forward {case} {precision}")
    sp = soft_plan(cm, (ha, wa), (hb, wb), qa, qb, precision)
    r = sp.compute(fdev(torch, c["PA"]), dev(torch, c["MA"]),
                   fdev(torch, c["PB"]), dev(torch, c["MB"]), mi=True, n=True)
    o = oracle.soft_direct(c["PA"], c["MA"], c["PB"], c["MB"])
    ov = oracle.cmif_direct(np.zeros((ha, wa), np.uint8), c["MA"],
                            np.zeros((hb, wb), np.uint8), c["MB"], 1, 1)
    mi = r["mi"][0][0].cpu().numpy()
    n = r["n"][0][0].cpu().numpy()
    assert np.array_equal(n, ov["n"]), "mask overlap count differs"
    e = eligible(ov["n"])
    err = np.abs(mi - o["mi"])[e].max()
    full = np.abs(mi - o["mi"])[ov["n"] >= 16].max()
    say(f"soft {precision}: eligible max|dMI| {err:.3e}, N>=16 {full:.3e}")
    assert err <= (1e-5 if precision == "fp32" else 1e-9)
    assert full <= (1e-2 if precision == "fp32" else 1e-7)


def torch_grads(oracle, c, w):
    import torch
    pa = torch.tensor(c["PA"], dtype=torch.float64, requires_grad=True)
    pb = torch.tensor(c["PB"], dtype=torch.float64, requires_grad=True)
    ma = torch.tensor(c["MA"], dtype=torch.float64)
    mb = torch.tensor(c["MB"], dtype=torch.float64)
    mi, _ = oracle.soft_mi_torch(oracle.soft_joint_torch(pa, ma, pb, mb))
    (mi * torch.tensor(w)).sum().backward()
    return pa.grad.numpy(), pb.grad.numpy(), mi.detach().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", [(30, 26, 24, 33, 3, 4, 0.85),
                                  (48, 48, 48, 48, 4, 4, None)],
                         ids=["30x26-24x33-q34-mask", "48-q4"])
def test_soft_gradients(gpu, oracle, precision, case):
    cm, torch = gpu
    ha, wa, hb, wb, qa, qb, dens = case
    c = synth.random_soft_case(900 + ha * wb, ha, wa, hb, wb, qa, qb=qb,
                               mask_density=dens)
    ov = oracle.cmif_direct(np.zeros((ha, wa), np.uint8), c["MA"],
                            np.zeros((hb, wb), np.uint8), c["MB"], 1, 1)
    rng = np.random.default_rng(5)
    w = rng.standard_normal(ov["n"].shape) * eligible(ov["n"])
    ga_o, gb_o, _ = torch_grads(oracle, c, w)
    say(f"[gpu] soft gradients {case} {precision}")
    sp = soft_plan(cm, (ha, wa), (hb, wb), qa, qb, precision)
    A, B = fdev(torch, c["PA"]), fdev(torch, c["PB"])
    MA, MB = dev(torch, c["MA"]), dev(torch, c["MB"])
    sp.compute(A, MA, B, MB, mi=True, n=False)
    gm = torch.from_numpy(w[None]).cuda()
    ga, gb = sp.backward(A, MA, B, MB, [gm])
    ea = rel_l2(ga[0].cpu().numpy(), ga_o)
    eb = rel_l2(gb[0].cpu().numpy(), gb_o)
    say(f"grad rel L2: A {ea:.3e}  B {eb:.3e}")
    tol = 1e-3 if precision == "fp32" else 2e-7
    assert ea <= tol and eb <= tol
    # masked-out pixels get exactly zero gradient
    assert np.all(ga[0].cpu().numpy()[:, c["MA"] == 0] == 0)
    assert np.all(gb[0].cpu().numpy()[:, c["MB"] == 0] == 0)


def test_soft_cmif_autograd_loss(gpu, oracle):
    """SoftCMIF through torch autograd with the batch loss (logsumexp of
    MI / 0.01 over eligible displacements) against the oracle loss."""
    cm, torch = gpu
    c = synth.random_soft_case(1234, 52, 47, 44, 50, 4, qb=3)
    ha, wa = c["MA"].shape
    hb, wb = c["MB"].shape
    sp = soft_plan(cm, (ha, wa), (hb, wb), 4, 3, "fp32")
    say("[gpu] SoftCMIF autograd loss 52x47/44x50 q4,3")
    A = fdev(torch, c["PA"]).requires_grad_(True)
    B = fdev(torch, c["PB"]).requires_grad_(True)
    MA, MB = dev(torch, c["MA"]), dev(torch, c["MB"])
    n = sp.compute(A.detach(), MA, B.detach(), MB, mi=False, n=True)["n"][0][0]
    e = n >= 0.5 * n.max()
    mi = cm.soft_cmif(A, B, sp, MA, MB)[0]
    loss = torch.logsumexp(mi[e] / 0.01, dim=0)
    loss.backward()
    pa = torch.tensor(c["PA"], dtype=torch.float64, requires_grad=True)
    pb = torch.tensor(c["PB"], dtype=torch.float64, requires_grad=True)
    lo, _, el = oracle.soft_loss_torch(
        [(pa, torch.tensor(c["MA"], dtype=torch.float64), pb,
          torch.tensor(c["MB"], dtype=torch.float64))], 0.5, 0.01)
    lo.backward()
    assert np.array_equal(e.cpu().numpy(), el[0].numpy())
    say(f"loss gpu {loss.item():.9f} oracle {lo.item():.9f}")
    assert abs(loss.item() - lo.item()) <= 1e-3
    assert rel_l2(A.grad.cpu().numpy(), pa.grad.numpy()) <= 1e-3
    assert rel_l2(B.grad.cpu().numpy(), pb.grad.numpy()) <= 1e-3


def test_soft_batch_uneven_pairs(gpu, oracle):
    """Several soft pairs of different sizes in one plan (the C5 layout,
    smaller sizes): forward against the FP64 torch oracle per pair."""
    cm, torch = gpu
    cfg = synth.config5(n_pairs=4, q=8, lo=60, hi=140, shift_max=12)
    pairs = cfg["pairs"]
    sizes = [(*p["MA"].shape, *p["MB"].shape) for p in pairs]
    say(f"[gpu] soft batch {sizes}")
    plan = cm.Plan(sizes, 8, 8, mode="soft", precision="fp32", flags=SAVE)
    A = [fdev(torch, p["PA"]) for p in pairs]
    B = [fdev(torch, p["PB"]) for p in pairs]
    MA = [dev(torch, p["MA"]) for p in pairs]
    MB = [dev(torch, p["MB"]) for p in pairs]
    r = plan.compute(A, MA, B, MB, mi=True, n=True, best=True)
    for k, p in enumerate(pairs):
        f64 = lambda a: torch.tensor(a, dtype=torch.float64)
        omi, _ = oracle.soft_mi_torch(oracle.soft_joint_torch(
            f64(p["PA"]), f64(p["MA"]), f64(p["PB"]), f64(p["MB"])))
        omi = omi.numpy()
        n = r["n"][k][0].cpu().numpy()
        e = eligible(n)
        err = np.abs(r["mi"][k][0].cpu().numpy() - omi)[e].max()
        b = r["best"][k]
        ha, wa = p["MA"].shape
        say(f"pair {k} {sizes[k]}: eligible max|dMI| {err:.3e} best "
            f"({b['dy']},{b['dx']}) planted {p['shift']}")
        assert err <= 1e-5
        # Alg. 1 on the soft map: the pick is eligible and within the
        # forward tolerance of the oracle's eligible maximum
        i, j = b["dy"] + ha - 1, b["dx"] + wa - 1
        assert e[i, j]
        assert abs(omi[i, j] - omi[e].max()) <= 2e-5


def test_soft_adjoint_vs_central_differences(gpu):
    """The library's FP64 adjoint against central differences of its own
    FP64 forward, on a tiny case (12x10 against 9x11, Q 3): L = sum_chi
    w(chi) MI(chi) with fixed weights on eligible displacements."""
    cm, torch = gpu
    c = synth.random_soft_case(31, 12, 10, 9, 11, 3, mask_density=0.9)
    sp = soft_plan(cm, (12, 10), (9, 11), 3, 3, "fp64")
    MA, MB = dev(torch, c["MA"]), dev(torch, c["MB"])
    n = sp.compute(fdev(torch, c["PA"]), MA, fdev(torch, c["PB"]), MB, mi=False,
                   n=True)["n"][0][0].cpu().numpy()
    w = np.random.default_rng(7).standard_normal(n.shape) * eligible(n)

    def loss(pa, pb):
        mi = sp.compute(fdev(torch, pa), MA, fdev(torch, pb), MB, mi=True,
                        n=False)["mi"][0][0].cpu().numpy()
        return float((mi * w).sum())

    sp.compute(fdev(torch, c["PA"]), MA, fdev(torch, c["PB"]), MB, mi=True, n=False)
    ga, gb = sp.backward(fdev(torch, c["PA"]), MA, fdev(torch, c["PB"]), MB,
                         [torch.from_numpy(w[None]).cuda()])
    ga, gb = ga[0].cpu().numpy(), gb[0].cpu().numpy()
    rng = np.random.default_rng(11)
    worst = 0.0
    for side, base, g in (("A", c["PA"], ga), ("B", c["PB"], gb)):
        mask = c["MA"] if side == "A" else c["MB"]
        for _ in range(6):
            q = int(rng.integers(0, base.shape[0]))
            y = int(rng.integers(0, base.shape[1]))
            x = int(rng.integers(0, base.shape[2]))
            if not mask[y, x]:
                continue
            hp = base.copy()
            hm = base.copy()
            hp[q, y, x] = np.float32(base[q, y, x] + np.float32(2.0 ** -10))
            hm[q, y, x] = np.float32(base[q, y, x] - np.float32(2.0 ** -10))
            step = float(hp[q, y, x]) - float(hm[q, y, x])
            if side == "A":
                fd = (loss(hp, c["PB"]) - loss(hm, c["PB"])) / step
            else:
                fd = (loss(c["PA"], hp) - loss(c["PA"], hm)) / step
            err = abs(fd - g[q, y, x]) / max(abs(fd), 1e-3)
            worst = max(worst, err)
            assert err <= 1e-3, (side, q, y, x, fd, g[q, y, x])
    say(f"adjoint vs central differences: worst relative error {worst:.2e}")


def test_spatially_weighted_mi(gpu, oracle):
    """Spatially weighted MI (Sec. 3.3, Eq. 13) through the soft path: the
    memberships are the level-set indicators times the weight maps, so each
    displacement's joint is the weighted histogram sum_x W_A(x) W_B(x + chi)
    [A(x) = a][B(x + chi) = b]."""
    cm, torch = gpu
    c = synth.random_case(1313, 50, 44, 41, 52, 4, 5, mask_density=None)
    rng = np.random.default_rng(1313)
    wa = rng.uniform(0.0, 1.0, c["A"].shape).astype(np.float32)
    wb = rng.uniform(0.0, 1.0, c["B"].shape).astype(np.float32)
    pa = one_hot(c["A"], 4) * wa[None]
    pb = one_hot(c["B"], 5) * wb[None]
    sp = soft_plan(cm, (50, 44), (41, 52), 4, 5, "fp64", flags=0)
    r = sp.compute(fdev(torch, pa), None, fdev(torch, pb), None, mi=True, n=True)
    o = oracle.soft_direct(pa, np.ones_like(c["MA"]), pb, np.ones_like(c["MB"]))
    n = r["n"][0][0].cpu().numpy()
    e = eligible(n)
    err = np.abs(r["mi"][0][0].cpu().numpy() - o["mi"])[e].max()
    say(f"SWMI fp64: eligible max|dMI| {err:.3e}")
    assert err <= 1e-9
