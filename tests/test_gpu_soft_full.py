"""GPU: the soft-membership batch at its own sizes (16 pairs, sides drawn in
128..384, Q 8), against the FP64 torch oracle, and soft pairs large enough
for the 1024-point row and adjoint kernels (two-wave teams with
workgroup-level exchanges).

The batch reaches FFT sides 256, 512 and 768 (3 * 2^8: 12-point first
stages) in one plan.  Bars as in test_gpu_soft.py: forward |MI - oracle| <=
1e-5 on eligible displacements (FP32 transforms), gradients relative L2 <=
1e-3 against FP64 autograd of the oracle, and the FP64 adjoint against
central differences of the FP64 forward."""

import numpy as np
import pytest

import synth
from gpu_common import dev, say

pytestmark = pytest.mark.gpu

SAVE = 1 << 2  # CMIF_FLAG_SAVE_FOR_BACKWARD

FWD_PAIRS = (0, 3, 9, 15)
GRAD_PAIRS = (0, 3, 8)
SIZES = (128, 256, 512, 768, 1024, 1536, 2048)


def fft_side(n):
    return min(p for p in SIZES if p >= n)


def fdev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def f64(torch, a):
    return torch.tensor(np.asarray(a), dtype=torch.float64)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def batch(gpu):
    cm, torch = gpu
    cfg = synth.config5()
    pairs = cfg["pairs"]
    sizes = [(*p["MA"].shape, *p["MB"].shape) for p in pairs]
    say(f"[gpu] soft batch at full size: {sizes}")
    plan = cm.Plan(sizes, 8, 8, mode="soft", precision="fp32", flags=SAVE)
    A = [fdev(torch, p["PA"]) for p in pairs]
    B = [fdev(torch, p["PB"]) for p in pairs]
    MA = [dev(torch, p["MA"]) for p in pairs]
    MB = [dev(torch, p["MB"]) for p in pairs]
    return dict(cm=cm, torch=torch, cfg=cfg, pairs=pairs, sizes=sizes,
                plan=plan, A=A, B=B, MA=MA, MB=MB)


def test_soft_batch_full_size_covers_fft_sides(batch):
    sides = {fft_side(s[0] + s[2] - 1) for s in batch["sizes"]} | \
        {fft_side(s[1] + s[3] - 1) for s in batch["sizes"]}
    assert {512, 768} <= sides
    plan = batch["cm"].Plan([batch["sizes"][3]], 8, 8, mode="soft",
                            precision="fp32")
    assert (plan.info()["fft_h"], plan.info()["fft_w"]) == (768, 768)


def test_soft_batch_full_size_forward(batch, oracle):
    torch, plan, pairs = batch["torch"], batch["plan"], batch["pairs"]
    r = plan.compute(batch["A"], batch["MA"], batch["B"], batch["MB"],
                     mi=True, n=True, best=True)
    for k in FWD_PAIRS:
        p = pairs[k]
        omi, on = oracle.soft_mi_torch(oracle.soft_joint_torch(
            f64(torch, p["PA"]), f64(torch, p["MA"]), f64(torch, p["PB"]),
            f64(torch, p["MB"])))
        omi = omi.numpy()
        n = r["n"][k][0].cpu().numpy()
        # all-ones masks: N is the rectangle overlap, the oracle's joint sum
        assert np.array_equal(n, np.rint(on.numpy()).astype(np.int64))
        e = n >= 0.5 * n.max()
        err = float(np.abs(r["mi"][k][0].cpu().numpy() - omi)[e].max())
        b = r["best"][k]
        ha, wa = p["MA"].shape
        i, j = b["dy"] + ha - 1, b["dx"] + wa - 1
        say(f"pair {k} {batch['sizes'][k]}: eligible max|dMI| {err:.3e}, best "
            f"({b['dy']},{b['dx']}) planted {p['shift']}")
        assert err <= 1e-5
        assert e[i, j] and abs(omi[i, j] - omi[e].max()) <= 2e-5


def test_soft_batch_full_size_gradients(batch, oracle):
    cm, torch, plan, pairs = batch["cm"], batch["torch"], batch["plan"], batch["pairs"]
    r = plan.compute(batch["A"], batch["MA"], batch["B"], batch["MB"], mi=True,
                     n=True)
    rng = np.random.default_rng(55)
    weights = []
    for k in range(len(pairs)):
        n = r["n"][k][0].cpu().numpy()
        weights.append(rng.standard_normal(n.shape) * (n >= 0.5 * n.max()))
    gm = [torch.from_numpy(w[None]).cuda() for w in weights]
    ga, gb = plan.backward(batch["A"], batch["MA"], batch["B"], batch["MB"], gm)
    for k in GRAD_PAIRS:
        p = pairs[k]
        pa = f64(torch, p["PA"]).requires_grad_(True)
        pb = f64(torch, p["PB"]).requires_grad_(True)
        mi, _ = oracle.soft_mi_torch(oracle.soft_joint_torch(
            pa, f64(torch, p["MA"]), pb, f64(torch, p["MB"])))
        (mi * torch.from_numpy(weights[k])).sum().backward()
        ea = rel_l2(ga[k].cpu().numpy(), pa.grad.numpy())
        eb = rel_l2(gb[k].cpu().numpy(), pb.grad.numpy())
        say(f"pair {k} {batch['sizes'][k]}: grad rel L2 A {ea:.3e} B {eb:.3e}")
        assert ea <= 1e-3 and eb <= 1e-3


def _pair_1024():
    """A soft pair whose FFT sides are 1024 (420 x 400 against 410 x 430,
    Q 4): two-wave teams in the soft row and adjoint kernels."""
    return synth.random_soft_case(1024, 420, 400, 410, 430, 4, smooth=4.0)


def test_soft_1024_forward_and_gradients(gpu, oracle):
    cm, torch = gpu
    c = _pair_1024()
    size = (*c["MA"].shape, *c["MB"].shape)
    plan = cm.Plan([size], 4, 4, mode="soft", precision="fp32", flags=SAVE)
    assert (plan.info()["fft_h"], plan.info()["fft_w"]) == (1024, 1024)
    say(f"[gpu] soft pair at FFT side 1024 {size}")
    A, B = fdev(torch, c["PA"]), fdev(torch, c["PB"])
    MA, MB = dev(torch, c["MA"]), dev(torch, c["MB"])
    r = plan.compute(A, MA, B, MB, mi=True, n=True)
    pa = f64(torch, c["PA"]).requires_grad_(True)
    pb = f64(torch, c["PB"]).requires_grad_(True)
    omi, _ = oracle.soft_mi_torch(oracle.soft_joint_torch(
        pa, f64(torch, c["MA"]), pb, f64(torch, c["MB"])))
    n = r["n"][0][0].cpu().numpy()
    e = n >= 0.5 * n.max()
    err = float(np.abs(r["mi"][0][0].cpu().numpy() - omi.detach().numpy())[e].max())
    w = np.random.default_rng(77).standard_normal(n.shape) * e
    (omi * torch.from_numpy(w)).sum().backward()
    ga, gb = plan.backward(A, MA, B, MB, [torch.from_numpy(w[None]).cuda()])
    ea = rel_l2(ga[0].cpu().numpy(), pa.grad.numpy())
    eb = rel_l2(gb[0].cpu().numpy(), pb.grad.numpy())
    say(f"eligible max|dMI| {err:.3e}; grad rel L2 A {ea:.3e} B {eb:.3e}")
    assert err <= 1e-5
    assert ea <= 1e-3 and eb <= 1e-3


@pytest.mark.parametrize("which", ["1024", "768"])
def test_soft_adjoint_central_differences_large(gpu, which):
    """FP64 adjoint against central differences of the library's own FP64
    forward, L = sum_chi w(chi) MI(chi) with fixed weights on eligible
    displacements: a pair at FFT side 1024 (two-wave teams in the adjoint's
    row and output kernels) and a batch pair at 768 (12-point stages)."""
    cm, torch = gpu
    if which == "1024":
        p = _pair_1024()
        pa0, pb0, q = p["PA"], p["PB"], 4
    else:
        p = synth.config5()["pairs"][3]
        pa0, pb0, q = p["PA"], p["PB"], 8
    ha, wa = p["MA"].shape
    hb, wb = p["MB"].shape
    sp = cm.Plan([(ha, wa, hb, wb)], q, q, precision="fp64", mode="soft",
                 flags=SAVE)
    assert sp.info()["fft_h"] == int(which)
    say(f"[gpu] soft FP64 adjoint vs central differences {(ha, wa, hb, wb)} "
        f"fft {sp.info()['fft_h']}x{sp.info()['fft_w']}")
    MA, MB = dev(torch, p["MA"]), dev(torch, p["MB"])
    n = sp.compute(fdev(torch, pa0), MA, fdev(torch, pb0), MB,
                   mi=False, n=True)["n"][0][0].cpu().numpy()
    w = np.random.default_rng(9).standard_normal(n.shape) * (n >= 0.5 * n.max())

    def loss(pa, pb):
        mi = sp.compute(fdev(torch, pa), MA, fdev(torch, pb), MB, mi=True,
                        n=False)["mi"][0][0].cpu().numpy()
        return float((mi * w).sum())

    sp.compute(fdev(torch, pa0), MA, fdev(torch, pb0), MB, mi=True, n=False)
    ga, gb = sp.backward(fdev(torch, pa0), MA, fdev(torch, pb0), MB,
                         [torch.from_numpy(w[None]).cuda()])
    ga, gb = ga[0].cpu().numpy(), gb[0].cpu().numpy()
    rng = np.random.default_rng(21)
    worst = 0.0
    h = np.float32(2.0 ** -9)
    for side, base, g in (("A", pa0, ga), ("B", pb0, gb)):
        for _ in range(3):
            k = int(rng.integers(0, base.shape[0]))
            y = int(rng.integers(0, base.shape[1]))
            x = int(rng.integers(0, base.shape[2]))
            hp = base.copy()
            hm = base.copy()
            hp[k, y, x] = np.float32(base[k, y, x] + h)
            hm[k, y, x] = np.float32(base[k, y, x] - h)
            step = float(hp[k, y, x]) - float(hm[k, y, x])
            if side == "A":
                fd = (loss(hp, pb0) - loss(hm, pb0)) / step
            else:
                fd = (loss(pa0, hp) - loss(pa0, hm)) / step
            err = abs(fd - g[k, y, x]) / max(abs(fd), 1e-6)
            say(f"  {side}[{k},{y},{x}] fd {fd:.6e} adjoint {g[k, y, x]:.6e} "
                f"rel {err:.2e}")
            worst = max(worst, err)
            assert err <= 1e-3, (side, k, y, x, fd, g[k, y, x])
    say(f"adjoint vs central differences: worst {worst:.2e}")


def test_soft_cmif_two_forwards_share_a_plan(gpu, oracle):
    """Two SoftCMIF forwards on one plan before backward (a loss summed over
    two pairs of one size): each gradient must be its own pair's, although
    the second forward overwrote the plan's saved state."""
    cm, torch = gpu
    c1 = synth.random_soft_case(41, 40, 44, 38, 36, 3, qb=4)
    c2 = synth.random_soft_case(42, 40, 44, 38, 36, 3, qb=4)
    plan = cm.Plan([(40, 44, 38, 36)], 3, 4, mode="soft", precision="fp32",
                   flags=SAVE)
    say("[gpu] two SoftCMIF forwards on one plan, one backward")
    A1 = fdev(torch, c1["PA"]).requires_grad_(True)
    B1 = fdev(torch, c1["PB"]).requires_grad_(True)
    A2 = fdev(torch, c2["PA"]).requires_grad_(True)
    B2 = fdev(torch, c2["PB"]).requires_grad_(True)
    m1 = cm.soft_cmif(A1, B1, plan)[0]
    m2 = cm.soft_cmif(A2, B2, plan)[0]
    # weights on eligible displacements only (all-ones masks: N is the
    # rectangle overlap)
    ov = oracle.cmif_direct(np.zeros((40, 44), np.uint8), None,
                            np.zeros((38, 36), np.uint8), None, 1, 1)["n"]
    elig = ov >= 0.5 * ov.max()
    rng = np.random.default_rng(3)
    w1 = torch.from_numpy(rng.standard_normal(elig.shape) * elig).cuda()[None]
    w2 = torch.from_numpy(rng.standard_normal(elig.shape) * elig).cuda()[None]
    ((m1 * w1).sum() + (m2 * w2).sum()).backward()
    assert plan.recomputed_forwards >= 1
    for c, A, B, w in ((c1, A1, B1, w1), (c2, A2, B2, w2)):
        pa = f64(torch, c["PA"]).requires_grad_(True)
        pb = f64(torch, c["PB"]).requires_grad_(True)
        mi, _ = oracle.soft_mi_torch(oracle.soft_joint_torch(
            pa, f64(torch, c["MA"]), pb, f64(torch, c["MB"])))
        (mi * w[0].cpu()).sum().backward()
        ea = rel_l2(A.grad.cpu().numpy(), pa.grad.numpy())
        eb = rel_l2(B.grad.cpu().numpy(), pb.grad.numpy())
        say(f"grad rel L2 A {ea:.3e} B {eb:.3e}")
        assert ea <= 1e-3 and eb <= 1e-3
