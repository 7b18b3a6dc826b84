"""GPU: the soft-membership batch at its own sizes (16 pairs, sides drawn in
128..384, Q 8), against the FP64 torch oracle.

These sizes reach the FFT lengths whose row and adjoint kernels run
two-wave teams with workgroup-level exchanges (1024 points), next to
one-wave teams (512 points), in one plan.  Bars as in test_gpu_soft.py:
forward |MI - oracle| <= 1e-5 on eligible displacements (FP32 transforms),
gradients relative L2 <= 1e-3 against FP64 autograd of the oracle, and the
FP64 adjoint against central differences of the FP64 forward."""

import numpy as np
import pytest

import synth
from gpu_common import dev, say

pytestmark = pytest.mark.gpu

SAVE = 1 << 2  # CMIF_FLAG_SAVE_FOR_BACKWARD

# pairs of the batch whose FFT sides are (512, 512), (1024, 1024),
# (1024, 1024) and (1024, 512)
FWD_PAIRS = (0, 3, 9, 15)
GRAD_PAIRS = (0, 3, 8)


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


def _p2(v):
    p = 128
    while p < v:
        p *= 2
    return p


def test_soft_batch_full_size_covers_both_team_shapes(batch):
    sides = {(_p2(s[0] + s[2] - 1), _p2(s[1] + s[3] - 1)) for s in batch["sizes"]}
    assert (1024, 1024) in sides and (512, 512) in sides
    for k in FWD_PAIRS + GRAD_PAIRS:
        s = batch["sizes"][k]
        assert max(_p2(s[0] + s[2] - 1), _p2(s[1] + s[3] - 1)) >= 512


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


def test_soft_adjoint_central_differences_1024(gpu):
    """FP64 adjoint of one batch pair whose FFT sides are 1024 (two-wave
    teams in the adjoint's row and output kernels) against central
    differences of the library's own FP64 forward: L = sum_chi w(chi)
    MI(chi), fixed weights on eligible displacements."""
    cm, torch = gpu
    p = synth.config5()["pairs"][3]
    ha, wa = p["MA"].shape
    hb, wb = p["MB"].shape
    assert _p2(ha + hb - 1) == 1024 and _p2(wa + wb - 1) == 1024
    say(f"[gpu] soft FP64 adjoint vs central differences {(ha, wa, hb, wb)}")
    sp = cm.Plan([(ha, wa, hb, wb)], 8, 8, precision="fp64", mode="soft",
                 flags=SAVE)
    MA, MB = dev(torch, p["MA"]), dev(torch, p["MB"])
    n = sp.compute(fdev(torch, p["PA"]), MA, fdev(torch, p["PB"]), MB,
                   mi=False, n=True)["n"][0][0].cpu().numpy()
    w = np.random.default_rng(9).standard_normal(n.shape) * (n >= 0.5 * n.max())

    def loss(pa, pb):
        mi = sp.compute(fdev(torch, pa), MA, fdev(torch, pb), MB, mi=True,
                        n=False)["mi"][0][0].cpu().numpy()
        return float((mi * w).sum())

    sp.compute(fdev(torch, p["PA"]), MA, fdev(torch, p["PB"]), MB, mi=True,
               n=False)
    ga, gb = sp.backward(fdev(torch, p["PA"]), MA, fdev(torch, p["PB"]), MB,
                         [torch.from_numpy(w[None]).cuda()])
    ga, gb = ga[0].cpu().numpy(), gb[0].cpu().numpy()
    rng = np.random.default_rng(21)
    worst = 0.0
    h = np.float32(2.0 ** -9)
    for side, base, g in (("A", p["PA"], ga), ("B", p["PB"], gb)):
        for _ in range(3):
            q = int(rng.integers(0, base.shape[0]))
            y = int(rng.integers(0, base.shape[1]))
            x = int(rng.integers(0, base.shape[2]))
            hp = base.copy()
            hm = base.copy()
            hp[q, y, x] = np.float32(base[q, y, x] + h)
            hm[q, y, x] = np.float32(base[q, y, x] - h)
            step = float(hp[q, y, x]) - float(hm[q, y, x])
            if side == "A":
                fd = (loss(hp, p["PB"]) - loss(hm, p["PB"])) / step
            else:
                fd = (loss(p["PA"], hp) - loss(p["PA"], hm)) / step
            err = abs(fd - g[q, y, x]) / max(abs(fd), 1e-6)
            say(f"  {side}[{q},{y},{x}] fd {fd:.6e} adjoint {g[q, y, x]:.6e} "
                f"rel {err:.2e}")
            worst = max(worst, err)
            assert err <= 1e-3, (side, q, y, x, fd, g[q, y, x])
    say(f"adjoint vs central differences at 1024 points: worst {worst:.2e}")


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
