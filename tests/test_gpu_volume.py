"""GPU: the 3-D (volume) CMIF through cmif_compute_volume against the
oracle's 3-D direct method: N exact everywhere, every label pair's count
digest exact, MI within 1e-12 everywhere, Alg. 1's pick by the oracle's
rule (near-ties as in 2-D), the planted displacement recovered; depth-1
volumes against the 2-D plan."""

import numpy as np
import pytest

import synth
from gpu_common import MI_TOL, argmax_ok, dev, say

pytestmark = pytest.mark.gpu


def _check(cm, torch, oracle, c, qa, qb, precision, tag):
    say(f"[gpu] volume {tag} A{c['A'].shape} B{c['B'].shape} q=({qa},{qb}) "
        f"{precision}")
    r = cm.compute_volume(dev(torch, c["A"]), dev(torch, c["MA"]),
                          dev(torch, c["B"]), dev(torch, c["MB"]), qa, qb,
                          precision=precision, digest=True)
    o = oracle.cmif_direct3d(c["A"], c["MA"], c["B"], c["MB"], qa, qb,
                             digest=True)
    n = r["n"].cpu().numpy()
    mi = r["mi"].cpu().numpy()
    assert np.array_equal(n, o["n"]), "N differs"
    assert np.array_equal(r["digest"].cpu().numpy().view(np.uint64), o["digest"])
    err = float(np.abs(mi - o["mi"]).max())
    assert err <= MI_TOL, err
    b = r["best"]
    da, ha, wa = c["A"].shape
    sd, sh, sw = o["mi"].shape
    g_idx = ((b["dz"] + da - 1) * sh + b["dy"] + ha - 1) * sw + b["dx"] + wa - 1
    ok, near = argmax_ok(oracle, o["mi"].reshape(sd * sh, sw),
                         o["n"].reshape(sd * sh, sw), 0.5, g_idx)
    assert ok, b
    st = r["stats"]
    say(f"  max|dMI| {err:.2e} best ({b['dz']},{b['dy']},{b['dx']}) mi "
        f"{b['mi']:.6f} residual {st['max_residual']:.4f} near-tie {near}")
    assert st["unresolved_pairs"] == 0 and st["label_errors"] == 0
    return r


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_volume_small_with_masks(gpu, oracle, precision):
    cm, torch = gpu
    c = synth.volume_pair(31, (12, 14, 10), (9, 11, 13), 3, (2, -3, 1),
                          mask_density=0.8)
    # B relabelled into 4 labels to exercise Q_A != Q_B
    c["B"] = (c["B"].astype(np.int64) * 4 // 3).astype(np.uint8)
    _check(cm, torch, oracle, c, 3, 4, precision, "small masked")


def test_volume_planted_shift(gpu, oracle):
    cm, torch = gpu
    c = synth.volume_pair(32, (40, 36, 44), (30, 40, 34), 4, (3, -5, 7))
    r = _check(cm, torch, oracle, c, 4, 4, "fp32", "planted")
    b = r["best"]
    assert (b["dz"], b["dy"], b["dx"]) == c["chi"]


def test_volume_depth_one_is_the_2d_map(gpu, oracle):
    cm, torch = gpu
    c = synth.random_case(33, 40, 50, 37, 45, 4, 5, mask_density=0.85)
    A, MA, B, MB = (c[k][None] for k in ("A", "MA", "B", "MB"))
    r3 = cm.compute_volume(dev(torch, A), dev(torch, MA), dev(torch, B),
                           dev(torch, MB), 4, 5, digest=True)
    plan = cm.Plan([(40, 50, 37, 45)], 4, 5)
    r2 = plan.compute(dev(torch, c["A"]), dev(torch, c["MA"]),
                      dev(torch, c["B"]), dev(torch, c["MB"]), mi=True, n=True,
                      digest=True)
    assert np.array_equal(r3["n"].cpu().numpy()[0], r2["n"][0][0].cpu().numpy())
    assert np.array_equal(r3["digest"].cpu().numpy(), r2["digest"][0][0].cpu().numpy())
    err = float(np.abs(r3["mi"].cpu().numpy()[0] - r2["mi"][0][0].cpu().numpy()).max())
    say(f"[gpu] depth-1 volume vs 2-D plan: max|dMI| {err:.2e}")
    assert err <= MI_TOL
