"""GPU: cmif_compute_noalloc (both workspaces in the library's own device
array, no allocation) against cmif_compute with caller workspaces, on two
calls in a row, the second with a smaller input: counts, N and digests
bit-exact, MI within 1e-12 (bitwise in practice: same kernels, same launch
shapes), same Alg. 1 results.  Also the host-side rejection of plans whose
workspace exceeds the array."""

import ctypes
import math

import numpy as np
import pytest

import synth
from gpu_common import MI_TOL, dev, say

pytestmark = pytest.mark.gpu


def _run(cm, torch, c, precision, angles, noalloc):
    A, MA, B, MB = c["A"], c["MA"], c["B"], c["MB"]
    plan = cm.Plan([(*A.shape, *B.shape)], c["qa"], c["qb"], angles=angles,
                   precision=precision)
    r = plan.compute(dev(torch, A), dev(torch, MA), dev(torch, B), dev(torch, MB),
                     mi=True, n=True, counts=True, digest=True, best=True,
                     per_angle=True, noalloc=noalloc)
    return dict(mi=r["mi"][0].cpu().numpy(), n=r["n"][0].cpu().numpy(),
                counts=r["counts"][0].cpu().numpy(),
                digest=r["digest"][0].cpu().numpy(), best=r["best"][0],
                per_angle=r["per_angle"][0], stats=r["stats"])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_matches_compute_two_calls(gpu, precision):
    cm, torch = gpu
    big = synth.random_case(9101, 100, 120, 110, 90, 6, 5, mask_density=0.85)
    small = synth.random_case(9102, 40, 52, 47, 38, 3, 4, mask_density=0.9)
    cases = ((big, [0.0, math.radians(17.0), math.radians(200.0)], "100x120/110x90"),
             (small, [0.0, math.radians(-40.0)], "40x52/47x38"))
    for c, angles, tag in cases:
        plan = cm.Plan([(*c["A"].shape, *c["B"].shape)], c["qa"], c["qb"],
                       angles=angles, precision=precision)
        need = plan.persistent_bytes + plan.scratch_bytes
        assert need <= cm.NOALLOC_BYTES, need
        del plan
        say(f"[gpu] cmif_compute_noalloc {tag} q=({c['qa']},{c['qb']}) "
            f"{precision} angles={len(angles)}")
        ref = _run(cm, torch, c, precision, angles, noalloc=False)
        got = _run(cm, torch, c, precision, angles, noalloc=True)
        assert np.array_equal(got["counts"], ref["counts"])
        assert np.array_equal(got["n"], ref["n"])
        assert np.array_equal(got["digest"], ref["digest"])
        err = float(np.abs(got["mi"] - ref["mi"]).max())
        bitwise = np.array_equal(got["mi"].view(np.uint64), ref["mi"].view(np.uint64))
        say(f"  max|dMI| {err:.3e} bitwise {bitwise}")
        assert err <= MI_TOL
        assert got["best"] == ref["best"]
        for a, b in zip(got["per_angle"], ref["per_angle"]):
            assert (a["dy"], a["dx"], a["n"]) == (b["dy"], b["dx"], b["n"])
            assert abs(a["mi"] - b["mi"]) <= MI_TOL
        for k in ("label_errors", "flagged_pairs", "fallback_pairs",
                  "fallback_overflow", "unresolved_pairs"):
            assert got["stats"][k] == ref["stats"][k], k


def test_noalloc_rejects_large_plans(gpu):
    cm, torch = gpu
    plan = cm.Plan([(1024, 1024, 1024, 1024)], 16, 16)
    need = plan.persistent_bytes + plan.scratch_bytes
    assert need > cm.NOALLOC_BYTES
    A = torch.zeros((1024, 1024), dtype=torch.uint8, device="cuda")
    with pytest.raises(cm.CmifError) as ei:
        plan.compute(A, None, A, None, mi=True, n=False, noalloc=True)
    assert ei.value.status == cm.CMIF_ERR_UNSUPPORTED
    say(f"[gpu] noalloc rejects a plan needing {need} bytes: {ei.value}")
