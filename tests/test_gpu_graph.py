"""GPU: launch sequences captured into HIP graphs and replayed.

A plan captures its launch sequence on the first call and replays it while
the pointers repeat.  Every replay must give what the eager schedule
(CMIF_FLAG_NO_GRAPH) gives, bitwise, with the inputs' contents changed in
place between replays and unrelated eager work (and synchronisations) in
between; new pointers capture again."""

import math

import numpy as np
import pytest

import synth
from gpu_common import dev, say

pytestmark = pytest.mark.gpu

NO_GRAPH = 1 << 1
FORCE = 1 << 0


def _fill(torch, dst, arr):
    dst.copy_(torch.from_numpy(np.ascontiguousarray(arr)).cuda())


def _eager_noise(torch):
    x = torch.randn(1 << 16, device="cuda")
    y = (x * 3.0).cumsum(0).sum()
    torch.cuda.synchronize()
    return float(y)


@pytest.mark.parametrize("flags,prec", [(0, "fp32"), (FORCE, "fp32"),
                                        (0, "fp64")],
                         ids=["fp32", "fp32-forced-rerun", "fp64"])
def test_compute_replays_match_eager(gpu, oracle, flags, prec):
    cm, torch = gpu
    ha, wa, hb, wb, qa, qb = 45, 50, 39, 44, 4, 5
    angles = [0.0, math.radians(30.0), math.radians(200.0)]
    pg = cm.Plan([(ha, wa, hb, wb)], qa, qb, angles=angles, precision=prec,
                 flags=flags)
    pe = cm.Plan([(ha, wa, hb, wb)], qa, qb, angles=angles, precision=prec,
                 flags=flags | NO_GRAPH)
    A = torch.empty((ha, wa), dtype=torch.uint8, device="cuda")
    MA = torch.empty_like(A)
    B = torch.empty((hb, wb), dtype=torch.uint8, device="cuda")
    MB = torch.empty_like(B)
    for rep in range(4):
        c = synth.random_case(500 + rep, ha, wa, hb, wb, qa, qb, mask_density=0.8)
        for t, k in ((A, "A"), (MA, "MA"), (B, "B"), (MB, "MB")):
            _fill(torch, t, c[k])
        say(f"[gpu] graph replay {rep} {prec} flags={flags}")
        rg = pg.compute(A, MA, B, MB, mi=True, n=True, counts=True, digest=True,
                        best=True, per_angle=True, reuse=True)
        _eager_noise(torch)
        re = pe.compute(A, MA, B, MB, mi=True, n=True, counts=True, digest=True,
                        best=True, per_angle=True)
        for name in ("mi", "n", "counts", "digest"):
            g = rg[name][0].cpu().numpy()
            e = re[name][0].cpu().numpy()
            assert np.array_equal(g.view(np.uint8), e.view(np.uint8)), (rep, name)
        assert rg["best"] == re["best"]
        assert rg["per_angle"] == re["per_angle"]
        assert rg["stats"] == re["stats"]
        bw, mw = oracle.warp_nn(c["B"], c["MB"], angles[1])
        o = oracle.cmif_direct(c["A"], c["MA"], bw, mw, qa, qb, counts=True)
        assert np.array_equal(rg["counts"][0][1].cpu().numpy(), o["counts"])
    info = pg.info()
    say(f"graph info {info}")
    assert info["graph_captures"] == 1 and info["graph_replays"] == 3


def test_align_replays_and_recapture(gpu, oracle):
    cm, torch = gpu
    c = synth.config3(n_angles=10, size=96, q=8)
    angles = [math.radians(36.0 * i) for i in range(10)]
    ins = [dev(torch, c[k]) for k in ("A", "MA", "B", "MB")]
    pg = cm.Plan([(96, 96, 96, 96)], 8, 8, angles=angles, angle_batch=3)
    pe = cm.Plan([(96, 96, 96, 96)], 8, 8, angles=angles, angle_batch=3,
                 flags=NO_GRAPH)
    ref = pe.align(*ins, per_angle=True)
    for rep in range(3):
        say(f"[gpu] align replay {rep}")
        r = pg.align(*ins, per_angle=True)
        _eager_noise(torch)
        assert r["best"] == ref["best"] and r["per_angle"] == ref["per_angle"]
    assert pg.info()["graph_replays"] == 2
    # new input pointers: captured again, same result
    ins2 = [t.clone() for t in ins]
    r2 = pg.align(*ins2, per_angle=True)
    assert r2["best"] == ref["best"]
    assert pg.info()["graph_captures"] == 2
    o = oracle.align(c["A"], c["MA"], c["B"], c["MB"], 8, 8, angles, 0.5)
    assert abs(r2["best"][0]["mi"] - o["mi"]) <= 1e-12


def test_soft_compute_replays(gpu):
    cm, torch = gpu
    c = synth.random_soft_case(77, 40, 44, 38, 35, 3, qb=4, mask_density=0.9)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    A, B = f32(c["PA"]), f32(c["PB"])
    MA, MB = dev(torch, c["MA"]), dev(torch, c["MB"])
    pg = cm.Plan([(40, 44, 38, 35)], 3, 4, mode="soft")
    pe = cm.Plan([(40, 44, 38, 35)], 3, 4, mode="soft", flags=NO_GRAPH)
    e = pe.compute(A, MA, B, MB, mi=True, n=True, best=True)
    for rep in range(3):
        g = pg.compute(A, MA, B, MB, mi=True, n=True, best=True, reuse=True)
        _eager_noise(torch)
        assert np.array_equal(g["mi"][0].cpu().numpy().view(np.uint64),
                              e["mi"][0].cpu().numpy().view(np.uint64))
        assert np.array_equal(g["n"][0].cpu().numpy(), e["n"][0].cpu().numpy())
        assert g["best"] == e["best"]
    assert pg.info()["graph_replays"] == 2
