"""GPU: the launch-shape autotuner (CMIF_FLAG_AUTOTUNE).

The first call of a tuned plan times every candidate shape of the pair row
and column kernels on its own buffers, keeps the fastest, and writes the
choice to the cache file; a second plan with the same file reads it at plan
time and times nothing.  Counts, digests and N must match the default
shapes bit for bit, MI to the summation-order tolerance, and the oracle at
sampled displacements of one angle."""

import math

import numpy as np
import pytest

import synth
from gpu_common import MI_TOL, dev, say

pytestmark = pytest.mark.gpu

FORCE = 1 << 0
AUTOTUNE = 1 << 4


def _run(plan, ins):
    return plan.compute(*ins, mi=True, n=True, counts=True, digest=True,
                        best=True, per_angle=True)


def _same(r, ref):
    for name in ("n", "counts", "digest"):
        g = r[name][0].cpu().numpy()
        e = ref[name][0].cpu().numpy()
        assert np.array_equal(g.view(np.uint8), e.view(np.uint8)), name
    err = np.abs(r["mi"][0].cpu().numpy() - ref["mi"][0].cpu().numpy()).max()
    assert err <= MI_TOL, err
    return err


@pytest.mark.parametrize("size,q,prec,flags", [
    ((100, 90, 80, 110), (4, 12), "fp32", 0),
    ((100, 90, 80, 110), (4, 12), "fp32", FORCE),
    ((300, 260, 280, 310), (8, 8), "fp32", 0),
    ((160, 150, 170, 140), (6, 5), "fp64", 0),
    # 4096-point rows (two workgroups per map row): every row shape the
    # tuner times, the spilling 1024-lane one included, must agree too
    ((40, 1100, 36, 1000), (4, 5), "fp32", 0),
], ids=["fp32-q4x12", "fp32-forced-rerun", "fp32-p768", "fp64", "fp32-rows4096"])
def test_tuned_plan_matches_default(gpu, oracle, tmp_path, size, q, prec, flags):
    cm, torch = gpu
    ha, wa, hb, wb = size
    qa, qb = q
    angles = [0.0, math.radians(40.0), math.radians(250.0)]
    c = synth.random_case(710 + qa, ha, wa, hb, wb, qa, qb, mask_density=0.8)
    ins = [dev(torch, c[k]) for k in ("A", "MA", "B", "MB")]
    cache = str(tmp_path / "tune.txt")
    say(f"[gpu] autotune {size} q={q} {prec} flags={flags}")
    base = cm.Plan([size], qa, qb, angles=angles, precision=prec, flags=flags)
    ref = _run(base, ins)
    tuned = cm.Plan([size], qa, qb, angles=angles, precision=prec,
                    flags=flags | AUTOTUNE, tune_cache_path=cache)
    assert tuned.info()["tuned"] == 0
    r1 = _run(tuned, ins)
    info = tuned.info()
    say(f"tuned info {info}")
    assert info["tuned"] == 1 and info["tune_runs"] >= 3
    assert info["rows_per_wg"] in (1, 2, 4)
    assert info["labels_per_team"] in (0, 4, 8, 16)
    assert info["xcd_grouping"] in (0, 1)
    err = _same(r1, ref)
    assert r1["best"] == ref["best"] or err > 0.0
    # later calls (graph capture, then replay) with the chosen shapes
    for _ in range(2):
        _same(_run(tuned, ins), ref)
    assert tuned.info()["tune_runs"] == info["tune_runs"]
    # the cache file now holds the choice; a new plan times nothing
    again = cm.Plan([size], qa, qb, angles=angles, precision=prec,
                    flags=flags | AUTOTUNE, tune_cache_path=cache)
    i2 = again.info()
    assert i2["tuned"] == 2 and i2["tune_runs"] == 0
    assert (i2["rows_per_wg"], i2["labels_per_team"], i2["xcd_grouping"]) == \
        (info["rows_per_wg"], info["labels_per_team"], info["xcd_grouping"])
    r2 = _run(again, ins)
    assert again.info()["tune_runs"] == 0
    _same(r2, ref)
    # sampled displacements of one angle against the oracle
    bw, mw = oracle.warp_nn(c["B"], c["MB"], angles[1])
    mi = r2["mi"][0][1].cpu().numpy()
    n = r2["n"][0][1].cpu().numpy()
    cnt = r2["counts"][0][1].cpu().numpy()
    rng = np.random.default_rng(3)
    sh, sw = mi.shape
    for _ in range(24):
        i, j = int(rng.integers(sh)), int(rng.integers(sw))
        mo, no, jo = oracle.cmif_at(c["A"], c["MA"], bw, mw, qa, qb,
                                    i - (ha - 1), j - (wa - 1))
        assert n[i, j] == no and np.array_equal(cnt[:, :, i, j], jo), (i, j)
        assert abs(mi[i, j] - mo) <= MI_TOL, (i, j)


@pytest.mark.parametrize("size,qa,qb", [((400, 400, 400, 400), 4, 4),
                                        ((300, 260, 280, 310), 4, 4),
                                        ((400, 400, 400, 400), 3, 5)],
                         ids=["fft1024", "fft768", "fft1024-q3x5"])
def test_every_column_shape_matches_default(gpu, tmp_path, size, qa, qb):
    """Each FP32 column-pass shape (launch or XCD-grouped workgroup order,
    the latter with each workgroup's labels b rotated x half or whole tile of
    columns per workgroup x radix cap 16 or 8 x one or two labels of A per
    workgroup), forced through the tune cache, gives the default shape's
    counts, N and digests bit for bit and the same MI bitwise (the row pass
    sums the same integers in the same order).  An odd Q_B makes the rotated
    label order wrap at an odd length."""
    import itertools
    cm, torch = gpu
    ha, wa, hb, wb = size
    angles = [0.0, math.radians(70.0)]
    c = synth.random_case(7300 + ha + qb, ha, wa, hb, wb, qa, qb, mask_density=0.8)
    ins = [dev(torch, c[k]) for k in ("A", "MA", "B", "MB")]
    base = cm.Plan([size], qa, qb, angles=angles)
    ref = _run(base, ins)
    info = base.info()
    sh, sw = ha + hb - 1, wa + wb - 1
    key = (f"cmif-tune v1 gfx950 {info['fft_h']}x{info['fft_w']}:{sh}x{sw} "
           f"qa={qa} qb={qb} prec=0 batch={info['angle_batch']}")
    for xcd, half, maxr, ba in itertools.product((0, 1), (0, 1), (16, 8), (1, 2)):
        f = tmp_path / f"tune_{xcd}_{half}_{maxr}_{ba}.txt"
        f.write_text(f"{key} rows_per_wg=1 bpw=0 xcd={xcd} half={half} maxr={maxr} "
                     f"ba={ba}\n")
        plan = cm.Plan([size], qa, qb, angles=angles, flags=AUTOTUNE,
                       tune_cache_path=str(f))
        pi = plan.info()
        assert pi["tuned"] == 2
        assert (pi["xcd_grouping"], pi["cols_half"], pi["cols_maxr"],
                pi["cols_ba"]) == (xcd, half, maxr, ba)
        say(f"[gpu] column shape xcd={xcd} half={half} maxr={maxr} ba={ba} {size}")
        r = _run(plan, ins)
        for name in ("n", "counts", "digest"):
            g = r[name][0].cpu().numpy()
            e = ref[name][0].cpu().numpy()
            assert np.array_equal(g.view(np.uint8), e.view(np.uint8)), name
        assert np.array_equal(r["mi"][0].cpu().numpy().view(np.uint64),
                              ref["mi"][0].cpu().numpy().view(np.uint64))
