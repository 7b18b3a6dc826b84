"""Host-side checks of the C ABI: the library loads, exports every function
the header declares, the ctypes mirrors match the C struct layouts, and the
plan/argument validation rejects bad input before any device work.  None of
these needs a GPU (cmif_plan is host-only)."""

import ctypes
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cmif.h")


@pytest.fixture(scope="module")
def cm():
    import paper_2106_14699_amd as cm
    return cm


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cmif_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(cm):
    names = header_functions()
    assert set(names) == set(cm.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", cm.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    for n in names:
        assert n in exported, n
        assert hasattr(cm._lib, n)


def test_struct_layouts_match_header(cm, tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "cmif.h"
#define P(s, f) printf(#s "." #f " %zu\n", offsetof(s, f))
int main(void) {
  printf("desc %zu\n", sizeof(cmif_plan_desc));
  printf("stats %zu\n", sizeof(cmif_stats));
  printf("best %zu\n", sizeof(cmif_best));
  printf("inputs %zu\n", sizeof(cmif_inputs));
  printf("outputs %zu\n", sizeof(cmif_outputs));
  P(cmif_plan_desc, gamma); P(cmif_plan_desc, angle_batch);
  P(cmif_plan_desc, angles_rad); P(cmif_best, angle_rad); P(cmif_best, n);
  P(cmif_stats, max_residual); P(cmif_outputs, stats);
  printf("vdesc %zu\n", sizeof(cmif_volume_desc));
  printf("best3d %zu\n", sizeof(cmif_best3d));
  P(cmif_volume_desc, gamma); P(cmif_volume_desc, device);
  P(cmif_best3d, mi); P(cmif_best3d, n);
  printf("info %zu\n", sizeof(cmif_plan_info));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog),
                    "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run(
        [str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
        if l)
    assert int(got["desc"]) == ctypes.sizeof(cm.cmif_plan_desc)
    assert int(got["stats"]) == ctypes.sizeof(cm.cmif_stats)
    assert int(got["best"]) == ctypes.sizeof(cm.cmif_best)
    assert int(got["inputs"]) == ctypes.sizeof(cm.cmif_inputs)
    assert int(got["outputs"]) == ctypes.sizeof(cm.cmif_outputs)
    assert int(got["cmif_plan_desc.gamma"]) == cm.cmif_plan_desc.gamma.offset
    assert int(got["cmif_plan_desc.angle_batch"]) == cm.cmif_plan_desc.angle_batch.offset
    assert int(got["cmif_plan_desc.angles_rad"]) == cm.cmif_plan_desc.angles_rad.offset
    assert int(got["cmif_best.angle_rad"]) == cm.cmif_best.angle_rad.offset
    assert int(got["cmif_best.n"]) == cm.cmif_best.n.offset
    assert int(got["cmif_stats.max_residual"]) == cm.cmif_stats.max_residual.offset
    assert int(got["cmif_outputs.stats"]) == cm.cmif_outputs.stats.offset
    assert int(got["vdesc"]) == ctypes.sizeof(cm.cmif_volume_desc)
    assert int(got["best3d"]) == ctypes.sizeof(cm.cmif_best3d)
    assert int(got["info"]) == ctypes.sizeof(cm.cmif_plan_info)
    for st, f in (("cmif_volume_desc", "gamma"), ("cmif_volume_desc", "device"),
                  ("cmif_best3d", "mi"), ("cmif_best3d", "n")):
        assert int(got[f"{st}.{f}"]) == getattr(getattr(cm, st), f).offset


def make_desc(cm, sizes=((64, 64, 64, 64),), qa=4, qb=4, angles=(0.0,),
              gamma=0.5, precision=0, mode=0, flags=0):
    n = len(sizes)
    arrs = [(ctypes.c_int32 * n)(*[s[k] for s in sizes]) for k in range(4)]
    ang = (ctypes.c_double * max(len(angles), 1))(*angles) if angles else None
    d = cm.cmif_plan_desc()
    d.n_pairs = n
    d.h_a, d.w_a, d.h_b, d.w_b = [ctypes.cast(a, ctypes.POINTER(ctypes.c_int32))
                                  for a in arrs]
    d.q_a, d.q_b = qa, qb
    d.n_angles = len(angles) if angles else 1
    d.angles_rad = ctypes.cast(ang, ctypes.POINTER(ctypes.c_double)) if ang else None
    d.gamma = gamma
    d.precision, d.mode, d.flags = precision, mode, flags
    d._keep = (arrs, ang)
    return d


def plan_status(cm, d):
    h = ctypes.c_void_p()
    s = cm._lib.cmif_plan(ctypes.byref(d), ctypes.byref(h))
    if s == 0:
        cm.cmif_plan_free(h.value)
    return s


@pytest.mark.parametrize("field,value,expect", [
    ("q_a", 0, 1), ("q_a", 65, 1), ("q_b", 0, 1), ("gamma", -0.1, 1),
    ("gamma", 1.5, 1), ("gamma", float("nan"), 1), ("precision", 7, 1),
    ("mode", 3, 1), ("flags", 1 << 20, 1), ("n_pairs", 0, 1),
    ("n_angles", 0, 1), ("angle_batch", -1, 1), ("fallback_capacity", -1, 1),
    ("fallback_capacity", 4097, 1),
])
def test_plan_rejects_bad_fields(cm, field, value, expect):
    d = make_desc(cm)
    setattr(d, field, value)
    assert plan_status(cm, d) == expect


def test_plan_rejects_bad_sizes_and_pointers(cm):
    assert plan_status(cm, make_desc(cm, sizes=((0, 5, 5, 5),))) == 1
    assert plan_status(cm, make_desc(cm, sizes=((5, 5, 4097, 5),))) == 1
    # sides up to 4096 are valid, but the full set of two such images needs
    # a transform above 4096: unsupported without a window
    assert plan_status(cm, make_desc(cm, sizes=((5, 5, 1025, 5),))) == 0
    assert plan_status(cm, make_desc(cm, sizes=((1500, 5, 1025, 5),))) == 0
    assert plan_status(cm, make_desc(cm, sizes=((2100, 5, 2100, 5),))) == 2
    # 4096-point transforms: FP32-rounded HARD plans of the fused schedule
    # only (FP64 precision, SOFT mode and the plain schedule: unsupported)
    big = ((1500, 5, 1025, 5),)
    assert plan_status(cm, make_desc(cm, sizes=big, precision=1)) == 2
    assert plan_status(cm, make_desc(cm, sizes=big, mode=1)) == 2
    assert plan_status(cm, make_desc(cm, sizes=big, precision=1,
                                     flags=cm.CMIF_FLAG_PLAIN_SCHEDULE)) == 2
    assert plan_status(cm, make_desc(cm, sizes=((1000, 5, 1025, 5),), precision=1)) == 0
    d = make_desc(cm)
    d.h_a = None
    assert plan_status(cm, d) == 1
    d = make_desc(cm, angles=(0.0, 1.0))
    d.angles_rad = None
    assert plan_status(cm, d) == 1
    d = make_desc(cm, angles=(float("inf"),))
    assert plan_status(cm, d) == 1
    h = ctypes.c_void_p()
    assert cm._lib.cmif_plan(None, ctypes.byref(h)) == 1
    assert cm._lib.cmif_plan(ctypes.byref(make_desc(cm)), None) == 1


def test_plan_and_workspace_sizes(cm):
    d = make_desc(cm, sizes=((512, 512, 512, 512),), qa=16, qb=16,
                  angles=tuple(math.radians(2 * i) for i in range(180)))
    h = cm.cmif_plan(d)
    try:
        p, s = cm.cmif_workspace_size(h)
        assert p > 0 and s > 0 and p % 256 == 0
        # Z of at least one angle: 256 pairs x 512 columns x 1023 rows x 8 B
        assert s >= 256 * 512 * 1023 * 8
    finally:
        cm.cmif_plan_free(h)
    dd = make_desc(cm, sizes=((64, 64, 64, 64), (30, 40, 20, 70)), qa=3, qb=5)
    h = cm.cmif_plan(dd)
    try:
        assert cm.cmif_workspace_size(h)[1] > 0
    finally:
        cm.cmif_plan_free(h)


def test_calls_validate_before_device_work(cm):
    h = cm.cmif_plan(make_desc(cm))
    try:
        p, s = cm.cmif_workspace_size(h)
        inp = cm.cmif_inputs()
        out = cm.cmif_outputs()
        lib = cm._lib
        # workspace too small is caught on the host
        assert lib.cmif_compute(ctypes.c_void_p(h), ctypes.byref(inp),
                                ctypes.byref(out), None, 0, None, 0,
                                None) == cm.CMIF_ERR_WORKSPACE_TOO_SMALL
        # NULL inputs
        assert lib.cmif_compute(ctypes.c_void_p(h), None, ctypes.byref(out),
                                None, p, None, s, None) == 1
        # NULL workspace with sufficient sizes
        assert lib.cmif_compute(ctypes.c_void_p(h), ctypes.byref(inp),
                                ctypes.byref(out), None, p, None, s,
                                None) == 1
        # misaligned workspace
        assert lib.cmif_align(ctypes.c_void_p(h), ctypes.byref(inp),
                              ctypes.c_void_p(256), None, None,
                              ctypes.c_void_p(8), p, ctypes.c_void_p(256), s,
                              None) == 1
        # NULL best for align
        assert lib.cmif_align(ctypes.c_void_p(h), ctypes.byref(inp), None,
                              None, None, ctypes.c_void_p(256), p,
                              ctypes.c_void_p(512), s, None) == 1
        # backward on a HARD plan
        assert lib.cmif_backward(ctypes.c_void_p(h), ctypes.byref(inp), None,
                                 None, None, None, p, None, s,
                                 None) == cm.CMIF_ERR_WRONG_MODE
        assert cm.cmif_last_error() != ""
        assert lib.cmif_workspace_size(None, None, None) == 1
    finally:
        cm.cmif_plan_free(h)
    cm.cmif_plan_free(0)  # NULL is ignored


def test_soft_plans(cm):
    save = cm.CMIF_FLAG_SAVE_FOR_BACKWARD
    d = make_desc(cm, sizes=((40, 36, 33, 45),), qa=3, qb=4)
    d.mode = cm.CMIF_MODE_SOFT
    assert plan_status(cm, d) == 0
    # the adjoint takes the single angle 0 only
    d = make_desc(cm, angles=(0.0, 0.5))
    d.mode, d.flags = cm.CMIF_MODE_SOFT, save
    assert plan_status(cm, d) == cm.CMIF_ERR_UNSUPPORTED
    d = make_desc(cm, angles=(0.25,))
    d.mode, d.flags = cm.CMIF_MODE_SOFT, save
    assert plan_status(cm, d) == cm.CMIF_ERR_UNSUPPORTED
    # saved state lives in the persistent workspace:
    # (q_a + q_b + 2) float planes of the 72 x 80 map
    sizes = ((40, 36, 33, 45),)
    d0 = make_desc(cm, sizes=sizes, qa=3, qb=4)
    d0.mode = cm.CMIF_MODE_SOFT
    d1 = make_desc(cm, sizes=sizes, qa=3, qb=4)
    d1.mode, d1.flags = cm.CMIF_MODE_SOFT, save
    h0, h1 = cm.cmif_plan(d0), cm.cmif_plan(d1)
    try:
        p0, s0 = cm.cmif_workspace_size(h0)
        p1, s1 = cm.cmif_workspace_size(h1)
        assert p1 - p0 >= (3 + 4 + 2) * 72 * 80 * 4
        lib = cm._lib
        inp = cm.cmif_inputs()
        # backward needs SAVE_FOR_BACKWARD; then NULL memberships are caught
        assert lib.cmif_backward(ctypes.c_void_p(h0), ctypes.byref(inp), None,
                                 None, None, None, p0, None, s0,
                                 None) == cm.CMIF_ERR_WRONG_MODE
        gm = (ctypes.c_void_p * 1)(None)
        assert lib.cmif_backward(ctypes.c_void_p(h1), ctypes.byref(inp),
                                 ctypes.cast(gm, cm._PP), None, None,
                                 ctypes.c_void_p(256), p1, ctypes.c_void_p(512),
                                 s1, None) == cm.CMIF_ERR_INVALID_ARGUMENT
        # compute on a SOFT plan without memberships
        out = cm.cmif_outputs()
        assert lib.cmif_compute(ctypes.c_void_p(h1), ctypes.byref(inp),
                                ctypes.byref(out), ctypes.c_void_p(256), p1,
                                ctypes.c_void_p(512), s1,
                                None) == cm.CMIF_ERR_INVALID_ARGUMENT
    finally:
        cm.cmif_plan_free(h0)
        cm.cmif_plan_free(h1)


def test_plain_schedule_plans(cm):
    plain = cm.CMIF_FLAG_PLAIN_SCHEDULE
    d = make_desc(cm)
    d.flags, d.precision = plain, cm.CMIF_PREC_FP64
    assert plan_status(cm, d) == 0
    d = make_desc(cm)
    d.flags, d.precision = plain, cm.CMIF_PREC_FP32_ROUNDED
    assert plan_status(cm, d) == cm.CMIF_ERR_UNSUPPORTED
    d = make_desc(cm)
    d.flags, d.precision, d.mode = plain, cm.CMIF_PREC_FP64, cm.CMIF_MODE_SOFT
    assert plan_status(cm, d) == cm.CMIF_ERR_UNSUPPORTED


def _tune_plan(cm, path, flags=None, mode=0):
    d = make_desc(cm, sizes=((64, 64, 64, 64),), qa=4, qb=4)
    d.flags = cm.CMIF_FLAG_AUTOTUNE if flags is None else flags
    d.mode = mode
    keep = path.encode() if path else None
    d.tune_cache_path = keep
    h = cm.cmif_plan(d)
    try:
        return cm.cmif_plan_query(h)
    finally:
        cm.cmif_plan_free(h)


def test_autotune_plan_and_cache_file(cm, tmp_path):
    # no file: default shapes, not yet tuned
    info = _tune_plan(cm, None)
    assert (info["tuned"], info["tune_runs"]) == (0, 0)
    # power-of-two column length (128): the XCD-grouped column order
    assert (info["rows_per_wg"], info["labels_per_team"], info["xcd_grouping"]) \
        == (1, 0, 1)
    assert (info["cols_half"], info["cols_maxr"], info["cols_ba"]) == (0, 16, 1)
    ph, pw = info["fft_h"], info["fft_w"]
    key = (f"cmif-tune v1 gfx950 {ph}x{pw}:127x127 qa=4 qb=4 prec=0 "
           f"batch={info['angle_batch']}")
    f = tmp_path / "tune.txt"
    # a missing file, then malformed or out-of-range lines, are ignored
    assert _tune_plan(cm, str(f))["tuned"] == 0
    f.write_text("garbage\n" + key + " rows_per_wg=9 bpw=4 xcd=0\n"
                 + key + " rows_per_wg=1 bpw=5 xcd=0\n"
                 + key.replace("qa=4", "qa=3") + " rows_per_wg=4 bpw=8 xcd=0\n")
    assert _tune_plan(cm, str(f))["tuned"] == 0
    # a matching line is taken at plan time (no timing on the first call)
    f.write_text(f.read_text() + key + " rows_per_wg=4 bpw=8 xcd=0\n")
    info = _tune_plan(cm, str(f))
    assert info["tuned"] == 2 and info["tune_runs"] == 0
    assert (info["rows_per_wg"], info["labels_per_team"], info["xcd_grouping"]) \
        == (4, 8, 0)
    # the column-pass fields of the current format
    f.write_text(key + " rows_per_wg=2 bpw=0 xcd=1 half=1 maxr=8 ba=2\n")
    info = _tune_plan(cm, str(f))
    assert info["tuned"] == 2 and (info["rows_per_wg"], info["xcd_grouping"]) == (2, 1)
    assert (info["cols_half"], info["cols_maxr"], info["cols_ba"]) == (1, 8, 2)
    f.write_text(key + " rows_per_wg=2 bpw=0 xcd=1 half=1 maxr=12 ba=2\n")
    assert _tune_plan(cm, str(f))["tuned"] == 0
    f.write_text(f.read_text() + key + " rows_per_wg=4 bpw=8 xcd=0\n")
    # without the flag, or for SOFT, the file is not consulted
    assert _tune_plan(cm, str(f), flags=0)["tuned"] == 0
    assert _tune_plan(cm, str(f), mode=cm.CMIF_MODE_SOFT)["tuned"] == 0


def _window_desc(cm, sizes, windows, **kw):
    d = make_desc(cm, sizes=sizes, **kw)
    if windows is not None:
        arr = (ctypes.c_int32 * (4 * len(windows)))(*[v for w in windows for v in w])
        d.window = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
        d._keep = (d._keep, arr)
    return d


def _fft_sides(cm, d):
    h = cm.cmif_plan(d)
    try:
        info = cm.cmif_plan_query(h)
        return (info["fft_h"], info["fft_w"]), cm.cmif_workspace_size(h)[1]
    finally:
        cm.cmif_plan_free(h)


@pytest.mark.parametrize("side,fft", [(64, 128), (65, 256), (129, 512),
                                      (257, 768), (385, 1024), (513, 1536),
                                      (769, 2048), (1024, 2048), (1025, 4096),
                                      (2048, 4096)])
def test_fft_side_rule(cm, side, fft):
    """FFT side per axis: the smallest of 128, 256, 512, 768, 1024, 1536,
    2048, 4096 that reaches h_a + h_b - 1 (alias-free circular correlation)."""
    d = make_desc(cm, sizes=((side, side, side, side),))
    assert _fft_sides(cm, d)[0] == (fft, fft)
    # one more row or column moves to the next length exactly at the boundary
    s = 2 * side - 1
    d = make_desc(cm, sizes=((side, 1, side, 1),))
    assert _fft_sides(cm, d)[0][0] == fft and fft >= s


def test_window_validation_and_fft_sides(cm):
    s = ((400, 400, 400, 400),)
    # full set: 799 -> 1024; +-100 needs max(100 + 400, 400 + 100) -> 512
    full, scr_full = _fft_sides(cm, _window_desc(cm, s, None))
    assert full == (1024, 1024)
    win, scr_win = _fft_sides(cm, _window_desc(cm, s, [(-100, 100, -100, 100)]))
    assert win == (512, 512) and scr_win < scr_full
    # one displacement at 0 needs only max(h_a, h_b)
    assert _fft_sides(cm, _window_desc(cm, s, [(0, 0, 0, 0)]))[0] == (512, 512)
    # a window on one side only: max(300 + 400, 400 - 10) -> 768 rows
    # (3 * 2^8, the smallest compiled length >= 700)
    assert _fft_sides(cm, _window_desc(cm, s, [(10, 300, -5, 5)]))[0] == (768, 512)
    # windows on one side of 0 with unequal sides: the transform still
    # holds both images (500 + 1 and 1000 - 500 alone would give 512)
    assert _fft_sides(cm, _window_desc(cm, ((1, 1, 1000, 1000),),
                                       [(500, 500, 500, 500)]))[0] == (1024, 1024)
    assert _fft_sides(cm, _window_desc(cm, ((1000, 1000, 1, 1),),
                                       [(-500, -500, -500, -500)]))[0] == (1024, 1024)
    # the full set written out is the same plan as NULL
    assert _fft_sides(cm, _window_desc(cm, s, [(-399, 399, -399, 399)]))[0] == full
    for bad in [(5, 4, 0, 0), (0, 0, 3, 2), (-400, 0, 0, 0), (0, 400, 0, 0),
                (0, 0, -400, 0), (0, 0, 0, 400)]:
        assert plan_status(cm, _window_desc(cm, s, [bad])) == cm.CMIF_ERR_INVALID_ARGUMENT, bad
    # SOFT and the plain schedule take the full set only
    d = _window_desc(cm, ((64, 64, 64, 64),), [(-3, 3, -3, 3)])
    d.mode = cm.CMIF_MODE_SOFT
    assert plan_status(cm, d) == cm.CMIF_ERR_UNSUPPORTED
    d = _window_desc(cm, ((64, 64, 64, 64),), [(-3, 3, -3, 3)])
    d.precision, d.flags = cm.CMIF_PREC_FP64, cm.CMIF_FLAG_PLAIN_SCHEDULE
    assert plan_status(cm, d) == cm.CMIF_ERR_UNSUPPORTED


def test_kmeans_validates_before_device_work(cm):
    lib = cm._lib
    P = 0x1000  # never dereferenced: every call below fails validation
    E = cm.CMIF_ERR_INVALID_ARGUMENT
    ok = dict(image=P, mask=None, n=100, m=1, k=4, init=P, batches=P, iters=5,
              batch=10, centers=P, labels=P, bad=None, stream=None)
    def call(**kw):
        d = dict(ok, **kw)
        return lib.cmif_kmeans(d["image"], d["mask"], d["n"], d["m"], d["k"],
                               d["init"], d["batches"], d["iters"], d["batch"],
                               d["centers"], d["labels"], d["bad"], d["stream"])
    for bad in [dict(image=None), dict(centers=None), dict(labels=None),
                dict(n=0), dict(k=0), dict(k=65), dict(m=0), dict(m=9),
                dict(iters=-1), dict(iters=100001), dict(batches=None),
                dict(batch=0), dict(batch=8193)]:
        assert call(**bad) == E, bad


def test_status_strings(cm):
    seen = set()
    for s in range(8):
        t = cm.cmif_status_string(s)
        assert t and t not in seen
        seen.add(t)
    assert cm.cmif_status_string(99) == "unknown status"


def test_volume_workspace_size_validation(cm):
    d = cm.volume_desc((12, 14, 10), (9, 11, 13), 3, 4)
    assert cm.cmif_volume_workspace_size(d) > 0
    # depth transform above 512 points, in-plane above 2048
    for shape_b, status in (((600, 11, 13), cm.CMIF_ERR_UNSUPPORTED),
                            ((9, 2040, 13), cm.CMIF_ERR_UNSUPPORTED),
                            ((0, 11, 13), cm.CMIF_ERR_INVALID_ARGUMENT)):
        with pytest.raises(cm.CmifError) as ei:
            cm.cmif_volume_workspace_size(cm.volume_desc((12, 14, 10), shape_b, 3, 4))
        assert ei.value.status == status
    for q in (0, 65):
        with pytest.raises(cm.CmifError):
            cm.cmif_volume_workspace_size(cm.volume_desc((4, 4, 4), (4, 4, 4), q, 2))
    d = cm.volume_desc((4, 4, 4), (4, 4, 4), 2, 2)
    d.gamma = 1.5
    with pytest.raises(cm.CmifError):
        cm.cmif_volume_workspace_size(d)
