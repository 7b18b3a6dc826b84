#!/usr/bin/env python3
"""Throughput of the CMIF rotation-sweep alignment on one MI355X.

Workload: A, B 512x512 uint8 labels, Q_A = Q_B = 16 (256 label pairs), B a
rotated and moved copy of A's field through a non-monotone relabelling, 180
angles at 2 degree steps, gamma = 0.5; every angle's full 1023x1023 CMIF map
is computed (FP32 FFTs, counts rounded to integers, FP64 entropy sums) and the
Alg. 1 argmax is taken over displacements and angles.  One step = one
cmif_align call over all 180 angles; value = CMIF maps per second (180 maps
per step).

The JSON line also carries:
  roofline      the dominant kernel's algorithmic bytes per launch divided by
                its mean launch time (HIP events on the library's stream,
                recorded inside the timed steps), against 8 TB/s HBM;
                traffic = measured HBM bytes per launch from the rocprofv3
                counter summary in profiles/ when its source hash matches;
  cpu_baseline  the CPU oracle (direct method) on a bounded sample: one
                angle's full map on all host threads;
  plain_fp64    the same alignment through the library's plain FP64
                schedule (paper-shaped: every level set, mask and
                correlation transformed on its own, materialised FP64 maps,
                a separate entropy kernel, host sync per angle) and the
                speed-up of the batched FP32 path over it;
  soft          the soft-membership batch (16 pairs, sides 128-384, Q 8):
                forward, logsumexp(MI/0.01) over eligible shifts and the
                library's backward, per step.

--copy-gib G adds a plain device copy of G GiB (three times) after the
measurement: rocprofv3 counter passes use it to calibrate FETCH_SIZE and
WRITE_SIZE against bytes known to move.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("CMIF maps/s at 512², 16×16 labels; batched-FP32 vs "
          "plain-FP64 speedup; HBM GB/s")
HBM_PEAK_GBS = 8000.0


def kernel_source_sha(path):
    h = hashlib.sha256()
    for p in sorted(path):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def hot_sources():
    c = os.path.join(ROOT, "paper_2106_14699_amd", "csrc")
    return [os.path.join(c, f) for f in ("k_rows.hip", "k_pair.hip",
                                         "fft_core.h", "entropy.h",
                                         "internal.h", "rows_common.h")]


def read_traffic(stage):
    """HBM bytes per launch of `stage` from the counter summary in profiles/,
    or None when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"{stage}_sweep512_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"source_sha:\s*([0-9a-f]+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_sha or not m_b or m_sha.group(1) != kernel_source_sha(hot_sources()):
        return None
    return float(m_b.group(1))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(c, np):
    """The oracle (direct method) on one angle's full map on all host
    threads, plus a one-thread rate measured on a 256x256 crop of the same
    pair and scaled to the full map by the pixel visits sum_chi N(chi) =
    |M_A| |M_B'| that the direct method makes."""
    import oracle
    nt = oracle.max_threads()
    B, MB = oracle.warp_nn(c["B"], c["MB"], c["angles"][0])
    t0 = time.perf_counter()
    oracle.cmif_direct(c["A"], c["MA"], B, MB, c["qa"], c["qb"])
    dt = time.perf_counter() - t0
    visits = float(c["MA"].astype(np.int64).sum()) * float(MB.astype(np.int64).sum())
    crop = (slice(128, 384), slice(128, 384))
    va = float(c["MA"][crop].astype(np.int64).sum()) * float(MB[crop].astype(np.int64).sum())
    t1 = time.perf_counter()
    oracle.cmif_direct(c["A"][crop], c["MA"][crop], B[crop], MB[crop], c["qa"],
                       c["qb"], nthreads=1)
    d1 = time.perf_counter() - t1
    one = va / d1
    return dict(value=1.0 / dt, unit="maps/s", cores=nt, kind="oracle",
                sample=f"1 of 180 angles (full {2 * 512 - 1}x{2 * 512 - 1} map,"
                       f" direct method, {visits:.3g} pixel visits) in "
                       f"{dt:.1f} s on {nt} threads",
                cpu_model=cpu_model(),
                visits_per_s=round(visits / dt, 1),
                one_thread=dict(value=round(one / visits, 6), unit="maps/s",
                                visits_per_s=round(one, 1),
                                sample="256x256 crops of A and the rotated B "
                                       f"({va:.3g} visits) in {d1:.1f} s on "
                                       "1 thread, scaled by visits"))


def soft_bench(cm, torch, np, synth, steps):
    """Soft batch: one step = forward MI maps of all 16 pairs, the loss
    sum_pairs logsumexp(MI/0.01 over eligible shifts) and its gradient
    w.r.t. every membership map through the library's adjoint."""
    cfg = synth.config5()
    pairs = cfg["pairs"]
    sizes = [(*p["MA"].shape, *p["MB"].shape) for p in pairs]
    plan = cm.Plan(sizes, cfg["q"], cfg["q"], mode="soft", precision="fp32",
                   flags=cm.CMIF_FLAG_SAVE_FOR_BACKWARD)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    u8 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.uint8)).cuda()
    A = [f32(p["PA"]) for p in pairs]
    B = [f32(p["PB"]) for p in pairs]
    MA = [u8(p["MA"]) for p in pairs]
    MB = [u8(p["MB"]) for p in pairs]
    # eligibility (gamma 0.5 of the mask overlap) does not depend on the
    # memberships: computed once
    n = plan.compute(A, MA, B, MB, mi=False, n=True)["n"]
    elig = [(nk[0] >= cfg["gamma"] * nk[0].max()) for nk in n]

    def step():
        mi = plan.compute(A, MA, B, MB, mi=True, n=False)["mi"]
        grads, loss = [], 0.0
        for k in range(len(pairs)):
            m = mi[k][0].detach().requires_grad_(True)
            lk = torch.logsumexp(m[elig[k]] / cfg["temperature"], dim=0)
            lk.backward()
            grads.append(m.grad[None])
            loss = loss + lk.detach()
        ga, gb = plan.backward(A, MA, B, MB, grads)
        return float(loss), ga, gb

    step()
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        t0 = time.perf_counter()
        loss, ga, gb = step()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    med = float(np.median(times))
    return dict(ms_per_step_median=round(med, 3), pairs=len(pairs),
                pairs_per_s=round(len(pairs) * 1000.0 / med, 2),
                sizes=sizes, loss=loss,
                note="wall time per forward + loss + backward step "
                     "(host syncs included)")


class OracleMap:
    """The oracle's full direct map of the 1024x1024 stress pair, computed
    on host threads in the background (the C oracle releases the GIL) while
    the GPU sections run."""

    def __init__(self, c, nthreads):
        import threading
        self.c = c
        self.nthreads = nthreads
        self.res = None
        self.err = None
        self.seconds = None
        self.t = threading.Thread(target=self._run, daemon=True)
        self.t.start()

    def _run(self):
        try:
            import oracle
            t0 = time.perf_counter()
            c = self.c
            self.res = oracle.cmif_direct(c["A"], c["MA"], c["B"], c["MB"],
                                          c["qa"], c["qb"], digest=True,
                                          nthreads=self.nthreads)
            self.seconds = time.perf_counter() - t0
        except Exception as e:  # reported in the bench line
            self.err = repr(e)

    def get(self):
        self.t.join()
        return self.res


def stress_bench(cm, torch, np, synth, dev, reps=3, omap=None):
    """1024x1024, Q 16, all-ones masks (joint counts up to 2^20), FFT 2048:
    the FP32-rounded path with its residual check and FP64 re-run against
    the full-FP64 path on the same GPU, and both against the oracle's full
    direct map (N, digests, max |dMI|).  Median of `reps` computes each
    (MI, N and digests emitted)."""
    print("[bench] precision stress 1024x1024", file=sys.stderr, flush=True)
    c = synth.config4() if omap is None else omap.c
    n = 1024
    ins = [dev(c[k]) for k in ("A", "MA", "B", "MB")]
    out = {}
    for prec in ("fp32", "fp64"):
        plan = cm.Plan([(n, n, n, n)], c["qa"], c["qb"], angles=c["angles"],
                       gamma=c["gamma"], precision=prec)
        res = plan.compute(*ins, mi=True, n=True, digest=True, best=True)
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            res = plan.compute(*ins, mi=True, n=True, digest=True, best=True)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        out[prec] = dict(ms=float(np.median(times)), res=res,
                         fft=plan.info()["fft_h"])
        del plan
    r32, r64 = out["fp32"]["res"], out["fp64"]["res"]
    dmi = float((r32["mi"][0] - r64["mi"][0]).abs().max())
    same_digests = bool(torch.equal(r32["digest"][0], r64["digest"][0]))
    st = r32["stats"]
    b32, b64 = r32["best"][0], r64["best"][0]
    vs_oracle = None
    if omap is not None:
        print("[bench] waiting for the oracle's 1024x1024 map", file=sys.stderr,
              flush=True)
        o = omap.get()
        if o is not None:
            n32 = r32["n"][0][0].cpu().numpy()
            vs_oracle = dict(
                max_abs_dmi_fp32=float(np.abs(r32["mi"][0][0].cpu().numpy() -
                                              o["mi"]).max()),
                max_abs_dmi_fp64=float(np.abs(r64["mi"][0][0].cpu().numpy() -
                                              o["mi"]).max()),
                n_equal=bool(np.array_equal(n32, o["n"])),
                digests_equal=bool(np.array_equal(
                    r32["digest"][0][0].cpu().numpy().view(np.uint64),
                    o["digest"])),
                oracle_s=round(omap.seconds, 1), oracle_threads=omap.nthreads)
        else:
            vs_oracle = dict(error=omap.err)
    return dict(workload="1024x1024 uint8, Q_A=Q_B=16, all-ones masks, one "
                         "angle, full 2047x2047 map",
                fft=out["fp32"]["fft"],
                fp32_rounded_ms=round(out["fp32"]["ms"], 3),
                fp64_ms=round(out["fp64"]["ms"], 3),
                speedup=round(out["fp64"]["ms"] / out["fp32"]["ms"], 3),
                max_residual=st["max_residual"],
                flagged_pairs=st["flagged_pairs"],
                fallback_pairs=st["fallback_pairs"],
                fallback_overflow=st["fallback_overflow"],
                unresolved_pairs=st["unresolved_pairs"],
                vs_oracle=vs_oracle,
                max_abs_dmi_vs_fp64=dmi, digests_equal=same_digests,
                same_best=(b32["dy"], b32["dx"]) == (b64["dy"], b64["dx"]),
                planted_shift=list(c["shift"]), best=[b32["dy"], b32["dx"]])


# The paper's Table 1 times (k = 16, 200 grid + 32 refinement angles), on
# its stated GPU and including k-means quantisation on the CPU.
PAPER_TABLE1_S = {300: 6.1, 834: 32.9}


def table1_context(cm, torch, np, synth, dev):
    """Alg. 1 end to end on intensity images shaped like the paper's
    alignment benchmark: both images quantised to 16 labels by the GPU
    mini-batch k-means (batch 1000, 25 iterations, as for the paper's
    Table 1), then the two-stage global alignment (200 equispaced grid
    angles in [-pi, pi), then 32 random angles around the best), FP32-rounded
    over the full displacement set.  Wall time of one run after a warm-up
    run (plans, workspaces and graphs included), next to the paper's time
    for the same k and angle counts."""
    out = []
    for n in (300, 834):
        print(f"[bench] Alg. 1 end to end {n}x{n}", file=sys.stderr, flush=True)
        c = synth.table1_intensities(n)
        A, B, MB = dev(c["A"]), dev(c["B"]), dev(c["MB"])
        grid = [-math.pi + 2.0 * math.pi * i / 200 for i in range(200)]

        def run(seed):
            rng = np.random.default_rng(seed)
            qa = cm.kmeans_quantize(A, 16, iters=25, batch=1000, rng=rng)
            qb = cm.kmeans_quantize(B, 16, iters=25, batch=1000, rng=rng, mask=MB)
            return cm.align_two_stage(qa["labels"], None, qb["labels"], MB,
                                      (n, n, n, n), 16, 16, grid, rng=rng)
        run(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = run(2)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        b = r["best"]
        cerr = cm.cmif_corner_error(b, (n, n, n, n), c["truth"])
        out.append(dict(image=[n, n], k=16, angles="200+32", wall_s=round(wall, 3),
                        corner_error_px=round(cerr, 3),
                        success=bool(cerr < 0.02 * n),
                        paper_s=PAPER_TABLE1_S[n],
                        paper_over_ours=round(PAPER_TABLE1_S[n] / wall, 1),
                        best=dict(angle_deg=round(math.degrees(b["angle_rad"]), 3),
                                  dy=b["dy"], dx=b["dx"], stage=r["stage"]),
                        truth=dict(angle_deg=round(c["theta_deg"], 3),
                                   shift=list(c["shift"]))))
    return dict(runs=out, note="context only: the paper's times are on its "
                "stated GPU (GTX 2080, 11 GB) with k-means on the CPU; ours "
                "start from FP32 intensity images already in HBM and include "
                "the GPU k-means")


def template_bench(cm, torch, np, synth, dev, reps=5):
    """The paper's run-time experiment shape: reference side 256 .. 4096,
    floating image half of it, the CMIF map over every placement of the
    floating image inside the reference (a displacement window; FFT side =
    the reference side), Q 16, FP32-rounded, one angle.  Median time per map
    (cmif_compute of MI and N) and the planted offset."""
    out = []
    for ref in (256, 512, 1024, 2048, 4096):
        print(f"[bench] template {ref}/{ref // 2}", file=sys.stderr, flush=True)
        c = synth.template_pair(ref)
        half = ref // 2
        w = c["window"]
        plan = cm.Plan([(ref, ref, half, half)], 16, 16, windows=[w])
        A, B = dev(c["A"]), dev(c["B"])
        res = plan.compute(A, None, B, None, mi=True, n=True, best=True,
                           reuse=True)
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            # plan-owned outputs: stable pointers replay the captured graph
            res = plan.compute(A, None, B, None, mi=True, n=True, best=True,
                               reuse=True)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        b = res["best"][0]
        row = dict(reference=ref, floating=half, map=[half + 1, half + 1],
                   fft=plan.info()["fft_h"], ms_per_map=round(float(np.median(times)), 3),
                   found=[-b["dy"], -b["dx"]], planted=list(c["offset"]))
        out.append(row)
        del plan
    return out


def volume_bench(cm, torch, np, synth, dev, reps=3):
    """3-D volumes (the nD case of the paper's discussion): two 64^3 label
    volumes, Q 8, the second moved by a planted displacement, FP32-rounded;
    the full 127^3 map (FFT 128 per axis) and Alg. 1 over it.  Median ms per
    map and the recovered displacement."""
    print("[bench] volumes 64^3", file=sys.stderr, flush=True)
    c = synth.volume_pair(2106, (64, 64, 64), (64, 64, 64), 8, (5, -9, 3))
    A, B = dev(c["A"]), dev(c["B"])
    r = cm.compute_volume(A, None, B, None, 8, 8, mi=True, n=True)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        r = cm.compute_volume(A, None, B, None, 8, 8, mi=True, n=True)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    b = r["best"]
    return dict(volumes=[[64, 64, 64], [64, 64, 64]], labels=[8, 8],
                map=list(r["mi"].shape), fft=[128, 128, 128],
                ms_per_map=round(float(np.median(times)), 3),
                found=[b["dz"], b["dy"], b["dx"]], planted=list(c["chi"]),
                max_residual=r["stats"]["max_residual"],
                note="wall time of one cmif_compute_volume call (eager "
                     "launches, workspace allocated per call)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain per-angle FP64 comparator")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-soft", action="store_true",
                    help="skip the soft-membership batch")
    ap.add_argument("--soft-steps", type=int, default=5)
    ap.add_argument("--no-template", action="store_true",
                    help="skip the template-matching maps")
    ap.add_argument("--no-table1", action="store_true",
                    help="skip the paper-shaped two-stage alignments")
    ap.add_argument("--no-stress", action="store_true",
                    help="skip the 1024x1024 precision-stress comparison")
    ap.add_argument("--no-window", action="store_true",
                    help="skip the windowed sweep (Alg. 1's padded window)")
    ap.add_argument("--no-volume", action="store_true",
                    help="skip the 3-D volume map")
    ap.add_argument("--copy-gib", type=float, default=0.0)
    ap.add_argument("--tune-cache", default=None,
                    help="text file of tuned launch shapes: read at plan time "
                         "when it holds this workload, written after tuning")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes instead of timing "
                         "the candidates in the warm-up call "
                         "(CMIF_FLAG_AUTOTUNE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not "
              "supported (the library runs on one GPU; sharding the angles "
              "across GPUs with one all-gather of the per-GPU best is not "
              "implemented)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2106_14699_amd as cm
    import synth

    torch.cuda.set_device(0)
    c = synth.config3()
    n = 512
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    A, MA, B, MB = dev(c["A"]), dev(c["MA"]), dev(c["B"]), dev(c["MB"])
    plan = cm.Plan([(n, n, n, n)], c["qa"], c["qb"], angles=c["angles"],
                   gamma=c["gamma"], precision="fp32",
                   flags=0 if args.no_autotune else cm.CMIF_FLAG_AUTOTUNE,
                   tune_cache_path=args.tune_cache)
    n_maps = len(c["angles"])

    # warm-up: the first call captures the launch graph the timed steps replay
    plan.align(A, MA, B, MB)
    for _ in range(max(args.warmup - 1, 0)):
        plan.align(A, MA, B, MB)
    torch.cuda.synchronize()
    info0 = plan.info()
    t0 = time.perf_counter()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record()
    for k in range(args.steps):
        out = plan.align(A, MA, B, MB, sync=False)
        evs[k + 1].record()
        print(f"[bench] step {k + 1}/{args.steps} enqueued", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = evs[0].elapsed_time(evs[-1])
    step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
    info1 = plan.info()
    replays = info1["graph_replays"] - info0["graph_replays"]
    ms_per_step = ms_total / args.steps
    # stage times: the same steps launched eagerly with a HIP event pair
    # around every launch on the library's stream (same kernels, same
    # launch configuration as the replayed graph)
    stage_steps = min(args.steps, 3)
    cm.cmif_profile_read(plan.handle)          # clear
    cm.cmif_profile_enable(plan.handle, True)
    for _ in range(stage_steps):
        plan.align(A, MA, B, MB, sync=False)
    torch.cuda.synchronize()
    stages = cm.cmif_profile_read(plan.handle)
    cm.cmif_profile_enable(plan.handle, False)
    eager_ms = sum(s["total_ms"] for s in stages) / stage_steps
    value = n_maps * 1000.0 / ms_per_step
    best = cm.best_from_bytes(bytes(out["best_raw"][0].cpu().numpy()))
    # exactness of the timed calls: no flagged pair left without its FP64
    # re-run (the last timed call's stats; every call has the same inputs)
    hstats = cm.stats_from_raw(out["stats_raw"])
    if hstats["unresolved_pairs"] != 0:
        raise SystemExit(f"timed alignment left flagged pairs unresolved: {hstats}")

    # the oracle's full map of the stress pair, on host threads while the
    # remaining GPU sections run (two threads stay free for the GPU driver)
    omap = None
    if not args.no_stress and not args.no_cpu:
        import oracle
        omap = OracleMap(synth.config4(), max(1, oracle.max_threads() - 2))

    dom = max(stages, key=lambda s: s["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    bytes_per_launch = dom["bytes"] / dom["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = read_traffic(dom["name"])
    roofline = dict(bound="hbm", achieved=round(achieved, 1),
                    peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=traffic, kernel=dom["name"],
                    launches=dom["launches"],
                    avg_launch_ms=round(avg_ms, 4),
                    bytes_per_launch=bytes_per_launch)

    plain = None
    if not args.no_plain:
        print("[bench] plain FP64 schedule", file=sys.stderr, flush=True)
        pplan = cm.Plan([(n, n, n, n)], c["qa"], c["qb"], angles=c["angles"],
                        gamma=c["gamma"], precision="fp64",
                        flags=cm.CMIF_FLAG_PLAIN_SCHEDULE)
        pplan.align(A, MA, B, MB)
        torch.cuda.synchronize()
        pms = []
        for k in range(args.plain_steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            pres = pplan.align(A, MA, B, MB)
            e1.record()
            torch.cuda.synchronize()
            pms.append(e0.elapsed_time(e1))
            print(f"[bench] plain step {k + 1}: {pms[-1]:.1f} ms", file=sys.stderr,
                  flush=True)
        pmed = float(np.median(pms))
        pb = pres["best"][0]
        plain = dict(ms_per_step_median=round(pmed, 3),
                     ms_per_step_all=[round(v, 3) for v in pms],
                     value=round(n_maps * 1000.0 / pmed, 2), unit="maps/s",
                     schedule="FP64; per angle 34 forward and 289 inverse "
                              "transforms each launched alone, separate "
                              "product and entropy kernels, materialised "
                              "FP64 maps, host sync per angle",
                     same_best=(pb["angle_index"], pb["dy"], pb["dx"]) ==
                     (best["angle_index"], best["dy"], best["dx"]))
        del pplan

    window = None
    if not args.no_window:
        # Alg. 1's padded search window for gamma = 0.5: |chi| <= H_B (1 - gamma)
        # per axis; only those 513 x 513 displacements are stored and reduced
        r = int(math.ceil(n * (1.0 - c["gamma"])))
        print(f"[bench] windowed sweep +-{r}", file=sys.stderr, flush=True)
        wplan = cm.Plan([(n, n, n, n)], c["qa"], c["qb"], angles=c["angles"],
                        gamma=c["gamma"], precision="fp32",
                        flags=0 if args.no_autotune else cm.CMIF_FLAG_AUTOTUNE,
                        tune_cache_path=args.tune_cache,
                        windows=[(-r, r, -r, r)])
        wplan.align(A, MA, B, MB)
        torch.cuda.synchronize()
        we = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        we[0].record()
        for k in range(args.steps):
            wout = wplan.align(A, MA, B, MB, sync=False)
            we[k + 1].record()
        torch.cuda.synchronize()
        wms = we[0].elapsed_time(we[-1]) / args.steps
        wb = cm.best_from_bytes(bytes(wout["best_raw"][0].cpu().numpy()))
        winfo = wplan.info()
        window = dict(window=[-r, r, -r, r], map=[2 * r + 1, 2 * r + 1],
                      fft=[winfo["fft_h"], winfo["fft_w"]],
                      ms_per_step=round(wms, 3),
                      value=round(n_maps * 1000.0 / wms, 2), unit="maps/s",
                      same_best=(wb["angle_index"], wb["dy"], wb["dx"]) ==
                      (best["angle_index"], best["dy"], best["dx"]))
        del wplan

    template = None
    if not args.no_template:
        print("[bench] template matching", file=sys.stderr, flush=True)
        template = template_bench(cm, torch, np, synth, dev)

    table1 = None
    if not args.no_table1:
        table1 = table1_context(cm, torch, np, synth, dev)

    stress = None
    if not args.no_stress:
        stress = stress_bench(cm, torch, np, synth, dev, omap=omap)

    # attainable HBM bandwidth of a plain device copy (context for the
    # roofline): 1 GiB read + 1 GiB written per copy, median of 5
    csrc = torch.empty(1 << 30, dtype=torch.uint8, device="cuda").fill_(1)
    cdst = torch.empty_like(csrc)
    cdst.copy_(csrc)
    cts = []
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        cdst.copy_(csrc)
        e1.record()
        torch.cuda.synchronize()
        cts.append(e0.elapsed_time(e1))
    copy_gbs = 2.0 * (1 << 30) / (float(np.median(cts)) * 1e-3) / 1e9
    del csrc, cdst

    volume = None
    if not args.no_volume:
        volume = volume_bench(cm, torch, np, synth, dev)

    soft = None
    if not args.no_soft:
        print("[bench] soft batch", file=sys.stderr, flush=True)
        soft = soft_bench(cm, torch, np, synth, args.soft_steps)

    if args.copy_gib > 0:
        # calibration copies of known size: a contiguous device copy (wide
        # requests), then 64-byte rows out of 128-byte rows (requests of one
        # 64-byte segment, like the library's row and tile accesses)
        nbytes = int(args.copy_gib * (1 << 30))
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        rows = src.view(-1, 128)[:, :64]
        half = torch.empty((rows.shape[0], 64), dtype=torch.uint8, device="cuda")
        for _ in range(3):
            half.copy_(rows)
        torch.cuda.synchronize()
        del src, dst, rows, half

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(c, np)
        cpu["value"] = round(cpu["value"], 5)

    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "maps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "rotation-sweep alignment: A,B 512x512 uint8, "
                        "Q_A=Q_B=16, 180 angles at 2 deg, gamma 0.5, full "
                        "1023x1023 CMIF map per angle",
            "image": [n, n], "labels": [16, 16], "angles": n_maps,
            "fft": [1024, 1024], "precision": "fp32-rounded",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "hbm_copy": dict(gbs=round(copy_gbs, 1),
                         frac_of_peak=round(copy_gbs / HBM_PEAK_GBS, 4),
                         kernel_frac_of_copy=round(achieved / copy_gbs, 4),
                         note="torch device copy of 1 GiB, read + write "
                              "bytes, median of 5"),
        "exactness": dict(unresolved_pairs=hstats["unresolved_pairs"],
                          fallback_overflow=hstats["fallback_overflow"],
                          flagged_pairs=hstats["flagged_pairs"],
                          fallback_pairs=hstats["fallback_pairs"],
                          max_residual=hstats["max_residual"]),
        "ms_per_step_median": round(float(np.median(step_ms)), 3),
        "plain_fp64": plain,
        "speedup_vs_plain_fp64": (round(plain["ms_per_step_median"] /
                                        float(np.median(step_ms)), 3)
                                  if plain else None),
        "window_sweep": window,
        "precision_stress": stress,
        "template_matching": template,
        "paper_table1_context": table1,
        "soft": soft,
        "volume": volume,
        "launch_shapes": {k: info1[k] for k in ("rows_per_wg", "labels_per_team",
                                                "xcd_grouping", "cols_half",
                                                "cols_maxr", "cols_ba", "tuned",
                                                "tune_runs")},
        "graph": dict(replays=replays, captures=info1["graph_captures"],
                      stage_steps=stage_steps,
                      eager_kernel_ms_per_step=round(eager_ms, 3)),
        "stages": {s["name"]: dict(launches=s["launches"],
                                   ms_per_step=round(s["total_ms"] / stage_steps, 3),
                                   gbs=round(s["bytes"] / (s["total_ms"] * 1e-3) / 1e9, 1)
                                   if s["total_ms"] > 0 else None)
                   for s in stages},
        "best": dict(angle_deg=round(math.degrees(best["angle_rad"]), 3),
                     dy=best["dy"], dx=best["dx"], mi=best["mi"], n=best["n"],
                     corner_error_px=round(cm.cmif_corner_error(
                         best, (n, n, n, n), c["truth"]), 3),
                     success=bool(cm.cmif_corner_error(
                         best, (n, n, n, n), c["truth"]) < 0.02 * n),
                     truth_deg=round(c["theta_deg"], 3),
                     truth_shift=list(c["shift"])),
        "wall_s": round(wall, 3),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
