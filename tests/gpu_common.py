"""Helpers shared by the GPU parity tests (HIP path through the C ABI
against the CPU oracle)."""

import sys

import numpy as np

MI_TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(torch, a):
    if a is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(a, np.uint8)).cuda()


def run_compute(gpu, c, precision="fp32", angles=None, counts=True,
                digest=False, best=True, per_angle=False, tag="", flags=0,
                fallback_capacity=0, angle_batch=0):
    cm, torch = gpu
    A, MA, B, MB = c["A"], c["MA"], c["B"], c["MB"]
    ha, wa = A.shape
    hb, wb = B.shape
    angles = c.get("angles", [0.0]) if angles is None else angles
    say(f"[gpu] compute {tag} A{A.shape} B{B.shape} q=({c['qa']},{c['qb']}) "
        f"{precision} angles={len(angles)} counts={counts} digest={digest} "
        f"flags={flags} cap={fallback_capacity} batch={angle_batch}")
    plan = cm.Plan([(ha, wa, hb, wb)], c["qa"], c["qb"], angles=angles,
                   gamma=c.get("gamma", 0.5), precision=precision, flags=flags,
                   fallback_capacity=fallback_capacity,
                   angle_batch=angle_batch)
    res = plan.compute(dev(torch, A), dev(torch, MA), dev(torch, B),
                       dev(torch, MB), mi=True, n=True, counts=counts,
                       digest=digest, best=best, per_angle=per_angle)
    out = dict(mi=res["mi"][0].cpu().numpy(), n=res["n"][0].cpu().numpy(),
               stats=res["stats"])
    if counts:
        out["counts"] = res["counts"][0].cpu().numpy()
    if digest:
        out["digest"] = res["digest"][0].cpu().numpy().view(np.uint64)
    if best:
        out["best"] = res["best"][0]
    if per_angle:
        out["per_angle"] = res["per_angle"][0]
    return out


def check_map(oracle, g, o, angle=0):
    assert np.array_equal(g["n"][angle], o["n"]), "N map differs"
    if "counts" in g and o.get("counts") is not None:
        gc = g["counts"][angle]
        assert gc.shape == o["counts"].shape
        bad = np.argwhere(gc != o["counts"])
        assert bad.size == 0, f"{len(bad)} counts differ, first {bad[:3]}"
    err = np.abs(g["mi"][angle] - o["mi"]).max()
    assert err <= MI_TOL, f"max |dMI| = {err}"
    return err


def argmax_ok(oracle, mi_o, n_o, gamma, g_idx):
    """c12 acceptance: the oracle's own value at the GPU pick is within
    MI_TOL of the oracle's maximum over eligible displacements."""
    idx, v, _ = oracle.argmax(mi_o, n_o, gamma)
    if idx == g_idx:
        return True, False
    flat_mi = mi_o.ravel()
    flat_n = n_o.ravel()
    thr = gamma * flat_n.max()
    ok = flat_n[g_idx] >= thr and abs(flat_mi[g_idx] - v) <= MI_TOL
    return ok, True
