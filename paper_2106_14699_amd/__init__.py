"""Python binding of libcmif (include/cmif.h), the gfx950 CMIF library.

The functions named like the C entry points (cmif_plan, cmif_workspace_size,
cmif_compute, cmif_align, cmif_backward, cmif_plan_free, cmif_status_string,
cmif_last_error) marshal arguments through ctypes and call the library; every
step of the computation runs in the library's HIP kernels.  `Plan` is a thin
convenience wrapper that takes torch tensors, allocates the outputs and the
workspace with torch on the plan's device, and passes torch's current stream.

Importing this module loads libcmif.so and raises if it is missing: there is
no CPU or PyTorch fallback.
"""

from __future__ import annotations

import ctypes
import math
import os
from typing import Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcmif.so")

CMIF_OK = 0
CMIF_ERR_INVALID_ARGUMENT = 1
CMIF_ERR_UNSUPPORTED = 2
CMIF_ERR_WORKSPACE_TOO_SMALL = 3
CMIF_ERR_DEVICE = 4
CMIF_ERR_WRONG_MODE = 5
CMIF_ERR_NO_DEVICE = 6
CMIF_ERR_HOST_MEMORY = 7

CMIF_PREC_FP32_ROUNDED = 0
CMIF_PREC_FP64 = 1
CMIF_MODE_HARD = 0
CMIF_MODE_SOFT = 1
CMIF_FLAG_FORCE_FALLBACK = 1 << 0
CMIF_FLAG_NO_GRAPH = 1 << 1
CMIF_FLAG_SAVE_FOR_BACKWARD = 1 << 2
CMIF_FLAG_PLAIN_SCHEDULE = 1 << 3
CMIF_FLAG_AUTOTUNE = 1 << 4

EXPORTED = ("cmif_plan", "cmif_plan_free", "cmif_workspace_size",
            "cmif_compute", "cmif_align", "cmif_backward",
            "cmif_profile_enable", "cmif_profile_read", "cmif_plan_query",
            "cmif_status_string", "cmif_last_error", "cmif_kmeans",
            "cmif_compute_noalloc", "cmif_align_two_stage",
            "cmif_corner_error", "cmif_volume_workspace_size",
            "cmif_compute_volume")
NOALLOC_BYTES = 128 << 20  # CMIF_NOALLOC_BYTES

_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)


class cmif_plan_desc(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int32),
                ("h_a", ctypes.POINTER(ctypes.c_int32)),
                ("w_a", ctypes.POINTER(ctypes.c_int32)),
                ("h_b", ctypes.POINTER(ctypes.c_int32)),
                ("w_b", ctypes.POINTER(ctypes.c_int32)),
                ("q_a", ctypes.c_int32), ("q_b", ctypes.c_int32),
                ("n_angles", ctypes.c_int32),
                ("angles_rad", ctypes.POINTER(ctypes.c_double)),
                ("gamma", ctypes.c_double),
                ("precision", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("device", ctypes.c_int32),
                ("angle_batch", ctypes.c_int32),
                ("fallback_capacity", ctypes.c_int32),
                ("tune_cache_path", ctypes.c_char_p),
                ("window", ctypes.POINTER(ctypes.c_int32))]


class cmif_stats(ctypes.Structure):
    _fields_ = [("label_errors", ctypes.c_uint32),
                ("flagged_pairs", ctypes.c_uint32),
                ("fallback_pairs", ctypes.c_uint32),
                ("fallback_overflow", ctypes.c_uint32),
                ("max_residual", ctypes.c_float),
                ("nonfinite_inputs", ctypes.c_uint32),
                ("unresolved_pairs", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class cmif_best(ctypes.Structure):
    _fields_ = [("angle_index", ctypes.c_int32), ("dy", ctypes.c_int32),
                ("dx", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("angle_rad", ctypes.c_double), ("mi", ctypes.c_double),
                ("n", ctypes.c_int64)]


class cmif_volume_desc(ctypes.Structure):
    _fields_ = [("d_a", ctypes.c_int32), ("h_a", ctypes.c_int32),
                ("w_a", ctypes.c_int32), ("d_b", ctypes.c_int32),
                ("h_b", ctypes.c_int32), ("w_b", ctypes.c_int32),
                ("q_a", ctypes.c_int32), ("q_b", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("precision", ctypes.c_int32),
                ("device", ctypes.c_int32)]


class cmif_best3d(ctypes.Structure):
    _fields_ = [("dz", ctypes.c_int32), ("dy", ctypes.c_int32),
                ("dx", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("mi", ctypes.c_double), ("n", ctypes.c_int64)]


class cmif_inputs(ctypes.Structure):
    _fields_ = [("labels_a", _PP), ("mask_a", _PP), ("labels_b", _PP),
                ("mask_b", _PP), ("memb_a", _PP), ("memb_b", _PP)]


class cmif_outputs(ctypes.Structure):
    _fields_ = [("mi", _PP), ("n", _PP), ("counts", _PP), ("digest", _PP),
                ("best", _P), ("per_angle", _P), ("stats", _P)]


class cmif_plan_info(ctypes.Structure):
    _fields_ = [("angle_batch", ctypes.c_int32),
                ("fallback_capacity", ctypes.c_int32),
                ("graph_captures", ctypes.c_int32),
                ("graph_replays", ctypes.c_int32),
                ("fft_h", ctypes.c_int32), ("fft_w", ctypes.c_int32),
                ("rows_per_wg", ctypes.c_int32),
                ("labels_per_team", ctypes.c_int32),
                ("xcd_grouping", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("tune_runs", ctypes.c_int32), ("cols_half", ctypes.c_int32),
                ("cols_maxr", ctypes.c_int32), ("cols_ba", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class cmif_stage_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class CmifError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: {cmif_status_string(status)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


class CmifInexactError(CmifError):
    """A call finished, but some label pairs whose FP32 rounding residual
    reached 0.25 were not recomputed in FP64 (the plan's fallback capacity
    was too small), so their counts are not guaranteed exact.  The results
    are attached as `.results`."""

    def __init__(self, where: str, stats: dict, results=None):
        self.stats = stats
        self.results = results
        super().__init__(CMIF_OK, where,
                         f"{stats['unresolved_pairs']} flagged label pairs "
                         "beyond the FP64 re-run capacity; raise "
                         "fallback_capacity, or pass allow_inexact=True")


def _load_lib():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libcmif.so not found at {LIB_PATH}; build it with "
            "`python paper_2106_14699_amd/build.py` (there is no fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    S = ctypes.c_size_t
    lib.cmif_plan.argtypes = [ctypes.POINTER(cmif_plan_desc), ctypes.POINTER(_P)]
    lib.cmif_plan.restype = ctypes.c_int
    lib.cmif_plan_free.argtypes = [_P]
    lib.cmif_plan_free.restype = None
    lib.cmif_workspace_size.argtypes = [_P, ctypes.POINTER(S), ctypes.POINTER(S)]
    lib.cmif_workspace_size.restype = ctypes.c_int
    lib.cmif_compute.argtypes = [_P, ctypes.POINTER(cmif_inputs),
                                 ctypes.POINTER(cmif_outputs), _P, S, _P, S, _P]
    lib.cmif_compute.restype = ctypes.c_int
    lib.cmif_align.argtypes = [_P, ctypes.POINTER(cmif_inputs), _P, _P, _P, _P,
                               S, _P, S, _P]
    lib.cmif_align.restype = ctypes.c_int
    lib.cmif_compute_noalloc.argtypes = [_P, ctypes.POINTER(cmif_inputs),
                                         ctypes.POINTER(cmif_outputs), _P]
    lib.cmif_compute_noalloc.restype = ctypes.c_int
    lib.cmif_align_two_stage.argtypes = [_P, ctypes.POINTER(cmif_inputs),
                                         ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_double), _P,
                                         _P, _P, _P, _P, S, _P, S, _P]
    lib.cmif_align_two_stage.restype = ctypes.c_int
    lib.cmif_corner_error.argtypes = [ctypes.POINTER(cmif_best), ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
    lib.cmif_corner_error.restype = ctypes.c_int
    lib.cmif_volume_workspace_size.argtypes = [ctypes.POINTER(cmif_volume_desc),
                                               ctypes.POINTER(S)]
    lib.cmif_volume_workspace_size.restype = ctypes.c_int
    lib.cmif_compute_volume.argtypes = [ctypes.POINTER(cmif_volume_desc), _P, _P,
                                        _P, _P, _P, _P, _P, _P, _P, _P, S, _P]
    lib.cmif_compute_volume.restype = ctypes.c_int
    lib.cmif_backward.argtypes = [_P, ctypes.POINTER(cmif_inputs), _PP, _PP,
                                  _PP, _P, S, _P, S, _P]
    lib.cmif_backward.restype = ctypes.c_int
    lib.cmif_kmeans.argtypes = [_P, _P, ctypes.c_int64, ctypes.c_int32,
                                ctypes.c_int32, _P, _P, ctypes.c_int32,
                                ctypes.c_int32, _P, _P, _P, _P]
    lib.cmif_kmeans.restype = ctypes.c_int
    lib.cmif_plan_query.argtypes = [_P, ctypes.POINTER(cmif_plan_info)]
    lib.cmif_plan_query.restype = ctypes.c_int
    lib.cmif_profile_enable.argtypes = [_P, ctypes.c_int32]
    lib.cmif_profile_enable.restype = ctypes.c_int
    lib.cmif_profile_read.argtypes = [_P, ctypes.POINTER(cmif_stage_time),
                                      ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32)]
    lib.cmif_profile_read.restype = ctypes.c_int
    lib.cmif_status_string.argtypes = [ctypes.c_int]
    lib.cmif_status_string.restype = ctypes.c_char_p
    lib.cmif_last_error.argtypes = []
    lib.cmif_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load_lib()


# -- entry points with the C names (marshalling only) ------------------------

def cmif_status_string(status: int) -> str:
    return _lib.cmif_status_string(int(status)).decode()


def cmif_last_error() -> str:
    return _lib.cmif_last_error().decode()


def _check(status: int, where: str):
    if status != CMIF_OK:
        raise CmifError(status, where, cmif_last_error())


def cmif_plan(desc: cmif_plan_desc) -> int:
    h = _P()
    _check(_lib.cmif_plan(ctypes.byref(desc), ctypes.byref(h)), "cmif_plan")
    return h.value


def cmif_plan_free(plan: int) -> None:
    _lib.cmif_plan_free(_P(plan))


def cmif_workspace_size(plan: int) -> tuple[int, int]:
    p = ctypes.c_size_t()
    s = ctypes.c_size_t()
    _check(_lib.cmif_workspace_size(_P(plan), ctypes.byref(p), ctypes.byref(s)),
           "cmif_workspace_size")
    return p.value, s.value


def cmif_compute(plan, inputs, outputs, persistent, persistent_bytes, scratch,
                 scratch_bytes, stream) -> None:
    _check(_lib.cmif_compute(_P(plan), ctypes.byref(inputs),
                             ctypes.byref(outputs), _P(persistent),
                             persistent_bytes, _P(scratch), scratch_bytes,
                             _P(stream)), "cmif_compute")


def cmif_compute_noalloc(plan, inputs, outputs, stream) -> None:
    _check(_lib.cmif_compute_noalloc(_P(plan), ctypes.byref(inputs),
                                     ctypes.byref(outputs), _P(stream)),
           "cmif_compute_noalloc")


def cmif_align(plan, inputs, best, per_angle, stats, persistent,
               persistent_bytes, scratch, scratch_bytes, stream) -> None:
    _check(_lib.cmif_align(_P(plan), ctypes.byref(inputs), _P(best),
                           _P(per_angle), _P(stats), _P(persistent),
                           persistent_bytes, _P(scratch), scratch_bytes,
                           _P(stream)), "cmif_align")


def cmif_align_two_stage(plan, inputs, n_refine, refine_offsets, best,
                         grid_best, refine_best, stats, persistent,
                         persistent_bytes, scratch, scratch_bytes,
                         stream) -> None:
    _check(_lib.cmif_align_two_stage(_P(plan), ctypes.byref(inputs),
                                     int(n_refine), refine_offsets, _P(best),
                                     _P(grid_best), _P(refine_best), _P(stats),
                                     _P(persistent), persistent_bytes,
                                     _P(scratch), scratch_bytes, _P(stream)),
           "cmif_align_two_stage")


def cmif_corner_error(result: dict, sizes, truth) -> float:
    """Mean corner (landmark) error in reference pixels of an Alg. 1
    result dict (best_from_bytes) for image sides (h_a, w_a, h_b, w_b)
    against the true A -> B affine map truth (6 numbers)."""
    b = cmif_best()
    b.angle_index = int(result["angle_index"])
    b.dy, b.dx = int(result["dy"]), int(result["dx"])
    b.angle_rad = float(result["angle_rad"])
    b.mi = float(result.get("mi", 0.0))
    b.n = int(result.get("n", 0))
    t = (ctypes.c_double * 6)(*[float(v) for v in truth])
    e = ctypes.c_double()
    ha, wa, hb, wb = (int(v) for v in sizes)
    _check(_lib.cmif_corner_error(ctypes.byref(b), ha, wa, hb, wb, t,
                                  ctypes.byref(e)), "cmif_corner_error")
    return e.value


def cmif_volume_workspace_size(desc: cmif_volume_desc) -> int:
    b = ctypes.c_size_t()
    _check(_lib.cmif_volume_workspace_size(ctypes.byref(desc), ctypes.byref(b)),
           "cmif_volume_workspace_size")
    return b.value


def cmif_compute_volume(desc, labels_a, mask_a, labels_b, mask_b, mi, n,
                        digest, best, stats, workspace, workspace_bytes,
                        stream) -> None:
    _check(_lib.cmif_compute_volume(ctypes.byref(desc), _P(labels_a),
                                    _P(mask_a), _P(labels_b), _P(mask_b),
                                    _P(mi), _P(n), _P(digest), _P(best),
                                    _P(stats), _P(workspace), workspace_bytes,
                                    _P(stream)), "cmif_compute_volume")


def volume_desc(shape_a, shape_b, q_a, q_b, gamma=0.5, precision="fp32",
                device=0) -> cmif_volume_desc:
    d = cmif_volume_desc()
    d.d_a, d.h_a, d.w_a = (int(v) for v in shape_a)
    d.d_b, d.h_b, d.w_b = (int(v) for v in shape_b)
    d.q_a, d.q_b = int(q_a), int(q_b)
    d.gamma = float(gamma)
    d.precision = {"fp32": CMIF_PREC_FP32_ROUNDED,
                   "fp64": CMIF_PREC_FP64}[precision]
    d.device = int(device)
    return d


def compute_volume(A, MA, B, MB, q_a, q_b, *, gamma=0.5, precision="fp32",
                   mi=True, n=True, digest=False, best=True,
                   allow_inexact=False):
    """3-D CMIF of two uint8 label volumes (device tensors [D][H][W],
    masks or None) through cmif_compute_volume.  Returns dict(mi, n [S_d,
    S_h, S_w] tensors, digest [q_a, q_b] int64 tensor, best dict(dz, dy,
    dx, mi, n), stats).  Raises CmifInexactError when FP32 label pairs were
    flagged (volumes have no FP64 re-run), unless allow_inexact=True."""
    import torch
    dev = A.device
    for t, name in ((A, "A"), (B, "B"), (MA, "MA"), (MB, "MB")):
        if t is None:
            continue
        if t.dtype != torch.uint8 or t.dim() != 3 or not t.is_contiguous() \
                or t.device != dev:
            raise ValueError(f"{name} must be a contiguous uint8 [D][H][W] "
                             f"tensor on {dev}")
    if MA is not None and tuple(MA.shape) != tuple(A.shape):
        raise ValueError("MA must have A's shape")
    if MB is not None and tuple(MB.shape) != tuple(B.shape):
        raise ValueError("MB must have B's shape")
    d = volume_desc(A.shape, B.shape, q_a, q_b, gamma, precision,
                    dev.index or 0)
    nbytes = cmif_volume_workspace_size(d)
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    ws = buf.data_ptr() + (-buf.data_ptr()) % 256
    shape = tuple(a + b - 1 for a, b in zip(A.shape, B.shape))
    mi_t = torch.empty(shape, dtype=torch.float64, device=dev) if mi else None
    n_t = torch.empty(shape, dtype=torch.int32, device=dev) if n else None
    dg_t = (torch.empty((q_a, q_b), dtype=torch.int64, device=dev)
            if digest else None)
    b_t = (torch.empty((ctypes.sizeof(cmif_best3d),), dtype=torch.uint8,
                       device=dev) if best else None)
    st_t = torch.zeros((ctypes.sizeof(cmif_stats),), dtype=torch.uint8,
                       device=dev)
    ptr = lambda t: t.data_ptr() if t is not None else None
    cmif_compute_volume(d, A.data_ptr(), ptr(MA), B.data_ptr(), ptr(MB),
                        ptr(mi_t), ptr(n_t), ptr(dg_t), ptr(b_t),
                        st_t.data_ptr(), ws, nbytes,
                        torch.cuda.current_stream(dev).cuda_stream)
    torch.cuda.current_stream(dev).synchronize()
    res = dict(mi=mi_t, n=n_t, digest=dg_t, stats=_stats_dict(st_t))
    if best:
        b = cmif_best3d.from_buffer_copy(bytes(b_t.cpu().numpy()))
        res["best"] = dict(dz=b.dz, dy=b.dy, dx=b.dx, mi=b.mi, n=b.n)
    del buf
    if res["stats"]["unresolved_pairs"] and not allow_inexact:
        raise CmifInexactError("cmif_compute_volume", res["stats"], res)
    return res


def cmif_backward(plan, inputs, grad_mi, grad_a, grad_b, persistent,
                  persistent_bytes, scratch, scratch_bytes, stream) -> None:
    _check(_lib.cmif_backward(_P(plan), ctypes.byref(inputs), grad_mi, grad_a,
                              grad_b, _P(persistent), persistent_bytes,
                              _P(scratch), scratch_bytes, _P(stream)),
           "cmif_backward")


def cmif_plan_query(plan: int) -> dict:
    info = cmif_plan_info()
    _check(_lib.cmif_plan_query(_P(plan), ctypes.byref(info)), "cmif_plan_query")
    return {k: getattr(info, k) for k, _ in cmif_plan_info._fields_
            if k != "reserved"}


def cmif_profile_enable(plan: int, enable: bool) -> None:
    _check(_lib.cmif_profile_enable(_P(plan), 1 if enable else 0),
           "cmif_profile_enable")


def cmif_profile_read(plan: int) -> list[dict]:
    """Per-stage launch counts, summed event milliseconds and algorithmic
    bytes recorded since the last read (waits for the recorded events)."""
    cap = 32
    buf = (cmif_stage_time * cap)()
    n = ctypes.c_int32()
    _check(_lib.cmif_profile_read(_P(plan), buf, cap, ctypes.byref(n)),
           "cmif_profile_read")
    return [dict(name=buf[i].name.decode(), launches=buf[i].launches,
                 total_ms=buf[i].total_ms, bytes=buf[i].bytes)
            for i in range(n.value)]


# -- torch convenience layer ----------------------------------------------------

def _ptr_array(ptrs):
    if ptrs is None:
        return None
    arr = (ctypes.c_void_p * len(ptrs))(*[p if p else None for p in ptrs])
    return ctypes.cast(arr, _PP), arr


BEST_DTYPE_FIELDS = ("angle_index", "dy", "dx", "reserved", "angle_rad", "mi",
                     "n")


def best_from_bytes(raw: bytes) -> dict:
    b = cmif_best.from_buffer_copy(raw)
    return {k: getattr(b, k) for k in BEST_DTYPE_FIELDS if k != "reserved"}


class Plan:
    """A plan for n image pairs (sizes given per pair) with fixed Q_A, Q_B,
    angle list and gamma.  Tensors passed in must live on the plan's device
    (uint8 labels/masks, row-major)."""

    def __init__(self, sizes: Sequence[tuple[int, int, int, int]], q_a: int,
                 q_b: int, angles: Sequence[float] | None = None,
                 gamma: float = 0.5, precision: str = "fp32",
                 mode: str = "hard", flags: int = 0, device: int = 0,
                 angle_batch: int = 0, fallback_capacity: int = 0,
                 tune_cache_path: str | None = None,
                 windows: Sequence[tuple[int, int, int, int]] | None = None):
        import torch
        self._torch = torch
        self.sizes = [tuple(int(v) for v in s) for s in sizes]
        n = len(self.sizes)
        self.q_a, self.q_b = int(q_a), int(q_b)
        self.angles = [0.0] if angles is None else [float(a) for a in angles]
        self.gamma = float(gamma)
        self.device = int(device)
        i32 = ctypes.c_int32 * n
        self._keep = [i32(*[s[k] for s in self.sizes]) for k in range(4)]
        ang = (ctypes.c_double * len(self.angles))(*self.angles)
        self._keep.append(ang)
        d = cmif_plan_desc()
        d.n_pairs = n
        d.h_a, d.w_a, d.h_b, d.w_b = [ctypes.cast(a, ctypes.POINTER(ctypes.c_int32))
                                      for a in self._keep[:4]]
        d.q_a, d.q_b = self.q_a, self.q_b
        d.n_angles = len(self.angles)
        d.angles_rad = ctypes.cast(ang, ctypes.POINTER(ctypes.c_double))
        d.gamma = self.gamma
        d.precision = {"fp32": CMIF_PREC_FP32_ROUNDED,
                       "fp64": CMIF_PREC_FP64}[precision]
        d.mode = {"hard": CMIF_MODE_HARD, "soft": CMIF_MODE_SOFT}[mode]
        self.mode = mode
        d.flags = int(flags)
        d.device = self.device
        d.angle_batch = int(angle_batch)
        d.fallback_capacity = int(fallback_capacity)
        self._tune_path = (tune_cache_path.encode() if tune_cache_path
                           else None)
        d.tune_cache_path = self._tune_path
        # displacement windows (y0, y1, x0, x1) per pair; None = full set
        self.windows = None if windows is None else [
            tuple(int(v) for v in w) for w in windows]
        if self.windows is not None:
            if len(self.windows) != n:
                raise ValueError("one window per image pair")
            win = (ctypes.c_int32 * (4 * n))(*[v for w in self.windows for v in w])
            self._keep.append(win)
            d.window = ctypes.cast(win, ctypes.POINTER(ctypes.c_int32))
        self.handle = cmif_plan(d)
        # kept for __del__: module globals may already be gone at exit
        self._free = _lib.cmif_plan_free
        self.persistent_bytes, self.scratch_bytes = cmif_workspace_size(
            self.handle)
        self._ws = None
        self._forward_gen = 0        # cmif_compute calls made by this plan
        self.recomputed_forwards = 0  # SoftCMIF backwards that re-ran theirs

    def __del__(self):
        h = getattr(self, "handle", None)
        free = getattr(self, "_free", None)
        if h and free is not None:
            free(h)  # argtypes convert the int handle
            self.handle = None

    def window(self, p: int = 0):
        """Displacement window (y0, y1, x0, x1) of pair p: map entry [i][j]
        holds chi = (y0 + i, x0 + j)."""
        if self.windows is not None:
            return self.windows[p]
        ha, wa, hb, wb = self.sizes[p]
        return 1 - ha, hb - 1, 1 - wa, wb - 1

    def map_shape(self, p: int = 0):
        y0, y1, x0, x1 = self.window(p)
        return y1 - y0 + 1, x1 - x0 + 1

    def _aligned(self, nbytes: int):
        torch = self._torch
        buf = torch.empty(max(nbytes, 1) + 256, dtype=torch.uint8,
                          device=f"cuda:{self.device}")
        off = (-buf.data_ptr()) % 256
        return buf, buf.data_ptr() + off

    def workspace(self):
        if self._ws is None:
            pb, pp = self._aligned(self.persistent_bytes)
            sb, sp = self._aligned(self.scratch_bytes)
            self._ws = (pb, pp, sb, sp)
        return self._ws

    def _inputs(self, A, MA, B, MB):
        """HARD: A, B uint8 label images [H][W]; SOFT: float32 memberships
        [Q][H][W].  MA, MB uint8 masks or None."""
        import torch
        A, B = _listify(A), _listify(B)
        MA, MB = _listify(MA, len(A)), _listify(MB, len(B))
        n = len(self.sizes)
        if len(A) != n or len(B) != n:
            raise ValueError("one A and one B per image pair")
        soft = self.mode == "soft"
        for p in range(n):
            ha, wa, hb, wb = self.sizes[p]
            if soft:
                _check_tensor(A[p], (self.q_a, ha, wa), self.device, "A",
                              torch.float32)
                _check_tensor(B[p], (self.q_b, hb, wb), self.device, "B",
                              torch.float32)
            else:
                _check_tensor(A[p], (ha, wa), self.device, "A")
                _check_tensor(B[p], (hb, wb), self.device, "B")
            if MA[p] is not None:
                _check_tensor(MA[p], (ha, wa), self.device, "MA")
            if MB[p] is not None:
                _check_tensor(MB[p], (hb, wb), self.device, "MB")
        keep = []
        inp = cmif_inputs()
        names = (("memb_a", A), ("mask_a", MA), ("memb_b", B), ("mask_b", MB)) \
            if soft else (("labels_a", A), ("mask_a", MA), ("labels_b", B),
                          ("mask_b", MB))
        for name, ts in names:
            ptrs = [t.data_ptr() if t is not None else 0 for t in ts]
            pa, arr = _ptr_array(ptrs)
            keep.append(arr)
            setattr(inp, name, pa)
        return inp, keep

    def _stream(self):
        return self._torch.cuda.current_stream(self.device).cuda_stream

    def _buffer(self, reuse, key, shape, dtype):
        """Output tensor: fresh, or (reuse=True) kept by the plan so that
        repeated calls pass the same pointers and replay the captured
        launch graph (the returned tensor is overwritten by the next call)."""
        torch = self._torch
        dev = f"cuda:{self.device}"
        if not reuse:
            return torch.empty(shape, dtype=dtype, device=dev)
        cache = self.__dict__.setdefault("_bufs", {})
        t = cache.get(key)
        if t is None or tuple(t.shape) != tuple(shape) or t.dtype != dtype:
            t = torch.empty(shape, dtype=dtype, device=dev)
            cache[key] = t
        return t

    def compute(self, A, MA=None, B=None, MB=None, *, mi=True, n=True,
                counts=False, digest=False, best=False, per_angle=False,
                reuse=False, allow_inexact=False, noalloc=False):
        """CMIF maps for every pair and angle.  Returns a dict of lists (one
        entry per pair) of torch tensors, plus 'stats' (dict).  With
        reuse=True the output tensors belong to the plan and are overwritten
        by its next call (stable pointers replay the captured graph).
        Raises CmifInexactError when flagged label pairs were left without
        their FP64 re-run (stats['unresolved_pairs'] > 0), unless
        allow_inexact=True.  noalloc=True calls cmif_compute_noalloc (the
        library's own workspace array) instead of cmif_compute."""
        torch = self._torch
        inp, keep = self._inputs(A, MA, B, MB)
        na = len(self.angles)
        res = {}
        outs = cmif_outputs()
        for name, want, dtype, shape_fn in (
                ("mi", mi, torch.float64, lambda s: (na, *s)),
                ("n", n, torch.int32, lambda s: (na, *s)),
                ("counts", counts, torch.int32,
                 lambda s: (na, self.q_a, self.q_b, *s)),
                ("digest", digest, torch.int64,
                 lambda s: (na, self.q_a, self.q_b))):
            if want:
                ts = [self._buffer(reuse, ("c", name, p),
                                   shape_fn(self.map_shape(p)), dtype)
                      for p in range(len(self.sizes))]
                res[name] = ts
                pa, arr = _ptr_array([t.data_ptr() for t in ts])
                keep.append(arr)
                setattr(outs, name, pa)
        nbest = ctypes.sizeof(cmif_best)
        best_t = self._buffer(reuse, ("c", "best"), (len(self.sizes), nbest),
                              torch.uint8) if best else None
        pa_t = self._buffer(reuse, ("c", "pa"), (len(self.sizes), na, nbest),
                            torch.uint8) if per_angle else None
        stats_t = self._buffer(reuse, ("c", "stats"),
                               (ctypes.sizeof(cmif_stats),), torch.uint8)
        stats_t.zero_()
        outs.best = best_t.data_ptr() if best else None
        outs.per_angle = pa_t.data_ptr() if per_angle else None
        outs.stats = stats_t.data_ptr()
        if noalloc:
            cmif_compute_noalloc(self.handle, inp, outs, self._stream())
        else:
            pb, pp, sb, sp = self.workspace()
            cmif_compute(self.handle, inp, outs, pp, self.persistent_bytes, sp,
                         self.scratch_bytes, self._stream())
        torch.cuda.current_stream(self.device).synchronize()
        res["stats"] = _stats_dict(stats_t)
        if best:
            res["best"] = [best_from_bytes(bytes(best_t[p].cpu().numpy()))
                           for p in range(len(self.sizes))]
        if per_angle:
            raw = pa_t.cpu().numpy()
            res["per_angle"] = [[best_from_bytes(bytes(raw[p, k]))
                                 for k in range(na)]
                                for p in range(len(self.sizes))]
        del keep
        self._forward_gen += 1
        if res["stats"]["unresolved_pairs"] and not allow_inexact:
            raise CmifInexactError("cmif_compute", res["stats"], res)
        return res

    def info(self) -> dict:
        return cmif_plan_query(self.handle)

    def align(self, A, MA=None, B=None, MB=None, *, per_angle=False,
              sync=True, allow_inexact=False):
        """Alg. 1 over the plan's angles for every pair.  Returns a list of
        best dicts (and per-angle lists), plus stats.  The small result
        buffers belong to the plan (stable pointers replay the captured
        graph): with sync=False the returned raw tensors are overwritten by
        the next call, and the caller checks stats_raw itself (see
        stats_from_raw).  With sync=True, raises CmifInexactError when
        flagged label pairs were left without their FP64 re-run, unless
        allow_inexact=True."""
        torch = self._torch
        inp, keep = self._inputs(A, MA, B, MB)
        na = len(self.angles)
        nbest = ctypes.sizeof(cmif_best)
        best_t = self._buffer(True, ("a", "best"), (len(self.sizes), nbest),
                              torch.uint8)
        pa_t = self._buffer(True, ("a", "pa"), (len(self.sizes), na, nbest),
                            torch.uint8) if per_angle else None
        stats_t = self._buffer(True, ("a", "stats"),
                               (ctypes.sizeof(cmif_stats),), torch.uint8)
        stats_t.zero_()
        pb, pp, sb, sp = self.workspace()
        cmif_align(self.handle, inp, best_t.data_ptr(),
                   pa_t.data_ptr() if per_angle else None, stats_t.data_ptr(),
                   pp, self.persistent_bytes, sp, self.scratch_bytes,
                   self._stream())
        del keep
        if not sync:
            return dict(best_raw=best_t, per_angle_raw=pa_t, stats_raw=stats_t)
        torch.cuda.current_stream(self.device).synchronize()
        res = dict(best=[best_from_bytes(bytes(best_t[p].cpu().numpy()))
                         for p in range(len(self.sizes))],
                   stats=_stats_dict(stats_t))
        if per_angle:
            raw = pa_t.cpu().numpy()
            res["per_angle"] = [[best_from_bytes(bytes(raw[p, k]))
                                 for k in range(na)]
                                for p in range(len(self.sizes))]
        if res["stats"]["unresolved_pairs"] and not allow_inexact:
            raise CmifInexactError("cmif_align", res["stats"], res)
        return res


def _plan_align_two_stage(self, A, MA=None, B=None, MB=None, *,
                          refine_offsets, allow_inexact=False):
    """Sec. 3.6's two-stage alignment through cmif_align_two_stage: Alg. 1
    over the plan's angles, then per pair over theta* + u_k 2 pi / |angles|
    for the given offsets u_k in [-1, 1].  Returns dict(best, grid_best,
    refine_best: lists per pair, stats)."""
    torch = self._torch
    inp, keep = self._inputs(A, MA, B, MB)
    u = [float(v) for v in refine_offsets]
    uarr = (ctypes.c_double * len(u))(*u)
    n = len(self.sizes)
    nbest = ctypes.sizeof(cmif_best)
    bufs = [self._buffer(True, ("t", k), (n, nbest), torch.uint8)
            for k in ("best", "grid", "refine")]
    stats_t = self._buffer(True, ("t", "stats"), (ctypes.sizeof(cmif_stats),),
                           torch.uint8)
    stats_t.zero_()
    pb, pp, sb, sp = self.workspace()
    cmif_align_two_stage(self.handle, inp, len(u), uarr, bufs[0].data_ptr(),
                         bufs[1].data_ptr(), bufs[2].data_ptr(),
                         stats_t.data_ptr(), pp, self.persistent_bytes, sp,
                         self.scratch_bytes, self._stream())
    torch.cuda.current_stream(self.device).synchronize()
    del keep
    out = [[best_from_bytes(bytes(t[p].cpu().numpy())) for p in range(n)]
           for t in bufs]
    res = dict(best=out[0], grid_best=out[1], refine_best=out[2],
               stats=_stats_dict(stats_t))
    if res["stats"]["unresolved_pairs"] and not allow_inexact:
        raise CmifInexactError("cmif_align_two_stage", res["stats"], res)
    return res


Plan.align_two_stage = _plan_align_two_stage


def stats_from_raw(stats_t) -> dict:
    """cmif_stats (a device or host uint8 tensor of its bytes) as a dict."""
    return _stats_dict(stats_t)


def cmif_kmeans(image, mask, n_pixels, channels, k, init_idx, batches, iters,
                batch, centers, labels, bad_indices, stream) -> None:
    _check(_lib.cmif_kmeans(_P(image), _P(mask), int(n_pixels), int(channels),
                            int(k), _P(init_idx), _P(batches), int(iters),
                            int(batch), _P(centers), _P(labels),
                            _P(bad_indices), _P(stream)), "cmif_kmeans")


def kmeans_quantize(image, k, *, iters=25, batch=1000, rng=None, mask=None,
                    init_idx=None, batches=None):
    """Quantise a device FP32 image ([H, W] or [H, W, m]) into k labels by
    mini-batch k-means (cmif_kmeans).  The random draws are made here on the
    host with `rng` (numpy Generator) unless given: k distinct in-mask
    pixels seed the centres, and each of `iters` batches is `batch` in-mask
    pixel indices drawn uniformly with replacement.  Returns dict(labels
    uint8 [H, W], centers float64 [k, m], init_idx, batches, bad)."""
    import numpy as np
    import torch
    if image.dtype != torch.float32 or not image.is_cuda:
        raise ValueError("image must be a float32 device tensor")
    img = image.contiguous()
    h, w = img.shape[0], img.shape[1]
    m = 1 if img.dim() == 2 else img.shape[2]
    n = h * w
    dev = img.device
    msk = None
    if mask is not None:
        msk = mask.to(device=dev, dtype=torch.uint8).contiguous()
    if init_idx is None or (batches is None and iters > 0):
        if rng is None:
            raise ValueError("pass rng or both init_idx and batches")
        pool = (np.arange(n) if msk is None
                else np.flatnonzero(msk.reshape(-1).cpu().numpy()))
        if init_idx is None:
            init_idx = rng.choice(pool, size=k, replace=False)
        if batches is None and iters > 0:
            batches = pool[rng.integers(0, pool.size, size=(iters, batch))]
    init_t = torch.as_tensor(np.asarray(init_idx, np.int32), device=dev)
    bt = (torch.as_tensor(np.asarray(batches, np.int32).reshape(iters, batch),
                          device=dev) if iters > 0 else None)
    centers = torch.zeros((k, m), dtype=torch.float64, device=dev)
    labels = torch.empty((h, w), dtype=torch.uint8, device=dev)
    bad = torch.zeros((1,), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    cmif_kmeans(img.data_ptr(), msk.data_ptr() if msk is not None else None,
                n, m, k, init_t.data_ptr(),
                bt.data_ptr() if bt is not None else None, iters,
                batch if iters > 0 else 1, centers.data_ptr(), labels.data_ptr(),
                bad.data_ptr(), stream)
    torch.cuda.current_stream(dev).synchronize()
    return dict(labels=labels, centers=centers, init_idx=np.asarray(init_idx),
                batches=None if batches is None else np.asarray(batches),
                bad=int(bad.item()))


def align_two_stage(A, MA, B, MB, size, q_a, q_b, grid, *, n_refine=32,
                    rng=None, refine_offsets=None, gamma=0.5, precision="fp32",
                    flags=0, window=None, device=0):
    """Global rigid alignment run twice (Sec. 3.6) for one image pair of
    sides `size` = (h_a, w_a, h_b, w_b): one cmif_align_two_stage call, Alg.
    1 over the angles `grid`, then over n_refine angles drawn uniformly from
    [theta* - 2 pi/|grid|, theta* + 2 pi/|grid|] around the grid's best
    angle theta*.  The draws are offsets u_k uniform in [-1, 1] from `rng`
    (a numpy Generator), made on the host, or the caller passes
    refine_offsets.  Returns dict(best, stage ('grid' or 'refine'),
    grid_best, refine_best, refine_offsets)."""
    import numpy as np
    grid = [float(t) for t in grid]
    if refine_offsets is None:
        if rng is None:
            raise ValueError("pass rng (numpy Generator) or refine_offsets")
        refine_offsets = rng.uniform(-1.0, 1.0, int(n_refine))
    u = [float(v) for v in np.asarray(refine_offsets).ravel()]
    wins = None if window is None else [tuple(window)]
    plan = Plan([size], q_a, q_b, angles=grid, gamma=gamma, precision=precision,
                flags=flags, device=device, windows=wins)
    r = plan.align_two_stage(A, MA, B, MB, refine_offsets=u)
    del plan
    best = r["best"][0]
    return dict(best=best,
                stage="refine" if best["angle_index"] >= len(grid) else "grid",
                grid_best=r["grid_best"][0], refine_best=r["refine_best"][0],
                refine_offsets=u)


def _plan_backward(self, A, MA, B, MB, grad_mi, *, want_a=True, want_b=True):
    """SOFT plans with SAVE_FOR_BACKWARD, after compute() on the same
    inputs: dL/dA and dL/dB (float32, shapes of the memberships) for the
    upstream dL/dMI maps grad_mi (one float64 [n_angles][S_h][S_w] tensor
    per pair).  Returns (list or None, list or None)."""
    torch = self._torch
    inp, keep = self._inputs(A, MA, B, MB)
    dev = f"cuda:{self.device}"
    gm = _listify(grad_mi)
    n = len(self.sizes)
    if len(gm) != n:
        raise ValueError("one grad_mi per image pair")
    gm = [g.to(device=dev, dtype=torch.float64).contiguous() for g in gm]
    for p in range(n):
        if tuple(gm[p].shape) != (len(self.angles), *self.map_shape(p)):
            raise ValueError("grad_mi must have shape [n_angles, S_h, S_w]")
    ga = [torch.empty((self.q_a, s[0], s[1]), dtype=torch.float32, device=dev)
          for s in self.sizes] if want_a else None
    gb = [torch.empty((self.q_b, s[2], s[3]), dtype=torch.float32, device=dev)
          for s in self.sizes] if want_b else None
    pgm, agm = _ptr_array([t.data_ptr() for t in gm])
    pga, aga = _ptr_array([t.data_ptr() for t in ga]) if ga else (None, None)
    pgb, agb = _ptr_array([t.data_ptr() for t in gb]) if gb else (None, None)
    pb, pp, sb, sp = self.workspace()
    cmif_backward(self.handle, inp, pgm, pga, pgb, pp, self.persistent_bytes,
                  sp, self.scratch_bytes, self._stream())
    torch.cuda.current_stream(self.device).synchronize()
    del keep, agm, aga, agb
    return ga, gb


Plan.backward = _plan_backward


def _soft_cmif_function():
    import torch

    class SoftCMIF(torch.autograd.Function):
        """Differentiable soft CMIF maps of one image pair: forward returns
        the MI map [n_angles][S_h][S_w] (float64) of memberships A
        [Q_A][H_A][W_A] and B [Q_B][H_B][W_B] (float32, on the plan's
        device) under masks MA, MB (uint8 or None); backward runs the
        library's adjoint.  The plan must be SOFT with SAVE_FOR_BACKWARD and
        describe exactly one image pair.

        The adjoint reads the per-displacement state that the plan's last
        forward left in its persistent workspace.  Several forwards may share
        one plan before their backwards run (a loss summed over pairs of one
        size): each forward records the plan's forward count, and a backward
        whose forward is no longer the plan's last one first runs that
        forward again to restore its state."""

        @staticmethod
        def forward(ctx, A, B, plan, MA=None, MB=None):
            A = A.detach().contiguous()
            B = B.detach().contiguous()
            res = plan.compute(A, MA, B, MB, mi=True, n=False)
            ctx.plan = plan
            ctx.gen = plan._forward_gen
            ctx.save_for_backward(A, B)
            ctx.masks = (MA, MB)
            return res["mi"][0]

        @staticmethod
        def backward(ctx, grad_mi):
            A, B = ctx.saved_tensors
            MA, MB = ctx.masks
            need_a, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            if ctx.plan._forward_gen != ctx.gen:
                # another forward on this plan overwrote the saved state
                ctx.plan.compute(A, MA, B, MB, mi=False, n=False)
                ctx.plan.recomputed_forwards += 1
            ga, gb = ctx.plan.backward(A, MA, B, MB, grad_mi, want_a=need_a,
                                       want_b=need_b)
            return (ga[0] if ga else None, gb[0] if gb else None, None, None,
                    None)

    return SoftCMIF


def soft_cmif(A, B, plan, MA=None, MB=None):
    """MI maps of soft memberships with autograd support (see SoftCMIF)."""
    global SoftCMIF
    if SoftCMIF is None:
        SoftCMIF = _soft_cmif_function()
    return SoftCMIF.apply(A, B, plan, MA, MB)


SoftCMIF = None


def _listify(x, n=None):
    if isinstance(x, (list, tuple)):
        return list(x)
    if x is None:
        return [None] * (n or 1)
    return [x]


def _check_tensor(t, shape, device, name, dtype=None):
    import torch
    dtype = torch.uint8 if dtype is None else dtype
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be {dtype} of shape {shape}, got "
                         f"{t.dtype} {tuple(t.shape)}")
    if t.device.type != "cuda" or t.device.index != device:
        raise ValueError(f"{name} must be on cuda:{device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _stats_dict(stats_t):
    s = cmif_stats.from_buffer_copy(bytes(stats_t.cpu().numpy()))
    return dict(label_errors=s.label_errors, flagged_pairs=s.flagged_pairs,
                fallback_pairs=s.fallback_pairs,
                fallback_overflow=s.fallback_overflow,
                max_residual=s.max_residual,
                nonfinite_inputs=s.nonfinite_inputs,
                unresolved_pairs=s.unresolved_pairs)
