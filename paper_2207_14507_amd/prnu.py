"""ctypes binding of the C ABI in include/prnu.h (argument marshalling only).

Every function keeps the C name.  Host inputs are numpy arrays; device inputs are
torch CUDA/HIP tensors (their data pointer and current stream are passed through).
The library must have been built (``paper_2207_14507_amd.build``); importing this
module fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprnu.so")

PRNU_OK, PRNU_PENDING = 0, 1
PRNU_E_ARG, PRNU_E_SHAPE, PRNU_E_NOMEM, PRNU_E_DEVICE = -1, -2, -3, -4
PRNU_E_HANDLE, PRNU_E_BUSY, PRNU_E_NONFINITE, PRNU_E_CANCELLED = -5, -6, -7, -8
PRNU_F32, PRNU_BF16 = 0, 1
PRNU_NUM_KERNELS = 4
PRNU_FLAG_NO_GRAPHS, PRNU_FLAG_NO_AUTOTUNE = 1, 2

EXPORTED = [
    "prnu_create", "prnu_destroy", "prnu_status_string", "prnu_last_error", "prnu_supported_lengths",
    "prnu_open_fingerprint", "prnu_close_fingerprint", "prnu_search_frames", "prnu_score_grid",
    "prnu_submit_video", "prnu_poll", "prnu_cancel", "prnu_tune", "prnu_graph_stats", "prnu_profile_enable",
    "prnu_profile_read", "prnu_score_transforms", "prnu_search_with_transform", "prnu_candidates",
    "prnu_check_opts", "prnu_estimate_fingerprint", "prnu_extract_residuals", "prnu_score_grid_noalloc",
]


class prnu_config(C.Structure):
    _fields_ = [("device", C.c_int32), ("hbm_budget_bytes", C.c_uint64), ("max_slots", C.c_int32),
                ("tune_cache_path", C.c_char_p), ("flags", C.c_uint32)]


class prnu_grid(C.Structure):
    _fields_ = [("n_scale", C.c_int32), ("scale_lo", C.c_double), ("scale_hi", C.c_double),
                ("n_rot", C.c_int32), ("rot_lo_deg", C.c_double), ("rot_hi_deg", C.c_double)]


class prnu_search_opts(C.Structure):
    _fields_ = [("full", prnu_grid), ("shift_radius", C.c_int32), ("exclusion", C.c_int32),
                ("warm", C.c_int32), ("local_n_scale", C.c_int32), ("local_n_rot", C.c_int32),
                ("local_dscale", C.c_double), ("local_drot_deg", C.c_double), ("fallback_pce", C.c_double),
                ("has_init", C.c_int32), ("init_scale", C.c_double), ("init_rot_deg", C.c_double),
                ("tau", C.c_double), ("refine", C.c_int32), ("refine_half", C.c_int32),
                ("refine_max_iter", C.c_int32), ("refine_scale_step", C.c_double), ("refine_rot_step", C.c_double),
                ("refine_rot_lo_deg", C.c_double), ("refine_rot_hi_deg", C.c_double)]


class prnu_frames(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("frame_scale", C.c_void_p),
                ("n_frames", C.c_int32), ("height", C.c_int32), ("width", C.c_int32),
                ("frame_stride", C.c_int64), ("row_stride", C.c_int64), ("on_device", C.c_int32),
                ("stream", C.c_void_p)]


class prnu_frame_result(C.Structure):
    _fields_ = [("pce", C.c_double), ("rho", C.c_double), ("scale", C.c_double), ("rot_deg", C.c_double),
                ("dx", C.c_int32), ("dy", C.c_int32), ("cand_index", C.c_int32), ("fell_back", C.c_int32),
                ("n_evaluated", C.c_int32), ("status", C.c_int32), ("iterations", C.c_int32),
                ("used_init", C.c_int32)]


class prnu_video_summary(C.Structure):
    _fields_ = [("mean_pce", C.c_double), ("decision", C.c_int32), ("n_frames", C.c_int32),
                ("queue_s", C.c_double), ("latency_s", C.c_double)]


class prnu_kernel_stats(C.Structure):
    _fields_ = [("name", C.c_char_p), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("candidates", C.c_int64), ("algo_bytes", C.c_double)]


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2207_14507_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    sigs = {
        "prnu_create": (C.c_int, [P(prnu_config), P(C.c_void_p)]),
        "prnu_destroy": (None, [C.c_void_p]),
        "prnu_status_string": (C.c_char_p, [C.c_int]),
        "prnu_last_error": (C.c_char_p, []),
        "prnu_supported_lengths": (C.c_int32, [P(C.c_int32), C.c_int32]),
        "prnu_open_fingerprint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_int32,
                                            C.c_void_p, P(C.c_uint64)]),
        "prnu_close_fingerprint": (C.c_int, [C.c_void_p, C.c_uint64]),
        "prnu_search_frames": (C.c_int, [C.c_void_p, C.c_uint64, P(prnu_frames), P(prnu_search_opts),
                                         P(prnu_frame_result), P(prnu_video_summary)]),
        "prnu_score_grid": (C.c_int, [C.c_void_p, C.c_uint64, P(prnu_frames), C.c_int32, P(prnu_search_opts),
                                      P(C.c_double), P(C.c_double), P(C.c_int32), P(C.c_int32)]),
        "prnu_score_grid_noalloc": (C.c_int, [C.c_void_p, C.c_uint64, P(prnu_frames), C.c_int32,
                                              P(prnu_search_opts), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
        "prnu_submit_video": (C.c_int, [C.c_void_p, C.c_uint64, P(prnu_frames), P(prnu_search_opts),
                                        P(C.c_uint64)]),
        "prnu_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int32, P(prnu_frame_result), P(prnu_video_summary)]),
        "prnu_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
        "prnu_score_transforms": (C.c_int, [C.c_void_p, C.c_uint64, P(prnu_frames), C.c_int32, P(C.c_double),
                                            C.c_int32, C.c_int32, P(C.c_double), P(C.c_double), P(C.c_int32),
                                            P(C.c_int32)]),
        "prnu_search_with_transform": (C.c_int, [C.c_void_p, C.c_uint64, P(prnu_frames), P(prnu_search_opts),
                                                 P(C.c_double), P(prnu_frame_result), P(prnu_video_summary)]),
        "prnu_estimate_fingerprint": (C.c_int, [C.c_void_p, P(prnu_frames), P(prnu_frames), C.c_void_p, C.c_int32]),
        "prnu_extract_residuals": (C.c_int, [C.c_void_p, P(prnu_frames), C.c_double, C.c_void_p, C.c_int32]),
        "prnu_candidates": (C.c_int32, [P(prnu_search_opts), C.c_int32, C.c_int32, C.c_double, C.c_double,
                                        P(C.c_double), C.c_int32]),
        "prnu_check_opts": (C.c_int, [P(prnu_search_opts)]),
        "prnu_tune": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int, P(C.c_int32), P(C.c_int32),
                                P(C.c_double), P(C.c_int32)]),
        "prnu_graph_stats": (C.c_int, [C.c_void_p, P(C.c_int64), P(C.c_int64)]),
        "prnu_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
        "prnu_profile_read": (C.c_int, [C.c_void_p, P(prnu_kernel_stats)]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


class PrnuError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.prnu_last_error().decode(errors="replace")
        super().__init__(f"{where}: {lib.prnu_status_string(status).decode()} ({status}): {msg}")


def _check(st: int, where: str) -> int:
    if st < 0:
        raise PrnuError(st, where)
    return st


# ---------------------------------------------------------------------------
# Option helpers.

def make_grid(n_scale=41, scale_lo=0.85, scale_hi=1.15, n_rot=21, rot_lo=-2.0, rot_hi=2.0) -> prnu_grid:
    return prnu_grid(int(n_scale), float(scale_lo), float(scale_hi), int(n_rot), float(rot_lo), float(rot_hi))


def make_opts(grid=(41, 0.85, 1.15, 21, -2.0, 2.0), radius=64, warm=False, local=(9, 9, 0.005, 0.1),
              fallback_pce=60.0, init: Optional[Tuple[float, float]] = None, tau=19.5,
              exclusion=11, refine=None) -> prnu_search_opts:
    """refine: None (grid search) or a dict with any of half, max_iter, scale_step,
    rot_step, rot_lo, rot_hi (the paper's values 5, 3, 0.01, 0.1, -5, 5 by default)."""
    o = prnu_search_opts()
    o.full = make_grid(*grid)
    o.shift_radius = int(radius)
    o.exclusion = int(exclusion)
    o.warm = int(warm)
    o.local_n_scale, o.local_n_rot = int(local[0]), int(local[1])
    o.local_dscale, o.local_drot_deg = float(local[2]), float(local[3])
    o.has_init = int(init is not None)
    o.init_scale, o.init_rot_deg = (float(init[0]), float(init[1])) if init is not None else (1.0, 0.0)
    o.fallback_pce = float(fallback_pce)
    o.tau = float(tau)
    r = dict(half=5, max_iter=3, scale_step=0.01, rot_step=0.1, rot_lo=-5.0, rot_hi=5.0)
    if refine is not None:
        r.update(refine)
    o.refine = int(refine is not None)
    o.refine_half, o.refine_max_iter = int(r["half"]), int(r["max_iter"])
    o.refine_scale_step, o.refine_rot_step = float(r["scale_step"]), float(r["rot_step"])
    o.refine_rot_lo_deg, o.refine_rot_hi_deg = float(r["rot_lo"]), float(r["rot_hi"])
    return o


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _stream_of(t) -> int:
    import torch
    return torch.cuda.current_stream(t.device).cuda_stream


def _check_device_out(out, n: int, where: str, align: int = 4) -> None:
    """An output the library writes through a raw device pointer: a contiguous float32
    tensor on the device holding exactly n values."""
    import torch
    if not (_is_torch(out) and out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()):
        raise TypeError(f"{where}: out must be a contiguous float32 tensor on the device")
    if out.numel() != n:
        raise ValueError(f"{where}: out holds {out.numel()} values, the call writes {n}")
    if out.data_ptr() % align:
        raise ValueError(f"{where}: out must be {align}-byte aligned")


def make_frames(data, scales=None, keep: list = None) -> prnu_frames:
    """frames for a (F, M, N) or (M, N) array: numpy float32 / uint16 (bf16 bits) on the
    host, or a torch float32 / bfloat16 / int16 tensor on the device.  ``keep`` collects
    objects that must outlive the call."""
    keep = keep if keep is not None else []
    f = prnu_frames()
    if _is_torch(data):
        import torch
        t = data if data.dim() == 3 else data.unsqueeze(0)
        if t.dtype == torch.float32:
            f.dtype = PRNU_F32
        elif t.dtype in (torch.bfloat16, torch.int16, torch.uint16):
            f.dtype = PRNU_BF16
        else:
            raise TypeError(f"unsupported tensor dtype {t.dtype}")
        if t.stride(2) != 1:
            raise ValueError("rows must be contiguous")
        f.data = t.data_ptr()
        f.on_device = int(t.is_cuda)
        f.stream = _stream_of(t) if t.is_cuda else None
        f.n_frames, f.height, f.width = t.shape
        f.frame_stride, f.row_stride = t.stride(0), t.stride(1)
        keep.append(t)
        if f.dtype == PRNU_BF16:
            s = scales if _is_torch(scales) else torch.as_tensor(np.asarray(scales, np.float32), device=t.device)
            s = s.to(torch.float32).contiguous()
            keep.append(s)
            f.frame_scale = s.data_ptr()
    else:
        a = np.asarray(data)
        if a.ndim == 2:
            a = a[None]
        if a.dtype == np.float32:
            f.dtype = PRNU_F32
        elif a.dtype == np.uint16:
            f.dtype = PRNU_BF16
        else:
            raise TypeError(f"unsupported array dtype {a.dtype}")
        a = np.ascontiguousarray(a)
        keep.append(a)
        f.data = a.ctypes.data
        f.on_device = 0
        f.n_frames, f.height, f.width = a.shape
        f.frame_stride, f.row_stride = a.shape[1] * a.shape[2], a.shape[2]
        if f.dtype == PRNU_BF16:
            s = np.ascontiguousarray(np.asarray(scales, dtype=np.float32).reshape(-1))
            keep.append(s)
            f.frame_scale = s.ctypes.data
    return f


# ---------------------------------------------------------------------------
# Entry points (C names).

def prnu_create(device: int = 0, hbm_budget_bytes: int = 0, max_slots: int = 0,
                tune_cache_path: Optional[str] = None, flags: int = 0) -> C.c_void_p:
    cfg = prnu_config(device, hbm_budget_bytes, max_slots,
                      tune_cache_path.encode() if tune_cache_path else None, int(flags))
    ctx = C.c_void_p()
    _check(lib.prnu_create(C.byref(cfg), C.byref(ctx)), "prnu_create")
    return ctx


def prnu_destroy(ctx) -> None:
    lib.prnu_destroy(ctx)


def prnu_supported_lengths() -> list:
    buf = (C.c_int32 * 64)()
    n = lib.prnu_supported_lengths(buf, 64)
    return list(buf)[:n]


def prnu_open_fingerprint(ctx, K) -> int:
    out = C.c_uint64()
    if _is_torch(K):
        import torch
        if K.dtype != torch.float32 or K.dim() != 2 or K.stride(1) != 1:
            raise ValueError("fingerprint must be a 2-D float32 tensor with contiguous rows")
        st = lib.prnu_open_fingerprint(ctx, K.data_ptr(), K.shape[0], K.shape[1], K.stride(0), int(K.is_cuda),
                                       _stream_of(K) if K.is_cuda else None, C.byref(out))
    else:
        a = np.ascontiguousarray(np.asarray(K, dtype=np.float32))
        if a.ndim != 2:
            raise ValueError("fingerprint must be 2-D")
        st = lib.prnu_open_fingerprint(ctx, a.ctypes.data, a.shape[0], a.shape[1], a.shape[1], 0, None,
                                       C.byref(out))
    _check(st, "prnu_open_fingerprint")
    return out.value


def prnu_close_fingerprint(ctx, fp: int) -> None:
    _check(lib.prnu_close_fingerprint(ctx, fp), "prnu_close_fingerprint")


def prnu_search_frames(ctx, fp: int, frames, opts: prnu_search_opts, scales=None):
    """Returns (list of prnu_frame_result, prnu_video_summary)."""
    keep = []
    fr = make_frames(frames, scales, keep)
    out = (prnu_frame_result * max(1, fr.n_frames))()
    summ = prnu_video_summary()
    _check(lib.prnu_search_frames(ctx, fp, C.byref(fr), C.byref(opts), out, C.byref(summ)), "prnu_search_frames")
    return list(out)[:fr.n_frames], summ


def prnu_score_grid(ctx, fp: int, frames, frame: int, opts: prnu_search_opts, scales=None):
    """Per-candidate (pce, rho, dx, dy) arrays of the full grid for one frame."""
    keep = []
    fr = make_frames(frames, scales, keep)
    n = opts.full.n_scale * opts.full.n_rot
    pce = np.zeros(n, np.float64)
    rho = np.zeros(n, np.float64)
    dx = np.zeros(n, np.int32)
    dy = np.zeros(n, np.int32)
    P = C.POINTER
    _check(lib.prnu_score_grid(ctx, fp, C.byref(fr), frame, C.byref(opts),
                               pce.ctypes.data_as(P(C.c_double)), rho.ctypes.data_as(P(C.c_double)),
                               dx.ctypes.data_as(P(C.c_int32)), dy.ctypes.data_as(P(C.c_int32))),
           "prnu_score_grid")
    return pce, rho, dx, dy


def prnu_score_grid_noalloc(ctx, fp: int, frames, frame: int, opts: prnu_search_opts, pce, rho=None, dx=None,
                            dy=None, scales=None) -> None:
    """prnu_score_grid into device tensors, with no allocation: frames (and scales) are
    device tensors; pce and rho contiguous float64, dx and dy contiguous int32 device
    tensors of n_scale * n_rot entries (rho, dx, dy optional).  Asynchronous on the
    frames' stream."""
    import torch
    n = opts.full.n_scale * opts.full.n_rot
    outs = []
    for name, t, dt in (("pce", pce, torch.float64), ("rho", rho, torch.float64), ("dx", dx, torch.int32),
                        ("dy", dy, torch.int32)):
        if t is None:
            if name == "pce":
                raise TypeError("pce is required")
            outs.append(None)
            continue
        if not (_is_torch(t) and t.is_cuda and t.dtype == dt and t.is_contiguous() and t.numel() == n):
            raise TypeError(f"prnu_score_grid_noalloc: {name} must be a contiguous {dt} device tensor of {n} entries")
        outs.append(t.data_ptr())
    if not _is_torch(frames) or not frames.is_cuda:
        raise TypeError("prnu_score_grid_noalloc: frames must be a device tensor")
    keep = []
    fr = make_frames(frames, scales, keep)
    _check(lib.prnu_score_grid_noalloc(ctx, fp, C.byref(fr), frame, C.byref(opts), *outs), "prnu_score_grid_noalloc")


# Frame count of every video submitted through this binding and not yet retired, so that
# poll's result buffer always holds the video's results whatever n_frames the caller gives.
_video_frames = {}


def prnu_submit_video(ctx, fp: int, frames, opts: prnu_search_opts, scales=None) -> int:
    keep = []
    fr = make_frames(frames, scales, keep)
    t = C.c_uint64()
    _check(lib.prnu_submit_video(ctx, fp, C.byref(fr), C.byref(opts), C.byref(t)), "prnu_submit_video")
    _video_frames[(ctx.value, t.value)] = fr.n_frames
    return t.value


def prnu_poll(ctx, ticket: int, n_frames: int, timeout_ms: int = -1):
    """Returns (status, results or None, summary or None); status PRNU_PENDING while
    the video is in flight.  The results list has the video's frame count."""
    key = (ctx.value, ticket)
    n = _video_frames.get(key, n_frames)
    out = (prnu_frame_result * max(1, n, n_frames))()
    summ = prnu_video_summary()
    st = lib.prnu_poll(ctx, ticket, timeout_ms, out, C.byref(summ))
    if st == PRNU_PENDING:
        return st, None, None
    _video_frames.pop(key, None)  # retired (done, failed, cancelled or unknown)
    _check(st, "prnu_poll")
    return st, list(out)[:n], summ


def prnu_cancel(ctx, ticket: int) -> None:
    _check(lib.prnu_cancel(ctx, ticket), "prnu_cancel")


def prnu_profile_enable(ctx, enable: bool = True) -> None:
    _check(lib.prnu_profile_enable(ctx, int(enable)), "prnu_profile_enable")


def prnu_score_transforms(ctx, fp: int, frames, frame: int, T, radius: int, scales=None):
    """Per-transform (pce, rho, dx, dy) arrays for general Eq. (4) transforms T of shape
    (n, 3, 3) (centred coordinates) on one frame."""
    keep = []
    fr = make_frames(frames, scales, keep)
    Tm = np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(-1, 9))
    n = Tm.shape[0]
    pce = np.zeros(n, np.float64)
    rho = np.zeros(n, np.float64)
    dx = np.zeros(n, np.int32)
    dy = np.zeros(n, np.int32)
    P = C.POINTER
    _check(lib.prnu_score_transforms(ctx, fp, C.byref(fr), frame, Tm.ctypes.data_as(P(C.c_double)), n, int(radius),
                                     pce.ctypes.data_as(P(C.c_double)), rho.ctypes.data_as(P(C.c_double)),
                                     dx.ctypes.data_as(P(C.c_int32)), dy.ctypes.data_as(P(C.c_int32))),
           "prnu_score_transforms")
    return pce, rho, dx, dy


def prnu_search_with_transform(ctx, fp: int, frames, opts: prnu_search_opts, H, scales=None):
    """Refinement started from per-frame transforms H (n_frames, 3, 3) where they score
    higher than the frames as they are.  Returns (results, summary)."""
    keep = []
    fr = make_frames(frames, scales, keep)
    Hm = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(-1, 9))
    out = (prnu_frame_result * max(1, fr.n_frames))()
    summ = prnu_video_summary()
    _check(lib.prnu_search_with_transform(ctx, fp, C.byref(fr), C.byref(opts),
                                          Hm.ctypes.data_as(C.POINTER(C.c_double)), out, C.byref(summ)),
           "prnu_search_with_transform")
    return list(out)[:fr.n_frames], summ


def prnu_estimate_fingerprint(ctx, images, residuals, out=None):
    """Eq. (2) from (L, M, N) float32 images and residuals (numpy or torch).  Returns a
    numpy array, or fills ``out`` (a contiguous float32 torch tensor on the device)."""
    keep = []
    fi = make_frames(images, None, keep)
    fw = make_frames(residuals, None, keep)
    if out is None:
        K = np.zeros((fi.height, fi.width), np.float32)
        _check(lib.prnu_estimate_fingerprint(ctx, C.byref(fi), C.byref(fw), K.ctypes.data, 0),
               "prnu_estimate_fingerprint")
        return K
    _check_device_out(out, fi.height * fi.width, "prnu_estimate_fingerprint", align=16)
    _check(lib.prnu_estimate_fingerprint(ctx, C.byref(fi), C.byref(fw), out.data_ptr(), 1), "prnu_estimate_fingerprint")
    return out


def prnu_extract_residuals(ctx, images, sigma0: float = 3.0, out=None):
    """Noise residuals W(I) = I - F(I) of (L, M, N) float32 images (numpy or torch).
    Returns a numpy array, or fills ``out`` (a contiguous float32 torch tensor of the
    same shape on the device)."""
    keep = []
    fi = make_frames(images, None, keep)
    if out is None:
        W = np.zeros((fi.n_frames, fi.height, fi.width), np.float32)
        _check(lib.prnu_extract_residuals(ctx, C.byref(fi), float(sigma0), W.ctypes.data, 0), "prnu_extract_residuals")
        return W
    _check_device_out(out, fi.n_frames * fi.height * fi.width, "prnu_extract_residuals")
    _check(lib.prnu_extract_residuals(ctx, C.byref(fi), float(sigma0), out.data_ptr(), 1), "prnu_extract_residuals")
    return out


def prnu_candidates(opts: prnu_search_opts, kind: int, iteration: int = 1, centre=(1.0, 0.0)) -> list:
    """(scale, rotation) pairs of a candidate grid: kind 0 full, 1 local, 2 refinement."""
    n = _check(lib.prnu_candidates(C.byref(opts), int(kind), int(iteration), float(centre[0]), float(centre[1]),
                                   None, 0), "prnu_candidates")
    out = np.zeros(2 * max(n, 1), np.float64)
    _check(lib.prnu_candidates(C.byref(opts), int(kind), int(iteration), float(centre[0]), float(centre[1]),
                               out.ctypes.data_as(C.POINTER(C.c_double)), n), "prnu_candidates")
    return [(float(out[2 * i]), float(out[2 * i + 1])) for i in range(n)]


def prnu_check_opts(opts: prnu_search_opts) -> int:
    """The status a search would return for these options alone."""
    return lib.prnu_check_opts(C.byref(opts))


def prnu_tune(ctx, height: int, width: int, radius: int, dtype: int = PRNU_F32) -> dict:
    """Launch schedule of a shape (tuned now if it is not yet known)."""
    b, o, f = C.c_int32(), C.c_int32(), C.c_int32()
    ns = C.c_double()
    _check(lib.prnu_tune(ctx, int(height), int(width), int(radius), int(dtype), C.byref(b), C.byref(o),
                         C.byref(ns), C.byref(f)), "prnu_tune")
    return dict(batch=b.value, order=o.value, ns_per_candidate=ns.value, from_cache=bool(f.value))


def prnu_graph_stats(ctx) -> Tuple[int, int]:
    """(captures, replays) of the synchronous search's launch graphs."""
    c, r = C.c_int64(), C.c_int64()
    _check(lib.prnu_graph_stats(ctx, C.byref(c), C.byref(r)), "prnu_graph_stats")
    return c.value, r.value


def prnu_profile_read(ctx) -> list:
    out = (prnu_kernel_stats * PRNU_NUM_KERNELS)()
    _check(lib.prnu_profile_read(ctx, out), "prnu_profile_read")
    return [dict(name=s.name.decode(), launches=s.launches, total_ms=s.total_ms, candidates=s.candidates,
                 algo_bytes=s.algo_bytes) for s in out]
