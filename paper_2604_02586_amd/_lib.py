"""ctypes binding of libtg (see include/tg.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtg.so")

c_f = ctypes.c_float
c_d = ctypes.c_double
c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_vp = ctypes.c_void_p

TG_MAX_VIEWS = 32
TG_ACC_STRIDE = 16
TG_REC_STRIDE = 8
TG_MAX_SLOTS = 8
TG_MAX_FRAMES = 4
TG_BIN_SORT_STATIC_BYTES = 64 << 20

STATUS = {0: "ok", 1: "invalid argument", 2: "misaligned buffer", 3: "workspace too small",
          4: "capacity overflow", 5: "HIP runtime error", 6: "request exceeds the memory budget",
          7: "unsupported size"}


class TGError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {STATUS.get(code, code)} ({code})")
        self.code = code


class Camera(ctypes.Structure):
    _fields_ = [("R", c_f * 9), ("t", c_f * 3), ("fx", c_f), ("fy", c_f), ("cx", c_f), ("cy", c_f),
                ("width", c_i32), ("height", c_i32), ("pad", c_f * 2)]


class Params(ctypes.Structure):
    _fields_ = [("near_z", c_f), ("dilation", c_f), ("extent", c_f), ("j_clamp", c_f),
                ("alpha_min", c_f), ("alpha_max", c_f), ("t_min", c_f), ("static_px", c_f),
                ("det_min", c_d), ("iso_min", c_d), ("wsum_min", c_d), ("wsum_total_min", c_d),
                ("pix_min", c_i32), ("views_min", c_i32), ("pix_total_min", c_i32),
                ("coarse_shift", c_i32), ("reg_k", c_i32), ("static_min_pix", c_i32), ("static_frac", c_d),
                ("static_views", c_i32), ("reserved", c_i32)]


class Gaussians(ctypes.Structure):
    _fields_ = [("means", c_vp), ("quats", c_vp), ("scales", c_vp), ("opacity", c_vp), ("sh", c_vp),
                ("sh_degree", c_i32), ("scale_mode", c_i32), ("opacity_mode", c_i32), ("pad", c_i32)]


class Splats(ctypes.Structure):
    _fields_ = [("rec", c_vp), ("cov2d", c_vp), ("rect", c_vp), ("key", c_vp), ("colors", c_vp),
                ("clamped", c_vp)]


class Bins(ctypes.Structure):
    _fields_ = [("order", c_vp), ("cell_ids", c_vp), ("cell_ranges", c_vp), ("n_pairs", c_vp),
                ("overflow", c_vp), ("capacity", c_i64)]


class AccSlot(ctypes.Structure):
    _fields_ = [("s", c_vp), ("bins", c_vp), ("cams", c_vp), ("N", c_i64), ("V", c_i32), ("F", c_i32),
                ("disp", c_vp * TG_MAX_FRAMES), ("vis", c_vp * TG_MAX_FRAMES), ("acc", c_vp * TG_MAX_FRAMES),
                ("t_final", c_vp)]


class UpdSlot(ctypes.Structure):
    _fields_ = [("s", c_vp), ("g_in", c_vp), ("cams", c_vp), ("N", c_i64), ("V", c_i32), ("F", c_i32),
                ("acc", c_vp * TG_MAX_FRAMES), ("g_out", c_vp * TG_MAX_FRAMES), ("status", c_vp * TG_MAX_FRAMES)]


TG_SERVE_HOST_BYTES = 4096


class ServeConfig(ctypes.Structure):
    _fields_ = [("arena", c_vp), ("arena_bytes", ctypes.c_size_t), ("host_scratch", c_vp),
                ("compute_stream", c_vp), ("copy_stream", c_vp), ("max_inflight", c_i32), ("max_frames", c_i32),
                ("max_slots", c_i32), ("dry", c_i32)]


class ServeDone(ctypes.Structure):
    _fields_ = [("stream_id", c_i64), ("frame_id", c_i64), ("step", c_i64), ("arrival", c_d), ("done", c_d),
                ("status", c_i32), ("entry", c_i32)]


class ServeStats(ctypes.Structure):
    _fields_ = [(k, c_i64) for k in ("steps", "entries", "frames", "rebins", "max_admitted", "arena_used",
                                       "arena_peak", "waiting_streams", "admitted_streams", "inflight_steps")]


_lib = None


def lib():
    """Load libtg.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libtg.so not found at {LIB_PATH}; run __graft_entry__.build() "
                          "(or python paper_2604_02586_amd/build.py) first")
    L = ctypes.CDLL(LIB_PATH)
    P = c_vp
    st = c_i32
    sig = {
        "tg_abi_version": ([], c_i32),
        "tg_status_string": ([c_i32], ctypes.c_char_p),
        "tg_default_params": ([P], None),
        "tg_num_cells": ([P, c_i32, c_i64, P], c_i64),
        "tg_num_tiles": ([P, c_i32], c_i64),
        "tg_preprocess": ([P, c_i64, P, c_i32, P, P, P], st),
        "tg_acc_zero": ([P, c_i64, P], st),
        "tg_bin_sort": ([P, c_i64, P, c_i32, P, P, P, P, P], st),
        "tg_bin_sort_static": ([P, c_i64, P, c_i32, P, P, P], st),
        "tg_splat_accumulate": ([P, P, c_i64, P, c_i32, P, P, P, P, P, P, P], st),
        "tg_splat_accumulate_batch": ([P, c_i32, P, P, P], st),
        "tg_regularize": ([P, P, P, P, c_i64, c_i32, P, P, P, P, P, P], st),
        "tg_solve_views": ([P, P, c_i64, c_i32, P, P, P, P, P, P], st),
        "tg_triangulate": ([P, P, P, P, P, P, c_i64, P, c_i32, P, P, P, P], st),
        "tg_solve_triangulate": ([P, P, P, c_i64, P, c_i32, P, P, P, P], st),
        "tg_solve_triangulate_batch": ([P, c_i32, P, P], st),
        "tg_bin_expand": ([P, P, c_i64, P, c_i32, P, P, P, c_i64, P, P, P, P], st),
        "tg_raster_fwd": ([P, P, c_i64, P, c_i32, P, P, P, P, P, P], st),
        "tg_raster_bwd": ([P, P, c_i64, P, c_i32, P, P, P, P, P, P], st),
        "tg_raster_fwd_counted": ([P, P, c_i64, P, c_i32, P, P, P, P, P, P, P], st),
        "tg_raster_bwd_counted": ([P, P, c_i64, P, c_i32, P, P, P, P, P, P, P], st),
        "tg_project_bwd": ([P, P, c_i64, P, c_i32, P, P, P, P], st),
        "tg_l1_loss_grad": ([P, P, c_i64, c_f, P, P, P], st),
        "tg_scale_by": ([P, P, c_i64, P, P], st),
        "tg_scalar_affine": ([P, P, c_i32, P, c_f, P], st),
        "tg_ssim_loss_grad": ([P, P, c_i32, c_i32, c_i32, c_f, P, P, P, P, P], st),
        "tg_adam_step": ([P, P, P, P, c_i64, c_f, c_f, c_f, c_f, c_i32, P], st),
        "tg_adam_step_rows": ([P, P, P, P, c_i64, c_i32, c_i32, c_f, c_f, c_f, c_f, c_f, c_i32, P], st),
        "tg_serve_create": ([P, P, P], st),
        "tg_serve_destroy": ([P], st),
        "tg_serve_now": ([P], c_d),
        "tg_serve_open_stream": ([P, P, c_i64, P, c_i32, c_d, P], st),
        "tg_serve_submit": ([P, c_i64, c_i64, P, P, c_i32, P, P, c_d], st),
        "tg_serve_close_stream": ([P, c_i64], st),
        "tg_serve_step": ([P, P], st),
        "tg_serve_poll": ([P, P, c_i32, P], st),
        "tg_serve_get_stats": ([P, P], st),
        "tg_serve_dry_complete": ([P, c_i32, c_d], st),
        "tg_serve_stream_bytes": ([P, c_i32, c_i64, P, P, P, P], st),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def exported_symbols():
    return [n for n in ("tg_abi_version", "tg_status_string", "tg_default_params", "tg_num_cells",
                        "tg_num_tiles", "tg_preprocess", "tg_acc_zero", "tg_bin_sort", "tg_bin_sort_static", "tg_splat_accumulate",
                        "tg_splat_accumulate_batch", "tg_regularize", "tg_solve_views", "tg_triangulate",
                        "tg_solve_triangulate", "tg_solve_triangulate_batch", "tg_bin_expand", "tg_raster_fwd", "tg_raster_bwd",
                        "tg_raster_fwd_counted", "tg_raster_bwd_counted",
                        "tg_project_bwd", "tg_l1_loss_grad", "tg_scale_by", "tg_scalar_affine", "tg_ssim_loss_grad",
                        "tg_adam_step",
                        "tg_adam_step_rows", "tg_serve_create", "tg_serve_destroy", "tg_serve_now",
                        "tg_serve_open_stream", "tg_serve_submit", "tg_serve_close_stream", "tg_serve_step",
                        "tg_serve_poll", "tg_serve_get_stats", "tg_serve_dry_complete", "tg_serve_stream_bytes")]


def check(fn, code):
    if code != 0:
        raise TGError(fn, code)


def default_params() -> Params:
    p = Params()
    lib().tg_default_params(ctypes.byref(p))
    return p


def cameras(cams) -> ctypes.Array:
    """Host camera array from synth.Camera objects or a [V,20] float32 array."""
    import numpy as np
    if isinstance(cams, np.ndarray):
        arr = np.ascontiguousarray(cams, np.float32)
        out = (Camera * arr.shape[0])()
        ctypes.memmove(out, arr.ctypes.data, arr.nbytes)
        return out
    out = (Camera * len(cams))()
    for i, c in enumerate(cams):
        out[i].R[:] = [float(x) for x in c.R.reshape(-1)]
        out[i].t[:] = [float(x) for x in c.t]
        out[i].fx, out[i].fy, out[i].cx, out[i].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        out[i].width, out[i].height = int(c.W), int(c.H)
    return out
