"""ctypes binding of libcgv2r.so (the C ABI declared in include/cgv2r.h).

Argument marshalling only: every step of the rasterizer runs in the library's HIP kernels.
Loading fails loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcgv2r.so")

CGV2_OK, CGV2_EINVAL, CGV2_EWORKSPACE, CGV2_EUNSUPPORTED, CGV2_EHIP = 0, -1, -2, -3, -4
NOALLOC_SCRATCH_BYTES = 16 << 20  # CGV2_NOALLOC_SCRATCH_BYTES
TILE = 16
REC_FLOATS = 24
F_VISIBLE, F_NEAR, F_OPACITY, F_BEHIND, F_NONFINITE, F_LOWPASS = 1, 2, 4, 8, 16, 32

EXPORTS = ["cgv2_project", "cgv2_project_compact", "cgv2_bin_sort_workspace", "cgv2_bin_sort", "cgv2_render_fwd", "cgv2_loss_workspace",
           "cgv2_loss", "cgv2_render_bwd_workspace", "cgv2_render_bwd", "cgv2_render_bwd_records",
           "cgv2_project_bwd", "cgv2_zero_grads", "cgv2_densify_workspace",
           "cgv2_densify_stats", "cgv2_densify_stats_noalloc", "cgv2_render_count", "cgv2_contribution_workspace", "cgv2_contribution",
           "cgv2_trim_workspace", "cgv2_trim_mask", "cgv2_densify_plan_workspace", "cgv2_densify_plan",
           "cgv2_densify_apply", "cgv2_densify_gather", "cgv2_visibility_workspace", "cgv2_visibility_count",
           "cgv2_crop_workspace", "cgv2_crop_volume", "cgv2_compact_order_workspace", "cgv2_compact_order",
           "cgv2_vq_init", "cgv2_vq_assign_workspace", "cgv2_vq_assign", "cgv2_vq_update_workspace", "cgv2_vq_update",
           "cgv2_compact_write", "cgv2_strerror", "cgv2_last_hip_error"]

P = ctypes.c_void_p


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("R", ctypes.c_float * 9),
                ("t", ctypes.c_float * 3), ("znear", ctypes.c_float), ("bg", ctypes.c_float * 3)]


class Surfels(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("mean", P), ("log_scale", P), ("quat", P),
                ("opacity_logit", P), ("sh", P)]


class SurfelsCompact(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_full", ctypes.c_int64), ("sh_degree", ctypes.c_int32),
                ("codebook_size", ctypes.c_int32), ("mean", P), ("log_scale", P), ("quat", P),
                ("opacity_logit", P), ("sh", P), ("code", P), ("codebook", P)]


class CompactOut(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("mean", P), ("log_scale", P), ("quat", P),
                ("opacity_logit", P), ("sh", P), ("codebook", P)]


class Proj(ctypes.Structure):
    _fields_ = [("rec", P), ("rect", P), ("radius", P), ("flags", P), ("visible", P), ("visible_start", P)]


class Bins(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("ids", P), ("ranges", P), ("status", P), ("needed", P), ("order", P)]


class Image(ctypes.Structure):
    _fields_ = [("rgb", P), ("depth", P), ("depth_med", P), ("normal", P), ("alpha", P), ("T_final", P),
                ("last", P), ("med", P), ("qmask", P)]


class ImageGrad(ctypes.Structure):
    _fields_ = [("d_rgb", P), ("d_depth", P), ("d_depth_med", P), ("d_normal", P), ("d_alpha", P),
                ("d_rgb_ssim", P)]


class Grads(ctypes.Structure):
    _fields_ = [("d_mean", P), ("d_log_scale", P), ("d_quat", P), ("d_opacity_logit", P), ("d_sh", P),
                ("g_view_total", P), ("g_view_ssim", P)]


class DensifyParams(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_float), ("eta_min", ctypes.c_float), ("grad_threshold", ctypes.c_float)]


class DensifyState(ctypes.Structure):
    _fields_ = [("accum_dgd", P), ("accum_total", P), ("max_radius", P), ("denom", P), ("mask", P),
                ("counters", P), ("scale", P)]


class ActionParams(ctypes.Structure):
    _fields_ = [("dense_scale", ctypes.c_float), ("min_opacity", ctypes.c_float), ("split_shrink", ctypes.c_float)]


class SurfelsOut(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("mean", P), ("log_scale", P), ("quat", P),
                ("opacity_logit", P), ("sh", P)]


_lib = None


class Cgv2Error(RuntimeError):
    pass


def lib():
    """The loaded library with typed entry points (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise Cgv2Error(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "cgv2_project": (ctypes.c_int, [ctypes.POINTER(Surfels), ctypes.POINTER(Camera), i32, ctypes.POINTER(Proj), P]),
        "cgv2_project_compact": (ctypes.c_int, [ctypes.POINTER(SurfelsCompact), ctypes.POINTER(Camera), i32,
                                                ctypes.POINTER(Proj), P]),
        "cgv2_bin_sort_workspace": (sz, [i64, i32, i32, i64]),
        "cgv2_bin_sort": (ctypes.c_int, [ctypes.POINTER(Proj), ctypes.POINTER(Camera), i32, i64, ctypes.POINTER(Bins),
                                         P, sz, P]),
        "cgv2_render_fwd": (ctypes.c_int, [ctypes.POINTER(Proj), ctypes.POINTER(Bins), ctypes.POINTER(Camera), i32, i64,
                                           ctypes.POINTER(Image), P]),
        "cgv2_render_count": (ctypes.c_int, [ctypes.POINTER(Proj), ctypes.POINTER(Bins), ctypes.POINTER(Camera), i32,
                                             i64, P, P]),
        "cgv2_loss_workspace": (sz, [i32, i32, i32]),
        "cgv2_loss": (ctypes.c_int, [P, P, i32, i32, i32, ctypes.c_float, P, P, P, P, sz, P]),
        "cgv2_render_bwd_workspace": (sz, [i64, i32]),
        "cgv2_render_bwd": (ctypes.c_int, [ctypes.POINTER(Surfels), ctypes.POINTER(Proj), ctypes.POINTER(Bins),
                                           ctypes.POINTER(Camera), i32, ctypes.POINTER(Image),
                                           ctypes.POINTER(ImageGrad), ctypes.POINTER(Grads), P, sz, P]),
        "cgv2_render_bwd_records": (ctypes.c_int, [ctypes.POINTER(Proj), ctypes.POINTER(Bins), ctypes.POINTER(Camera),
                                                   i32, i64, ctypes.POINTER(Image), ctypes.POINTER(ImageGrad), P, sz,
                                                   P]),
        "cgv2_project_bwd": (ctypes.c_int, [ctypes.POINTER(Surfels), ctypes.POINTER(Proj), ctypes.POINTER(Camera), i32,
                                            P, sz, ctypes.POINTER(Grads), P]),
        "cgv2_zero_grads": (ctypes.c_int, [ctypes.POINTER(Grads), i64, i32, P]),
        "cgv2_densify_workspace": (sz, [i64, i32]),
        "cgv2_densify_stats": (ctypes.c_int, [ctypes.POINTER(Surfels), ctypes.POINTER(Proj), ctypes.POINTER(Grads), i32,
                                              ctypes.POINTER(DensifyParams), ctypes.POINTER(DensifyState), P, sz, P]),
        "cgv2_densify_stats_noalloc": (ctypes.c_int, [ctypes.POINTER(Surfels), ctypes.POINTER(Proj),
                                                      ctypes.POINTER(Grads), i32, ctypes.POINTER(DensifyParams),
                                                      ctypes.POINTER(DensifyState), P]),
        "cgv2_contribution_workspace": (sz, [i64, i32]),
        "cgv2_contribution": (ctypes.c_int, [ctypes.POINTER(Proj), ctypes.POINTER(Bins), ctypes.POINTER(Camera), i32,
                                             i64, ctypes.c_float, P, P, P, P, sz, P]),
        "cgv2_trim_workspace": (sz, [i64]),
        "cgv2_trim_mask": (ctypes.c_int, [P, i64, ctypes.c_float, P, P, P, P, sz, P]),
        "cgv2_densify_plan_workspace": (sz, [i64]),
        "cgv2_densify_plan": (ctypes.c_int, [ctypes.POINTER(Surfels), P, P, ctypes.POINTER(ActionParams), P, P, P, P,
                                             sz, P]),
        "cgv2_densify_apply": (ctypes.c_int, [ctypes.POINTER(Surfels), P, P, P, P, ctypes.POINTER(ActionParams),
                                              ctypes.POINTER(SurfelsOut), P, P]),
        "cgv2_densify_gather": (ctypes.c_int, [P, i64, i32, i32, P, P, i32, P, i64, P]),
        "cgv2_visibility_workspace": (sz, [i32]),
        "cgv2_visibility_count": (ctypes.c_int, [P, i64, ctypes.POINTER(Camera), i32, ctypes.c_float, ctypes.c_float, P,
                                                 P, sz, P]),
        "cgv2_crop_workspace": (sz, [i64]),
        "cgv2_crop_volume": (ctypes.c_int, [P, i64, P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double), P, P, P, P, P,
                                            sz, P]),
        "cgv2_compact_order_workspace": (sz, [i64]),
        "cgv2_compact_order": (ctypes.c_int, [P, i64, P, P, P, sz, P]),
        "cgv2_vq_init": (ctypes.c_int, [P, i32, P, i64, i32, P, P]),
        "cgv2_vq_assign_workspace": (sz, [i32]),
        "cgv2_vq_assign": (ctypes.c_int, [P, i32, P, i64, P, i32, i32, P, P, sz, P]),
        "cgv2_vq_update_workspace": (sz, [i32, i32]),
        "cgv2_vq_update": (ctypes.c_int, [P, i32, P, i64, P, i32, P, P, P, sz, P]),
        "cgv2_compact_write": (ctypes.c_int, [ctypes.POINTER(Surfels), P, P, P, i32, ctypes.POINTER(CompactOut), P]),
        "cgv2_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "cgv2_last_hip_error": (ctypes.c_int, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(rc: int, what: str):
    if rc != CGV2_OK:
        L = lib()
        msg = L.cgv2_strerror(rc).decode()
        if rc == CGV2_EHIP:
            msg += f" (hipError {L.cgv2_last_hip_error()})"
        raise Cgv2Error(f"{what}: {msg} [{rc}]")


def ptr(t):
    """Device pointer of a tensor (None -> NULL)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def camera_struct(cam) -> Camera:
    """Camera from the generators' Camera (R, t rounded to float32, as the oracle sees them)."""
    import numpy as np
    c = Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R, np.float64).reshape(-1)
    t = np.asarray(cam.t, np.float64).reshape(-1)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
        c.bg[k] = float(cam.bg[k])
    c.znear = float(cam.znear)
    return c


def camera_array(cams):
    arr = (Camera * len(cams))()
    for k, cam in enumerate(cams):
        arr[k] = camera_struct(cam)
    return arr
