"""ctypes declarations of the C ABI in include/rtg.h (argument marshalling only).

Loading fails loudly when librtg.so has not been built: there is no fallback
path; every step of the rasterizer runs in the HIP kernels of the library.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtg.so")

RTG_OK = 0
RTG_ERR_INVALID = -1
RTG_ERR_HIP = -2
RTG_ERR_CAPACITY = -3
RTG_ERR_OOM = -4
RTG_ERR_UNSUPPORTED = -5

_c = ctypes
i32, i64, f32, vp = _c.c_int32, _c.c_int64, _c.c_float, _c.c_void_p


class Camera(_c.Structure):
    _fields_ = [("width", i32), ("height", i32), ("fx", f32), ("fy", f32), ("cx", f32), ("cy", f32),
                ("R", f32 * 9), ("T", f32 * 3)]


class Settings(_c.Structure):
    _fields_ = [("tile_w", i32), ("tile_h", i32), ("batch", i32), ("T_min", f32), ("alpha_min", f32),
                ("alpha_max", f32), ("z_near", f32), ("eps2d", f32), ("max_instances", i64),
                ("isotropic", i32), ("reserved", i32)]


class Gaussians(_c.Structure):
    _fields_ = [("n", i64), ("means", vp), ("log_scales", vp), ("quats", vp), ("opacity", vp),
                ("colors", vp), ("uncert", vp)]


class Grads(_c.Structure):
    _fields_ = [("d_means", vp), ("d_log_scales", vp), ("d_quats", vp), ("d_opacity", vp),
                ("d_colors", vp)]


# device scratch allocator callbacks (rtg_set_allocator)
ALLOC_FN = _c.CFUNCTYPE(_c.c_void_p, _c.c_void_p, _c.c_size_t)
FREE_FN = _c.CFUNCTYPE(None, _c.c_void_p, _c.c_void_p)

# name -> (restype, argtypes)
SIGNATURES = {
    "rtg_set_allocator": (i32, [vp, ALLOC_FN, FREE_FN, vp]),
    "rtg_last_error": (_c.c_char_p, []),
    "rtg_default_settings": (i32, [_c.POINTER(Settings)]),
    "rtg_device_count": (i32, []),
    "rtg_create": (i32, [i32, _c.POINTER(vp)]),
    "rtg_destroy": (None, [vp]),
    "rtg_project": (i32, [vp, _c.POINTER(Gaussians), _c.POINTER(Camera), i32, _c.POINTER(Settings),
                          _c.POINTER(vp), vp]),
    "rtg_bin_sort": (i32, [vp, vp, _c.POINTER(i64), vp]),
    "rtg_render": (i32, [vp, vp, vp, vp, vp, vp, vp]),
    "rtg_loss": (i32, [vp, vp, vp, vp, vp, vp, f32, vp, vp, vp, vp]),
    "rtg_render_backward": (i32, [vp, vp, vp, vp, vp, vp, _c.POINTER(Grads), vp]),
    "rtg_frame_destroy": (None, [vp]),
    "rtg_frame_export": (i32, [vp, vp, vp, vp, vp, vp]),
    "rtg_frame_export_records": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
    "rtg_frame_info": (i32, [vp, _c.POINTER(i64)]),
    "rtg_score_views": (i32, [vp, _c.POINTER(Gaussians), _c.POINTER(Camera), i32, _c.POINTER(Settings),
                              vp, i32, i32, vp]),
    "rtg_score_graph_create": (i32, [vp, _c.POINTER(Gaussians), i32, i32, i32, _c.POINTER(Settings), i32,
                                     _c.POINTER(Camera), i32, _c.POINTER(vp), vp]),
    "rtg_score_graph_launch": (i32, [vp, _c.POINTER(Camera), i32, vp, vp]),
    "rtg_score_graph_status": (i32, [vp]),
    "rtg_score_graph_destroy": (None, [vp]),
    "rtg_autotune": (i32, [vp, _c.POINTER(Gaussians), _c.POINTER(Camera), i32, i32,
                           _c.POINTER(Settings), vp]),
    "rtg_frame_stats": (i32, [vp, vp, _c.POINTER(i64), vp]),
    "rtg_map_graph_create": (i32, [vp, _c.POINTER(Gaussians), _c.POINTER(Camera), i32, _c.POINTER(Settings),
                                   vp, vp, f32, vp, vp, vp, _c.POINTER(Grads), _c.POINTER(vp), vp]),
    "rtg_map_graph_create_ssim": (i32, [vp, _c.POINTER(Gaussians), _c.POINTER(Camera), i32, _c.POINTER(Settings),
                                        vp, vp, f32, f32, f32, vp, vp, vp, _c.POINTER(Grads), _c.POINTER(vp), vp]),
    "rtg_map_graph_launch": (i32, [vp, vp]),
    "rtg_map_graph_status": (i32, [vp]),
    "rtg_map_graph_destroy": (None, [vp]),
    "rtg_view_utility": (i32, [vp, _c.POINTER(Gaussians), _c.POINTER(Camera), i32, _c.POINTER(Settings), f32,
                               vp, _c.c_double, vp, vp, vp, vp, vp]),
    "rtg_uncertainty_thresholds": (i32, [vp, vp, i64, _c.c_double, vp, vp]),
    "rtg_trajectory_select": (i32, [vp, vp, vp, i32, vp, vp, vp]),
    "rtg_uncertainty_update": (i32, [vp, i64, vp, vp, vp, i32, vp, vp]),
    "rtg_region_grid": (i32, [_c.POINTER(_c.c_double), _c.c_double, _c.POINTER(i32)]),
    "rtg_region_utility": (i32, [vp, i64, vp, vp, _c.POINTER(_c.c_double), _c.c_double, vp, vp, vp, vp]),
    "rtg_loss_ssim": (i32, [vp, vp, vp, vp, vp, vp, f32, f32, f32, vp, vp, vp, vp]),
    "rtg_collision_check": (i32, [vp, _c.POINTER(Gaussians), vp, i64, f32, f32, vp, vp, vp]),
    "rtg_collision_check_noalloc": (i32, [vp, _c.POINTER(Gaussians), vp, i64, f32, f32, vp, vp, vp]),
    "rtg_timing_enable": (i32, [vp, i32]),
    "rtg_timing_read": (i32, [vp, i32, _c.POINTER(_c.c_double), _c.POINTER(i64)]),
    "rtg_timing_reset": (i32, [vp]),
}

TIMER_IDS = {"project": 0, "depth_sort": 1, "binning": 2, "render": 3, "loss": 4,
             "render_backward": 5, "project_backward": 6, "score": 7, "map_graph": 8}

_lib = None


class RtgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rtg error {code}: {msg}")
        self.code = code


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2409_18122_amd.build` (hipcc, gfx950)")
        L = _c.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code):
    if code != RTG_OK:
        raise RtgError(code, lib().rtg_last_error().decode())
    return code
