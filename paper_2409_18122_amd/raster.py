"""PyTorch-facing wrappers over the C ABI (device memory and streams only).

Every function here marshals tensors into the library's structs and calls one
entry point of include/rtg.h; all arithmetic runs in the HIP kernels.
Tensors must be float32, contiguous and on the context's device.
"""
from __future__ import annotations

import atexit
import ctypes
import json
import os
import weakref

import numpy as np
import torch

from . import _lib as _lib_mod
from ._lib import (Camera, Gaussians, Grads, RtgError, Settings, check, lib, RTG_ERR_CAPACITY,
                   RTG_ERR_UNSUPPORTED)

DEFAULTS = {
    "tile_w": 16, "tile_h": 16, "batch": 0,
    "T_min": 1e-4, "alpha_min": 1.0 / 255.0, "alpha_max": 0.99,
    "z_near": 0.2, "eps2d": 0.0, "max_instances": 0, "isotropic": 0,
}

GAUSS_KEYS = ("means", "log_scales", "quats", "opacity", "colors", "uncert")
GRAD_KEYS = ("means", "log_scales", "quats", "opacity", "colors")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous() or t.dtype not in (torch.float32, torch.float64,
                                                                   torch.int64, torch.int32):
        raise ValueError("expected a contiguous CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def make_settings(settings=None) -> Settings:
    s = dict(DEFAULTS)
    if settings:
        s.update({k: v for k, v in settings.items() if k in DEFAULTS})
    return Settings(int(s["tile_w"]), int(s["tile_h"]), int(s["batch"]), float(s["T_min"]),
                    float(s["alpha_min"]), float(s["alpha_max"]), float(s["z_near"]),
                    float(s["eps2d"]), int(s["max_instances"]), int(s["isotropic"]), 0)


def _host_f64(x):
    if isinstance(x, torch.Tensor):
        x = x.detach().cpu().numpy()
    return np.asarray(x, dtype=np.float64)


def make_cameras(cams):
    """The C camera array of a list of camera dicts; an array made by this
    function is passed through unchanged (build it once to call an entry
    point many times on the same views)."""
    if isinstance(cams, ctypes.Array):
        return cams
    arr = (Camera * len(cams))()
    for i, c in enumerate(cams):
        R = _host_f64(c["R"]).reshape(9).tolist()
        T = _host_f64(c["T"]).reshape(3).tolist()
        arr[i] = Camera(int(c["width"]), int(c["height"]), float(c["fx"]), float(c["fy"]),
                        float(c["cx"]), float(c["cy"]), (ctypes.c_float * 9)(*R),
                        (ctypes.c_float * 3)(*T))
    return arr


def make_gaussians(g) -> Gaussians:
    n = int(g["opacity"].shape[0])
    for k in GAUSS_KEYS:
        t = g.get(k)
        if t is not None and (t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda):
            raise ValueError(f"gaussian array {k} must be a contiguous float32 CUDA tensor")
    return Gaussians(n, *[_ptr(g.get(k)) for k in GAUSS_KEYS])


def to_device(scene, device="cuda"):
    """numpy scene (planar float32) -> dict of CUDA tensors."""
    return {k: torch.as_tensor(v).to(device=device, dtype=torch.float32).contiguous()
            for k, v in scene.items()}


def image_sizes(cams):
    return [int(c["width"]) * int(c["height"]) for c in cams]


# contexts whose scratch comes from PyTorch: closed at exit while torch is still alive
_TORCH_ALLOC_CTXS = weakref.WeakSet()


def _close_torch_alloc_contexts():
    for c in list(_TORCH_ALLOC_CTXS):
        c.close()


atexit.register(_close_torch_alloc_contexts)


class Context:
    """One library context bound to a device (one per stream)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        check(lib().rtg_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device
        self._callbacks = None

    def use_torch_allocator(self):
        """Serve this context's device scratch from PyTorch's caching
        allocator (rtg_set_allocator); no frame or graph may be alive."""
        dev = self.device

        def _alloc(user, nbytes):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev,
                                                          stream=torch.cuda.current_stream(dev))
            except RuntimeError:  # out of memory: the library reports RTG_ERR_OOM
                return None

        def _free(user, ptr):
            torch.cuda.caching_allocator_delete(ptr)

        cbs = (_lib_mod.ALLOC_FN(_alloc), _lib_mod.FREE_FN(_free))
        check(lib().rtg_set_allocator(self.handle, cbs[0], cbs[1], None))
        self._callbacks = cbs  # kept alive as long as the library may call them
        _TORCH_ALLOC_CTXS.add(self)

    def use_hip_allocator(self):
        """Back to the library's own hipMalloc-based cache."""
        check(lib().rtg_set_allocator(self.handle, _lib_mod.ALLOC_FN(), _lib_mod.FREE_FN(), None))
        self._callbacks = None

    def close(self):
        if self.handle:
            lib().rtg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def timing_enable(ctx, on=True):
    check(lib().rtg_timing_enable(ctx.handle, int(bool(on))))


def timing_reset(ctx):
    check(lib().rtg_timing_reset(ctx.handle))


def timing_read(ctx):
    """{kernel name: (total ms, launches)} accumulated since the last reset."""
    from ._lib import TIMER_IDS
    out = {}
    for name, i in TIMER_IDS.items():
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        check(lib().rtg_timing_read(ctx.handle, i, ctypes.byref(ms), ctypes.byref(n)))
        out[name] = (float(ms.value), int(n.value))
    return out


class Frame:
    """Projection of the map into a batch of views, with its binning."""

    def __init__(self, ctx: Context, g, cams, settings=None):
        self.ctx = ctx
        self._g = g  # keeps the tensors alive
        self._gs = make_gaussians(g)
        self.cams = cams
        self._cams = make_cameras(cams)
        self.settings = make_settings(settings)
        h = ctypes.c_void_p()
        check(lib().rtg_project(ctx.handle, ctypes.byref(self._gs), self._cams, len(cams),
                                ctypes.byref(self.settings), ctypes.byref(h), _stream()))
        self.handle = h
        self.n_instances = None

    def bin_sort(self):
        k = ctypes.c_int64()
        check(lib().rtg_bin_sort(self.ctx.handle, self.handle, ctypes.byref(k), _stream()))
        self.n_instances = int(k.value)
        return self.n_instances

    def stats(self):
        a = (ctypes.c_int64 * 4)()
        check(lib().rtg_frame_stats(self.ctx.handle, self.handle, a, _stream()))
        return {"records": a[0], "instances": a[1], "contrib_pairs": a[2], "walked_pairs": a[3]}

    def info(self):
        a = (ctypes.c_int64 * 6)()
        check(lib().rtg_frame_info(self.handle, a))
        return {"records": a[0], "instances": a[1], "tiles": a[2], "pixels": a[3],
                "tile_w": a[4], "tile_h": a[5]}

    def render(self, want=("rgb", "depth", "alpha", "unc")):
        P = sum(image_sizes(self.cams))
        dev = self._g["means"].device
        out = {}
        if "rgb" in want:
            out["rgb"] = torch.empty(3 * P, device=dev, dtype=torch.float32)
        for k in ("depth", "alpha", "unc"):
            if k in want:
                out[k] = torch.empty(P, device=dev, dtype=torch.float32)
        check(lib().rtg_render(self.ctx.handle, self.handle, _ptr(out.get("rgb")),
                               _ptr(out.get("depth")), _ptr(out.get("alpha")), _ptr(out.get("unc")),
                               _stream()))
        return out

    def loss(self, rgb, depth, target_rgb, target_depth, w_depth=0.5, want_grad=True):
        dev = rgb.device
        loss = torch.empty(1, device=dev, dtype=torch.float64)
        d_rgb = torch.empty_like(rgb) if want_grad else None
        d_depth = torch.empty_like(depth) if want_grad else None
        check(lib().rtg_loss(self.ctx.handle, self.handle, _ptr(rgb), _ptr(depth), _ptr(target_rgb),
                             _ptr(target_depth), float(w_depth), _ptr(d_rgb), _ptr(d_depth),
                             _ptr(loss), _stream()))
        return loss, d_rgb, d_depth

    def loss_ssim(self, rgb, depth, target_rgb, target_depth, w_depth=1.0, lambda1=0.4, lambda2=0.1,
                  want_grad=True):
        """The full loss of eq. (4): L1 depth + lambda1 L1 colour + lambda2 (1 - SSIM), per view."""
        dev = rgb.device
        loss = torch.empty(1, device=dev, dtype=torch.float64)
        d_rgb = torch.empty_like(rgb) if want_grad else None
        d_depth = torch.empty_like(depth) if want_grad else None
        check(lib().rtg_loss_ssim(self.ctx.handle, self.handle, _ptr(rgb), _ptr(depth), _ptr(target_rgb),
                                  _ptr(target_depth), float(w_depth), float(lambda1), float(lambda2),
                                  _ptr(d_rgb), _ptr(d_depth), _ptr(loss), _stream()))
        return loss, d_rgb, d_depth

    def backward(self, d_rgb, d_depth, d_alpha=None, d_unc=None, grads=None):
        """Adds dL/dparams into `grads` (dict of tensors shaped like the map)."""
        if grads is None:
            grads = {k: torch.zeros_like(self._g[k]) for k in GRAD_KEYS if self._g.get(k) is not None}
        gr = Grads(*[_ptr(grads.get(k)) for k in GRAD_KEYS])
        check(lib().rtg_render_backward(self.ctx.handle, self.handle, _ptr(d_rgb), _ptr(d_depth),
                                        _ptr(d_alpha), _ptr(d_unc), ctypes.byref(gr), _stream()))
        return grads

    def export(self):
        """Sorted (tile << 32 | depth bits) keys, Gaussian indices, tile ranges."""
        inf = self.info()
        dev = self._g["means"].device
        K = max(inf["instances"], 0)
        keys = torch.empty(K, device=dev, dtype=torch.int64)
        vals = torch.empty(K, device=dev, dtype=torch.int32)
        ranges = torch.empty(2 * inf["tiles"], device=dev, dtype=torch.int32)
        check(lib().rtg_frame_export(self.ctx.handle, self.handle, _ptr(keys) if K else None,
                                     _ptr(vals) if K else None,
                                     _ptr(ranges) if inf["tiles"] else None, _stream()))
        return keys, vals, ranges

    def export_records(self):
        """The projected records (Gaussian-major, views ascending): dict of
        mean2d (2, R) and conic (3, R) float64, pbox (4, R) int32 (u0, u1, v0,
        v1), depth_bits, gid, view and ntiles (R,) int32 views of uint32."""
        R = max(self.info()["records"], 0)
        dev = self._g["means"].device
        out = {"mean2d": torch.empty(2 * R, device=dev, dtype=torch.float64),
               "conic": torch.empty(3 * R, device=dev, dtype=torch.float64),
               "pbox": torch.empty(4 * R, device=dev, dtype=torch.int32)}
        for k in ("depth_bits", "gid", "view", "ntiles"):
            out[k] = torch.empty(R, device=dev, dtype=torch.int32)
        if R:
            check(lib().rtg_frame_export_records(self.ctx.handle, self.handle, _ptr(out["mean2d"]),
                                                 _ptr(out["conic"]), _ptr(out["pbox"]), _ptr(out["depth_bits"]),
                                                 _ptr(out["gid"]), _ptr(out["view"]), _ptr(out["ntiles"]),
                                                 _stream()))
        for k, rows in (("mean2d", 2), ("conic", 3), ("pbox", 4)):
            out[k] = out[k].view(rows, R)
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().rtg_frame_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def render(ctx, g, cams, settings=None, want=("rgb", "depth", "alpha", "unc")):
    """Forward render of several views; returns (images, frame)."""
    f = Frame(ctx, g, cams, settings)
    f.bin_sort()
    return f.render(want), f


class RasterizeFn(torch.autograd.Function):
    """Differentiable render: (means, log_scales, quats, opacity, colors) ->
    (rgb, depth, alpha, unc), packed per view; uncertainty has no gradient."""

    @staticmethod
    def forward(fctx, means, log_scales, quats, opacity, colors, uncert, cams, settings, rctx):
        g = {"means": means.detach(), "log_scales": log_scales.detach(),
             "quats": None if quats is None else quats.detach(),
             "opacity": opacity.detach(), "colors": colors.detach(),
             "uncert": None if uncert is None else uncert.detach()}
        frame = Frame(rctx, g, cams, settings)
        frame.bin_sort()
        out = frame.render(("rgb", "depth", "alpha") + (("unc",) if uncert is not None else ()))
        fctx.frame = frame
        fctx.has_unc = uncert is not None
        unc = out.get("unc", torch.zeros_like(out["alpha"]))
        return out["rgb"], out["depth"], out["alpha"], unc

    @staticmethod
    def backward(fctx, d_rgb, d_depth, d_alpha, d_unc):
        frame = fctx.frame
        grads = frame.backward(d_rgb.contiguous(), d_depth.contiguous(), d_alpha.contiguous(),
                               d_unc.contiguous() if fctx.has_unc else None)
        frame.close()
        fctx.frame = None
        return (grads["means"], grads["log_scales"], grads.get("quats"), grads["opacity"],
                grads["colors"], None, None, None, None)


def rasterize(rctx, g, cams, settings=None):
    return RasterizeFn.apply(g["means"], g["log_scales"], g.get("quats"), g["opacity"], g["colors"],
                             g.get("uncert"), cams, settings, rctx)


SCORE_MODES = {"rendered": 0, "binary": 1}


def score_views(ctx, g, cams, settings=None, persistent=True, mode="rendered"):
    """Per-view score (float64 tensor of len(cams)): mode "rendered" sums the
    composited uncertainty sum_i u_i a_i T_i over the pixels, "binary" sums u_i
    over the contributing Gaussians of each pixel (the binary-J trace)."""
    gs = make_gaussians(g)
    cs = make_cameras(cams)
    st = make_settings(settings)
    out = torch.empty(len(cams), device=g["means"].device, dtype=torch.float64)
    check(lib().rtg_score_views(ctx.handle, ctypes.byref(gs), cs, len(cams), ctypes.byref(st),
                                _ptr(out), int(bool(persistent)), SCORE_MODES[mode], _stream()))
    return out


class ScoreGraph:
    """The batched scoring pipeline captured once, replayed for new poses."""

    def __init__(self, ctx, g, max_views, max_width, max_height, settings=None, probe=None, mode="rendered"):
        self.ctx = ctx
        self._g = g
        self._gs = make_gaussians(g)
        self.settings = make_settings(settings)
        pr = make_cameras(probe) if probe else None
        h = ctypes.c_void_p()
        check(lib().rtg_score_graph_create(ctx.handle, ctypes.byref(self._gs), int(max_views),
                                           int(max_width), int(max_height),
                                           ctypes.byref(self.settings), SCORE_MODES[mode], pr,
                                           len(probe) if probe else 0, ctypes.byref(h), _stream()))
        self.handle = h

    def launch(self, cams, out=None):
        cs = make_cameras(cams)
        if out is None:
            out = torch.empty(len(cams), device=self._g["means"].device, dtype=torch.float64)
        check(lib().rtg_score_graph_launch(self.handle, cs, len(cams), _ptr(out), _stream()))
        return out

    def status(self):
        code = lib().rtg_score_graph_status(self.handle)
        if code == RTG_ERR_CAPACITY:
            return False
        check(code)
        return True

    def close(self):
        if getattr(self, "handle", None):
            lib().rtg_score_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MapGraph:
    """One mapping iteration (render, loss, backward) on fixed keyframes,
    captured once and replayed; gradients are added into `grads`.  The loss is
    the L1 form of rtg_loss, or with lambda1 / lambda2 given the full eq. (4)
    of rtg_loss_ssim."""

    def __init__(self, ctx, g, cams, target_rgb, target_depth, w_depth=0.5, settings=None, grads=None,
                 lambda1=None, lambda2=None):
        self.ctx = ctx
        self._g = g
        self._gs = make_gaussians(g)
        self.cams = cams
        self._cams = make_cameras(cams)
        self.settings = make_settings(settings)
        P = sum(image_sizes(cams))
        dev = g["means"].device
        self.rgb = torch.empty(3 * P, device=dev, dtype=torch.float32)
        self.depth = torch.empty(P, device=dev, dtype=torch.float32)
        self.loss = torch.zeros(1, device=dev, dtype=torch.float64)
        self.grads = grads if grads is not None else {k: torch.zeros_like(g[k]) for k in GRAD_KEYS
                                                      if g.get(k) is not None}
        self._targets = (target_rgb, target_depth)
        gr = Grads(*[_ptr(self.grads.get(k)) for k in GRAD_KEYS])
        h = ctypes.c_void_p()
        if lambda1 is None and lambda2 is None:
            check(lib().rtg_map_graph_create(ctx.handle, ctypes.byref(self._gs), self._cams, len(cams),
                                             ctypes.byref(self.settings), _ptr(target_rgb), _ptr(target_depth),
                                             float(w_depth), _ptr(self.rgb), _ptr(self.depth), _ptr(self.loss),
                                             ctypes.byref(gr), ctypes.byref(h), _stream()))
        else:
            check(lib().rtg_map_graph_create_ssim(ctx.handle, ctypes.byref(self._gs), self._cams, len(cams),
                                                  ctypes.byref(self.settings), _ptr(target_rgb), _ptr(target_depth),
                                                  float(w_depth), float(0.4 if lambda1 is None else lambda1),
                                                  float(0.1 if lambda2 is None else lambda2), _ptr(self.rgb),
                                                  _ptr(self.depth), _ptr(self.loss), ctypes.byref(gr),
                                                  ctypes.byref(h), _stream()))
        self.handle = h

    def launch(self):
        check(lib().rtg_map_graph_launch(self.handle, _stream()))
        return self.loss

    def status(self):
        code = lib().rtg_map_graph_status(self.handle)
        if code == RTG_ERR_CAPACITY:
            return False
        check(code)
        return True

    def close(self):
        if getattr(self, "handle", None):
            lib().rtg_map_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def uncertainty_thresholds(ctx, uncert, k_std=0.5):
    """Device tensor [mean - k sd, mean + k sd] of the uncertainties."""
    out = torch.empty(2, device=uncert.device, dtype=torch.float64)
    check(lib().rtg_uncertainty_thresholds(ctx.handle, _ptr(uncert), int(uncert.numel()), float(k_std),
                                           _ptr(out), _stream()))
    return out


def view_utility(ctx, g, cams, lo_hi, settings=None, range_=5.0, lambda_xi=1.0):
    """Paper-literal utility per view: dict of n_high, n_low (int64), sum_u, xi (float64)."""
    gs = make_gaussians(g)
    cs = make_cameras(cams)
    st = make_settings(settings)
    dev = g["means"].device
    V = len(cams)
    out = {"n_high": torch.empty(V, device=dev, dtype=torch.int64),
           "n_low": torch.empty(V, device=dev, dtype=torch.int64),
           "sum_u": torch.empty(V, device=dev, dtype=torch.float64),
           "xi": torch.empty(V, device=dev, dtype=torch.float64)}
    check(lib().rtg_view_utility(ctx.handle, ctypes.byref(gs), cs, V, ctypes.byref(st), float(range_),
                                 _ptr(lo_hi), float(lambda_xi), _ptr(out["n_high"]), _ptr(out["n_low"]),
                                 _ptr(out["sum_u"]), _ptr(out["xi"]), _stream()))
    return out


def trajectory_select(ctx, xi, offsets):
    """eq. (10): per-trajectory sums of xi over [offsets[t], offsets[t+1]) and the best index."""
    off = offsets.to(device=xi.device, dtype=torch.int32).contiguous()
    n = off.numel() - 1
    util = torch.empty(n, device=xi.device, dtype=torch.float64)
    best = torch.empty(1, device=xi.device, dtype=torch.int32)
    check(lib().rtg_trajectory_select(ctx.handle, _ptr(xi), _ptr(off), n, _ptr(util), _ptr(best), _stream()))
    return util, best


def tune_key(g, cams, mode, settings=None):
    """Cache key of a tuning result: the device, mode, resolution(s), view
    count, the power-of-two bucket of the Gaussian count, and the settings
    that change the work (alpha_min, T_min, alpha_max, eps2d, isotropic)."""
    n = int(g["opacity"].shape[0])
    res = sorted({(int(c["width"]), int(c["height"])) for c in cams})
    st = make_settings(settings)
    t = g["opacity"]
    name = torch.cuda.get_device_name(t.device) if isinstance(t, torch.Tensor) and t.is_cuda else "host"
    work = (f"amin{st.alpha_min:.9g}:tmin{st.T_min:.9g}:amax{st.alpha_max:.9g}:eps{st.eps2d:.9g}"
            f":iso{int(st.isotropic)}")
    return (f"{name}:mode{int(mode)}:" + ",".join(f"{w}x{h}" for w, h in res) +
            f":v{len(cams)}:n2^{max(n, 1).bit_length() - 1}:{work}")


def autotune(ctx, g, cams, mode, settings=None, cache=None):
    """Fastest tile and staging batch for `mode` (0 forward, 1 forward +
    backward, 2 scoring).  With `cache` (a JSON file path), a result stored
    under the same tune_key is returned without timing, and a new result is
    stored there."""
    out = dict(settings or DEFAULTS)
    key = tune_key(g, cams, mode, settings)
    table = {}
    if cache is not None and os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
        if key in table:
            out.update({k: int(table[key][k]) for k in ("tile_w", "tile_h", "batch")})
            return out
    st = make_settings(settings)
    gs = make_gaussians(g)
    cs = make_cameras(cams)
    check(lib().rtg_autotune(ctx.handle, ctypes.byref(gs), cs, len(cams), int(mode),
                             ctypes.byref(st), _stream()))
    out["tile_w"], out["tile_h"], out["batch"] = st.tile_w, st.tile_h, st.batch
    if cache is not None:
        table[key] = {"tile_w": st.tile_w, "tile_h": st.tile_h, "batch": st.batch}
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return out


def uncertainty_update(ctx, means_prev, means_cur, u_prev, squared=False, out=None):
    """Per-Gaussian ||mu_cur - mu_prev|| (squared with squared=True); a
    Gaussian whose mean did not change keeps u_prev (Sec. IV-A bookkeeping).
    Means: (3, N) float32 device tensors; returns (N,) float32 (out may be
    u_prev for an in-place update)."""
    n = int(u_prev.shape[0])
    if out is None:
        out = torch.empty_like(u_prev)
    check(lib().rtg_uncertainty_update(ctx.handle, n, _ptr(means_prev.contiguous()),
                                       _ptr(means_cur.contiguous()), _ptr(u_prev), int(bool(squared)),
                                       _ptr(out), _stream()))
    return out


def region_grid(box, size=2.5):
    b = (ctypes.c_double * 6)(*[float(x) for x in box])
    d = (ctypes.c_int32 * 3)()
    check(lib().rtg_region_grid(b, float(size), d))
    return tuple(int(x) for x in d)


def region_utility(ctx, means, u, box, size=2.5):
    """(count int64, sum float64, mean float64) per cuboid region of edge
    `size` of box = (lo x, y, z, hi x, y, z), region ix + nx (iy + ny iz)."""
    nx, ny, nz = region_grid(box, size)
    nr = nx * ny * nz
    dev = u.device
    count = torch.empty(nr, device=dev, dtype=torch.int64)
    sm = torch.empty(nr, device=dev, dtype=torch.float64)
    mean = torch.empty(nr, device=dev, dtype=torch.float64)
    b = (ctypes.c_double * 6)(*[float(x) for x in box])
    check(lib().rtg_region_utility(ctx.handle, int(u.shape[0]), _ptr(means.contiguous()), _ptr(u), b, float(size),
                                   _ptr(count), _ptr(sm), _ptr(mean), _stream()))
    return count, sm, mean


def collision_check(ctx, g, points, r_robot, lambda_g=3.0, clearance=True, no_alloc=False):
    """(collide int32[P], clearance float32[P] or None) of the points
    (planar 3 x P) against the Gaussians' principal-axis spheres.
    no_alloc=True calls rtg_collision_check_noalloc (the library's fixed
    scratch, no device allocation; up to 96 MiB of scratch)."""
    for k in ("means", "log_scales"):
        t = g[k]
        if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda or t.dim() != 2 or t.shape[0] != 3:
            raise ValueError(f"gaussian array {k} must be a contiguous planar 3 x N float32 CUDA tensor")
    gs = Gaussians(int(g["means"].shape[1]), *[_ptr(g[k]) if k in ("means", "log_scales") else None
                                              for k in GAUSS_KEYS])
    pts = points.contiguous()
    if pts.dtype != torch.float32:
        raise ValueError("points must be float32")
    P = int(pts.shape[1]) if pts.dim() == 2 else 0
    dev = g["means"].device
    hit = torch.empty(P, device=dev, dtype=torch.int32)
    clr = torch.empty(P, device=dev, dtype=torch.float32) if clearance else None
    fn = lib().rtg_collision_check_noalloc if no_alloc else lib().rtg_collision_check
    check(fn(ctx.handle, ctypes.byref(gs), _ptr(pts), P, float(r_robot), float(lambda_g), _ptr(hit), _ptr(clr),
             _stream()))
    return hit, clr


def unpack_images(out, cams):
    """Split packed per-view outputs into lists of (C, H, W) / (H, W) tensors."""
    res = []
    off = 0
    for c in cams:
        W, H = int(c["width"]), int(c["height"])
        P = W * H
        d = {}
        if "rgb" in out:
            d["rgb"] = out["rgb"][3 * off:3 * off + 3 * P].view(3, H, W)
        for k in ("depth", "alpha", "unc"):
            if k in out:
                d[k] = out[k][off:off + P].view(H, W)
        res.append(d)
        off += P
    return res


__all__ = ["Context", "Frame", "RasterizeFn", "rasterize", "render", "score_views", "ScoreGraph", "MapGraph", "tune_key",
           "uncertainty_update", "region_grid", "region_utility", "collision_check",
           "autotune", "to_device", "unpack_images", "RtgError", "DEFAULTS"]
