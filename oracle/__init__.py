"""FP64 CPU oracle for the RT-GuIDE rasterizer (arXiv 2409.18122).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library under ``paper_2409_18122_amd`` and never imports it.

The arithmetic lives in ``rtg_oracle.c`` (plain C, binary64, OpenMP over
pixels); this module only marshals numpy arrays.  Float32 inputs are promoted
exactly to float64.  See the C file's header for which passage of the paper
each function follows.

Functions: ``project``, ``render``, ``count``, ``keys``, ``loss``,
``loss_ssim``, ``score``, ``adjoint``, ``thresholds``, ``view_utility``,
``traj_select``, ``uncertainty_update``, ``region_utility``, ``collision``.
Parity status: every function here is pinned by the ``-m "not gpu"`` tests
(closed forms, invariants, brute force, finite differences); see
tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rtg_oracle.c")
_LIB = os.path.join(_HERE, "librtgo.so")

# Relative widths of the near-threshold bands: a per-pixel decision whose
# operand lies this close (relative) to its threshold is taken both ways by the
# oracle, since another evaluation may legitimately fall on either side.
#  * alpha_min: the HIP path re-takes every decision within 2e-3 of alpha_min
#    in binary64 from the binary64 conic and a mean exact to ~2^-48, so only
#    binary64 rounding-order differences (~1e-11 relative) separate the two:
#    1e-5 covers them with a wide margin;
#  * T_min: the HIP path decides it in binary32.  After the contributors of a
#    pixel, binary32 T differs from binary64 by at most
#    sum_i [2^-24 + eps_a a_i / (1 - a_i)] relative (eps_a ~ 2.4e-7, the
#    relative error of binary32 alpha); with T >= T_min = 1e-4 at the stop
#    and a_i <= 0.99 this stays below 7e-5 (two clamped splats give 5e-5,
#    300 roundings 1.8e-5), so the band is 1e-4.
EV_ALPHA = 1e-5
EV_T = 1e-4


# binary64 throughout, no contraction and no reassociation: the optimisation
# level and target only change speed, never a result
_CFLAGS = ["-std=c99", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = False) -> str:
    """Compile rtg_oracle.c with gcc (binary64, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", *_CFLAGS, "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def use_native_build(directory: str) -> str:
    """Compile rtg_oracle.c at -O3 -march=native for the host it runs on, into
    `directory`, and make it the library this module calls (for timing the
    oracle as a CPU baseline; results are the same as the in-tree build's).
    Returns the gcc flags used."""
    global _lib, _lib_path
    path = os.path.join(directory, "librtgo_native.so")
    flags = ["-O3", "-march=native"]
    subprocess.run(["gcc", *flags, *_CFLAGS, "-o", path, _SRC, "-lm"], check=True)
    _lib = None
    _lib_path = path
    lib()
    return " ".join(flags)


_lib = None
_lib_path = None  # None: the in-tree build


def lib():
    global _lib
    if _lib is None:
        if _lib_path is None:
            build()
        L = ctypes.CDLL(_lib_path or _LIB)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.rtgo_project.argtypes = [i64] + [p] * 6 + [p] * 8
        L.rtgo_project.restype = ctypes.c_int
        L.rtgo_render.argtypes = ([i64] + [p] * 8 + [ctypes.c_int] * 3 + [p] +
                                  [ctypes.c_double] * 2 + [p] * 7 + [i64, p, p])
        L.rtgo_render.restype = i64
        L.rtgo_count.argtypes = [i64] + [p] * 6 + [ctypes.c_int] * 3 + [p, p]
        L.rtgo_count.restype = ctypes.c_int
        L.rtgo_keys.argtypes = [i64] + [p] * 6 + [ctypes.c_int] * 3 + [i64, p, p]
        L.rtgo_keys.restype = ctypes.c_int
        L.rtgo_loss.argtypes = [i64, p, p, p, p, ctypes.c_double, p, p]
        L.rtgo_loss.restype = ctypes.c_double
        L.rtgo_loss_ssim.argtypes = [ctypes.c_int, ctypes.c_int] + [p] * 4 + [ctypes.c_double] * 3 + [p] * 3
        L.rtgo_loss_ssim.restype = ctypes.c_double
        L.rtgo_score.argtypes = [i64] + [p] * 7 + [ctypes.c_int, p, ctypes.c_int, ctypes.c_int, ctypes.c_int, p]
        L.rtgo_score.restype = ctypes.c_int
        L.rtgo_adjoint.argtypes = ([i64] + [p] * 8 + [ctypes.c_int] * 2 + [p] * 11 + [ctypes.c_double] * 2)
        L.rtgo_adjoint.restype = ctypes.c_int
        L.rtgo_thresholds.argtypes = [i64, p, ctypes.c_double, p, p]
        L.rtgo_thresholds.restype = None
        L.rtgo_view_utility.argtypes = ([i64, p, p, p, ctypes.c_int] + [ctypes.c_double] * 5 + [p] * 4)
        L.rtgo_view_utility.restype = ctypes.c_int
        L.rtgo_uncertainty_update.argtypes = [i64, p, p, p, ctypes.c_int, p]
        L.rtgo_uncertainty_update.restype = None
        L.rtgo_region_grid.argtypes = [p, ctypes.c_double, p]
        L.rtgo_region_grid.restype = ctypes.c_int
        L.rtgo_region_utility.argtypes = [i64, p, p, p, ctypes.c_double, p, p, p]
        L.rtgo_region_utility.restype = ctypes.c_int
        L.rtgo_collision.argtypes = [i64, p, p, i64, p, ctypes.c_double, ctypes.c_double, p, p]
        L.rtgo_collision.restype = None
        L.rtgo_traj_select.argtypes = [ctypes.c_int, p, p, p]
        L.rtgo_traj_select.restype = ctypes.c_int
        L.rtgo_set_threads.argtypes = [ctypes.c_int]
        L.rtgo_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().rtgo_set_threads(int(n))


def max_threads() -> int:
    return int(lib().rtgo_max_threads())


def _d(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data


class _G:
    """Scene promoted to float64 (kept alive while pointers are in use)."""

    def __init__(self, s):
        self.n = int(np.asarray(s["opacity"]).shape[0])
        self.means = _d(s["means"]).reshape(3, self.n)
        # isotropic scenes carry one log-radius per Gaussian (1 x N) and no quaternion
        ls = _d(s["log_scales"])
        self.ls = ls.reshape(-1, self.n)
        self.q = _d(s["quats"]).reshape(4, self.n) if s.get("quats") is not None else None
        self.o = _d(s["opacity"]).reshape(self.n)
        self.c = _d(s.get("colors", np.zeros((3, self.n)))).reshape(3, self.n)
        self.u = _d(s.get("uncert", np.zeros(self.n))).reshape(self.n)

    def geo(self):
        return [_ptr(self.means), _ptr(self.ls), _ptr(self.q) if self.q is not None else None, _ptr(self.o)]

    def all(self):
        return self.geo() + [_ptr(self.c), _ptr(self.u)]


def cam_array(cam):
    R = np.asarray(cam["R"], dtype=np.float64).reshape(9)
    T = np.asarray(cam["T"], dtype=np.float64).reshape(3)
    return _d([cam["width"], cam["height"], cam["fx"], cam["fy"], cam["cx"], cam["cy"],
               *R, *T])


def set_array(settings):
    """Settings are taken at their binary32 values, as the library receives them."""
    f = lambda k: float(np.float32(settings[k]))
    return _d([f("T_min"), f("alpha_min"), f("alpha_max"), f("z_near"), f("eps2d"),
               1.0 if settings.get("isotropic", 0) else 0.0])


def project(scene, cam, settings):
    g = _G(scene)
    n = g.n
    out = {
        "valid": np.zeros(n, np.int32), "mean2d": np.zeros((2, n)),
        "cov2d": np.zeros((3, n)), "conic": np.zeros((3, n)),
        "depth": np.zeros(n), "depth_bits": np.zeros(n, np.uint32),
        "half": np.zeros((2, n)), "box": np.zeros((4, n), np.int32),
    }
    ca, sa = cam_array(cam), set_array(settings)
    lib().rtgo_project(n, *g.geo(), _ptr(ca), _ptr(sa),
                       *[_ptr(out[k]) for k in ("valid", "mean2d", "cov2d", "conic",
                                                "depth", "depth_bits", "half", "box")])
    out["valid"] = out["valid"].astype(bool)
    return out


def render(scene, cam, settings, mode="tiled", tile=None, roi=None,
           ev_alpha=EV_ALPHA, ev_t=EV_T, alt_cap=None):
    """Render one camera. Returns dict with rgb (3,H,W), depth, alpha, unc,
    T (H,W), ncontrib, nevents (H,W int32) and the alternatives of event pixels:
    alt_pix (m,), alt_val (m, 4, 6) over (r, g, b, depth, alpha, unc)."""
    g = _G(scene)
    W, H = int(cam["width"]), int(cam["height"])
    P = W * H
    tw, th = tile if tile is not None else (settings.get("tile_w", 16), settings.get("tile_h", 16))
    m = {"brute": 0, "tiled": 1}[mode]
    ca, sa = cam_array(cam), set_array(settings)
    roi_a = None if roi is None else np.ascontiguousarray(np.asarray(roi, np.int32))
    rgb = np.zeros((3, H, W)); dep = np.zeros((H, W)); alp = np.zeros((H, W))
    unc = np.zeros((H, W)); T = np.ones((H, W))
    nc = np.zeros((H, W), np.int32); ne = np.zeros((H, W), np.int32)
    cap = alt_cap if alt_cap is not None else max(4096, P // 8)
    apix = np.zeros(cap, np.int64); aval = np.zeros((cap, 4, 6))
    nalt = lib().rtgo_render(g.n, *g.all(), _ptr(ca), _ptr(sa), m, int(tw), int(th), _ptr(roi_a),
                             float(ev_alpha), float(ev_t), _ptr(rgb), _ptr(dep), _ptr(alp),
                             _ptr(unc), _ptr(T), _ptr(nc), _ptr(ne), cap, _ptr(apix), _ptr(aval))
    if nalt < 0:
        raise MemoryError("oracle render failed")
    k = min(int(nalt), cap)
    return {"rgb": rgb, "depth": dep, "alpha": alp, "unc": unc, "T": T,
            "ncontrib": nc, "nevents": ne, "alt_pix": apix[:k], "alt_val": aval[:k],
            "alt_overflow": int(nalt) > cap}


def count(scene, cam, settings, tile=(16, 16), support=False):
    """(visible Gaussians, binned pairs).  Pairs are every tile a pixel box
    meets, or with support=True only tiles with a pixel centre where the
    Gaussian's alpha >= alpha_min."""
    g = _G(scene)
    nv = ctypes.c_int64(); npairs = ctypes.c_int64()
    ca, sa = cam_array(cam), set_array(settings)
    lib().rtgo_count(g.n, *g.geo(), _ptr(ca), _ptr(sa), int(tile[0]), int(tile[1]), int(bool(support)),
                     ctypes.addressof(nv), ctypes.addressof(npairs))
    return int(nv.value), int(npairs.value)


def keys(scene, cams, settings, tile=(16, 16), support=False):
    """Sorted (tile<<32 | depth bits, Gaussian index) pairs over several cameras,
    global tile ids offset by the tiles of the preceding cameras; `support` as
    in count()."""
    g = _G(scene)
    sa = set_array(settings)
    tw, th = int(tile[0]), int(tile[1])
    all_k, all_v = [], []
    base = 0
    for cam in cams:
        _, npairs = count(scene, cam, settings, tile, support)
        k = np.zeros(npairs, np.uint64); v = np.zeros(npairs, np.uint32)
        ca = cam_array(cam)
        lib().rtgo_keys(g.n, *g.geo(), _ptr(ca), _ptr(sa), tw, th, int(bool(support)), base, _ptr(k), _ptr(v))
        all_k.append(k); all_v.append(v)
        base += ((int(cam["width"]) + tw - 1) // tw) * ((int(cam["height"]) + th - 1) // th)
    return np.concatenate(all_k), np.concatenate(all_v)


def loss(rgb, depth, target_rgb, target_depth, w_depth=0.5):
    rgb = _d(rgb); dep = _d(depth); trgb = _d(target_rgb); tdep = _d(target_depth)
    P = dep.size
    grgb = np.zeros_like(rgb); gdep = np.zeros_like(dep)
    L = lib().rtgo_loss(P, _ptr(rgb), _ptr(dep), _ptr(trgb), _ptr(tdep), float(w_depth),
                        _ptr(grgb), _ptr(gdep))
    return float(L), grgb, gdep


def loss_ssim(rgb, depth, target_rgb, target_depth, width, height, w_depth=1.0, lambda1=0.4, lambda2=0.1,
              ssim_map=False):
    """Mapping loss of eq. (4) for one view: (L, dL/dC (3, P), dL/dD (P,)[, S map (3, P)]),
    L = mean_p (w_depth |D - D*| + lambda1 sum_ch |C - C*|) + lambda2 (1 - SSIM(C, C*))."""
    rgb = _d(rgb).reshape(3, -1); dep = _d(depth).reshape(-1)
    trgb = _d(target_rgb).reshape(3, -1); tdep = _d(target_depth).reshape(-1)
    P = int(width) * int(height)
    assert rgb.shape == (3, P) and trgb.shape == (3, P) and dep.size == P and tdep.size == P
    grgb = np.zeros_like(rgb); gdep = np.zeros_like(dep)
    smap = np.zeros_like(rgb) if ssim_map else None
    L = lib().rtgo_loss_ssim(int(width), int(height), _ptr(rgb), _ptr(dep), _ptr(trgb), _ptr(tdep),
                             float(w_depth), float(lambda1), float(lambda2), _ptr(grgb), _ptr(gdep),
                             _ptr(smap) if smap is not None else None)
    if L != L:
        raise MemoryError("oracle loss_ssim failed")
    return (float(L), grgb, gdep, smap) if ssim_map else (float(L), grgb, gdep)


def score(scene, cams, settings, tile=(16, 16), mode=0):
    """Per-view score: mode 0 the rendered trace proxy sum_p sum_i u_i a_i T_i,
    mode 1 the binary-J trace sum_p sum_{i contributing at p} u_i."""
    g = _G(scene)
    ca = np.ascontiguousarray(np.concatenate([cam_array(c) for c in cams]))
    sa = set_array(settings)
    out = np.zeros(len(cams))
    rc = lib().rtgo_score(g.n, *g.all(), _ptr(ca), len(cams), _ptr(sa), int(tile[0]),
                          int(tile[1]), int(mode), _ptr(out))
    if rc:
        raise MemoryError("oracle score failed")
    return out


def adjoint(scene, cam, settings, g_rgb=None, g_depth=None, g_alpha=None, g_unc=None,
            tile=(16, 16), want_2d=False):
    """Gradient of sum_p <g_img(p), image(p)> for one camera with respect to
    means (3,N), log_scales (3,N), quats (4,N), opacity (N,), colors (3,N).
    out["touched"] (N,) bool marks the Gaussians that may contribute at a
    pixel holding a near-threshold decision (their gradient may legitimately
    follow another decision set)."""
    g = _G(scene)
    n = g.n
    out = {"means": np.zeros((3, n)), "log_scales": np.zeros((3, n)),
           "quats": np.zeros((4, n)), "opacity": np.zeros(n), "colors": np.zeros((3, n))}
    g2d = np.zeros((n, 10)) if want_2d else None
    touched = np.zeros(n, np.int32)
    planes = [None if a is None else _d(a) for a in (g_rgb, g_depth, g_alpha, g_unc)]
    ca, sa = cam_array(cam), set_array(settings)
    rc = lib().rtgo_adjoint(n, *g.all(), _ptr(ca), _ptr(sa), int(tile[0]), int(tile[1]),
                            *[_ptr(a) for a in planes],
                            _ptr(out["means"]), _ptr(out["log_scales"]), _ptr(out["quats"]),
                            _ptr(out["opacity"]), _ptr(out["colors"]), _ptr(g2d), _ptr(touched),
                            float(EV_ALPHA), float(EV_T))
    if rc:
        raise MemoryError("oracle adjoint failed")
    if want_2d:
        out["screen"] = g2d
    out["touched"] = touched.astype(bool)
    return out


def thresholds(uncert, k=0.5):
    """(mean - k std, mean + k std) of the uncertainties (Sec. IV-C: k = 1/2)."""
    u = _d(uncert).reshape(-1)
    lo = ctypes.c_double(); hi = ctypes.c_double()
    lib().rtgo_thresholds(u.size, _ptr(u), float(k), ctypes.addressof(lo), ctypes.addressof(hi))
    return float(lo.value), float(hi.value)


def view_utility(scene, cams, settings, lo, hi, range_=5.0, lam=1.0):
    """Per-camera (n_high, n_low, sum_u, xi) of the view utility of eq. (8)."""
    g = _G(scene)
    ca = np.ascontiguousarray(np.concatenate([cam_array(c) for c in cams]))
    nv = len(cams)
    nh = np.zeros(nv, np.int64); nl = np.zeros(nv, np.int64)
    su = np.zeros(nv); xi = np.zeros(nv)
    z_near = float(np.float32(settings["z_near"]))
    lib().rtgo_view_utility(g.n, _ptr(g.means), _ptr(g.u), _ptr(ca), nv, z_near,
                            float(np.float32(range_)), float(lo), float(hi), float(lam),
                            _ptr(nh), _ptr(nl), _ptr(su), _ptr(xi))
    return nh, nl, su, xi


def traj_select(xi, offsets):
    """(utilities float64[n_traj], best index) of eq. (10): trajectory t sums
    xi[offsets[t]:offsets[t+1]]; the first of the highest totals is chosen."""
    x = _d(xi).reshape(-1)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1))
    nt = off.size - 1
    if nt < 1 or off[0] < 0 or off[-1] > x.size or np.any(np.diff(off) < 0):
        raise ValueError("offsets must be non-decreasing within [0, len(xi)] with at least two entries")
    util = np.zeros(nt)
    best = lib().rtgo_traj_select(nt, _ptr(x), _ptr(off), _ptr(util))
    return util, int(best)


def uncertainty_update(means_prev, means_cur, u_prev, squared=False):
    """Per-Gaussian ||mu_k - mu_{k-1}|| (squared with squared=True); Gaussians
    whose mean did not change keep u_prev.  Means 3 x N."""
    mp, mc, up = _d(means_prev), _d(means_cur), _d(u_prev)
    n = up.size
    out = np.zeros(n)
    lib().rtgo_uncertainty_update(n, _ptr(mp), _ptr(mc), _ptr(up), int(bool(squared)), _ptr(out))
    return out


def region_grid(box, size):
    b = _d(box)
    dims = np.zeros(3, np.int32)
    if lib().rtgo_region_grid(_ptr(b), float(size), _ptr(dims)):
        raise ValueError("bad region box or size")
    return tuple(int(x) for x in dims)


def region_utility(means, u, box, size=2.5):
    """(count, sum, mean) per cuboid region of edge `size` of box (lo xyz, hi
    xyz), region index ix + nx (iy + ny iz)."""
    m, uu, b = _d(means), _d(u), _d(box)
    nx, ny, nz = region_grid(box, size)
    nr = nx * ny * nz
    cnt = np.zeros(nr, np.int64); sm = np.zeros(nr); mean = np.zeros(nr)
    if lib().rtgo_region_utility(uu.size, _ptr(m), _ptr(uu), _ptr(b), float(size), _ptr(cnt), _ptr(sm), _ptr(mean)):
        raise ValueError("bad region box or size")
    return cnt, sm, mean


def collision(means, log_scales, points, r_robot, lambda_g=3.0):
    """(collide int32[P], clearance float64[P]): point p collides when
    ||p - mu_i|| < r_robot + lambda_g exp(max log-scale_i) for some i;
    clearance = min_i (||p - mu_i|| - lambda_g r_i).  Planar 3 x N / 3 x P."""
    m, l, pts = _d(means), _d(log_scales), _d(points)
    n = m.shape[1] if m.ndim == 2 else 0
    npt = pts.shape[1] if pts.ndim == 2 else 0
    hit = np.zeros(npt, np.int32)
    clr = np.zeros(npt)
    lib().rtgo_collision(n, _ptr(m), _ptr(l), npt, _ptr(pts), float(r_robot), float(lambda_g), _ptr(hit), _ptr(clr))
    return hit, clr
