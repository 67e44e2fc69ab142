"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and the oracle.

This module only draws random numbers and builds camera poses. It holds none of
the rasterizer's arithmetic (no projection, compositing, loss or scoring), so
both sides can take their inputs from it without sharing any of the method.

Conventions
-----------
* A scene is a dict of contiguous float32 numpy arrays in planar
  structure-of-arrays layout: ``means`` (3, N), ``log_scales`` (3, N),
  ``quats`` (4, N; w, x, y, z), ``opacity`` (N,), ``colors`` (3, N),
  ``uncert`` (N,).
* A camera is a dict with ``width``, ``height``, ``fx``, ``fy``, ``cx``,
  ``cy`` and a pose ``R`` (3x3, camera-to-world, column k is camera axis k in
  world coordinates) and ``T`` (camera centre in the world) - the pose
  (R_k, T_k) of the projection in Sec. III (Gaussian Splatting paragraph).
  Camera axes follow OpenCV: x right, y down, z forward.
* Random draws use ``numpy.random.default_rng(seed)`` in FP64 in the fixed
  order means, log-scales, quaternions, opacity, colours, uncertainty, poses,
  and are then rounded to float32. Perturbations for targets use
  ``default_rng(seed + 1000)``. ``N(a, b)`` means mean a, standard deviation b.

The five workloads mirror the shapes of the paper's use of the rasterizer: a
small forward render, a 640x480 mapping step (Sec. III eq. (2)/(4)), batched
scoring of candidate views (Sec. IV-A eq. (7), "hundreds of viewpoints" in
Sec. V-A), multi-keyframe mapping, and uneven batched scoring. The paper's
datasets (iTHOR, MP3D, robot logs) are not available; these seeded scenes
stand in for them.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(F32))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def make_camera(width, height, fx, fy, cx, cy, R=None, T=None):
    R = np.eye(3) if R is None else np.asarray(R, dtype=np.float64)
    T = np.zeros(3) if T is None else np.asarray(T, dtype=np.float64)
    return {
        "width": int(width), "height": int(height),
        "fx": float(F32(fx)), "fy": float(F32(fy)),
        "cx": float(F32(cx)), "cy": float(F32(cy)),
        "R": _f32(R).reshape(3, 3), "T": _f32(T).reshape(3),
    }


def default_intrinsics(width, height):
    """f = 525 * W / 640 and principal point at the image centre."""
    f = 525.0 * width / 640.0
    return f, f, width / 2.0, height / 2.0


def yaw_pose(x, y, z, yaw):
    """Level camera (zero pitch/roll) in a z-up world, looking along yaw."""
    fwd = np.array([np.cos(yaw), np.sin(yaw), 0.0])
    right = np.array([np.sin(yaw), -np.cos(yaw), 0.0])
    down = np.array([0.0, 0.0, -1.0])
    R = np.stack([right, down, fwd], axis=1)
    return R, np.array([x, y, z], dtype=np.float64)


def random_rotation(rng):
    """Uniformly distributed rotation matrix (QR of a Gaussian matrix, sign-fixed)."""
    m = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(m)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _gaussians(rng, n, lo, hi, ls_mean=-3.0, ls_std=0.5, opacity="sigmoid"):
    lo = np.asarray(lo, dtype=np.float64)[:, None]
    hi = np.asarray(hi, dtype=np.float64)[:, None]
    means = lo + (hi - lo) * rng.random((3, n))
    log_scales = rng.normal(ls_mean, ls_std, (3, n))
    quats = _unit_quats(rng, n)
    if opacity == "sigmoid":
        op = _sigmoid(rng.standard_normal(n))
    elif opacity == "beta":
        op = rng.beta(0.5, 0.5, n)
    else:
        raise ValueError(opacity)
    colors = rng.random((3, n))
    uncert = rng.random(n)
    return means, log_scales, quats, op, colors, uncert


def _pack(means, log_scales, quats, op, colors, uncert):
    return {
        "means": _f32(means), "log_scales": _f32(log_scales),
        "quats": _f32(quats), "opacity": _f32(op),
        "colors": _f32(colors), "uncert": _f32(uncert),
    }


def _cluster_uncertainty(rng, means, uncert, lo, hi, n_centres=8, frac=0.1):
    """Mark the frac*N Gaussians nearest any of n_centres random centres as u=1."""
    lo = np.asarray(lo, dtype=np.float64)[:, None]
    hi = np.asarray(hi, dtype=np.float64)[:, None]
    centres = lo + (hi - lo) * rng.random((3, n_centres))
    d2 = np.full(means.shape[1], np.inf)
    for k in range(n_centres):
        d2 = np.minimum(d2, ((means - centres[:, k:k + 1]) ** 2).sum(0))
    m = int(frac * means.shape[1])
    idx = np.argsort(d2, kind="stable")[:m]
    uncert = uncert.copy()
    uncert[idx] = 1.0
    return uncert


def perturbed(scene, seed):
    """Target scene: means + N(0, 0.01), colours clip(c + N(0, 0.05), 0, 1)."""
    rng = np.random.default_rng(seed + 1000)
    m = scene["means"].astype(np.float64)
    c = scene["colors"].astype(np.float64)
    m = m + rng.normal(0.0, 0.01, m.shape)
    c = np.clip(c + rng.normal(0.0, 0.05, c.shape), 0.0, 1.0)
    out = dict(scene)
    out["means"] = _f32(m)
    out["colors"] = _f32(c)
    return out


ROOM_LO = (-10.0, -10.0, 0.0)
ROOM_HI = (10.0, 10.0, 4.0)


def config1(n=2000, seed=1):
    """Plain forward: 2,000 Gaussians, one 128x96 camera, identity pose."""
    rng = np.random.default_rng(seed)
    g = _pack(*_gaussians(rng, n, (-2, -2, 2), (2, 2, 6)))
    cams = [make_camera(128, 96, 100.0, 100.0, 64.0, 48.0)]
    return g, cams


def config2(n=200_000, seed=2, width=640, height=480):
    """Mapping step: 200k Gaussians in a 10 x 4 x 10 m camera-frame box, 640x480."""
    rng = np.random.default_rng(seed)
    g = _pack(*_gaussians(rng, n, (-5, -2, 2), (5, 2, 12)))
    f = 525.0 * width / 640.0
    cams = [make_camera(width, height, f, f, width / 2.0, height / 2.0)]
    return g, cams, perturbed(g, seed)


def _yaw_poses(rng, n_views, width, height, f=None):
    fx, fy, cx, cy = default_intrinsics(width, height)
    if f is not None:
        fx = fy = f
    cams = []
    xy = rng.uniform(-9.5, 9.5, (n_views, 2))
    yaw = rng.uniform(0.0, 2.0 * np.pi, n_views)
    for v in range(n_views):
        R, T = yaw_pose(xy[v, 0], xy[v, 1], 1.0, yaw[v])
        cams.append(make_camera(width, height, fx, fy, cx, cy, R, T))
    return cams


def config3(n=500_000, seed=3, n_views=64, width=320, height=240):
    """Batched scoring: 500k Gaussians in a 20x20x4 m room, 64 level poses."""
    rng = np.random.default_rng(seed)
    means, ls, q, op, col, unc = _gaussians(rng, n, ROOM_LO, ROOM_HI)
    unc = _cluster_uncertainty(rng, means, unc, ROOM_LO, ROOM_HI)
    g = _pack(means, ls, q, op, col, unc)
    cams = _yaw_poses(rng, n_views, width, height)
    return g, cams


def config4(n=1_000_000, seed=4, n_views=8, width=1280, height=720):
    """Batched keyframe backward: 1M Gaussians, 8 keyframes of 1280x720."""
    rng = np.random.default_rng(seed)
    g = _pack(*_gaussians(rng, n, ROOM_LO, ROOM_HI))
    cams = _yaw_poses(rng, n_views, width, height, f=1050.0 * width / 1280.0)
    return g, cams, perturbed(g, seed)


RES5 = ((160, 120), (320, 240), (640, 480))


def config5(n=2_000_000, seed=5, n_views=256):
    """Uneven batched scoring: 2M Gaussians, 256 views of mixed resolution."""
    rng = np.random.default_rng(seed)
    means, ls, q, op, col, unc = _gaussians(rng, n, ROOM_LO, ROOM_HI,
                                            ls_mean=-3.5, ls_std=0.7,
                                            opacity="beta")
    unc = _cluster_uncertainty(rng, means, unc, ROOM_LO, ROOM_HI)
    g = _pack(means, ls, q, op, col, unc)
    res = rng.integers(0, len(RES5), n_views)
    pos = np.stack([rng.uniform(-9.5, 9.5, n_views),
                    rng.uniform(-9.5, 9.5, n_views),
                    rng.uniform(0.2, 3.8, n_views)], axis=1)
    cams = []
    for v in range(n_views):
        w, h = RES5[res[v]]
        fx, fy, cx, cy = default_intrinsics(w, h)
        cams.append(make_camera(w, h, fx, fy, cx, cy,
                                random_rotation(rng), pos[v]))
    return g, cams


def trajectory_states(n_traj=64, L=8, seed=7, width=320, height=240, step=0.5, z=1.0, curvature=0.6):
    """Candidate trajectories of the trajectory planner (Sec. IV-B): n_traj
    motion primitives of L steps of `step` metres (the candidate spacing of
    Sec. V-A) in the C3-C5 room, each a level camera at height z that looks
    along its heading; start uniform in the room, heading U(0, 2 pi),
    curvature U(-c, c) per metre.  Returns (cameras, offsets): the n_traj
    (L + 1) states trajectory after trajectory, and offsets[t] = t (L + 1)."""
    rng = np.random.default_rng(seed)
    fx, fy, cx, cy = default_intrinsics(width, height)
    xy0 = rng.uniform(-8.0, 8.0, (n_traj, 2))
    th0 = rng.uniform(0.0, 2.0 * np.pi, n_traj)
    kap = rng.uniform(-curvature, curvature, n_traj)
    cams = []
    for t in range(n_traj):
        x, y, th = xy0[t, 0], xy0[t, 1], th0[t]
        for l in range(L + 1):
            R, T = yaw_pose(x, y, z, th)
            cams.append(make_camera(width, height, fx, fy, cx, cy, R, T))
            x += step * np.cos(th)
            y += step * np.sin(th)
            th += kap[t] * step
    offsets = np.arange(n_traj + 1, dtype=np.int32) * (L + 1)
    return cams, offsets


LOT_HALF = 20.0  # a 40 m x 40 m lot


def lot_scene(n=3_000_000, seed=6, n_obstacles=80, ground=0.6):
    """A 40 m x 40 m outdoor lot of n Gaussians lying on surfaces: a fraction
    `ground` on the ground plane (z ~ N(0, 0.02)), the rest on the mantles of
    `n_obstacles` upright cylinders (radius U(0.3, 2), height U(0.5, 3)).
    Log-scales N(-3.5, 0.3); the other attributes as in the room scenes.  The
    means come from default_rng(seed + 2000)."""
    rng = np.random.default_rng(seed)
    _, ls, q, op, col, unc = _gaussians(rng, n, (-LOT_HALF, -LOT_HALF, 0.0), (LOT_HALF, LOT_HALF, 3.0),
                                        ls_mean=-3.5, ls_std=0.3)
    r2 = np.random.default_rng(seed + 2000)
    n_g = int(round(ground * n))
    m = np.empty((3, n))
    m[0, :n_g] = r2.uniform(-LOT_HALF, LOT_HALF, n_g)
    m[1, :n_g] = r2.uniform(-LOT_HALF, LOT_HALF, n_g)
    m[2, :n_g] = r2.normal(0.0, 0.02, n_g)
    cx = r2.uniform(-LOT_HALF + 2, LOT_HALF - 2, n_obstacles)
    cy = r2.uniform(-LOT_HALF + 2, LOT_HALF - 2, n_obstacles)
    rad = r2.uniform(0.3, 2.0, n_obstacles)
    hgt = r2.uniform(0.5, 3.0, n_obstacles)
    k = r2.integers(0, n_obstacles, n - n_g)
    phi = r2.uniform(0, 2 * np.pi, n - n_g)
    m[0, n_g:] = cx[k] + rad[k] * np.cos(phi) + r2.normal(0, 0.02, n - n_g)
    m[1, n_g:] = cy[k] + rad[k] * np.sin(phi) + r2.normal(0, 0.02, n - n_g)
    m[2, n_g:] = r2.uniform(0, 1, n - n_g) * hgt[k]
    return _pack(m, ls, q, op, col, unc)


def path_points(n_paths, seed, samples=129, length=5.0, z=0.5, curvature=0.3):
    """Points sampled on motion primitives: n_paths arcs of the given length
    at height z, start uniform in the lot, heading U(0, 2 pi), curvature
    U(-c, c) per metre, each sampled at `samples` evenly spaced arc lengths
    (both ends included).  Planar (3, n_paths * samples), path after path."""
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-LOT_HALF + 3, LOT_HALF - 3, (2, n_paths))
    th0 = rng.uniform(0, 2 * np.pi, n_paths)
    kap = rng.uniform(-curvature, curvature, n_paths)
    ds = length / max(samples - 1, 1)
    s = np.arange(samples) * ds
    th = th0[:, None] + kap[:, None] * s[None, :]
    px = x0[0][:, None] + np.concatenate([np.zeros((n_paths, 1)), np.cumsum(np.cos(th[:, :-1]) * ds, 1)], 1)
    py = x0[1][:, None] + np.concatenate([np.zeros((n_paths, 1)), np.cumsum(np.sin(th[:, :-1]) * ds, 1)], 1)
    pts = np.stack([px.ravel(), py.ravel(), np.full(n_paths * samples, z)])
    return _f32(pts)


def tiny_scene(n, seed, width=32, height=24, depth=(1.5, 4.0), ls=(-2.5, 0.5),
               opacity="sigmoid"):
    """Small random scene in front of an identity camera (for brute force)."""
    rng = np.random.default_rng(seed)
    f = 0.9 * width
    zlo, zhi = depth
    half_w = 0.5 * width / f * zlo
    half_h = 0.5 * height / f * zlo
    g = _pack(*_gaussians(rng, n, (-half_w, -half_h, zlo), (half_w, half_h, zhi),
                          ls_mean=ls[0], ls_std=ls[1], opacity=opacity))
    cam = make_camera(width, height, f, f, width / 2.0 - 0.5, height / 2.0 - 0.5)
    return g, [cam]


def isotropic_scene(scene):
    """The same map as the paper's isotropic Gaussians (Sec. III): one
    log-radius per Gaussian (the first log-scale row, 1 x N) and no
    quaternion."""
    out = {k: v for k, v in scene.items() if k != "quats"}
    out["log_scales"] = np.ascontiguousarray(scene["log_scales"][:1])
    return out


def subset(scene, idx):
    """Gaussians at positions idx (keeps planar layout)."""
    out = {}
    for k, a in scene.items():
        out[k] = np.ascontiguousarray(a[..., idx])
    return out


def n_gaussians(scene):
    return int(scene["opacity"].shape[0])


DEFAULT_SETTINGS = {
    "tile_w": 16, "tile_h": 16, "batch": 0,
    "T_min": 1e-4, "alpha_min": 1.0 / 255.0, "alpha_max": 0.99,
    "z_near": 0.2, "eps2d": 0.0,
}
