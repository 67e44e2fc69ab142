"""Pins of the oracle's reverse-mode adjoint.

The adjoint (gradient used to refine the map, Sec. IV-A) is checked against
FP64 central finite differences of the oracle's own forward render, which is
itself pinned by the closed forms in test_oracle_pins.py, and against
single-Gaussian analytic derivatives of the compositing formula of Sec. III.
"""
import math

import numpy as np
import pytest

import oracle
import scenes
from test_oracle_pins import AMIN, cam, one_gaussian, S

GROUPS = ("means", "log_scales", "quats", "opacity", "colors")
CHANNELS = ("r", "g", "b", "depth", "alpha", "unc")


def _objective(scene, c, w):
    r = oracle.render(scene, c, S(), mode="brute")
    img = np.concatenate([r["rgb"], r["depth"][None], r["alpha"][None], r["unc"][None]])
    return float((w * img).sum()), r["ncontrib"]


def _adjoint(scene, c, w):
    return oracle.adjoint(scene, c, S(), g_rgb=w[:3], g_depth=w[3], g_alpha=w[4], g_unc=w[5])


def _f64(scene):
    return {k: np.array(v, dtype=np.float64) for k, v in scene.items()}


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_adjoint_matches_finite_differences(seed):
    g, cams = scenes.tiny_scene(8, seed, 32, 24, ls=(-2.0, 0.3))
    g = _f64(g)
    c = cams[0]
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((6, c["height"], c["width"]))
    adj = _adjoint(g, c, w)
    _, nc0 = _objective(g, c, w)
    checked = 0
    for grp in GROUPS:
        arr = g[grp]
        flat = arr.reshape(-1)
        ref = adj[grp].reshape(-1)
        scale = np.sqrt(np.mean(ref ** 2)) + 1e-30
        for j in range(flat.size):
            h = 1e-6 * max(1.0, abs(flat[j]))
            vals = []
            ok = True
            for sgn in (1, -1):
                pert = {k: v.copy() for k, v in g.items()}
                pert[grp].reshape(-1)[j] += sgn * h
                f, nc = _objective(pert, c, w)
                ok &= np.array_equal(nc, nc0)
                vals.append(f)
            if not ok:
                continue  # a skip/stop decision changed inside the stencil
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - ref[j]) <= 1e-6 * (abs(ref[j]) + scale) + 1e-9, (grp, j, fd, ref[j])
            checked += 1
    assert checked >= 0.9 * 14 * 8


def test_single_gaussian_analytic_derivatives():
    c = cam()
    o = 0.6
    g = one_gaussian((0.0, 0.0, 2.5), (-1.6, -2.0, -2.0), opacity=o, color=(0.3, 0.6, 0.9))
    r = oracle.render(g, c, S(), mode="brute")
    a = r["alpha"]
    H, W = a.shape
    ones = np.ones((H, W))
    zero = np.zeros((H, W))
    # d(sum_p C_r(p)) / d c_r = sum_p alpha(p)
    adj = oracle.adjoint(g, c, S(), g_rgb=np.stack([ones, zero, zero]))
    assert adj["colors"][0, 0] == pytest.approx(a.sum(), rel=1e-13)
    assert adj["colors"][1, 0] == 0.0
    # d(sum_p C_r(p)) / d o = c_r * sum_p G(p) over supported pixels (unclamped)
    assert adj["opacity"][0] == pytest.approx(0.3 * a.sum() / o, rel=1e-12)
    # d(sum_p A(p)) / d mean: by symmetry of the on-axis footprint about the
    # principal point only the depth direction survives
    adj_a = oracle.adjoint(g, c, S(), g_alpha=ones)
    assert adj_a["opacity"][0] == pytest.approx(a.sum() / o, rel=1e-12)
    # d(sum_p D(p)) / d mean_z includes the direct term sum_p alpha(p)
    # (depth of the Gaussian enters D linearly) plus the footprint shrinkage
    adj_d = oracle.adjoint(g, c, S(), g_depth=ones, want_2d=True)
    assert adj_d["screen"][0, 9] == pytest.approx(a.sum(), rel=1e-13)


def test_screen_space_mean_gradient_closed_form():
    # dC/dmu_2D at one pixel = c * alpha * Q delta (unclamped), Sec. III formula
    c = cam()
    g = one_gaussian((0.0, 0.0, 2.5), (-1.6, -2.0, -2.0), opacity=0.6, color=(1.0, 0, 0))
    p = oracle.project(g, c, S())
    H, W = c["height"], c["width"]
    y, x = int(c["cy"]) + 2, int(c["cx"]) + 3
    sel = np.zeros((3, H, W))
    sel[0, y, x] = 1.0
    adj = oracle.adjoint(g, c, S(), g_rgb=sel, want_2d=True)
    r = oracle.render(g, c, S(), mode="brute")
    alpha = r["alpha"][y, x]
    cov = p["cov2d"][:, 0]
    Q = np.linalg.inv(np.array([[cov[0], cov[1]], [cov[1], cov[2]]]))
    delta = np.array([x - p["mean2d"][0, 0], y - p["mean2d"][1, 0]])
    np.testing.assert_allclose(adj["screen"][0, :2], alpha * Q @ delta, rtol=1e-12)


def test_unit_quaternion_gradient_is_tangent():
    # the loss depends on q only through q/|q|, so the gradient is orthogonal to q
    g, cams = scenes.tiny_scene(20, 41, 32, 24)
    c = cams[0]
    rng = np.random.default_rng(0)
    w = rng.standard_normal((6, c["height"], c["width"]))
    adj = _adjoint(_f64(g), c, w)
    q = g["quats"].astype(np.float64)
    dots = (adj["quats"] * q).sum(0)
    assert np.abs(dots).max() <= 1e-12 * (np.abs(adj["quats"]).max() + 1e-30)


def test_uncertainty_alpha_channels_share_weights():
    # with u = 1 the uncertainty image equals the alpha image, so their
    # adjoints coincide for every parameter
    g, cams = scenes.tiny_scene(15, 43, 32, 24)
    g = dict(_f64(g), uncert=np.ones(15))
    c = cams[0]
    ones = np.ones((c["height"], c["width"]))
    a = oracle.adjoint(g, c, S(), g_alpha=ones)
    u = oracle.adjoint(g, c, S(), g_unc=ones)
    for grp in GROUPS:
        np.testing.assert_allclose(a[grp], u[grp], rtol=1e-12, atol=1e-15)
