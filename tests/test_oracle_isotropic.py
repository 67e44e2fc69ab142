"""Pins of the oracle's isotropic mode: the paper's 8-parameter Gaussian of
Sec. III (colour, mean, radius, opacity), projected with r_2D = f r / d and
splatted as f_i(p) = alpha_i exp(-|p - mu_2D|^2 / (2 r_2D^2)), against the
closed forms of the paper's equations and finite differences."""
import math

import numpy as np
import pytest

import oracle
from test_oracle_pins import AMAX, AMIN, cam, S

ISO = {"isotropic": 1}


def iso_gaussians(means, log_r, opacity, colors, unc=None):
    n = len(log_r)
    return {
        "means": np.array(means, np.float64).reshape(3, n),
        "log_scales": np.array(log_r, np.float64).reshape(1, n),
        "opacity": np.array(opacity, np.float64).reshape(n),
        "colors": np.array(colors, np.float64).reshape(3, n),
        "uncert": np.array(unc if unc is not None else [0.5] * n, np.float64).reshape(n),
    }


@pytest.mark.parametrize("mean", [(0.0, 0.0, 3.0), (0.9, -0.6, 2.5), (-1.4, 1.1, 4.0)])
def test_projection_is_paper_radius_on_and_off_axis(mean):
    r = math.exp(-2.2)
    c = cam()
    p = oracle.project(iso_gaussians([[m] for m in mean], [-2.2], [0.8], [[0.1], [0.2], [0.3]]), c, S(**ISO))
    assert p["valid"][0]
    x, y, z = mean
    # mu_2D = K t / d, r_2D = f r / d per image axis, no off-diagonal term
    assert p["mean2d"][0, 0] == pytest.approx(c["fx"] * x / z + c["cx"], abs=1e-12)
    assert p["mean2d"][1, 0] == pytest.approx(c["fy"] * y / z + c["cy"], abs=1e-12)
    assert p["cov2d"][0, 0] == pytest.approx((c["fx"] * r / z) ** 2, rel=1e-14)
    assert p["cov2d"][1, 0] == 0.0
    assert p["cov2d"][2, 0] == pytest.approx((c["fy"] * r / z) ** 2, rel=1e-14)
    # the anisotropic EWA projection of the same sphere agrees on the optical axis only
    ewa = oracle.project({"means": np.array(mean, np.float64).reshape(3, 1),
                          "log_scales": np.full((3, 1), -2.2), "quats": np.array([[1.0], [0], [0], [0]]),
                          "opacity": np.array([0.8]), "colors": np.zeros((3, 1)), "uncert": np.zeros(1)}, c, S())
    same = np.allclose(ewa["cov2d"][:, 0], p["cov2d"][:, 0], rtol=1e-12, atol=0)
    assert same == (x == 0.0 and y == 0.0)


def test_single_gaussian_image_is_paper_formula():
    c = cam(w=40, h=30, fx=50.0, fy=50.0, cx=19.0, cy=14.0)
    lr, o = -1.6, 0.7
    col = (0.3, 0.6, 0.9)
    mean = (0.2, -0.1, 2.0)
    g = iso_gaussians([[m] for m in mean], [lr], [o], [[v] for v in col])
    rend = oracle.render(g, c, S(**ISO), mode="brute")
    f = c["fx"]
    r2d = f * math.exp(lr) / mean[2]
    mx = f * mean[0] / mean[2] + c["cx"]
    my = f * mean[1] / mean[2] + c["cy"]
    v, u = np.mgrid[0:30, 0:40]
    a = o * np.exp(-((u - mx) ** 2 + (v - my) ** 2) / (2 * r2d * r2d))
    a = np.minimum(a, AMAX)
    a = np.where(a >= AMIN, a, 0.0)
    for ch in range(3):
        assert np.abs(rend["rgb"][ch] - col[ch] * a).max() < 1e-12
    assert np.abs(rend["alpha"] - a).max() < 1e-12
    assert np.abs(rend["depth"] - mean[2] * a).max() < 1e-12


def test_two_gaussians_composite_in_depth_order():
    c = cam(w=24, h=20, fx=30.0, fy=30.0, cx=11.0, cy=9.0)
    # front (d = 2) red, back (d = 3) blue, overlapping
    g = iso_gaussians([[0.0, 0.05], [0.0, -0.02], [2.0, 3.0]], [-1.0, -0.8], [0.6, 0.9],
                      [[1.0, 0.0], [0.0, 0.0], [0.0, 1.0]])
    rend = oracle.render(g, c, S(**ISO), mode="brute")
    v, u = np.mgrid[0:20, 0:24]

    def f_i(k):
        z = g["means"][2, k]
        r2d = 30.0 * math.exp(g["log_scales"][0, k]) / z
        mx = 30.0 * g["means"][0, k] / z + 11.0
        my = 30.0 * g["means"][1, k] / z + 9.0
        a = np.minimum(g["opacity"][k] * np.exp(-((u - mx) ** 2 + (v - my) ** 2) / (2 * r2d * r2d)), AMAX)
        return np.where(a >= AMIN, a, 0.0)

    a0, a1 = f_i(0), f_i(1)
    # C = c_0 f_0 + c_1 f_1 (1 - f_0)
    assert np.abs(rend["rgb"][0] - a0).max() < 1e-12
    assert np.abs(rend["rgb"][2] - a1 * (1 - a0)).max() < 1e-12


def test_quaternion_and_extra_scales_are_not_read():
    c = cam()
    g = iso_gaussians([[0.3, -0.2], [0.1, 0.2], [2.5, 3.5]], [-2.0, -1.7], [0.8, 0.5],
                      [[0.1, 0.9], [0.4, 0.2], [0.7, 0.3]])
    base = oracle.render(g, c, S(**ISO), mode="brute")
    g2 = dict(g)
    g2["log_scales"] = np.vstack([g["log_scales"], [[5.0, -9.0]], [[np.nan, 1.0]]])
    g2["quats"] = np.array([[0.0, np.nan], [0.0, 2.0], [0.0, 0.1], [0.0, 0.3]])
    other = oracle.render(g2, c, S(**ISO), mode="brute")
    for k in ("rgb", "depth", "alpha", "unc"):
        assert np.array_equal(base[k], other[k])


def _objective(scene, c, w):
    r = oracle.render(scene, c, S(**ISO), mode="brute")
    img = np.concatenate([r["rgb"], r["depth"][None], r["alpha"][None], r["unc"][None]])
    return float((w * img).sum()), r["ncontrib"]


@pytest.mark.parametrize("seed", [41, 42])
def test_isotropic_adjoint_matches_finite_differences(seed):
    rng = np.random.default_rng(seed)
    n = 8
    c = cam(w=32, h=24, fx=28.0, fy=26.0, cx=15.0, cy=11.0)
    z = rng.uniform(1.5, 4.0, n)
    g = iso_gaussians(np.stack([rng.uniform(-0.5, 0.5, n) * z, rng.uniform(-0.4, 0.4, n) * z, z]),
                      rng.normal(-2.0, 0.3, n), rng.uniform(0.3, 0.95, n), rng.random((3, n)), rng.random(n))
    w = rng.standard_normal((6, 24, 32))
    adj = oracle.adjoint(g, c, S(**ISO), g_rgb=w[:3], g_depth=w[3], g_alpha=w[4], g_unc=w[5])
    assert not adj["quats"].any() and not adj["log_scales"][1:].any()
    _, nc0 = _objective(g, c, w)
    checked = 0
    for grp in ("means", "log_scales", "opacity", "colors"):
        flat = g[grp].reshape(-1)
        ref = adj[grp][:1].reshape(-1) if grp == "log_scales" else adj[grp].reshape(-1)
        scale = np.sqrt(np.mean(ref ** 2)) + 1e-30
        for j in range(flat.size):
            h = 1e-6 * max(1.0, abs(flat[j]))
            vals, ok = [], True
            for sgn in (1, -1):
                pert = {k: v.copy() for k, v in g.items()}
                pert[grp].reshape(-1)[j] += sgn * h
                f, nc = _objective(pert, c, w)
                ok &= np.array_equal(nc, nc0)
                vals.append(f)
            if not ok:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - ref[j]) <= 1e-6 * (abs(ref[j]) + scale) + 1e-9, (grp, j, fd, ref[j])
            checked += 1
    assert checked >= 0.9 * 8 * n
