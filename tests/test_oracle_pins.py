"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's formulas: each compares it with a
closed form derived independently (on-axis/off-axis projection, the
single-Gaussian image, two-Gaussian compositing, the transmittance cutoff),
with invariants of the compositing recursion, with a textbook sort, with brute
force, or with finite differences.
"""
import math

import numpy as np
import pytest

import oracle
import scenes

F32 = np.float32


def one_gaussian(mean, log_scales=(-2.0, -2.0, -2.0), quat=(1.0, 0.0, 0.0, 0.0),
                 opacity=0.8, color=(0.2, 0.5, 0.9), unc=0.7):
    return {
        "means": np.array(mean, np.float64).reshape(3, 1),
        "log_scales": np.array(log_scales, np.float64).reshape(3, 1),
        "quats": np.array(quat, np.float64).reshape(4, 1),
        "opacity": np.array([opacity], np.float64),
        "colors": np.array(color, np.float64).reshape(3, 1),
        "uncert": np.array([unc], np.float64),
    }


def stack(*gs):
    return {k: np.concatenate([g[k] for g in gs], axis=-1) for k in gs[0]}


def cam(w=64, h=48, fx=60.0, fy=55.0, cx=31.0, cy=23.0, R=None, T=None):
    return scenes.make_camera(w, h, fx, fy, cx, cy, R, T)


def S(**kw):
    s = dict(scenes.DEFAULT_SETTINGS)
    s.update(kw)
    return s


AMIN = float(F32(1.0 / 255.0))
AMAX = float(F32(0.99))
TMIN = float(F32(1e-4))


# --------------------------------------------------------------------------
# Projection (Sec. III: mu_2D = K R^T (mu - T) / d, r_2D = f r / d)
# --------------------------------------------------------------------------

def test_on_axis_isotropic_is_paper_radius():
    r, z = math.exp(-2.0), 3.0
    c = cam()
    p = oracle.project(one_gaussian((0, 0, z), (-2.0, -2.0, -2.0)), c, S())
    assert p["valid"][0]
    # paper: r_2D = f r / d, so Sigma_2D = diag(r_2D^2) per axis focal length
    assert p["cov2d"][0, 0] == pytest.approx((c["fx"] * r / z) ** 2, rel=1e-14)
    assert p["cov2d"][2, 0] == pytest.approx((c["fy"] * r / z) ** 2, rel=1e-14)
    assert abs(p["cov2d"][1, 0]) < 1e-14
    assert p["mean2d"][0, 0] == c["cx"] and p["mean2d"][1, 0] == c["cy"]
    assert p["depth"][0] == z


def test_on_axis_anisotropic_axis_aligned():
    sx, sy, z = math.exp(-1.5), math.exp(-2.5), 4.0
    c = cam()
    p = oracle.project(one_gaussian((0, 0, z), (-1.5, -2.5, -1.0)), c, S())
    assert p["cov2d"][0, 0] == pytest.approx((c["fx"] * sx / z) ** 2, rel=1e-14)
    assert p["cov2d"][2, 0] == pytest.approx((c["fy"] * sy / z) ** 2, rel=1e-14)


def test_off_axis_isotropic_closed_form():
    # isotropic Sigma = s^2 I  =>  Sigma_2D = s^2 J J^T with the perspective Jacobian
    s, x, y, z = math.exp(-2.2), 0.7, -0.4, 2.5
    c = cam()
    fx, fy = c["fx"], c["fy"]
    p = oracle.project(one_gaussian((x, y, z), (-2.2,) * 3), c, S())
    jxx = fx * fx / z ** 2 + fx * fx * x * x / z ** 4
    jxy = fx * fy * x * y / z ** 4
    jyy = fy * fy / z ** 2 + fy * fy * y * y / z ** 4
    np.testing.assert_allclose(p["cov2d"][:, 0], [s * s * jxx, s * s * jxy, s * s * jyy], rtol=1e-13)
    np.testing.assert_allclose(p["mean2d"][:, 0], [fx * x / z + c["cx"], fy * y / z + c["cy"]],
                               rtol=1e-15)
    cov = p["cov2d"][:, 0]
    det = cov[0] * cov[2] - cov[1] ** 2
    inv = np.linalg.inv(np.array([[cov[0], cov[1]], [cov[1], cov[2]]]))
    np.testing.assert_allclose(p["conic"][:, 0], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-12)
    assert det > 0


def test_quaternion_sign_and_norm_invariance():
    rng = np.random.default_rng(0)
    q = rng.standard_normal(4)
    base = one_gaussian((0.3, -0.2, 3.0), (-1.8, -2.4, -2.9), q)
    neg = one_gaussian((0.3, -0.2, 3.0), (-1.8, -2.4, -2.9), -q)
    big = one_gaussian((0.3, -0.2, 3.0), (-1.8, -2.4, -2.9), 3.7 * q)
    c = cam()
    a, b, d = (oracle.project(g, c, S()) for g in (base, neg, big))
    np.testing.assert_allclose(a["cov2d"], b["cov2d"], rtol=1e-13)
    np.testing.assert_allclose(a["cov2d"], d["cov2d"], rtol=1e-13)


def test_rotation_about_optical_axis_invariance():
    # s_x = s_y: rotating the Gaussian about the camera z axis leaves it unchanged
    c = cam()
    ref = oracle.project(one_gaussian((0, 0, 3.0), (-2.0, -2.0, -1.0)), c, S())
    for ang in (0.3, 1.1, 2.9):
        q = (math.cos(ang / 2), 0.0, 0.0, math.sin(ang / 2))
        p = oracle.project(one_gaussian((0, 0, 3.0), (-2.0, -2.0, -1.0), q), c, S())
        np.testing.assert_allclose(p["cov2d"], ref["cov2d"], rtol=1e-12, atol=1e-12)


def test_rotation_changes_axes():
    # 90 degrees about z swaps the x and y extents of an axis-aligned Gaussian
    c = cam(fx=50.0, fy=50.0)
    a = oracle.project(one_gaussian((0, 0, 3.0), (-1.5, -2.5, -2.0)), c, S())
    q = (math.cos(math.pi / 4), 0.0, 0.0, math.sin(math.pi / 4))
    b = oracle.project(one_gaussian((0, 0, 3.0), (-1.5, -2.5, -2.0), q), c, S())
    assert b["cov2d"][0, 0] == pytest.approx(a["cov2d"][2, 0], rel=1e-12)
    assert b["cov2d"][2, 0] == pytest.approx(a["cov2d"][0, 0], rel=1e-12)


def test_camera_pose_convention():
    # A Gaussian at p seen by the identity camera equals the Gaussian at R p + T
    # seen by the camera with pose (R, T) (R camera-to-world, T its centre).
    rng = np.random.default_rng(1)
    R = scenes.random_rotation(rng)
    T = rng.standard_normal(3)
    p_cam = np.array([0.4, -0.3, 2.7])
    world = R @ p_cam + T
    iso = (-2.1,) * 3
    c0 = cam()
    c1 = cam(R=R, T=T)
    # the camera stores R, T in binary32, so compare against that exact pose
    R32 = c1["R"].astype(np.float64)
    T32 = c1["T"].astype(np.float64)
    world = R32 @ p_cam + T32
    a = oracle.project(one_gaussian(p_cam, iso), c0, S())
    b = oracle.project(one_gaussian(world, iso), c1, S())
    np.testing.assert_allclose(b["mean2d"], a["mean2d"], rtol=1e-6)
    np.testing.assert_allclose(b["cov2d"], a["cov2d"], rtol=1e-5)
    assert b["depth"][0] == pytest.approx(2.7, rel=1e-6)


def test_rotated_anisotropic_on_axis_closed_form():
    # An on-axis Gaussian with s_x != s_y, rotated by +theta about the optical
    # axis (right-hand rule: its first axis turns towards the camera's +y,
    # i.e. down the image): Sigma = R_z(theta) diag(s^2) R_z(theta)^T, and with
    # J = diag(fx, fy) / z on the axis the 2D covariance is
    #   xx = (fx/z)^2 (sx^2 cos^2 + sy^2 sin^2), yy = (fy/z)^2 (sx^2 sin^2 + sy^2 cos^2),
    #   xy = (fx fy / z^2) (sx^2 - sy^2) sin cos.
    # The sign of xy fixes the orientation of the quaternion's rotation.
    c = cam(fx=60.0, fy=45.0)
    fx, fy = c["fx"], c["fy"]
    ls = (-1.2, -2.4, -1.8)
    sx, sy = math.exp(ls[0]), math.exp(ls[1])
    z = 3.0
    for deg in (30.0, -30.0, 75.0, 120.0):
        th = math.radians(deg)
        q = (math.cos(th / 2), 0.0, 0.0, math.sin(th / 2))
        p = oracle.project(one_gaussian((0, 0, z), ls, q), c, S())
        cs, sn = math.cos(th), math.sin(th)
        xx = (fx / z) ** 2 * (sx * sx * cs * cs + sy * sy * sn * sn)
        yy = (fy / z) ** 2 * (sx * sx * sn * sn + sy * sy * cs * cs)
        xy = fx * fy / z ** 2 * (sx * sx - sy * sy) * sn * cs
        np.testing.assert_allclose(p["cov2d"][:, 0], [xx, xy, yy], rtol=1e-12, atol=1e-12)
        # +30 degrees with s_x > s_y: the long axis runs right-down (xy > 0)
        if deg == 30.0:
            assert p["cov2d"][1, 0] > 0.0


def test_rotated_camera_equivalence_anisotropic():
    # A Gaussian at p with rotation q seen by the identity camera must project
    # exactly as the Gaussian at R p + T with rotation q_R * q (R applied after
    # q) seen by the camera with pose (R, T), R = rotation of q_R.  Rotations
    # and their composition come from scipy, not from the oracle's formulas; a
    # transposed Gaussian rotation or a transposed camera rotation (R Sigma R^T
    # in place of R^T Sigma R) breaks the equality.
    from scipy.spatial.transform import Rotation

    rng = np.random.default_rng(11)
    for trial in range(4):
        qg = rng.standard_normal(4)
        qg /= np.linalg.norm(qg)                      # w, x, y, z
        rot_g = Rotation.from_quat([qg[1], qg[2], qg[3], qg[0]])
        rot_c = Rotation.from_quat(rng.standard_normal(4))
        T = rng.standard_normal(3)
        # the camera stores R and T in binary32: use that exact pose, and
        # build the world rotation from it so that both sides share it
        c1 = cam(R=rot_c.as_matrix(), T=T)
        R32 = c1["R"].astype(np.float64).reshape(3, 3)
        T32 = c1["T"].astype(np.float64)
        rot_c32 = Rotation.from_matrix(R32)
        comp = (rot_c32 * rot_g).as_quat()            # x, y, z, w
        q_world = (comp[3], comp[0], comp[1], comp[2])
        p_cam = np.array([0.35, -0.25, 2.6]) + 0.1 * rng.standard_normal(3)
        ls = (-1.3, -2.6, -1.9)
        a = oracle.project(one_gaussian(p_cam, ls, tuple(qg)), cam(), S())
        b = oracle.project(one_gaussian(R32 @ p_cam + T32, ls, q_world), c1, S())
        assert a["valid"][0] and b["valid"][0]
        # R32 is orthogonal to ~1e-7 (binary32 rounding of a rotation)
        np.testing.assert_allclose(b["mean2d"], a["mean2d"], rtol=2e-6)
        np.testing.assert_allclose(b["cov2d"], a["cov2d"], rtol=2e-5, atol=2e-5 * np.abs(a["cov2d"]).max())
        # the off-diagonal term is not small here, so its sign is tested too
        assert abs(a["cov2d"][1, 0]) > 0.05 * math.sqrt(a["cov2d"][0, 0] * a["cov2d"][2, 0])
        assert np.sign(b["cov2d"][1, 0]) == np.sign(a["cov2d"][1, 0])


def test_depth_bits_are_binary32_of_depth():
    g, cams = scenes.config1(n=300)
    p = oracle.project(g, cams[0], S())
    v = p["valid"]
    assert np.array_equal(p["depth_bits"][v], p["depth"][v].astype(np.float32).view(np.uint32))


def test_culling_rules():
    c = cam()
    ok = one_gaussian((0, 0, 3.0))
    near = one_gaussian((0, 0, 0.2))          # depth <= z_near
    faint = one_gaussian((0, 0, 3.0), opacity=0.003)
    zeroq = one_gaussian((0, 0, 3.0), quat=(0, 0, 0, 0))
    nan = one_gaussian((0, float("nan"), 3.0))
    outside = one_gaussian((50.0, 0, 3.0))   # box entirely right of the image
    behind = one_gaussian((0, 0, -3.0))
    p = oracle.project(stack(ok, near, faint, zeroq, nan, outside, behind), c, S())
    assert p["valid"].tolist() == [True, False, False, False, False, False, False]


def test_box_is_exact_extent_of_support():
    # axis-aligned: half extent = sigma * sqrt(2 ln(o / alpha_min))
    c = cam()
    o = 0.6
    g = one_gaussian((0.05, -0.02, 2.0), (-2.0, -2.6, -2.0), opacity=o)
    p = oracle.project(g, c, S())
    sx = c["fx"] * math.exp(-2.0) / 2.0
    sy = c["fy"] * math.exp(-2.6) / 2.0
    rho = math.sqrt(2 * math.log(o / AMIN))
    # off-centre mean adds the small x-y coupling of the Jacobian; compare loosely
    assert p["half"][0, 0] == pytest.approx(sx * rho, rel=2e-3)
    assert p["half"][1, 0] == pytest.approx(sy * rho, rel=2e-3)
    # every pixel centre with o G >= alpha_min lies inside the box
    cov = p["cov2d"][:, 0]
    Q = np.linalg.inv(np.array([[cov[0], cov[1]], [cov[1], cov[2]]]))
    uu, vv = np.meshgrid(np.arange(c["width"]), np.arange(c["height"]))
    d = np.stack([uu - p["mean2d"][0, 0], vv - p["mean2d"][1, 0]], -1)
    a = o * np.exp(-0.5 * np.einsum("...i,ij,...j->...", d, Q, d))
    inside = a >= AMIN
    u0, u1, v0, v1 = p["box"][:, 0]
    assert inside.any()
    assert not inside[:, :u0].any() and not inside[:, u1 + 1:].any()
    assert not inside[:v0, :].any() and not inside[v1 + 1:, :].any()
    # and the box is tight: its extreme columns/rows contain support pixels
    assert inside[:, u0].any() or u0 == 0
    assert inside[v0, :].any() or v0 == 0


# --------------------------------------------------------------------------
# Compositing (Sec. III: C(p) = sum_i c_i f_i prod_{j<i} (1 - f_j); D likewise)
# --------------------------------------------------------------------------

def closed_form_single(c, g, settings):
    """Image of one axis-aligned on-axis Gaussian, derived independently."""
    z = g["means"][2, 0]
    sx = c["fx"] * math.exp(g["log_scales"][0, 0]) / z
    sy = c["fy"] * math.exp(g["log_scales"][1, 0]) / z
    mx = c["fx"] * g["means"][0, 0] / z + c["cx"]
    my = c["fy"] * g["means"][1, 0] / z + c["cy"]
    uu, vv = np.meshgrid(np.arange(c["width"], dtype=np.float64),
                         np.arange(c["height"], dtype=np.float64))
    a = g["opacity"][0] * np.exp(-0.5 * (((uu - mx) / sx) ** 2 + ((vv - my) / sy) ** 2))
    a = np.minimum(a, float(F32(settings["alpha_max"])))
    a = np.where(a >= float(F32(settings["alpha_min"])), a, 0.0)
    return a, z


@pytest.mark.parametrize("opacity", [0.5, 0.995])
def test_single_gaussian_closed_form(opacity):
    c = cam()
    g = one_gaussian((0.0, 0.0, 2.5), (-1.6, -2.0, -2.0), opacity=opacity)
    r = oracle.render(g, c, S(), mode="brute")
    a, z = closed_form_single(c, g, S())
    for ch in range(3):
        np.testing.assert_allclose(r["rgb"][ch], g["colors"][ch, 0] * a, atol=1e-12)
    np.testing.assert_allclose(r["alpha"], a, atol=1e-12)
    np.testing.assert_allclose(r["depth"], z * a, atol=1e-12)
    np.testing.assert_allclose(r["unc"], g["uncert"][0, ] * a, atol=1e-12)
    if opacity > AMAX:
        assert r["alpha"].max() == AMAX  # the clamp is hit at the centre


def test_two_gaussians_order_and_swap():
    c = cam()
    near = one_gaussian((0, 0, 2.0), (-1.0, -1.0, -1.0), opacity=0.6, color=(1, 0, 0))
    far = one_gaussian((0, 0, 3.0), (-0.8, -0.8, -0.8), opacity=0.7, color=(0, 1, 0))
    px = (int(c["cx"]), int(c["cy"]))
    for first, second in ((near, far), (far, near)):
        r = oracle.render(stack(first, second), c, S(), mode="brute")
        a1, _ = closed_form_single(c, near, S())
        a2, _ = closed_form_single(c, far, S())
        # whichever is listed first, the nearer one composites first
        expect_r = a1[px[1], px[0]]
        expect_g = a2[px[1], px[0]] * (1 - a1[px[1], px[0]])
        assert r["rgb"][0][px[1], px[0]] == pytest.approx(expect_r, rel=1e-14)
        assert r["rgb"][1][px[1], px[0]] == pytest.approx(expect_g, rel=1e-14)


def test_equal_depth_resolves_by_index():
    c = cam()
    a = one_gaussian((0, 0, 2.0), (-1.0,) * 3, opacity=0.6, color=(1, 0, 0))
    b = one_gaussian((0, 0, 2.0), (-1.0,) * 3, opacity=0.6, color=(0, 1, 0))
    r1 = oracle.render(stack(a, b), c, S(), mode="brute")
    r2 = oracle.render(stack(b, a), c, S(), mode="brute")
    y, x = int(c["cy"]), int(c["cx"])
    # lower index composites first: its colour gets the full weight alpha
    assert r1["rgb"][0][y, x] > r1["rgb"][1][y, x]
    assert r2["rgb"][1][y, x] > r2["rgb"][0][y, x]


def test_transmittance_cutoff_stack():
    # alpha = 0.95 at the centre: T = 0.05^n; 0.05^3 >= 1e-4 > 0.05^4, so
    # exactly three Gaussians contribute and A = 1 - 0.05^3 (to binary32 inputs)
    c = cam()
    gs = [one_gaussian((0, 0, 2.0 + 0.1 * k), (-1.0,) * 3, opacity=0.95,
                       color=(0.1 * (k + 1), 0, 0)) for k in range(6)]
    g = stack(*gs)
    g["opacity"] = g["opacity"].astype(np.float32).astype(np.float64)
    r = oracle.render(g, c, S(), mode="brute")
    y, x = int(c["cy"]), int(c["cx"])
    a = float(F32(0.95))
    assert r["ncontrib"][y, x] == 3
    assert r["alpha"][y, x] == pytest.approx(1 - (1 - a) ** 3, rel=1e-15)
    expect = sum(0.1 * (k + 1) * a * (1 - a) ** k for k in range(3))
    assert r["rgb"][0][y, x] == pytest.approx(expect, rel=1e-14)
    assert r["T"][y, x] >= TMIN


@pytest.mark.parametrize("seed,n", [(11, 50), (12, 500)])
def test_compositing_invariants(seed, n):
    g, cams = scenes.tiny_scene(n, seed, 64, 48)
    c = cams[0]
    g = {k: v.astype(np.float64) for k, v in g.items()}
    base = oracle.render(g, c, S())
    assert (base["T"] >= TMIN).all()
    assert (base["alpha"] >= 0).all() and (base["alpha"] <= 1).all()
    # u = 1 everywhere  =>  U = A  (sum of weights = 1 - T_final)
    g1 = dict(g, uncert=np.ones(n))
    r1 = oracle.render(g1, c, S())
    np.testing.assert_allclose(r1["unc"], r1["alpha"], atol=1e-13)
    # constant colour kappa  =>  C = kappa A
    g2 = dict(g, colors=np.full((3, n), 0.37))
    r2 = oracle.render(g2, c, S())
    for ch in range(3):
        np.testing.assert_allclose(r2["rgb"][ch], 0.37 * r2["alpha"], atol=1e-13)
    # all Gaussians at one depth z0  =>  D = z0 A
    m = g["means"].copy()
    m[2] = 3.0
    r3 = oracle.render(dict(g, means=m), c, S())
    np.testing.assert_allclose(r3["depth"], 3.0 * r3["alpha"], atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3, 10, 50, 500])
@pytest.mark.parametrize("size", [(32, 24), (64, 48)])
def test_brute_force_equals_tiled(n, size):
    g, cams = scenes.tiny_scene(n, 100 + n, *size)
    brute = oracle.render(g, cams[0], S(), mode="brute")
    for tile in ((8, 8), (16, 16), (32, 8)):
        tiled = oracle.render(g, cams[0], S(), mode="tiled", tile=tile)
        for k in ("rgb", "depth", "alpha", "unc", "T", "ncontrib"):
            assert np.array_equal(brute[k], tiled[k]), (k, tile)


def test_gaussian_order_permutation_invariance():
    g, cams = scenes.tiny_scene(200, 7, 64, 48)
    rng = np.random.default_rng(3)
    perm = rng.permutation(200)
    a = oracle.render(g, cams[0], S())
    b = oracle.render(scenes.subset(g, perm), cams[0], S())
    for k in ("rgb", "depth", "alpha", "unc"):
        assert np.array_equal(a[k], b[k])


def test_events_reported_near_thresholds():
    # on-axis Gaussian; choose the opacity so that the pixel 30 px right of the
    # centre has alpha = alpha_min (1 + 1e-7), i.e. inside the event band
    c = cam()
    z = 2.0
    sig = c["fx"] * math.exp(-1.0) / z
    k = 30
    o = AMIN * (1 + 1e-7) * math.exp(k * k / (2 * sig * sig))
    g = one_gaussian((0.0, 0.0, z), (-1.0, -1.0, -1.0), opacity=o)
    r = oracle.render(g, c, S(), mode="brute")
    y, x = int(c["cy"]), int(c["cx"]) + k
    assert r["nevents"][y, x] == 1
    assert r["alpha"][y, x] > 0.0  # the primary decision includes it
    j = list(r["alt_pix"]).index(y * c["width"] + x)
    alts = r["alt_val"][j]
    # the alternative takes the other decision: the Gaussian is skipped
    assert alts[0, 4] > 0.0 and alts[1, 4] == 0.0


# --------------------------------------------------------------------------
# Support tiles: a tile is binned only if one of its pixel centres has
# alpha >= alpha_min (the skip test of Sec. III's compositing loop)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ls,tile", [((-2.0, -2.0, -2.0), (16, 16)), ((-1.2, -3.0, -2.0), (8, 8)),
                                     ((-3.1, -1.4, -2.5), (32, 8))])
def test_support_tiles_of_axis_aligned_ellipse(ls, tile):
    # on the optical axis with identity rotation, Sigma_2D = diag((fx sx/z)^2, (fy sy/z)^2):
    # the support is the axis-aligned ellipse ((u-cx)/ax)^2 + ((v-cy)/ay)^2 <= 2 ln(o/amin),
    # and the smallest value over a tile's pixel centres is a sum of per-axis minima
    z, o = 2.5, 0.6
    c = cam(w=200, h=150, fx=180.0, fy=170.0, cx=97.3, cy=71.8)
    g = one_gaussian((0, 0, z), ls, opacity=o)
    ax = 180.0 * math.exp(ls[0]) / z
    ay = 170.0 * math.exp(ls[1]) / z
    rho2 = 2.0 * math.log(F32(o) / AMIN)
    tw, th = tile
    ntx, nty = -(-200 // tw), -(-150 // th)
    expect = []
    for ty in range(nty):
        vs = np.arange(ty * th, min(ty * th + th, 150))
        my = np.min(((vs - 71.8) / ay) ** 2)
        for tx in range(ntx):
            us = np.arange(tx * tw, min(tx * tw + tw, 200))
            mx = np.min(((us - 97.3) / ax) ** 2)
            assert abs(mx + my - rho2) > 1e-6  # no tile on the boundary
            if mx + my <= rho2:
                expect.append(ty * ntx + tx)
    k, v = oracle.keys(g, [c], S(), tile, support=True)
    assert np.array_equal((k >> np.uint64(32)).astype(np.int64), np.array(expect, np.int64))
    kb, _ = oracle.keys(g, [c], S(), tile)
    # the pixel box tiles hold the support tiles
    assert len(kb) >= len(k) and set((kb >> np.uint64(32)).tolist()) >= set(expect)
    assert oracle.count(g, c, S(), tile, support=True)[1] == len(expect)


def test_support_keys_are_the_box_keys_restricted():
    g, cams = scenes.config1(n=600)
    idx = np.concatenate([np.arange(600), np.arange(0, 600, 31)])
    g = scenes.subset(g, idx)
    for tile in ((16, 16), (8, 8), (32, 8)):
        kb, vb = oracle.keys(g, cams, S(), tile)
        ks, vs = oracle.keys(g, cams, S(), tile, support=True)
        box = (kb >> np.uint64(32)) << np.uint64(32) | vb.astype(np.uint64)
        sup = (ks >> np.uint64(32)) << np.uint64(32) | vs.astype(np.uint64)
        keep = np.isin(box, sup)
        # same order: the support pairs are a subsequence of the box pairs
        assert keep.sum() == len(ks) and len(ks) < len(kb)
        assert np.array_equal(kb[keep], ks) and np.array_equal(vb[keep], vs)
        # rendering from support tiles only is what the tiled render gives:
        # every pixel that composites Gaussian i lies in one of i's support tiles
        r = oracle.render(g, cams[0], S(), tile=tile)
        p = oracle.project(g, cams[0], S())
        tw, th = tile
        ntx = -(-cams[0]["width"] // tw)
        pairs = set(sup.tolist())
        rng = np.random.default_rng(1)
        for i in rng.choice(np.nonzero(p["valid"])[0], 40, replace=False):
            u0, u1, v0, v1 = p["box"][:, i]
            solo = oracle.render(scenes.subset(g, [i]), cams[0], S(), mode="brute")
            ys, xs = np.nonzero(solo["alpha"] > 0)
            for y, x in zip(ys, xs):
                assert ((y // th) * ntx + x // tw) << 32 | int(i) in pairs
        assert r["alpha"].max() > 0


# --------------------------------------------------------------------------
# Sorted binning keys: (tile << 32 | binary32 depth bits), ties by index
# --------------------------------------------------------------------------

def test_keys_match_textbook_sort():
    g, cams = scenes.config1(n=400)
    c = cams[0]
    # duplicate a few Gaussians to create exact depth ties
    idx = np.concatenate([np.arange(400), np.arange(0, 400, 37)])
    g = scenes.subset(g, idx)
    for tile in ((16, 16), (8, 8), (32, 8)):
        k, v = oracle.keys(g, [c], S(), tile)
        p = oracle.project(g, c, S())
        tw, th = tile
        ntx = (c["width"] + tw - 1) // tw
        ek, ev = [], []
        for i in np.nonzero(p["valid"])[0]:
            u0, u1, v0, v1 = p["box"][:, i]
            for ty in range(v0 // th, v1 // th + 1):
                for tx in range(u0 // tw, u1 // tw + 1):
                    ek.append((ty * ntx + tx) << 32 | int(p["depth_bits"][i]))
                    ev.append(i)
        ek = np.array(ek, np.uint64)
        ev = np.array(ev, np.uint32)
        order = np.lexsort((ev, ek))  # textbook stable ordering on (key, index)
        assert np.array_equal(k, ek[order]) and np.array_equal(v, ev[order])
        assert len(np.unique(k)) < len(k)  # ties exist and were ordered by index


# --------------------------------------------------------------------------
# Loss (Sec. III eq. (4), L1 terms; colour weight 1, depth weight 0.5)
# --------------------------------------------------------------------------

def test_loss_worked_example():
    rgb = np.array([[[0.5, 0.2]], [[0.1, 0.1]], [[0.9, 0.0]]])      # (3, 1, 2)
    trgb = np.array([[[0.4, 0.2]], [[0.3, 0.1]], [[0.9, 0.5]]])
    dep = np.array([[2.0, 1.0]])
    tdep = np.array([[1.0, 1.5]])
    L, grgb, gdep = oracle.loss(rgb, dep, trgb, tdep, 0.5)
    # pixel 0: 0.1 + 0.2 + 0 + 0.5*1 = 0.8 ; pixel 1: 0 + 0 + 0.5 + 0.5*0.5 = 0.75
    assert L == pytest.approx((0.8 + 0.75) / 2, rel=1e-15)
    np.testing.assert_array_equal(grgb[:, 0, 0], [0.5, -0.5, 0.0])
    np.testing.assert_array_equal(grgb[:, 0, 1], [0.0, 0.0, -0.5])
    np.testing.assert_array_equal(gdep[0], [0.25, -0.25])


# --------------------------------------------------------------------------
# Score: sum over pixels of the composited uncertainty (rendered form of the
# trace proxy, Sec. IV-A eq. (7))
# --------------------------------------------------------------------------

def test_score_unit_uncertainty_is_alpha_sum():
    g, cams = scenes.tiny_scene(300, 21, 64, 48)
    g = dict(g, uncert=np.ones(300, np.float32))
    s = oracle.score(g, cams, S())
    r = oracle.render(g, cams[0], S())
    assert s[0] == pytest.approx(r["alpha"].sum(), rel=1e-13)


def test_score_single_gaussian_integral():
    # one wide Gaussian fully inside the image: sum_p o G ~ 2 pi sx sy (o - alpha_min)
    c = cam(w=200, h=160, fx=100.0, fy=100.0, cx=100.0, cy=80.0)
    o = 0.7
    g = one_gaussian((0.0, 0.0, 2.0), (-1.2, -1.5, -1.0), opacity=o, unc=1.0)
    s = oracle.score(g, [c], S())[0]
    sx = 100.0 * math.exp(-1.2) / 2.0
    sy = 100.0 * math.exp(-1.5) / 2.0
    integral = 2 * math.pi * sx * sy * (o - AMIN)
    rho = math.sqrt(2 * math.log(o / AMIN))
    perimeter = 2 * math.pi * rho * math.sqrt((sx * sx + sy * sy) / 2)
    assert abs(s - integral) <= AMIN * perimeter + 1e-6 * integral


# Binary-J trace (eq. (7) with the Jacobian replaced by its sparsity
# pattern): per pixel, the sum of u over the Gaussians that contribute.

def test_binary_score_single_gaussian_footprint():
    # on the optical axis with identity rotation the support is the ellipse
    # ((u-cx)/ax)^2 + ((v-cy)/ay)^2 <= 2 ln(o/amin); each pixel inside adds u
    z, o, u = 2.5, 0.6, 0.37
    ls = (-1.2, -1.7, -2.0)
    c = cam(w=200, h=150, fx=180.0, fy=170.0, cx=97.3, cy=71.8)
    g = one_gaussian((0, 0, z), ls, opacity=o, unc=u)
    ax = 180.0 * math.exp(ls[0]) / z
    ay = 170.0 * math.exp(ls[1]) / z
    rho2 = 2.0 * math.log(o / AMIN)
    U, V = np.meshgrid(np.arange(200), np.arange(150))
    q = ((U - 97.3) / ax) ** 2 + ((V - 71.8) / ay) ** 2
    assert np.min(np.abs(q - rho2)) > 1e-6
    n_inside = int((q <= rho2).sum())
    assert oracle.score(g, [c], S(), mode=1)[0] == pytest.approx(u * n_inside, rel=1e-12)


def test_binary_score_equal_alpha_stack():
    # five coincident Gaussians (equal depth, ties by index): at a pixel with
    # alpha a >= alpha_min each, exactly k = min(5, floor(ln T_min / ln(1 - a)))
    # contribute, the first k in index order
    z, o = 2.0, 0.95
    c = cam(w=48, h=40, fx=60.0, fy=60.0, cx=23.5, cy=19.5)
    us = [0.11, 0.23, 0.35, 0.47, 0.59]
    g = stack(*[one_gaussian((0, 0, z), (-1.5,) * 3, opacity=o, unc=u) for u in us])
    sig = 60.0 * math.exp(-1.5) / z
    U, V = np.meshgrid(np.arange(48), np.arange(40))
    G = np.exp(-0.5 * ((U - 23.5) ** 2 + (V - 19.5) ** 2) / sig ** 2)
    a = np.minimum(AMAX, o * G)
    ratio = np.log(TMIN) / np.log1p(-a)
    keep = a >= AMIN
    assert np.min(np.abs(ratio - np.round(ratio))[keep]) > 1e-6 and np.min(np.abs(a - AMIN)) > 1e-9
    k = np.where(keep, np.minimum(5, np.floor(ratio)), 0).astype(int)
    cum = np.concatenate([[0.0], np.cumsum(us)])
    assert (k == 3).any() and (k == 5).any()
    want = cum[k].sum()
    assert oracle.score(g, [c], S(), mode=1)[0] == pytest.approx(want, rel=1e-12)


def test_binary_score_relations():
    g, cams = scenes.config3(n=3000, n_views=3, width=64, height=48)
    rendered = oracle.score(g, cams, S())
    binary = oracle.score(g, cams, S(), mode=1)
    assert np.all(binary >= rendered) and np.all(binary > 0)
    # u = 1: the binary score counts contributing (pixel, Gaussian) pairs
    g1 = dict(g, uncert=np.ones_like(g["uncert"]))
    b1 = oracle.score(g1, cams, S(), mode=1)
    for v, c in enumerate(cams):
        assert b1[v] == oracle.render(g1, c, S())["ncontrib"].sum()


def test_score_batch_invariance():
    g, cams = scenes.config3(n=3000, n_views=4, width=64, height=48)
    batch = oracle.score(g, cams, S())
    for v in range(4):
        assert oracle.score(g, [cams[v]], S())[0] == batch[v]
