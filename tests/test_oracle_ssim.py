"""Pins of the oracle's paper-faithful mapping loss (Sec. III eq. (4)): the L1
terms plus lambda2 (1 - SSIM), SSIM with an 11x11 Gaussian window (sigma 1.5),
zero padding, C1 = 0.01^2, C2 = 0.03^2."""
import numpy as np
import pytest
from scipy import ndimage

import oracle

C1 = 0.01 ** 2
C2 = 0.03 ** 2


def images(W, H, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((3, H * W))
    y = np.clip(x + rng.normal(0, 0.15, x.shape), 0, 1)
    d = rng.uniform(1, 5, H * W)
    td = d + rng.choice([-1, 1], H * W) * rng.uniform(0.01, 0.2, H * W)
    return x, y, d, td


def ssim_map_scipy(x, y, W, H):
    """The SSIM map from scipy's separable Gaussian filter (radius 5 =
    int(truncate * sigma + 0.5), zero padding)."""
    f = lambda a: ndimage.gaussian_filter(a, 1.5, mode="constant", cval=0.0, truncate=5.0 / 1.5)
    out = np.empty_like(x)
    for ch in range(3):
        a = x[ch].reshape(H, W)
        b = y[ch].reshape(H, W)
        mx, my = f(a), f(b)
        sx = f(a * a) - mx * mx
        sy = f(b * b) - my * my
        sxy = f(a * b) - mx * my
        s = (2 * mx * my + C1) * (2 * sxy + C2) / ((mx * mx + my * my + C1) * (sx + sy + C2))
        out[ch] = s.ravel()
    return out


@pytest.mark.parametrize("W,H", [(13, 9), (32, 24), (7, 30)])
def test_ssim_map_matches_scipy_filter(W, H):
    x, y, d, td = images(W, H, W * H)
    _, _, _, S = oracle.loss_ssim(x, d, y, td, W, H, ssim_map=True)
    ref = ssim_map_scipy(x, y, W, H)
    assert np.abs(S - ref).max() < 1e-12


def test_identical_images():
    W, H = 20, 11
    x, _, d, _ = images(W, H, 1)
    L, g, gd, S = oracle.loss_ssim(x, d, x, d, W, H, ssim_map=True)
    assert np.abs(S - 1.0).max() < 1e-15
    assert L == 0.0
    # SSIM is maximal at x = y, so its gradient vanishes; the L1 gradient is sign(0) = 0
    assert np.abs(g).max() < 1e-15 and np.abs(gd).max() == 0.0


def test_constant_images_interior_closed_form():
    W, H = 24, 20
    a, b = 0.3, 0.7
    x = np.full((3, W * H), a)
    y = np.full((3, W * H), b)
    d = np.ones(W * H)
    _, _, _, S = oracle.loss_ssim(x, d, y, d, W, H, ssim_map=True)
    S = S.reshape(3, H, W)
    interior = S[:, 5:H - 5, 5:W - 5]
    # no variance inside the window: the structure factor is C2 / C2, up to the
    # rounding of E[x^2] - mx^2 (~1e-17) relative to C2 = 9e-4
    assert np.abs(interior - (2 * a * b + C1) / (a * a + b * b + C1)).max() < 1e-12
    # at a corner the window is cut, so the local variance is not zero and S differs
    assert abs(S[0, 0, 0] - (2 * a * b + C1) / (a * a + b * b + C1)) > 1e-3


def test_single_pixel_closed_form():
    # a 1x1 image keeps only the window's centre weight w0 = g0^2
    g0 = 1.0 / np.exp(-np.arange(-5, 6) ** 2 / 4.5).sum()
    w0 = g0 * g0
    for xv, yv in ((0.2, 0.9), (0.5, 0.5), (1.0, 0.0)):
        x = np.full((3, 1), xv)
        y = np.full((3, 1), yv)
        _, _, _, S = oracle.loss_ssim(x, [1.0], y, [1.0], 1, 1, ssim_map=True)
        mx, my = w0 * xv, w0 * yv
        sx = w0 * xv * xv - mx * mx
        sy = w0 * yv * yv - my * my
        sxy = w0 * xv * yv - mx * my
        ref = (2 * mx * my + C1) * (2 * sxy + C2) / ((mx * mx + my * my + C1) * (sx + sy + C2))
        assert np.abs(S - ref).max() < 1e-15


def test_loss_value_composition():
    W, H = 16, 12
    x, y, d, td = images(W, H, 3)
    L, _, _, S = oracle.loss_ssim(x, d, y, td, W, H, w_depth=1.0, lambda1=0.4, lambda2=0.1, ssim_map=True)
    P = W * H
    l1 = (np.abs(d - td) + 0.4 * np.abs(x - y).sum(0)).sum() / P
    assert L == pytest.approx(l1 + 0.1 * (1 - S.mean()), rel=1e-14)
    # without the SSIM term, the L1 part is the one of the config-form loss
    L0, g0, gd0 = oracle.loss_ssim(x, d, y, td, W, H, w_depth=0.5, lambda1=1.0, lambda2=0.0)
    Lr, gr, gdr = oracle.loss(x, d, y, td, 0.5)
    assert L0 == pytest.approx(Lr, rel=1e-14)
    assert np.array_equal(g0, gr) and np.array_equal(gd0, gdr)


@pytest.mark.parametrize("lambda1,w_depth", [(0.0, 0.0), (0.4, 1.0)])
def test_gradient_finite_differences(lambda1, w_depth):
    W, H = 13, 9
    x, y, d, td = images(W, H, 5)
    # keep the L1 terms away from their kinks
    y = np.where(np.abs(x - y) < 0.02, np.clip(x + 0.05, 0, 1) - 0.1 * (x > 0.9), y)
    assert np.abs(x - y).min() > 1e-3
    kw = dict(w_depth=w_depth, lambda1=lambda1, lambda2=0.1)
    _, g, gd = oracle.loss_ssim(x, d, y, td, W, H, **kw)
    rng = np.random.default_rng(6)
    idx = [(int(c), int(p)) for c, p in zip(rng.integers(0, 3, 40), rng.integers(0, W * H, 40))]
    idx += [(0, 0), (1, W - 1), (2, W * H - 1), (0, (H // 2) * W + W // 2)]
    h = 1e-6
    for c, p in idx:
        xp = x.copy(); xp[c, p] += h
        xm = x.copy(); xm[c, p] -= h
        fd = (oracle.loss_ssim(xp, d, y, td, W, H, **kw)[0] - oracle.loss_ssim(xm, d, y, td, W, H, **kw)[0]) / (2 * h)
        assert abs(fd - g[c, p]) <= 1e-6 * max(abs(g[c, p]), 1e-4), (c, p, fd, g[c, p])
    if w_depth:
        for p in (0, 17, W * H - 1):
            dp = d.copy(); dp[p] += h
            dm = d.copy(); dm[p] -= h
            fd = (oracle.loss_ssim(x, dp, y, td, W, H, **kw)[0] - oracle.loss_ssim(x, dm, y, td, W, H, **kw)[0]) / (2 * h)
            assert abs(fd - gd[p]) <= 1e-8
