"""Parity of the paper-literal view utility (Sec. IV-B eq. (8)), the
uncertainty thresholds (Sec. IV-C) and trajectory selection (eq. (10)) with
the oracle.  Counts are integers decided in binary64 on both sides: they must
match exactly."""
import numpy as np
import pytest
import torch

import oracle
import scenes

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def raster():
    from paper_2409_18122_amd import raster as r
    return r


@pytest.fixture(scope="module")
def rctx(raster):
    oracle.set_threads(16)
    return raster.Context(0)


S = dict(scenes.DEFAULT_SETTINGS)


@pytest.mark.parametrize("which", ["c3", "c5"])
def test_view_utility_full_size(raster, rctx, which):
    if which == "c3":
        g, cams = scenes.config3()
    else:
        g, cams = scenes.config5()
    dev = raster.to_device(g)
    say(f"{which}: thresholds and utility over {len(cams)} views, {g['opacity'].shape[0]} Gaussians")
    th = raster.uncertainty_thresholds(rctx, dev["uncert"], 0.5).cpu().numpy()
    lo, hi = oracle.thresholds(g["uncert"], 0.5)
    assert abs(th[0] - lo) <= 1e-12 * max(1.0, abs(lo)) and abs(th[1] - hi) <= 1e-12 * max(1.0, abs(hi))
    lo_hi = torch.tensor([lo, hi], dtype=torch.float64, device="cuda")
    got = raster.view_utility(rctx, dev, cams, lo_hi, S, range_=5.0, lambda_xi=1.0)
    nh, nl, su, xi = oracle.view_utility(g, cams, S, lo, hi, range_=5.0, lam=1.0)
    assert np.array_equal(got["n_high"].cpu().numpy(), nh)
    assert np.array_equal(got["n_low"].cpu().numpy(), nl)
    assert np.array_equal(got["xi"].cpu().numpy(), xi)
    n = g["opacity"].shape[0]
    assert np.all(np.abs(got["sum_u"].cpu().numpy() - su) <= n * 2.0 ** -40 + 1e-12 * np.abs(su))
    say(f"{which}: xi range {xi.min()} .. {xi.max()}, visible high {nh.sum()}")


def test_view_utility_edges(raster, rctx):
    # points projecting exactly onto pixel centres around the image border,
    # at depths around the near plane and the range
    c = scenes.make_camera(20, 12, 64.0, 64.0, 9.0, 5.0)
    us, vs = np.meshgrid(np.arange(-2, 22), np.arange(-2, 14))
    pts = []
    for z in (0.2, 0.25, 2.0, 5.0, 5.5):
        pts.append(np.stack([(us.ravel() - 9.0) * z / 64.0, (vs.ravel() - 5.0) * z / 64.0,
                             np.full(us.size, z)], 1))
    xyz = np.concatenate(pts).astype(np.float32)
    n = xyz.shape[0]
    rng = np.random.default_rng(1)
    g = {"means": np.ascontiguousarray(xyz.T), "log_scales": np.full((3, n), -3.0, np.float32),
         "quats": np.tile(np.array([[1], [0], [0], [0]], np.float32), (1, n)),
         "opacity": np.full(n, 0.5, np.float32), "colors": np.zeros((3, n), np.float32),
         "uncert": rng.random(n).astype(np.float32)}
    dev = raster.to_device(g)
    lo, hi = oracle.thresholds(g["uncert"], 0.5)
    lo_hi = torch.tensor([lo, hi], dtype=torch.float64, device="cuda")
    got = raster.view_utility(rctx, dev, [c], lo_hi, S, range_=5.0)
    nh, nl, su, xi = oracle.view_utility(g, [c], S, lo, hi, range_=5.0)
    assert got["n_high"].item() == nh[0] and got["n_low"].item() == nl[0]


def test_trajectory_select(raster, rctx):
    rng = np.random.default_rng(2)
    lens = rng.integers(1, 7, 12)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    xi = rng.integers(-50, 50, int(off[-1])).astype(np.float64)
    util, best = raster.trajectory_select(rctx, torch.tensor(xi, device="cuda"), torch.tensor(off))
    exp, exp_best = oracle.traj_select(xi, off)
    assert np.array_equal(util.cpu().numpy(), exp)
    assert best.item() == exp_best
    # non-integer utilities, summed in the same order on both sides, and ties
    xr = rng.standard_normal(200)
    xr[100:110] = xr[0:10]
    offr = np.array([0, 10, 37, 100, 110, 150, 150, 200], np.int32)
    util, best = raster.trajectory_select(rctx, torch.tensor(xr, device="cuda"), torch.tensor(offr))
    exp, exp_best = oracle.traj_select(xr, offr)
    assert np.array_equal(util.cpu().numpy(), exp)
    assert best.item() == exp_best
