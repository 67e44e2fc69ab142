"""GPU parity of the uncertainty bookkeeping (Sec. IV-A) and the region
utility (Sec. IV-B, region size of Sec. IV-C) against the oracle, through the C ABI."""
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
    return raster.Context(0)


def moved_means(n, seed):
    rng = np.random.default_rng(seed)
    prev = rng.uniform(-10, 10, (3, n)).astype(np.float32)
    cur = (prev + rng.normal(0, 0.02, (3, n))).astype(np.float32)
    keep = rng.random(n) < 0.4
    cur[:, keep] = prev[:, keep]
    cur[0, :16] = prev[0, :16] + np.float32(1e-6)  # tiny moves still count as changes
    keep[:16] = False
    u_prev = rng.random(n).astype(np.float32)
    return prev, cur, u_prev, keep


@pytest.mark.parametrize("n", [0, 1, 777, 2_000_000])
@pytest.mark.parametrize("squared", [False, True])
def test_uncertainty_update_bit_exact(raster, rctx, n, squared):
    say(f"uncertainty update n={n} squared={squared}")
    prev, cur, up, keep = moved_means(n, 3 + n)
    t = {k: torch.as_tensor(v).cuda() for k, v in (("p", prev), ("c", cur), ("u", up))}
    got = raster.uncertainty_update(rctx, t["p"], t["c"], t["u"], squared=squared).cpu().numpy()
    ref = oracle.uncertainty_update(prev, cur, up, squared=squared).astype(np.float32)
    assert np.array_equal(got, ref)
    if n:
        assert np.array_equal(got[keep], up[keep])
    # in place
    raster.uncertainty_update(rctx, t["p"], t["c"], t["u"], squared=squared, out=t["u"])
    assert np.array_equal(t["u"].cpu().numpy(), ref)


def fixed_point_bound(count):
    # each value is rounded to 2^-32 before summing
    return count * 2.0 ** -33 + 1e-12


@pytest.mark.parametrize("size", [2.5, 0.4])  # 128 regions (LDS path) and 12,500 (global atomics)
def test_region_utility_matches_oracle(raster, rctx, size):
    g, _ = scenes.config5(n=2_000_000, n_views=1)
    box = [-10.0, -10.0, 0.0, 10.0, 10.0, 4.0]
    means = g["means"]
    u = np.abs(np.random.default_rng(11).normal(0, 0.05, means.shape[1])).astype(np.float32)
    say(f"region utility size {size}: grid {raster.region_grid(box, size)}")
    cnt, sm, mean = raster.region_utility(rctx, torch.as_tensor(means).cuda(), torch.as_tensor(u).cuda(), box, size)
    rc, rs, rm = oracle.region_utility(means, u, box, size)
    cnt, sm, mean = cnt.cpu().numpy(), sm.cpu().numpy(), mean.cpu().numpy()
    assert np.array_equal(cnt, rc)
    assert np.all(np.abs(sm - rs) <= fixed_point_bound(rc) + 1e-12 * np.abs(rs))
    assert np.all(np.abs(mean - rm) <= (fixed_point_bound(rc) + 1e-12 * np.abs(rs)) / np.maximum(rc, 1))
    assert np.all(mean[rc == 0] == 0.0)


def test_region_utility_edges(raster, rctx):
    box = [0.0, 0.0, 0.0, 10.0, 5.0, 2.5]
    pts = np.array([[1.0, 2.5, 2.49, 9.9, 10.0, -1e-6, 7.0, 7.5],
                    [1.0, 1.0, 4.99, 2.6, 1.0, 1.0, 3.0, 3.0],
                    [1.0, 1.0, 2.4, 0.0, 1.0, 1.0, 2.5, 1.0]], np.float32)
    u = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0, np.nan], np.float32)
    cnt, sm, mean = raster.region_utility(rctx, torch.as_tensor(pts).cuda(), torch.as_tensor(u).cuda(), box, 2.5)
    rc, rs, rm = oracle.region_utility(pts, u, box, 2.5)
    assert np.array_equal(cnt.cpu().numpy(), rc)
    # the NaN u makes its region NaN, as in the oracle; the others are exact
    sm = sm.cpu().numpy()
    assert np.array_equal(np.isnan(sm), np.isnan(rs))
    ok = ~np.isnan(rs)
    assert np.array_equal(sm[ok], rs[ok])
    # no Gaussians
    e = torch.zeros((3, 0), device="cuda")
    c0, s0, m0 = raster.region_utility(rctx, e, torch.zeros(0, device="cuda"), box, 2.5)
    assert int(c0.sum()) == 0 and float(s0.abs().sum()) == 0.0 and float(m0.abs().sum()) == 0.0
