"""Pins of the oracle's uncertainty bookkeeping (Sec. IV-A: the uncertainty
of a Gaussian is the magnitude of the change of its mean, kept when the mean
does not change) and region utility (Sec. IV-B, size of Sec. IV-C: mean uncertainty over
cuboidal regions of the enclosing space)."""
import numpy as np
import pytest

import oracle


def test_displacement_closed_forms_and_retention():
    prev = np.zeros((3, 6))
    cur = np.array([[3.0, 1.0, 0.0, 2.0, 0.0, -6.0],
                    [4.0, 2.0, 0.0, 3.0, 0.0, 0.0],
                    [0.0, 2.0, 0.0, 6.0, 0.0, 8.0]])
    cur[:, 4] = prev[:, 4]  # unchanged
    up = np.array([9.0, 9.0, 0.25, 9.0, 0.75, 9.0])
    u = oracle.uncertainty_update(prev, cur, up)
    # Pythagorean triples: (3, 4, 0) -> 5, (1, 2, 2) -> 3, (2, 3, 6) -> 7, (-6, 0, 8) -> 10;
    # unchanged means keep u_prev
    np.testing.assert_array_equal(u, [5.0, 3.0, 0.25, 7.0, 0.75, 10.0])
    u2 = oracle.uncertainty_update(prev, cur, up, squared=True)
    np.testing.assert_array_equal(u2, [25.0, 9.0, 0.25, 49.0, 0.75, 100.0])


def test_displacement_matches_numpy_norm():
    rng = np.random.default_rng(4)
    n = 5000
    prev = rng.uniform(-10, 10, (3, n)).astype(np.float32).astype(np.float64)
    cur = prev + rng.normal(0, 0.05, (3, n)).astype(np.float32)
    keep = rng.random(n) < 0.3
    cur[:, keep] = prev[:, keep]
    up = rng.random(n)
    u = oracle.uncertainty_update(prev, cur, up)
    assert np.array_equal(u[keep], up[keep])
    ref = np.linalg.norm(cur - prev, axis=0)
    np.testing.assert_allclose(u[~keep], ref[~keep], rtol=4e-16, atol=0)


def test_region_grid_dims():
    assert oracle.region_grid([0, 0, 0, 10, 5, 2.5], 2.5) == (4, 2, 1)
    assert oracle.region_grid([-10, -10, 0, 10.1, 10, 4], 2.5) == (9, 8, 2)
    with pytest.raises(ValueError):
        oracle.region_grid([0, 0, 0, 0, 1, 1], 2.5)


def test_region_utility_hand_placed():
    box = [0, 0, 0, 10, 5, 2.5]  # 4 x 2 x 1 regions of 2.5 m
    pts = np.array([[1.0, 2.5, 2.49, 9.9, 10.0, -1e-9, 7.0, 7.5],
                    [1.0, 1.0, 4.99, 2.6, 1.0, 1.0, 3.0, 3.0],
                    [1.0, 1.0, 2.4, 0.0, 1.0, 1.0, 2.5, 1.0]])
    u = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0, 8.0])
    cnt, sm, mean = oracle.region_utility(pts, u, box, 2.5)
    want_cnt = np.zeros(8, np.int64)
    want_sum = np.zeros(8)
    # x = 1 -> 0; x = 2.5 is the lower face of region 1; 2.49 -> 0 with y 4.99 -> 1;
    # (9.9, 2.6) -> (3, 1); x = 10 and x < 0 and z = 2.5 are outside
    for (ix, iy, val) in ((0, 0, 1.0), (1, 0, 2.0), (0, 1, 3.0), (3, 1, 4.0), (3, 1, 8.0)):
        r = ix + 4 * iy
        want_cnt[r] += 1
        want_sum[r] += val
    np.testing.assert_array_equal(cnt, want_cnt)
    np.testing.assert_array_equal(sm, want_sum)
    np.testing.assert_array_equal(mean, np.where(want_cnt > 0, want_sum / np.maximum(want_cnt, 1), 0.0))


def test_region_utility_matches_numpy_binning():
    rng = np.random.default_rng(8)
    n = 20000
    box = [-10.0, -10.0, 0.0, 10.0, 10.0, 4.0]
    pts = np.stack([rng.uniform(-11, 11, n), rng.uniform(-11, 11, n), rng.uniform(-0.5, 4.5, n)])
    u = rng.random(n)
    cnt, sm, mean = oracle.region_utility(pts, u, box, 2.5)
    d = oracle.region_grid(box, 2.5)
    idx = np.floor((pts - np.array(box[:3])[:, None]) / 2.5).astype(np.int64)
    inside = np.all((idx >= 0) & (idx < np.array(d)[:, None]), axis=0)
    r = idx[0] + d[0] * (idx[1] + d[1] * idx[2])
    ref_cnt = np.bincount(r[inside], minlength=int(np.prod(d)))
    ref_sum = np.bincount(r[inside], weights=u[inside], minlength=int(np.prod(d)))
    np.testing.assert_array_equal(cnt, ref_cnt)
    np.testing.assert_allclose(sm, ref_sum, rtol=1e-12)
    assert cnt.sum() < n  # some points fall outside the box
