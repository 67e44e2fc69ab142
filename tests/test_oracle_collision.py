"""Pins of the oracle's collision test (Sec. IV-B, trajectory planner, Collision Checking): a
sampled point of radius r_robot collides with a Gaussian whose mean is
closer than r_robot + lambda_g r, r = the Gaussian's principal axis."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle


def planar(xyz):
    return np.ascontiguousarray(np.asarray(xyz, np.float64).T)


def test_single_gaussian_closed_form():
    means = planar([[0.0, 0.0, 0.0]])
    ls = planar([[math.log(0.1)] * 3])  # r = 0.1, lambda_g r = 0.3
    pts = planar([[0.5, 0, 0], [0, 0.6, 0], [0, 0, -0.54], [0.3, 0.4, 0.0], [0.0, 0.0, 0.0]])
    hit, clr = oracle.collision(means, ls, pts, r_robot=0.25, lambda_g=3.0)
    # gamma = 0.55: distances 0.5, 0.6, 0.54, 0.5 (3-4-5), 0
    np.testing.assert_array_equal(hit, [1, 0, 1, 1, 1])
    np.testing.assert_allclose(clr, [0.2, 0.3, 0.24, 0.2, -0.3], atol=1e-15)


def test_principal_axis_is_the_radius():
    means = planar([[1.0, 2.0, 3.0]])
    ls = planar([[math.log(0.05), math.log(0.2), math.log(0.1)]])  # r = 0.2
    pts = planar([[1.0 + 0.95, 2.0, 3.0], [1.0, 2.0, 3.0 + 1.05]])
    hit, clr = oracle.collision(means, ls, pts, r_robot=0.4, lambda_g=3.0)
    # gamma = 1.0: 0.95 collides, 1.05 does not
    np.testing.assert_array_equal(hit, [1, 0])
    np.testing.assert_allclose(clr, [0.35, 0.45], atol=1e-14)
    # the boundary itself is no collision (strict inequality): distance exactly 1
    ls2 = planar([[math.log(0.25)] * 3])
    hit2, _ = oracle.collision(means, ls2, planar([[1.0, 2.0, 4.0]]), r_robot=0.25, lambda_g=3.0)
    assert hit2[0] == 0


def test_equal_radius_matches_nearest_neighbour():
    rng = np.random.default_rng(6)
    n, npt = 5000, 800
    means = rng.uniform(-5, 5, (3, n))
    ls = np.full((3, n), math.log(0.05))
    pts = rng.uniform(-5, 5, (3, npt))
    hit, clr = oracle.collision(means, ls, pts, r_robot=0.2, lambda_g=3.0)
    dist, _ = cKDTree(means.T).query(pts.T)
    np.testing.assert_allclose(clr, dist - 0.15, rtol=0, atol=1e-12)
    margin = np.abs(dist - 0.35) > 1e-9
    np.testing.assert_array_equal(hit[margin], (dist < 0.35)[margin].astype(np.int32))
    assert 0 < hit.sum() < npt


def test_ignored_and_empty():
    means = planar([[0.0, 0.0, 0.0], [np.nan, 0.0, 0.0]])
    ls = planar([[math.log(0.1)] * 3, [0.0] * 3])
    hit, clr = oracle.collision(means, ls, planar([[2.0, 0.0, 0.0]]), r_robot=0.1)
    assert hit[0] == 0 and clr[0] == pytest.approx(1.7, abs=1e-15)
    hit, clr = oracle.collision(np.zeros((3, 0)), np.zeros((3, 0)), planar([[0.0, 0.0, 0.0]]), r_robot=0.1)
    assert hit[0] == 0 and np.isinf(clr[0])
