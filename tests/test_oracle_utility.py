"""Pins of the oracle's paper-literal view utility (Sec. IV-B eq. (8)) and of
the high/low uncertainty thresholds (Sec. IV-C: half a standard deviation
around the mean)."""
import numpy as np
import pytest

import oracle
import scenes
from test_oracle_pins import cam, S


def points(xyz, u):
    xyz = np.asarray(xyz, np.float64).T.copy()
    n = xyz.shape[1]
    return {"means": xyz, "log_scales": np.full((3, n), -3.0), "quats": np.tile([[1.0], [0], [0], [0]], (1, n)),
            "opacity": np.full(n, 0.5), "colors": np.zeros((3, n)), "uncert": np.asarray(u, np.float64)}


def test_thresholds_match_numpy_population_std():
    rng = np.random.default_rng(3)
    u = rng.random(1001)
    lo, hi = oracle.thresholds(u, 0.5)
    assert lo == pytest.approx(u.mean() - 0.5 * u.std(), rel=1e-13)
    assert hi == pytest.approx(u.mean() + 0.5 * u.std(), rel=1e-13)
    # constant uncertainty: both thresholds equal the constant
    lo, hi = oracle.thresholds(np.full(10, 0.3), 0.5)
    assert lo == pytest.approx(0.3, abs=1e-15) and hi == pytest.approx(0.3, abs=1e-15)


def test_visibility_grid_counts_exactly_the_pixels_inside():
    # points at depth 2 that project exactly onto pixel centres u = -2 .. W+1,
    # v = -2 .. H+1: visible iff 0 <= u <= W-1 and 0 <= v <= H-1
    c = cam(w=20, h=12, fx=64.0, fy=64.0, cx=9.0, cy=5.0)
    us, vs = np.meshgrid(np.arange(-2, 22), np.arange(-2, 14))
    z = 2.0
    xyz = np.stack([(us.ravel() - 9.0) * z / 64.0, (vs.ravel() - 5.0) * z / 64.0, np.full(us.size, z)], 1)
    g = points(xyz, np.ones(us.size))
    nh, nl, su, xi = oracle.view_utility(g, [c], S(), lo=0.5, hi=0.5, range_=5.0)
    assert nh[0] == 20 * 12 and nl[0] == 0
    assert su[0] == 20 * 12 and xi[0] == 20 * 12


def test_range_and_near_plane():
    c = cam()
    depths = [0.1, 0.2, 0.21, 3.0, 4.99, 5.0, 5.01, 9.0, -1.0]
    xyz = [[0.0, 0.0, d] for d in depths]
    g = points(xyz, np.ones(len(depths)))
    nh, _, _, _ = oracle.view_utility(g, [c], S(), lo=0.5, hi=0.5, range_=5.0)
    # (0.2, 5.0]: 0.21, 3.0, 4.99, 5.0
    assert nh[0] == 4


def test_partition_and_lambda():
    c = cam()
    rng = np.random.default_rng(5)
    n = 300
    xyz = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.4, 0.4, n), rng.uniform(1.0, 4.0, n)], 1)
    u = rng.random(n)
    g = points(xyz, u)
    lo, hi = 0.3, 0.7
    nh, nl, su, xi = oracle.view_utility(g, [c], S(), lo, hi, range_=5.0, lam=1.0)
    # every point is in view here, so the counts are plain counts of u
    assert nh[0] == int((u > hi).sum()) and nl[0] == int((u < lo).sum())
    assert su[0] == pytest.approx(u.sum(), rel=1e-13)
    assert xi[0] == nh[0] - nl[0]
    _, _, _, xi0 = oracle.view_utility(g, [c], S(), lo, hi, range_=5.0, lam=0.0)
    assert xi0[0] == nh[0]
    _, _, _, xi2 = oracle.view_utility(g, [c], S(), lo, hi, range_=5.0, lam=2.5)
    assert xi2[0] == nh[0] - 2.5 * nl[0]
    # mirrored uncertainty swaps the high and low sets
    nh2, nl2, _, _ = oracle.view_utility(points(xyz, 1.0 - u), [c], S(), 1.0 - hi, 1.0 - lo, range_=5.0)
    assert nh2[0] == nl[0] and nl2[0] == nh[0]


def test_pose_convention_for_visibility():
    rng = np.random.default_rng(9)
    R = scenes.random_rotation(rng)
    T = rng.standard_normal(3)
    c0 = cam()
    c1 = cam(R=R, T=T)
    R32, T32 = c1["R"].astype(np.float64), c1["T"].astype(np.float64)
    n = 400
    p = np.stack([rng.uniform(-2, 2, n), rng.uniform(-2, 2, n), rng.uniform(-1, 7, n)], 1)
    w = p @ R32.T + T32
    u = rng.random(n)
    a = oracle.view_utility(points(p, u), [c0], S(), 0.4, 0.6)
    b = oracle.view_utility(points(w, u), [c1], S(), 0.4, 0.6)
    # the same points seen from the same relative pose (up to rounding at the borders)
    assert abs(int(a[0][0]) - int(b[0][0])) <= 1 and abs(int(a[1][0]) - int(b[1][0])) <= 1


# --------------------------------------------------------------------------
# Trajectory selection, Sec. IV-B eq. (10): argmax over trajectories of the
# sum of xi over the trajectory's L + 1 states.
# --------------------------------------------------------------------------

def test_traj_select_hand_example():
    # three trajectories of 3, 2 and 4 states
    xi = [4.0, -1.0, 2.0,   7.0, -2.0,   1.0, 1.0, 1.0, 1.0]
    off = [0, 3, 5, 9]
    util, best = oracle.traj_select(xi, off)
    assert util.tolist() == [5.0, 5.0, 4.0]
    # equal totals: the first trajectory is kept
    assert best == 0
    util, best = oracle.traj_select(xi[:8] + [3.0], off)
    assert util.tolist() == [5.0, 5.0, 6.0] and best == 2


def test_traj_select_single_states_and_empty():
    xi = [0.5, -3.0, 2.5, 2.5]
    util, best = oracle.traj_select(xi, [0, 1, 2, 3, 4])
    assert util.tolist() == xi and best == 2
    # a trajectory with no states has utility 0
    util, best = oracle.traj_select([-1.0, -2.0], [0, 1, 1, 2])
    assert util.tolist() == [-1.0, 0.0, -2.0] and best == 1


def test_traj_select_brute_force_integers():
    # integer utilities: every partial sum is exact, so the totals and the
    # choice equal a brute-force evaluation exactly
    rng = np.random.default_rng(8)
    for trial in range(20):
        n_traj = int(rng.integers(1, 12))
        lens = rng.integers(0, 9, n_traj)
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
        xi = rng.integers(-1000, 1000, int(off[-1])).astype(np.float64)
        util, best = oracle.traj_select(xi, off)
        ref = [sum(int(v) for v in xi[off[t]:off[t + 1]]) for t in range(n_traj)]
        assert util.tolist() == [float(r) for r in ref]
        top = max(ref)
        assert best == ref.index(top)
        # relabelling the trajectories permutes the totals
        perm = rng.permutation(n_traj)
        xi2 = np.concatenate([xi[off[t]:off[t + 1]] for t in perm]) if off[-1] else xi
        off2 = np.concatenate([[0], np.cumsum(lens[perm])]).astype(np.int32)
        util2, _ = oracle.traj_select(xi2, off2)
        assert util2.tolist() == [util[t] for t in perm]
