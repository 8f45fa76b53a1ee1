"""Pins of the oracle's motion undistortion (Sec. III-A.1) to things other than
itself: the least-squares line against numpy.polyfit and exact lines; the
per-point motion against scipy's matrix exponential (constant twist) and a
numerical solution of the pose kinematics (twist varying in time, on one
screw axis exactly, otherwise within the second Magnus term); and, end to
end, against the exact sensor trajectory of a moving-LiDAR scan."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

from oracle import far_oracle as orc
from paper_2606_26010_amd import synth


def hat(xi):
    """4x4 matrix of the twist (vx vy vz wx wy wz)."""
    v, w = xi[:3], xi[3:]
    return np.array([[0, -w[2], w[1], v[0]], [w[2], 0, -w[0], v[1]],
                     [-w[1], w[0], 0, v[2]], [0, 0, 0, 0]], dtype=np.float64)


def ulp(x):
    return np.spacing(np.abs(np.asarray(x, dtype=np.float32)))


def scatter(seed, n, t_lo=0.0, t_hi=0.1, r=100.0):
    g = np.random.default_rng(seed)
    d = g.normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0)
    xyz = (d * g.uniform(1.0, r, n)).astype(np.float32)
    t = np.sort(g.uniform(t_lo, t_hi, n)).astype(np.float32)
    return xyz, t


def test_fit_recovers_exact_line():
    g = np.random.default_rng(1)
    ts = g.uniform(-0.01, 0.1, 23)
    a0, b0, c = g.normal(size=6) * 10, g.normal(size=6) * 3, 0.037
    xi = a0 + np.outer(ts - c, b0)
    tb, a, b = orc.fit_twist(ts, xi)
    assert tb == pytest.approx(ts.mean(), abs=1e-15)
    np.testing.assert_allclose(b, b0, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(a, a0 + b0 * (tb - c), rtol=1e-12, atol=1e-12)


def test_fit_matches_polyfit():
    g = np.random.default_rng(2)
    ts = np.arange(-0.01, 0.1001, 0.005) + 12.5
    xi = g.normal(size=(ts.size, 6)) * [5, 1, 1, 0.1, 0.1, 0.5] + [70, 0, 0, 0, 0, 0.3]
    tb, a, b = orc.fit_twist(ts, xi)
    for k in range(6):
        slope, icept = np.polyfit(ts - tb, xi[:, k], 1)
        assert b[k] == pytest.approx(slope, rel=1e-10, abs=1e-12)
        assert a[k] == pytest.approx(icept, rel=1e-12, abs=1e-12)


def test_fit_degenerate_cases():
    tb, a, b = orc.fit_twist(np.zeros(0), np.zeros((0, 6)))
    assert tb == 0 and not a.any() and not b.any()
    x = np.arange(6.0) + 1
    tb, a, b = orc.fit_twist([0.3], x[None])
    assert tb == 0.3 and np.array_equal(a, x) and not b.any()
    xi = np.stack([x, 3 * x])
    tb, a, b = orc.fit_twist([0.5, 0.5], xi)
    np.testing.assert_allclose(a, 2 * x, rtol=1e-15)
    assert not b.any()
    # a sample with a non-finite entry is left out
    g = np.random.default_rng(3)
    ts, xi = g.uniform(0, 0.1, 9), g.normal(size=(9, 6))
    ref = orc.fit_twist(ts[1:], xi[1:])
    for bad in ((0, 2, np.nan), (0, 5, np.inf), (0, None, np.nan)):
        t2, x2 = ts.copy(), xi.copy()
        if bad[1] is None:
            t2[0] = bad[2]
        else:
            x2[0, bad[1]] = bad[2]
        got = orc.fit_twist(t2, x2)
        assert got[0] == ref[0] and np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])


def test_undistort_zero_motion_and_reference_points():
    xyz, t = scatter(4, 5000)
    out, tr = orc.undistort(xyz, t, [0.0, 0.1], np.zeros((2, 6)))
    assert tr == float(t.max())
    np.testing.assert_array_equal(out, xyz)
    # with motion: the points at the reference time stay exactly where they are
    xi = np.tile([30.0, 1.0, -2.0, 0.2, -0.1, 0.8], (2, 1))
    out, tr = orc.undistort(xyz, t, [0.0, 0.1], xi)
    last = t == t.max()
    np.testing.assert_array_equal(out[:, last], xyz[:, last])
    assert np.abs(out[:, ~last] - xyz[:, ~last]).max() > 1.0
    # non-finite times: copied unchanged and not taken as the reference
    t2 = t.copy()
    t2[[5, 77]] = [np.nan, np.inf]
    out2, tr2 = orc.undistort(xyz, t2, [0.0, 0.1], xi)
    assert tr2 == tr
    np.testing.assert_array_equal(out2[:, [5, 77]], xyz[:, [5, 77]])
    keep = np.ones(t.size, bool)
    keep[[5, 77]] = False
    np.testing.assert_array_equal(out2[:, keep], out[:, keep])
    out3, tr3 = orc.undistort(xyz[:, :3], np.full(3, np.nan, np.float32), [0.0], xi[:1])
    assert math.isnan(tr3)
    np.testing.assert_array_equal(out3, xyz[:, :3])
    out4, tr4 = orc.undistort(np.zeros((3, 0), np.float32), np.zeros(0, np.float32), [0.0], xi[:1])
    assert out4.shape == (3, 0) and math.isnan(tr4)


@pytest.mark.parametrize("xi", [[70.0, 2.0, -0.5, 0.05, -0.03, 0.9],
                                [5.0, -40.0, 3.0, 2.5, 1.0, -3.0],
                                [0.0, 0.0, 0.0, 1e-7, 0.0, 0.0],
                                [12.0, 0.0, 0.0, 0.0, 0.0, 0.0]])
def test_undistort_constant_twist_matches_matrix_exponential(xi):
    xi = np.asarray(xi)
    xyz, t = scatter(5, 600)
    out, tr = orc.undistort(xyz, t, [0.0, 0.05, 0.1], np.tile(xi, (3, 1)))
    p = xyz.astype(np.float64)
    for i in range(t.size):
        E = expm((float(t[i]) - tr) * hat(xi))
        want = E[:3, :3] @ p[:, i] + E[:3, 3]
        assert np.all(np.abs(out[:, i] - want) <= 0.51 * ulp(want) + 1e-12), i


def kinematics(xi_of, t_ref, times):
    """Pose of the sensor at each of `times` relative to t_ref, from
    dR/dt = R [w]x, dp/dt = R v with (v, w) = xi_of(t), integrated numerically."""
    def f(t, y):
        R = y[:9].reshape(3, 3)
        x = xi_of(t)
        W = np.array([[0, -x[5], x[4]], [x[5], 0, -x[3]], [-x[4], x[3], 0]])
        return np.concatenate([(R @ W).ravel(), R @ x[:3]])
    uniq = np.unique(times)[::-1]
    sol = solve_ivp(f, (t_ref, float(uniq[-1])), np.concatenate([np.eye(3).ravel(), np.zeros(3)]),
                    method="DOP853", t_eval=uniq, rtol=1e-13, atol=1e-13)
    assert sol.success
    return {float(tt): (sol.y[:9, j].reshape(3, 3), sol.y[9:, j]) for j, tt in enumerate(sol.t)}


def test_undistort_single_screw_axis_matches_kinematics():
    """A twist whose direction is fixed and whose size is linear in time:
    all its values commute, so the exponential of the integral is exact."""
    xi0 = np.array([40.0, 3.0, -1.0, 0.2, -0.1, 1.2])
    f = lambda s: 0.8 + 4.0 * (s - 0.02)
    ts = np.linspace(-0.01, 0.1, 23)
    xyz, t = scatter(6, 800)
    out, tr = orc.undistort(xyz, t, ts, np.outer(f(ts), xi0))
    poses = kinematics(lambda s: f(s) * xi0, tr, t.astype(np.float64))
    p = xyz.astype(np.float64)
    for i in range(t.size):
        R, q = poses[float(t[i])]
        want = R @ p[:, i] + q
        assert np.all(np.abs(out[:, i] - want) <= 0.51 * ulp(want) + 1e-9), i


def test_undistort_varying_twist_within_magnus_bound():
    """A twist linear in time along changing axes: the exponential of the
    integral differs from the true motion by the second Magnus term,
    tau^3 / 12 |[xi(t_ref), b]| to leading order."""
    x0 = np.array([20.0, 0.0, 0.0, 0.0, 0.0, 2.0])
    x1 = np.array([0.0, 5.0, 0.0, 3.0, 0.0, 0.0])
    ts = np.linspace(-0.01, 0.1, 23)
    xyz, t = scatter(7, 800)
    out, tr = orc.undistort(xyz, t, ts, x0 + np.outer(ts, x1))
    xi_at = lambda s: x0 + s * x1
    poses = kinematics(xi_at, tr, t.astype(np.float64))
    c = hat(xi_at(tr)) @ hat(x1) - hat(x1) @ hat(xi_at(tr))
    cw = np.linalg.norm([c[2, 1], c[0, 2], c[1, 0]])
    cv = np.linalg.norm(c[:3, 3])
    p = xyz.astype(np.float64)
    worst = 0.0
    for i in range(t.size):
        R, q = poses[float(t[i])]
        want = R @ p[:, i] + q
        tau = abs(float(t[i]) - tr)
        bound = tau ** 3 / 12 * (cw * np.linalg.norm(p[:, i]) + cv)
        err = np.abs(out[:, i] - want).max()
        worst = max(worst, err / max(bound, 1e-12))
        assert err <= 1.5 * bound + ulp(want).max(), (i, err, bound)
    assert worst > 0.2        # the bound is not vacuous: the term is seen


@pytest.mark.parametrize("noisy", [False, True])
def test_undistort_moving_lidar_scan_against_trajectory(noisy):
    kw = {} if noisy else dict(noise_v=0.0, noise_w=0.0)
    c = synth.make_deskew(6, n_scans=2, **kw)
    s = 1
    out, tr = orc.undistort(c.scans[s], c.times[s], c.vel_t[s], c.vel[s])
    assert tr == float(c.times[s].max())
    T_ref_inv = np.linalg.inv(c.poses[s])
    p = c.scans[s].astype(np.float64)
    err, raw = 0.0, 0.0
    for u in np.unique(c.times[s]):
        sel = c.times[s] == u
        D = T_ref_inv @ synth.trajectory_pose(c.starts[s] + float(u), **c.traj)
        truth = D[:3, :3] @ p[:, sel] + D[:3, 3:4]
        err = max(err, float(np.abs(out[:, sel] - truth).max()))
        raw = max(raw, float(np.abs(p[:, sel] - truth).max()))
    print(f"noisy={noisy}: undistorted {err:.4f} m, raw {raw:.3f} m")
    assert raw > 5.0
    assert err <= (0.03 if noisy else 0.01)


def test_odometry_with_undistortion_tracks_the_trajectory():
    """Scan-to-submap odometry over 20 scans of the racing line: with the
    scans undistorted the estimate stays within 0.2 m of the pose at each
    scan's last point time; without, it is several times farther off."""
    c = synth.make_deskew(6, n_scans=20)
    v1 = np.linalg.inv(c.poses[0]) @ c.poses[1]
    err = {}
    for deskew in (True, False):
        kw = dict(times=c.times, vel_t=c.vel_t, vel=c.vel) if deskew else {}
        ref, _ = orc.odometry(c.scans, c.poses[0], v1, c.voxel_size, c.max_pts_per_voxel,
                              c.min_spacing, c.k, c.map_capacity, c.downsample, c.sigma0,
                              c.r_max, max_iters=10, eps=0.0, **kw)
        assert all(r["status"] == 0 for r in ref)
        if deskew:
            assert [r["t_ref"] for r in ref] == [float(t.max()) for t in c.times]
        err[deskew] = max(np.linalg.norm(r["T"][:3, 3] - c.poses[s][:3, 3])
                          for s, r in enumerate(ref))
    print(f"odometry drift: undistorted {err[True]:.3f} m, raw {err[False]:.3f} m")
    assert err[True] <= 0.2 and err[True] <= 0.25 * err[False]
