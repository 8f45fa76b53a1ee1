"""Pins of the oracle's sequence-pipeline pieces: voxel downsampling, the
rigid transform of a scan, the adaptive threshold (KISS-ICP rule) and the
odometry loop that strings them together."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2606_26010_amd import synth


def first_per_voxel(x, v):
    """Plain definition: the first occurrence of every voxel key, via numpy."""
    fin = np.all(np.isfinite(x), axis=0)
    idx = np.nonzero(fin)[0]
    keys = np.floor(x[:, idx].astype(np.float64).T / v).astype(np.int64)
    _, first = np.unique(keys, axis=0, return_index=True)
    return np.sort(idx[first])


def test_downsample_is_first_point_per_voxel(orc):
    g = np.random.default_rng(1)
    x = g.uniform(-4, 4, (3, 30000)).astype(np.float32)
    x[:, 5000:5100] = x[:, 100:200]                          # duplicates
    x[:, 6000:6300] = (g.integers(-8, 8, (3, 300)) * 0.5).astype(np.float32)   # on faces
    x[0, 7000:7010] = np.nan
    x[2, 7010:7020] = np.inf
    keep = orc.downsample(x, 0.5)
    np.testing.assert_array_equal(keep, first_per_voxel(x, 0.5))
    assert not np.isin(np.arange(7000, 7020), keep).any()


def test_downsample_equals_cap_one_insert(orc):
    g = np.random.default_rng(2)
    x = g.uniform(-6, 6, (3, 20000)).astype(np.float32)
    keep = orc.downsample(x, 0.5)
    m = orc.Map(0.5, 1, 0.0, 1, point_capacity=1 << 16, voxel_capacity=1 << 16)
    m.insert(x)
    mx, _, _ = m.export()
    np.testing.assert_array_equal(mx, x[:, keep])


def test_downsample_edges(orc):
    assert orc.downsample(np.zeros((3, 0), np.float32), 0.5).size == 0
    np.testing.assert_array_equal(orc.downsample(np.zeros((3, 7), np.float32), 0.5), [0])
    bad = np.zeros((3, 3), np.float32)
    bad[1, 2] = 1e6                                          # key 2e6 > 2^20
    with pytest.raises(orc.OracleError):
        orc.downsample(bad, 0.5)


def test_transform_rounding(orc):
    g = np.random.default_rng(3)
    x = g.uniform(-100, 100, (3, 5000)).astype(np.float32)
    np.testing.assert_array_equal(orc.transform(x, np.eye(4)), x)
    T = np.eye(4)
    T[:3, 3] = (0.1, -7.25, 1e3 / 3)
    np.testing.assert_array_equal(
        orc.transform(x, T), (x.astype(np.float64) + T[:3, 3:4]).astype(np.float32))
    T = synth.pose(Rotation.from_rotvec([0.3, -0.2, 1.1]).as_matrix(), (5.0, -3.0, 2.0))
    ref = T[:3, :3] @ x.astype(np.float64) + T[:3, 3:4]
    got = orc.transform(x, T)
    ulp = np.spacing(np.abs(ref).astype(np.float32))
    assert np.all(np.abs(got - ref) <= ulp)                 # one rounding to float


def test_threshold_hand_sequence(orc):
    t = orc.Threshold(1.0 / 3.0, 100.0, 0.1)
    assert t.get() == pytest.approx((1.0, 1.0 / 9.0), rel=1e-15)
    I = np.eye(4)

    def trans(x, y, z):
        T = np.eye(4)
        T[:3, 3] = (x, y, z)
        return T

    # 5 cm deviation: below the minimum motion, no sample
    assert t.update(I, trans(0.05, 0, 0)) == pytest.approx(0.05, abs=1e-15)
    assert t.samples == 0 and t.get()[0] == pytest.approx(1.0, rel=1e-15)
    # 0.5 m deviation: sigma = 0.5
    assert t.update(I, trans(0.3, 0.4, 0)) == pytest.approx(0.5, abs=1e-15)
    assert t.get() == pytest.approx((1.5, 0.5 / 3.0), rel=1e-14)
    # deviation D = (rotation about z by 2 asin(1e-3), 0.1 m along z) applied
    # on the right of a non-trivial prediction P: 2 * 100 * 1e-3 + 0.1 = 0.3
    P = synth.pose(Rotation.from_euler("z", 30, degrees=True).as_matrix(), (5.0, -2.0, 1.0))
    D = synth.pose(Rotation.from_euler("z", 2 * math.asin(1e-3)).as_matrix(), (0, 0, 0.1))
    assert t.update(P, P @ D) == pytest.approx(0.3, abs=1e-9)
    s = math.sqrt((0.25 + 0.09) / 2)
    assert t.get() == pytest.approx((3 * s, s / 3), rel=1e-8)
    assert t.samples == 2


def test_nearest_rotation(orc):
    g = np.random.default_rng(6)
    for _ in range(20):
        R = Rotation.from_rotvec(g.normal(size=3)).as_matrix()
        np.testing.assert_allclose(orc._nearest_rotation(R), R, atol=1e-15)
        P = orc._nearest_rotation(R + 1e-3 * g.normal(size=(3, 3)))
        np.testing.assert_allclose(P.T @ P, np.eye(3), atol=1e-14)
        assert np.linalg.det(P) == pytest.approx(1.0, abs=1e-14)


def _angle_deg(A, B):
    E = A[:3, :3] @ B[:3, :3].T
    return math.degrees(math.acos(max(-1.0, min(1.0, (np.trace(E) - 1) / 2))))


def _polar_rotation(M):
    """Nearest rotation by Davenport's q-method (scipy's from_matrix), an
    algorithm other than the oracle's SVD polar factor."""
    return Rotation.from_matrix(M).as_matrix()


def _deviation(T_pred, T_est, r_max):
    """KISS-ICP model deviation of T_est from T_pred, written out with a
    general inverse and scipy's rotation angle."""
    D = np.linalg.inv(T_pred) @ T_est
    theta = Rotation.from_matrix(D[:3, :3]).magnitude()
    return 2.0 * r_max * math.sin(theta / 2.0) + float(np.linalg.norm(D[:3, 3]))


def check_odometry_structure(orc, c, out, m, n, max_iters=10, eps=0.0, asmd=False,
                             evict_radius=0.0, r_near=20.0, min_motion=0.1):
    """Replay the scan-to-submap loop (Sec. III-A, III-A.3) from the records it
    returned and check that each step consumed what the method says it does:

    * the downsampled scan is the first point of every downsample voxel;
    * the prediction of scan s >= 2 is T_{s-1} (T_{s-2}^-1 T_{s-1}) with its
      rotation projected onto SO(3); scan 1 uses the given first motion;
    * tau and kappa of scan s are 3 sigma and sigma / 3 of the deviations of
      the estimates of scans 1..s-1 from their predictions (sigma0 before the
      first sample), so the threshold is updated after the align;
    * the align of scan s starts at the prediction, on the map that holds
      scans 0..s-1 only, and returns the recorded estimate bit for bit;
    * the map after scan s equals a fresh map fed every downsampled scan at
      its returned estimate (sizes after every scan, the whole map at the
      end), with the density caps and eviction when they are on.
    """
    v1 = np.linalg.inv(c.poses[0]) @ c.poses[1]
    fm = orc.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.k,
                 point_capacity=c.map_capacity, voxel_capacity=c.map_capacity)
    samples, full = [], False
    for s in range(n):
        r = out[s]
        raw = c.scans[s]
        src = np.ascontiguousarray(raw[:, first_per_voxel(raw, c.downsample)])
        assert r["n"] == src.shape[1], f"scan {s}: downsampled size"
        if s == 0:
            np.testing.assert_array_equal(r["T"], c.poses[0])
        else:
            if s == 1:
                want = out[0]["T"] @ v1
            else:
                P1, P2 = out[s - 1]["T"], out[s - 2]["T"]
                want = P1 @ (np.linalg.inv(P2) @ P1)
            want[:3, :3] = _polar_rotation(want[:3, :3])
            np.testing.assert_allclose(r["T_pred"], want, rtol=0, atol=1e-11,
                                       err_msg=f"scan {s}: prediction")
            sigma = math.sqrt(sum(d * d for d in samples) / len(samples)) if samples \
                else c.sigma0
            assert r["tau"] == pytest.approx(3.0 * sigma, rel=1e-11), f"scan {s}: tau"
            assert r["kappa"] == pytest.approx(sigma / 3.0, rel=1e-11), f"scan {s}: kappa"
            cov, val = orc.scan_covariances(src, c.voxel_size, c.k)
            a = fm.align(src, cov.astype(np.float32), val, r["T_pred"], r["tau"], r["kappa"],
                         max_iters=max_iters, eps=eps)
            assert a["status"] == r["status"], f"scan {s}: align status"
            np.testing.assert_array_equal(a["T"] if a["status"] == 0 else r["T_pred"], r["T"],
                                          err_msg=f"scan {s}: align from the prediction")
            dev = _deviation(r["T_pred"], r["T"], c.r_max)
            assert r["deviation"] == pytest.approx(dev, rel=1e-9, abs=1e-12), \
                f"scan {s}: deviation"
            if dev > min_motion:
                samples.append(dev)
        if not full:
            moved = orc.transform(src, r["T"])
            caps = orc.asmd_caps(src, moved, c.voxel_size, c.k, c.max_pts_per_voxel, r_near,
                                 c.r_max)[0] if asmd else None
            rc, _, _ = fm.insert(moved, caps, check=False)
            full = rc == 2
        if evict_radius > 0:
            fm.evict(r["T"][:3, 3], evict_radius)
        assert fm.size == r["map_points"], f"scan {s}: map size after the insert"
    for a, b in zip(fm.export(), m.export()):
        np.testing.assert_array_equal(a, b, err_msg="map after the sequence")


def test_polar_rotation_agrees_with_svd():
    g = np.random.default_rng(9)
    for _ in range(20):
        M = Rotation.from_rotvec(g.normal(size=3)).as_matrix() + 1e-4 * g.normal(size=(3, 3))
        U, _, Vt = np.linalg.svd(M)
        np.testing.assert_allclose(_polar_rotation(M), U @ Vt, atol=1e-14)


def _run(orc, c, n, **kw):
    v1 = np.linalg.inv(c.poses[0]) @ c.poses[1]
    return orc.odometry(c.scans[:n], c.poses[0], v1, c.voxel_size, c.max_pts_per_voxel,
                        c.min_spacing, c.k, c.map_capacity, c.downsample, c.sigma0, c.r_max,
                        **kw)


def test_odometry_short_sequence_tracks_ground_truth(orc):
    n = 6
    c = synth.make_sequence(2, n_scans=n, lidar=synth.Lidar(beams=32, azimuths=512))
    out, m = _run(orc, c, n)
    assert [r["status"] for r in out] == [0] * n
    assert all(out[i]["map_points"] > out[i - 1]["map_points"] for i in range(1, n))
    for r, T in zip(out, c.poses):
        assert np.linalg.norm(r["T"][:3, 3] - T[:3, 3]) < 0.1 and _angle_deg(r["T"], T) < 0.3
    check_odometry_structure(orc, c, out, m, n)


def test_odometry_long_sequence_structure_and_drift(orc):
    # 60 scans: long enough for an unprojected constant-velocity predictor
    # (rounding growth about 2.4x per scan) to lose the rotation
    n = 60
    c = synth.make_sequence(2, n_scans=n, lidar=synth.Lidar(beams=32, azimuths=512))
    out, m = _run(orc, c, n)
    assert [r["status"] for r in out] == [0] * n
    assert all(out[i]["map_points"] > out[i - 1]["map_points"] for i in range(1, n))
    for r, T in zip(out, c.poses):
        assert np.linalg.norm(r["T"][:3, 3] - T[:3, 3]) < 2.0 and _angle_deg(r["T"], T) < 1.0
        np.testing.assert_allclose(r["T"][:3, :3].T @ r["T"][:3, :3], np.eye(3), atol=1e-13)
    check_odometry_structure(orc, c, out, m, n)


def test_odometry_structure_with_density_caps_and_eviction(orc):
    n = 12
    c = synth.make_sequence(2, n_scans=n, lidar=synth.Lidar(beams=32, azimuths=512))
    out, m = _run(orc, c, n, asmd=True, evict_radius=40.0)
    assert sum(r["evicted"] for r in out) > 0
    check_odometry_structure(orc, c, out, m, n, asmd=True, evict_radius=40.0)


MUTATIONS = ["insert_at_prediction", "threshold_before_align", "threshold_lag",
             "increment_on_wrong_side", "align_after_insert"]


def _loop_with_mistake(orc, c, n, mutation):
    """The odometry loop with one planted mistake (None: none), written out in
    the test so that the checker can be shown to catch each of them."""
    v1 = np.linalg.inv(c.poses[0]) @ c.poses[1]
    m = orc.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.k,
                point_capacity=c.map_capacity, voxel_capacity=c.map_capacity)
    thr = orc.Threshold(c.sigma0, c.r_max, 0.1)
    out, poses, pending, full = [], [], None, False
    for s in range(n):
        raw = c.scans[s]
        src = orc._soa(raw)[:, orc.downsample(raw, c.downsample)]
        rec = {"n": src.shape[1]}
        T_pred = None
        if s == 0:
            T = np.array(c.poses[0], dtype=np.float64)
            rec.update(T_pred=T.copy(), tau=None, kappa=None, status=0, iters=0)
        else:
            if s == 1:
                T_pred = poses[-1] @ v1
            elif mutation == "increment_on_wrong_side":
                T_pred = (orc._inv(poses[-2]) @ poses[-1]) @ poses[-1]
            else:
                T_pred = poses[-1] @ (orc._inv(poses[-2]) @ poses[-1])
            T_pred[:3, :3] = orc._nearest_rotation(T_pred[:3, :3])
            if mutation == "threshold_before_align":
                dev = thr.update(T_pred, poses[-1])
            tau, kappa = thr.get()
            if mutation == "threshold_lag" and pending is not None:
                thr.update(*pending)
            cov, val = orc.scan_covariances(src, c.voxel_size, c.k)
            if mutation == "align_after_insert" and not full:
                full = m.insert(orc.transform(src, T_pred), check=False)[0] == 2
            r = m.align(src, cov.astype(np.float32), val, T_pred, tau, kappa, max_iters=10,
                        eps=0.0)
            T = r["T"] if r["status"] == 0 else T_pred
            if mutation == "threshold_lag":
                pending = (T_pred, T)
                dev = orc.Threshold(c.sigma0, c.r_max, 0.1).update(T_pred, T)
            elif mutation != "threshold_before_align":
                dev = thr.update(T_pred, T)
            rec.update(T_pred=T_pred, tau=tau, kappa=kappa, status=r["status"],
                       iters=r["iters"], n_inliers=r["n_inliers"], cost=r["cost"],
                       deviation=dev)
        poses.append(T)
        if not full and not (mutation == "align_after_insert" and s > 0):
            at = T_pred if (mutation == "insert_at_prediction" and s > 0) else T
            rc, acc, _ = m.insert(orc.transform(src, at), None, check=False)
            full = rc == 2
            rec["inserted"] = acc
        rec.update(T=T, map_points=m.size, map_voxels=m.n_voxels)
        out.append(rec)
    return out, m


def test_mistake_harness_is_the_oracle_loop(orc):
    n = 6
    c = synth.make_sequence(2, n_scans=n, lidar=synth.Lidar(beams=32, azimuths=512))
    want, wm = _run(orc, c, n)
    got, gm = _loop_with_mistake(orc, c, n, None)
    for a, b in zip(want, got):
        for k in ("n", "T_pred", "tau", "kappa", "status", "iters", "T", "map_points"):
            np.testing.assert_array_equal(np.asarray(a[k], dtype=object if a[k] is None else None),
                                          np.asarray(b[k], dtype=object if b[k] is None else None))
    for a, b in zip(wm.export(), gm.export()):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("mutation", MUTATIONS)
def test_structure_check_catches_planted_mistake(orc, mutation):
    n = 6
    c = synth.make_sequence(2, n_scans=n, lidar=synth.Lidar(beams=32, azimuths=512))
    out, m = _loop_with_mistake(orc, c, n, mutation)
    with pytest.raises(AssertionError):
        check_odometry_structure(orc, c, out, m, n)


@pytest.mark.parametrize("angle", [1e-7, 3e-4, 0.3, 2.0, 3.1, math.pi])
def test_threshold_deviation_closed_form(orc, angle):
    # rotation only: the deviation is exactly 2 r_max sin(theta / 2), at small
    # angles and near pi (every quaternion branch) alike
    g = np.random.default_rng(int(angle * 1e3) + 7)
    for _ in range(5):
        axis = g.normal(size=3)
        axis /= np.linalg.norm(axis)
        P = synth.pose(Rotation.from_rotvec(g.normal(size=3)).as_matrix(), g.normal(size=3))
        D = synth.pose(Rotation.from_rotvec(axis * angle).as_matrix(), (0, 0, 0))
        t = orc.Threshold(1.0, 50.0, 0.0)
        want = 100.0 * math.sin(angle / 2)
        assert t.update(P, P @ D) == pytest.approx(want, rel=1e-7, abs=1e-12)
