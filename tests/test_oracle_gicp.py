"""Pins of the oracle's GICP linearisation, solve and align (paper Sec. III-A.2,
Eqs. (2)-(6)).

The checks do not reuse the oracle's arithmetic: correspondences against brute
force, the fused covariance against numpy, b against central finite
differences of the cost with correspondences and M frozen, H against the
finite-difference Hessian at zero residual, the SE(3) exponential against
scipy.linalg.expm, the solve against numpy.linalg.solve, and the align against
the Kabsch/Umeyama closed form and known ground truth.
"""
import math

import numpy as np
import pytest
import scipy.linalg

from paper_2606_26010_amd import synth
from tests.test_oracle_map import brute_knn


def twist_exp(delta):
    """SE(3) exponential via the matrix exponential of the 4x4 twist."""
    w, v = delta[:3], delta[3:]
    X = np.zeros((4, 4))
    X[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    X[:3, 3] = v
    return scipy.linalg.expm(X)


def frozen_cost(det, c, kappa, delta):
    """Sum of Cauchy costs with correspondences r, points p and W frozen, after
    moving the points by c + Exp(delta)(p - c)."""
    E = twist_exp(delta)
    p, r = det[:, 0:3], det[:, 3:6]
    W = det[:, 6:15].reshape(-1, 3, 3)
    q = (p - c) @ E[:3, :3].T + E[:3, 3] + c
    d = r - q
    e2 = np.einsum("ni,nij,nj->n", d, W, d)
    return float(np.sum(0.5 * kappa * kappa * np.log1p(e2 / (kappa * kappa))))


def built_tiny(orc, seed=1, n_batches=6):
    c = synth.make_tiny(seed, n_batches=n_batches)
    m = orc.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.k)
    for b in c.map_batches:
        m.insert(b)
    scov, sval = orc.scan_covariances(c.source, c.voxel_size, c.k)
    return c, m, scov.astype(np.float32), sval


@pytest.fixture(scope="module")
def tiny(orc):
    return built_tiny(orc)


def test_correspondences_equal_brute_force(orc, tiny):
    c, m, scov, sval = tiny
    xyz, _, _ = m.export()
    T = c.T_gt @ synth.random_offset(synth.rng(9), 0.1, 1.0)
    tau = 0.6
    out = m.linearize(c.source, scov, sval, T, tau, c.kappa, want_corr=True)
    s = c.source.astype(np.float64)
    R, t = T[:3, :3], T[:3, 3]
    # the FP64 transform, evaluated ((R0 sx + R1 sy) + R2 sz) + t
    p = np.stack([((R[a, 0] * s[0] + R[a, 1] * s[1]) + R[a, 2] * s[2]) + t[a]
                  for a in range(3)])
    r = min(tau, c.voxel_size)
    # brute force needs FP32 queries; compare on the subset whose FP64 point is
    # an FP32 value -- instead rank in FP64 directly:
    x = xyz.astype(np.float64)
    want = np.full(p.shape[1], -1, np.int32)
    for i in range(p.shape[1]):
        dx, dy, dz = x[0] - p[0, i], x[1] - p[1, i], x[2] - p[2, i]
        d2 = (dx * dx + dy * dy) + dz * dz
        mm = np.nonzero(d2 <= r * r)[0]
        if mm.size:
            want[i] = mm[np.lexsort((mm, d2[mm]))[0]]
    np.testing.assert_array_equal(out["corr"], want)
    assert out["n_inliers"] == int(np.sum(want >= 0))


def test_fused_covariance_and_sa_rule(orc, tiny):
    c, m, scov, sval = tiny
    _, mcov, mval = m.export()
    T = c.T_gt
    out = m.linearize(c.source, scov, sval, T, c.tau, c.kappa, want_corr=True,
                      want_detail=True)
    R = T[:3, :3]
    det, corr = out["detail"], out["corr"]
    n_sa = 0
    for i in np.nonzero(corr >= 0)[0][::5]:
        j = corr[i]
        if sval[i] and mval[j]:
            Sr = six(mcov[:, j])
            Ss = six(scov[:, i])
            M = Sr + R @ Ss @ R.T
        else:
            M = np.eye(3)
            n_sa += 1
        np.testing.assert_allclose(det[i, 6:15].reshape(3, 3), np.linalg.inv(M),
                                   rtol=1e-9, atol=1e-12)
        d = det[i, 3:6] - det[i, 0:3]
        e2 = d @ np.linalg.inv(M) @ d
        assert abs(det[i, 17] - e2) <= 1e-9 * max(e2, 1e-12)
        k2 = c.kappa ** 2
        assert abs(det[i, 15] - k2 / (k2 + e2)) < 1e-12
    assert n_sa > 0    # the case includes sparsity-aware (M = I) points


def six(c6):
    return np.array([[c6[0], c6[1], c6[2]], [c6[1], c6[3], c6[4]], [c6[2], c6[4], c6[5]]],
                    np.float64)


@pytest.mark.parametrize("kappa", [1.0 / 9.0, 0.5, 1e3])
def test_b_is_gradient_of_frozen_cost(orc, tiny, kappa):
    c, m, scov, sval = tiny
    T = c.T_gt @ synth.random_offset(synth.rng(10), 0.05, 0.5)
    cen = T[:3, 3].copy()
    out = m.linearize(c.source, scov, sval, T, c.tau, kappa, c=cen, want_detail=True)
    det = out["detail"]
    det = det[np.isfinite(det[:, 0])]
    assert det.shape[0] == out["n_inliers"]
    assert abs(frozen_cost(det, cen, kappa, np.zeros(6)) - out["cost"]) <= 1e-12 * out["cost"]
    h = 1e-6
    g = np.array([(frozen_cost(det, cen, kappa, h * e) - frozen_cost(det, cen, kappa, -h * e))
                  / (2 * h) for e in np.eye(6)])
    np.testing.assert_allclose(out["b"], g, rtol=2e-5, atol=2e-6 * np.abs(g).max())


def test_H_is_hessian_at_zero_residual(orc):
    # source = exact copies of map points at T = I: every residual is zero, so
    # the Gauss-Newton H equals the true Hessian of the cost
    c = synth.make_tiny(2, n_batches=2)
    m = orc.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.k)
    for b in c.map_batches:
        m.insert(b)
    xyz, _, _ = m.export()
    src = np.ascontiguousarray(xyz[:, ::4])
    scov, sval = orc.scan_covariances(src, c.voxel_size, c.k)
    cen = np.array([1.5, -2.0, 0.7])
    kappa = 1.0
    out = m.linearize(src, scov.astype(np.float32), sval, np.eye(4), c.tau, kappa, c=cen,
                      want_detail=True)
    det = out["detail"]
    det = det[np.isfinite(det[:, 0])]
    assert np.all(det[:, 17] == 0.0) and out["cost"] == 0.0
    # the Cauchy curvature enters at O(h^2 |p - c|^2 / kappa^2): keep h small
    h = 1e-5
    E = np.eye(6)
    Hfd = np.zeros((6, 6))
    f0 = frozen_cost(det, cen, kappa, np.zeros(6))
    for a in range(6):
        for bb in range(6):
            Hfd[a, bb] = (frozen_cost(det, cen, kappa, h * (E[a] + E[bb]))
                          - frozen_cost(det, cen, kappa, h * (E[a] - E[bb]))
                          - frozen_cost(det, cen, kappa, h * (E[bb] - E[a]))
                          + frozen_cost(det, cen, kappa, -h * (E[a] + E[bb]))) / (4 * h * h)
    assert f0 == 0.0
    np.testing.assert_allclose(out["H"], Hfd, rtol=1e-5, atol=1e-6 * np.abs(Hfd).max())


def test_H_symmetric_psd(orc, tiny):
    c, m, scov, sval = tiny
    out = m.linearize(c.source, scov, sval, np.eye(4), c.tau, c.kappa)
    H = out["H"]
    np.testing.assert_array_equal(H, H.T)
    lam = np.linalg.eigvalsh(H)
    assert lam.min() >= -1e-12 * np.abs(lam).max()


# ---------------------------------------------------------------- solve pieces
@pytest.mark.parametrize("scale", [0.0, 1e-9, 1e-7, 1e-5, 0.1, 1.0, 3.0])
def test_se3_exp_matches_expm(orc, scale):
    g = synth.rng(12)
    for _ in range(5):
        d = g.normal(size=6) * scale
        T = orc.se3_exp(d)
        np.testing.assert_allclose(T, twist_exp(d), rtol=0, atol=1e-13 * max(1.0, scale))
        R = T[:3, :3]
        assert np.abs(R.T @ R - np.eye(3)).max() < 1e-14
        np.testing.assert_allclose(T @ orc.se3_exp(-d), np.eye(4), atol=1e-13 * max(1, scale))


def test_cholesky_solve(orc):
    g = synth.rng(13)
    A = g.normal(size=(6, 6))
    H = A @ A.T + 0.1 * np.eye(6)
    b = g.normal(size=6)
    rc, x = orc.cholesky_solve6(H, b)
    assert rc == 0
    np.testing.assert_allclose(x, np.linalg.solve(H, b), rtol=1e-12, atol=1e-12)
    Hs = A[:, :5] @ A[:, :5].T          # rank 5
    assert orc.cholesky_solve6(Hs, b)[0] == 4


# ---------------------------------------------------------------- align
def kabsch(P, Q):
    """Rigid T minimising sum |Q - (R P + t)|^2 (Umeyama, no scale)."""
    mp, mq = P.mean(1, keepdims=True), Q.mean(1, keepdims=True)
    U, _, Vt = np.linalg.svd((Q - mq) @ (P - mp).T)
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(U @ Vt))])
    R = U @ D @ Vt
    return synth.pose(R, (mq - R @ mp).ravel())


def pose_err(A, B):
    E = np.linalg.inv(B) @ A
    ang = math.degrees(math.acos(max(-1.0, min(1.0, (np.trace(E[:3, :3]) - 1) / 2))))
    return float(np.linalg.norm(A[:3, 3] - B[:3, 3])), ang


def test_point_to_point_align_equals_kabsch(orc):
    c = synth.make_tiny(3, n_batches=4)
    m = orc.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.k)
    for b in c.map_batches:
        m.insert(b)
    xyz, _, _ = m.export()
    ref = np.ascontiguousarray(xyz[:, ::3])
    src = synth.apply(synth.pose_inverse(c.T_gt), ref)
    n = src.shape[1]
    zero_cov = np.zeros((6, n), np.float32)
    T0 = c.T_gt @ synth.random_offset(synth.rng(14), 0.04, 0.4)
    out = m.align(src, zero_cov, np.zeros(n, np.uint8), T0, 1.0, 1e8, max_iters=30,
                  eps=1e-12)
    assert out["status"] == 0 and out["n_inliers"] == n
    K = kabsch(src.astype(np.float64), ref.astype(np.float64))
    np.testing.assert_allclose(out["T"], K, atol=1e-9)
    dt, da = pose_err(out["T"], c.T_gt)
    assert dt < 1e-5 and da < 1e-4


def test_gicp_noise_free_recovers_pose(orc):
    c = synth.make_tiny(4, n_batches=6)
    m = orc.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.k)
    for b in c.map_batches:
        m.insert(b)
    xyz, _, _ = m.export()
    ref = np.ascontiguousarray(xyz[:, ::3])
    src = synth.apply(synth.pose_inverse(c.T_gt), ref)
    scov, sval = orc.scan_covariances(src, c.voxel_size, c.k)
    T0 = c.T_gt @ synth.random_offset(synth.rng(15), 0.05, 0.5)
    out = m.align(src, scov.astype(np.float32), sval, T0, c.tau, c.kappa, max_iters=20,
                  eps=1e-10)
    assert out["status"] == 0
    dt, da = pose_err(out["T"], c.T_gt)
    assert dt < 1e-6 and da < 1e-5, (dt, da)


def test_tiny_noisy_align_reaches_noise_level(orc, tiny):
    c, m, scov, sval = tiny
    # sanity only (not parity): converged error at the level of the 2 cm noise
    out = m.align(c.source, scov, sval, np.eye(4), c.tau, c.kappa, max_iters=40, eps=1e-6)
    assert out["status"] == 0 and out["converged"] == 1 and out["iters"] >= 2
    dt, da = pose_err(out["T"], c.T_gt)
    assert dt < 1e-2 and da < 0.05, (dt, da)


def test_few_correspondences_leave_pose(orc, tiny):
    c, m, scov, sval = tiny
    far = np.eye(4)
    far[:3, 3] = [500.0, 0.0, 0.0]
    out = m.align(c.source, scov, sval, far, c.tau, c.kappa)
    assert out["status"] == 5 and out["iters"] == 0
    np.testing.assert_array_equal(out["T"], far)
