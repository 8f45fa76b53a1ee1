"""Pins of the oracle's covariances: Eq. (1) regularisation and the k-neighbour
sample covariance (paper Sec. III-A.2, covariance paragraph).

Checked against numpy.cov on brute-force neighbour sets, closed forms derived
by hand from Eq. (1), and the invariants Eq. (1) implies.
"""
import math

import numpy as np
import pytest

from paper_2606_26010_amd import synth
from tests.test_oracle_map import brute_knn


def eq1_eigen(S_hat):
    """Eq. (1) via an eigendecomposition (numpy.linalg.eigh): C = Q diag(l) Q^T,
    C^-1 / ||C^-1||_F = Q diag(1/l) Q^T / sqrt(sum 1/l^2), inverted again."""
    C = S_hat + 1e-3 * np.eye(3)
    lam, Q = np.linalg.eigh(C)
    nrm = math.sqrt(float(np.sum(1.0 / lam ** 2)))
    return Q @ np.diag(lam * nrm) @ Q.T


def test_eq1_identical_points_closed_form(orc):
    # k identical points: Sigma_hat = 0, C = 1e-3 I, ||C^-1||_F = 1000 sqrt(3)
    Sig = orc.regularize_cov(np.zeros((3, 3)))
    np.testing.assert_allclose(Sig, math.sqrt(3.0) * np.eye(3), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("a,b", [(0.01, 0.04), (0.2, 0.2), (1e-6, 3.0)])
def test_eq1_planar_closed_form(orc, a, b):
    # planar neighbourhood with eigenvalues (0, a, b) in a rotated basis:
    # Sigma = sqrt(1e6 + (a+1e-3)^-2 + (b+1e-3)^-2) * diag(1e-3, a+1e-3, b+1e-3)
    Q = synth.random_offset(synth.rng(3), 0.0, 37.0)[:3, :3]
    S_hat = Q @ np.diag([0.0, a, b]) @ Q.T
    s = math.sqrt(1e6 + (a + 1e-3) ** -2 + (b + 1e-3) ** -2)
    want = Q @ np.diag([s * 1e-3, s * (a + 1e-3), s * (b + 1e-3)]) @ Q.T
    np.testing.assert_allclose(orc.regularize_cov(S_hat), want, rtol=1e-10,
                               atol=1e-12 * np.abs(want).max())


def test_eq1_invariants_random(orc):
    g = synth.rng(4)
    for _ in range(50):
        A = g.normal(size=(3, 7)) * g.uniform(0.001, 2.0, size=(3, 1))
        S_hat = np.cov(A, bias=True)
        Sig = orc.regularize_cov(S_hat)
        np.testing.assert_allclose(Sig, Sig.T, rtol=0, atol=1e-12 * np.abs(Sig).max())
        # ||Sigma^-1||_F = 1 and Sigma >= I (every eigenvalue at least 1)
        assert abs(np.linalg.norm(np.linalg.inv(Sig)) - 1.0) < 1e-10
        assert np.linalg.eigvalsh(Sig).min() >= 1.0 - 1e-10
        np.testing.assert_allclose(Sig, eq1_eigen(S_hat), rtol=1e-9,
                                   atol=1e-12 * np.abs(Sig).max())


def six_to_mat(c):
    return np.array([[c[0], c[1], c[2]], [c[1], c[3], c[4]], [c[2], c[4], c[5]]])


@pytest.mark.parametrize("k,v", [(5, 1.0), (10, 1.0), (5, 0.5)])
def test_scan_covariances_match_numpy(orc, k, v):
    cloud = synth.random_cloud(51, 2500, extent=2.5, dup_frac=0.02, on_faces=0.2, v=v)
    cov, valid = orc.scan_covariances(cloud, v, k)
    idx, _, cnt = brute_knn(cloud, np.arange(cloud.shape[1]), cloud, k, v)
    np.testing.assert_array_equal(valid, (cnt == k).astype(np.uint8))
    p64 = cloud.astype(np.float64)
    for i in np.nonzero(valid)[0][::3]:
        nb = p64[:, idx[i]]
        want = eq1_eigen(np.cov(nb, bias=True))
        np.testing.assert_allclose(six_to_mat(cov[:, i]), want, rtol=1e-7,
                                   atol=1e-9 * np.abs(want).max())
    assert np.all(cov[:, valid == 0] == 0)


def test_map_covariances_of_added_points_only(orc):
    # covariances are computed for added points on the updated map; existing
    # points keep theirs (Sec. III-A.3)
    v, k = 1.0, 5
    cloud = synth.random_cloud(52, 3000, extent=2.0, v=v)
    m = orc.Map(v, 1 << 20, 0.0, k)
    m.insert(cloud[:, :1000])
    _, cov_a, val_a = m.export()
    m.insert(cloud[:, 1000:])
    xyz, cov_b, val_b = m.export()
    np.testing.assert_array_equal(cov_b[:, :1000], cov_a)
    np.testing.assert_array_equal(val_b[:1000], val_a)
    # the first batch's covariances used only the first batch
    ref, rv = orc.scan_covariances(cloud[:, :1000], v, k)
    np.testing.assert_array_equal(val_a, rv)
    np.testing.assert_array_equal(cov_a, ref.astype(np.float32))
    # the added points' covariances use the whole updated map
    full, fv = orc.scan_covariances(xyz, v, k)
    np.testing.assert_array_equal(val_b[1000:], fv[1000:])
    np.testing.assert_array_equal(cov_b[:, 1000:], full[:, 1000:].astype(np.float32))


def test_sparse_points_are_invalid(orc):
    # isolated points (fewer than k neighbours within v) get no covariance
    pts = np.array([[0.0, 5.0, 10.0, 10.1, 10.2, 10.3, 10.4],
                    [0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0],
                    [0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]], np.float32)
    cov, valid = orc.scan_covariances(pts, 1.0, 5)
    np.testing.assert_array_equal(valid, [0, 0, 1, 1, 1, 1, 1])
