"""Pins of the oracle's GICP gradient (cost of Eq. 4 with the Cauchy rho of
Eq. 5; correspondences and source covariances held fixed): central finite
differences in FP64 (step 1e-6) of the cost with frozen correspondences, for
the 12 entries of [R | t], the 6 twist components and the source points; and
the reduction to b when every covariance is invalid."""
import numpy as np
import pytest

from paper_2606_26010_amd import synth

H_FD = 1e-6


@pytest.fixture(scope="module")
def case(orc):
    c = synth.make_tiny(1)
    m = orc.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.k)
    for b in c.map_batches:
        m.insert(b)
    cov, val = orc.scan_covariances(c.source, c.voxel_size, c.k)   # the whole scan's
    src = np.ascontiguousarray(c.source[:, :600])
    cov = np.ascontiguousarray(cov[:, :600].astype(np.float32))
    val = np.ascontiguousarray(val[:600])
    g = synth.rng(9)
    T = c.T_gt @ synth.random_offset(g, 0.05, 0.5)
    return c, m, src, cov, val, T


def fd(f, x0, h=H_FD):
    g = np.zeros(x0.size)
    for k in range(x0.size):
        e = np.zeros(x0.size)
        e[k] = h
        g[k] = (f(x0 + e) - f(x0 - e)) / (2 * h)
    return g


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def test_gradient_wrt_pose_entries(case):
    c, m, src, cov, val, T = case
    gr = m.gradient(src, cov, val, T, c.tau, c.kappa, c=T[:3, 3])
    assert gr["n_inliers"] > 500 and np.count_nonzero(val) > 300
    src64 = src.astype(np.float64)

    def cost(x):
        Tx = T.copy()
        Tx[:3, :] = x.reshape(3, 4)
        return m.cost_fixed(src64, cov, val, Tx, c.kappa, gr["corr"])

    assert cost(T[:3, :].ravel()) == pytest.approx(gr["cost"], rel=1e-12)
    assert rel(gr["grad_T"], fd(cost, T[:3, :].ravel())) <= 1e-6


def test_gradient_wrt_twist(case, orc):
    c, m, src, cov, val, T = case
    ctr = T[:3, 3].copy()
    gr = m.gradient(src, cov, val, T, c.tau, c.kappa, c=ctr)
    src64 = src.astype(np.float64)
    Tc, Tci = np.eye(4), np.eye(4)
    Tc[:3, 3], Tci[:3, 3] = ctr, -ctr

    def cost(d):
        return m.cost_fixed(src64, cov, val, Tc @ orc.se3_exp(d) @ Tci @ T, c.kappa, gr["corr"])

    num = fd(cost, np.zeros(6))
    assert rel(gr["grad_twist"], num) <= 1e-6
    # the covariance term of the rotation part is not negligible here, so a
    # gradient without it would fail the comparison above
    lin = m.linearize(src, cov, val, T, c.tau, c.kappa, c=ctr)
    assert rel(lin["b"], num) > 1e-4


def test_gradient_wrt_source_points(case):
    c, m, src, cov, val, T = case
    gr = m.gradient(src, cov, val, T, c.tau, c.kappa)
    src64 = src.astype(np.float64)
    pick = np.nonzero(gr["corr"] >= 0)[0][::13][:40]
    for i in pick:
        def cost(x, i=i):
            s = src64.copy()
            s[:, i] = x
            return m.cost_fixed(s, cov, val, T, c.kappa, gr["corr"])
        assert rel(gr["grad_src"][:, i], fd(cost, src64[:, i])) <= 1e-6, i
    out = np.nonzero(gr["corr"] < 0)[0]
    assert np.all(gr["grad_src"][:, out] == 0)


def test_gradient_reduces_to_b_without_covariances(case):
    c, m, src, cov, val, T = case
    none = np.zeros_like(val)
    ctr = T[:3, 3]
    gr = m.gradient(src, cov, none, T, c.tau, c.kappa, c=ctr)
    lin = m.linearize(src, cov, none, T, c.tau, c.kappa, c=ctr)
    assert rel(gr["grad_twist"], lin["b"]) <= 1e-12
    assert rel(gr["grad_T"][:, 3], lin["b"][3:]) <= 1e-12
    assert gr["cost"] == pytest.approx(lin["cost"], rel=1e-12)
