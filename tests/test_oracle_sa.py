"""Pins of the sparsity-aware switch of the oracle (Sec. III-A.2, the SA GICP
paragraph; Table III ablates it): with it off, a pair whose source or map
covariance is invalid is dropped instead of entering point-to-point.  Pinned
by reductions to other calls (all covariances valid: no change; only source
covariances invalid: the same as leaving those points out of the scan) and
by the correspondence sets; then the ablation on sparse scans."""
import math

import numpy as np
import pytest

from oracle import far_oracle as orc
from paper_2606_26010_amd import synth


@pytest.fixture(scope="module")
def tiny():
    c = synth.make_tiny(1)
    m = orc.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.k)
    for b in c.map_batches:
        m.insert(b)
    return c, m


def pose_err(A, B):
    E = A[:3, :3] @ B[:3, :3].T
    s = np.array([E[2, 1] - E[1, 2], E[0, 2] - E[2, 0], E[1, 0] - E[0, 1]])
    return (float(np.linalg.norm(A[:3, 3] - B[:3, 3])),
            math.degrees(math.atan2(0.5 * np.linalg.norm(s), 0.5 * (np.trace(E) - 1))))


def test_no_effect_when_every_covariance_is_valid(tiny):
    c, m = tiny
    cov, val = orc.scan_covariances(c.source, c.voxel_size, c.k)
    cov = cov.astype(np.float32)
    _, _, mval = m.export()
    T = c.T_gt @ synth.random_offset(synth.rng(3), 0.1, 1.0)
    on = m.linearize(c.source, cov, np.ones_like(val), T, c.tau, c.kappa, want_corr=True)
    hit = on["corr"] >= 0
    assert hit.sum() > 1000
    keep = np.zeros(c.source.shape[1], bool)
    keep[hit] = mval[on["corr"][hit]] != 0           # pairs whose map side is valid too
    src = np.ascontiguousarray(c.source[:, keep])
    ones = np.ones(src.shape[1], np.uint8)
    a = m.linearize(src, cov[:, keep], ones, T, c.tau, c.kappa, want_corr=True)
    b = m.linearize(src, cov[:, keep], ones, T, c.tau, c.kappa, want_corr=True, sa=False)
    np.testing.assert_array_equal(a["corr"], b["corr"])
    np.testing.assert_array_equal(a["H"], b["H"])
    np.testing.assert_array_equal(a["b"], b["b"])
    assert a["cost"] == b["cost"] and a["n_inliers"] == b["n_inliers"]


def test_invalid_source_covariances_are_left_out(tiny):
    """Correspondences kept exactly where both covariances are valid; and on
    the points whose match (if any) has a valid map covariance, dropping
    pairs equals removing the source points whose covariance is invalid."""
    c, m = tiny
    g = np.random.default_rng(5)
    sub = np.sort(g.choice(c.source.shape[1], 1500, replace=False))
    src = np.ascontiguousarray(c.source[:, sub])
    cov, val = orc.scan_covariances(src, c.voxel_size, c.k)
    cov = cov.astype(np.float32)
    assert 0.1 < val.mean() < 0.95                  # a sparse scan: some of each
    _, _, mval = m.export()
    T = c.T_gt @ synth.random_offset(synth.rng(4), 0.05, 0.5)
    on = m.linearize(src, cov, val, T, c.tau, c.kappa, want_corr=True)
    hit = on["corr"] >= 0
    map_ok = np.ones(src.shape[1], bool)
    map_ok[hit] = mval[on["corr"][hit]] != 0
    off = m.linearize(src, cov, val, T, c.tau, c.kappa, want_corr=True, sa=False)
    # the correspondences: kept exactly where both covariances are valid
    both = hit & (val != 0) & map_ok
    np.testing.assert_array_equal(off["corr"], np.where(both, on["corr"], -1))
    assert off["n_inliers"] == both.sum() < on["n_inliers"]
    # keep the points whose pair has a valid map side (a point's match does
    # not depend on the other source points): there, off = on over the points
    # with a valid source covariance
    assert (~map_ok).sum() > 0
    s2, c2, v2 = (np.ascontiguousarray(src[:, map_ok]), np.ascontiguousarray(cov[:, map_ok]),
                  val[map_ok])
    off2 = m.linearize(s2, c2, v2, T, c.tau, c.kappa, sa=False)
    keep = v2 != 0
    ref = m.linearize(np.ascontiguousarray(s2[:, keep]), np.ascontiguousarray(c2[:, keep]),
                      v2[keep], T, c.tau, c.kappa)
    np.testing.assert_array_equal(off2["H"], ref["H"])
    np.testing.assert_array_equal(off2["b"], ref["b"])
    assert off2["cost"] == ref["cost"] and off2["n_inliers"] == ref["n_inliers"] > 100


def test_gradient_follows_the_switch(tiny):
    c, m = tiny
    src = np.ascontiguousarray(c.source[:, ::4])
    cov, val = orc.scan_covariances(src, c.voxel_size, c.k)
    cov = cov.astype(np.float32)
    T = c.T_gt @ synth.random_offset(synth.rng(6), 0.05, 0.5)
    lin = m.linearize(src, cov, val, T, c.tau, c.kappa, want_corr=True, sa=False)
    gr = m.gradient(src, cov, val, T, c.tau, c.kappa, sa=False)
    np.testing.assert_array_equal(gr["corr"], lin["corr"])
    assert gr["n_inliers"] == lin["n_inliers"]
    assert gr["cost"] == pytest.approx(lin["cost"], rel=1e-12)
    dropped = lin["corr"] < 0
    assert not np.any(gr["grad_src"][:, dropped])


def sparse_scans(c, n_keep, n_scans, seed):
    g = np.random.default_rng(seed)
    for s in range(n_scans):
        sub = np.sort(g.choice(c.source.shape[1], n_keep, replace=False))
        yield s, np.ascontiguousarray(c.source[:, sub])


def test_ablation_on_sparse_scans(tiny):
    """Scans so sparse that almost no point has k neighbours within v (300
    and 600 of the 5000 points, at most 1 % valid covariances), 0.3 m / 2 deg
    from the truth: without the sparsity-aware case the align has too few
    correspondences (status 5) or lands farther off than it started; with it
    every scan converges and ends closer than it started.  (At moderate
    density the point-to-point terms add a bias instead: the ablation is
    reported, not pinned, there.)"""
    c, m = tiny
    for n_keep in (300, 600):
        err, fails = {True: [], False: []}, 0
        for s, src in sparse_scans(c, n_keep, 6, 21):
            cov, val = orc.scan_covariances(src, c.voxel_size, c.k)
            assert val.mean() <= 0.02
            cov = cov.astype(np.float32)
            T0 = c.T_gt @ synth.random_offset(synth.rng(40 + s), 0.3, 2.0)
            e0 = pose_err(T0, c.T_gt)[0]
            for sa in (True, False):
                r = m.align(src, cov, val, T0, c.tau, c.kappa, max_iters=20, eps=0.0, sa=sa)
                if sa:
                    assert r["status"] == 0
                    err[sa].append(pose_err(r["T"], c.T_gt)[0])
                    assert err[sa][-1] < e0
                elif r["status"] != 0:
                    fails += 1
                    err[sa].append(e0)
                else:
                    err[sa].append(pose_err(r["T"], c.T_gt)[0])
        on, off = float(np.mean(err[True])), float(np.mean(err[False]))
        print(f"ablation, {n_keep} points: SA on {on:.3f} m, off {off:.3f} m ({fails} of 6 "
              f"failed)")
        assert on < 0.5 * off
