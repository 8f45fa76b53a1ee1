"""The scan grid's two sort paths and the scratch pool on the GPU.

Scan covariances sort a batch's points by (scan, voxel key) in one pass over
compact keys when the batch's key range packs into 62 bits, and otherwise by
full keys and then by scan.  Both must give the oracle's covariances; the
cases sit on either side of the limit (a batch spanning the whole key range,
a scan at 2^20 voxels per axis, hundreds of scans); out-of-range keys are
found by the range pass that picks the path, and rejected.  Non-finite
points get the zero result with the outputs starting as junk.  The scratch
pool keeps its memory over repeated calls and gives it back on release."""
import numpy as np
import pytest
import torch

from paper_2606_26010_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def far():
    from paper_2606_26010_amd import far as f
    f.lib()
    return f


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)


def check_batch(far, orc, scans, v=1.0, k=5):
    sizes = [s.shape[1] for s in scans]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cov, val = far.far_scan_covariances_batch(dev(np.concatenate(scans, 1)), dev(offs), v, k)
    cov, val = host(cov), host(val)
    for s, sc in enumerate(scans):
        if sc.shape[1] == 0:
            continue
        oc, ov = orc.scan_covariances(np.ascontiguousarray(sc), v, k)
        np.testing.assert_array_equal(val[offs[s]:offs[s + 1]], ov)
        np.testing.assert_allclose(cov[:, offs[s]:offs[s + 1]], oc, rtol=2e-6, atol=1e-6)
    return cov, val


def scene(seed, n):
    if n == 0:
        return np.zeros((3, 0), np.float32)
    return synth.random_cloud(seed, n, extent=3.0, dup_frac=0.05, on_faces=0.2, v=1.0)


def corners(scale):
    """The eight corners of a cube of half-width scale (metres) plus a few
    points beside each, so that the far voxels hold covariances too."""
    g = np.random.default_rng(3)
    c = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)],
                 np.float64).T * scale
    pts = np.repeat(c, 8, axis=1) + g.uniform(0.05, 0.45, size=(3, 64)) * -np.sign(
        np.repeat(c, 8, axis=1))
    return np.ascontiguousarray(pts.astype(np.float32))


def test_compact_and_full_sort_paths_agree(far, orc):
    base = [scene(21, 3000), scene(22, 257), np.zeros((3, 0), np.float32), scene(23, 1500)]
    # compact path: the batch spans a few metres
    cov_a, val_a = check_batch(far, orc, base)
    # full-key path: one scan reaches voxel keys near +-2^20 on every axis
    wide = base + [np.concatenate([scene(24, 500), corners(1.0e6)], 1)]
    cov_b, val_b = check_batch(far, orc, wide)
    n = sum(s.shape[1] for s in base)
    np.testing.assert_array_equal(cov_a, cov_b[:, :n])
    np.testing.assert_array_equal(val_a, val_b[:n])
    say(f"compact / full sort: {n} shared points identical, {int(val_b.sum())} valid")


def test_single_scan_spanning_2_20_voxels(far, orc):
    # keys 0 .. 2^20 - 1 per axis: 60 key bits, still the compact path
    pts = np.concatenate([scene(25, 2000), corners(5.2e5) + 5.2e5], 1)
    gcov, gval = far.far_scan_covariances(dev(pts), 1.0, 5)
    ocov, oval = orc.scan_covariances(pts, 1.0, 5)
    np.testing.assert_array_equal(host(gval), oval)
    np.testing.assert_allclose(host(gcov), ocov, rtol=2e-6, atol=1e-6)
    assert oval[-64:].sum() > 0


def test_many_small_scans(far, orc):
    g = np.random.default_rng(26)
    scans = [scene(100 + s, int(g.integers(0, 200))) for s in range(300)]
    check_batch(far, orc, scans)


@pytest.mark.parametrize("wide", [False, True])
def test_out_of_range_keys_rejected(far, wide):
    pts = scene(27, 1000)
    if wide:                       # the rest of the batch alone takes the full-key path
        pts = np.concatenate([pts, corners(1.0e6)], 1)
    pts = np.concatenate([pts, np.array([[4.0e6], [0.0], [0.0]], np.float32)], 1)
    offs = np.array([0, 600, pts.shape[1]], np.int64)
    with pytest.raises(far.FarError, match="outside"):
        far.far_scan_covariances_batch(dev(pts), dev(offs), 1.0, 5)
    with pytest.raises(far.FarError, match="outside"):
        far.far_scan_covariances(dev(pts), 1.0, 5)


def test_scratch_pool_keeps_and_releases(far):
    pts = dev(np.concatenate([scene(28 + s, 20000) for s in range(4)], 1))
    far.far_scan_covariances(pts, 1.0, 5)
    torch.cuda.synchronize()
    held = far.far_scratch_reserved()
    assert held > 0
    for _ in range(3):
        far.far_scan_covariances(pts, 1.0, 5)
    torch.cuda.synchronize()
    assert far.far_scratch_reserved() == held       # reused, not grown
    far.far_scratch_release()
    after = far.far_scratch_reserved()
    say(f"scratch pool: {held} bytes held, {after} after release")
    assert after < held
    cov, val = far.far_scan_covariances(pts, 1.0, 5)     # and usable again
    torch.cuda.synchronize()
    assert far.far_scratch_reserved() > after and int(host(val).sum()) > 0


@pytest.mark.parametrize("dense", [0, 16])
def test_non_finite_points_get_the_zero_result(far, orc, dense):
    """Every output is written, also where the input is not finite: the
    outputs start as junk; a batch with scattered NaN / inf points and a scan
    with no finite point at all (the whole result zero)."""
    g = np.random.default_rng(29)
    scans = [scene(30, 3000), scene(31, 500), scene(32, 800)]
    for sc in scans[:2]:
        m = g.uniform(size=sc.shape[1]) < 0.03
        sc[0, m] = np.nan
        sc[2, m[::-1]] = np.inf
    scans[2][:] = np.nan
    sizes = [s.shape[1] for s in scans]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(offs[-1])
    cov = torch.full((6, n), 7.0, dtype=torch.float32, device="cuda")
    val = torch.full((n,), 3, dtype=torch.uint8, device="cuda")
    old = far.far_get_covariance_schedule()
    far.far_set_covariance_schedule(dense)
    try:
        far.far_scan_covariances_batch(dev(np.concatenate(scans, 1)), dev(offs), 1.0, 5,
                                       out=(cov, val))
        c, v = host(cov), host(val)
        for s, sc in enumerate(scans):
            oc, ov = orc.scan_covariances(np.ascontiguousarray(sc), 1.0, 5)
            np.testing.assert_array_equal(v[offs[s]:offs[s + 1]], ov)
            np.testing.assert_allclose(c[:, offs[s]:offs[s + 1]], oc, rtol=2e-6, atol=1e-6)
        bad = ~np.isfinite(np.concatenate(scans, 1)).all(axis=0)
        assert bad.sum() > 900 and np.all(c[:, bad] == 0) and np.all(v[bad] == 0)
        # one scan, nothing finite
        cov1 = torch.full((6, 800), 7.0, dtype=torch.float32, device="cuda")
        val1 = torch.full((800,), 3, dtype=torch.uint8, device="cuda")
        far.far_scan_covariances_batch(dev(scans[2]), dev(np.array([0, 800], np.int64)), 1.0,
                                       5, out=(cov1, val1))
        assert np.all(host(cov1) == 0) and np.all(host(val1) == 0)
    finally:
        far.far_set_covariance_schedule(old)
