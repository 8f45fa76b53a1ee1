"""Pins of the oracle's submap update (Sec. III-A.3): adaptive submap density
caps and eviction of distant voxels."""
import math

import numpy as np
import pytest

from paper_2606_26010_amd import synth


def test_asmd_caps_hand_example(orc):
    # near range 2 m: 10 points in voxel (0,0,0) and 2 in voxel (1,0,0) ->
    # mean 12 / 2 = 6; far points at ranges 5 and 9.5 (r_max 10, k 3, nmax 20)
    near = [(0.1 * i, 0.05, 0.05) for i in range(10)] + [(1.2, 0.1, 0.1), (1.5, 0.1, 0.1)]
    far = [(5.0, 0.0, 0.0), (0.0, 9.5, 0.0)]
    s = np.array(near + far, np.float32).T.copy()
    caps, mean = orc.asmd_caps(s, s, 1.0, 3, 20, r_near=2.0, r_max=10.0)
    assert mean == 6.0
    r = np.sqrt((s.astype(np.float64) ** 2).sum(0))
    want = [max(3, min(20, math.floor(6.0 * (1 - ri / 10.0) + 0.5))) for ri in r]
    assert caps.tolist() == want
    assert caps[12] == 3 and caps[13] == 3          # 6 * 0.5 = 3; 6 * 0.05 -> floor k
    assert caps[0] == 6                              # range 0.07 m: round(5.96)


def test_asmd_caps_bounds_and_no_near_points(orc):
    g = np.random.default_rng(2)
    s = g.uniform(-60, 60, (3, 5000)).astype(np.float32)
    caps, mean = orc.asmd_caps(s, s, 1.0, 5, 20, r_near=20.0, r_max=120.0)
    assert np.all((caps >= 5) & (caps <= 20))
    r = np.sqrt((s.astype(np.float64) ** 2).sum(0))
    order = np.argsort(r)
    assert np.all(np.diff(caps[order]) <= 0)        # never grows with range
    far = s[:, r > 30]
    caps2, mean2 = orc.asmd_caps(far, far, 1.0, 5, 20, r_near=20.0, r_max=120.0)
    assert mean2 == 20.0                             # no near points: N_max


def test_asmd_insert_respects_caps(orc):
    c = synth.make_tiny(1)
    src = c.map_batches[0]
    caps, _ = orc.asmd_caps(src, src, 1.0, 3, 20, r_near=10.0, r_max=30.0)
    m = orc.Map(1.0, 20, 0.0, 3)
    m.insert(src, caps)
    x, _, _ = m.export()
    keys = np.floor(x.astype(np.float64).T).astype(np.int64)
    _, inv, cnt = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    # a voxel never holds more points than the largest cap among its candidates
    skeys = np.floor(src.astype(np.float64).T).astype(np.int64)
    for k_, n_ in zip(map(tuple, np.unique(keys, axis=0)), cnt):
        sel = np.all(skeys == np.array(k_), axis=1)
        assert n_ <= caps[sel].max()


def filtered_export(x, c, v, val, center, radius):
    keys = np.floor(x.astype(np.float64) / v)
    ctr = (keys + 0.5) * v
    d = ctr - np.asarray(center, np.float64)[:, None]
    keep = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2] <= radius * radius
    return x[:, keep], c[:, keep], val[keep], keep


def test_evict_is_the_filtered_map(orc):
    c = synth.make_tiny(1)
    m = orc.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.k)
    for b in c.map_batches:
        m.insert(b)
    x, cv, val = m.export()
    center, radius = (3.0, -4.0, 1.0), 12.5
    fx, fc, fv, keep = filtered_export(x, cv, 1.0, val, center, radius)
    assert 0 < keep.sum() < keep.size
    removed = m.evict(center, radius)
    assert removed == keep.size - keep.sum()
    ex, ec, ev = m.export()
    np.testing.assert_array_equal(ex, fx)
    np.testing.assert_array_equal(ec, fc)
    np.testing.assert_array_equal(ev, fv)
    # the rebuilt map answers neighbour queries like a brute force over the survivors
    q = synth.random_cloud(5, 2000, extent=20.0)
    idx, d2, cnt = m.knn(q, 3, 1.0)
    P, Q = fx.astype(np.float64), q.astype(np.float64)
    for j in range(0, q.shape[1], 97):
        d = (P[0] - Q[0, j]) ** 2 + (P[1] - Q[1, j]) ** 2 + (P[2] - Q[2, j]) ** 2
        cand = np.nonzero(d <= 1.0)[0]
        cand = cand[np.lexsort((cand, d[cand]))][:3]
        np.testing.assert_array_equal(idx[j, :len(cand)], cand)


def test_evict_extremes(orc):
    c = synth.make_tiny(1)
    m = orc.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.k)
    m.insert(c.map_batches[0])
    x0, c0, v0 = m.export()
    assert m.evict((0.0, 0.0, 0.0), 1e9) == 0
    x1, c1, v1 = m.export()
    np.testing.assert_array_equal(x0, x1)
    assert m.evict((0.0, 0.0, 0.0), 0.0) == x0.shape[1]   # no voxel centre at the origin
    assert m.size == 0 and m.n_voxels == 0


def test_odometry_with_asmd_and_eviction(orc):
    n = 30
    c = synth.make_sequence(2, n_scans=n, lidar=synth.Lidar(beams=32, azimuths=512))
    v1 = np.linalg.inv(c.poses[0]) @ c.poses[1]
    out, m = orc.odometry(c.scans, c.poses[0], v1, c.voxel_size, c.max_pts_per_voxel,
                          c.min_spacing, c.k, c.map_capacity, c.downsample, c.sigma0, c.r_max,
                          asmd=True, evict_radius=60.0)
    assert [r["status"] for r in out] == [0] * n
    assert sum(r["evicted"] for r in out) > 0
    x, _, _ = m.export()
    d = np.linalg.norm(np.floor(x.astype(np.float64)) + 0.5 - out[-1]["T"][:3, 3:4], axis=0)
    assert d.max() <= 60.0
    for r, T in zip(out, c.poses):
        assert np.linalg.norm(r["T"][:3, 3] - T[:3, 3]) < 1.0
