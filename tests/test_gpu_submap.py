"""Submap update (Sec. III-A.3) on the GPU against the oracle: adaptive
submap density caps bit-exact, eviction of distant voxels (the rebuilt map
identical to the oracle's, then searched and extended), and the sequence
odometry with both."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from paper_2606_26010_amd import synth

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)


def angle_deg(A, B):
    E = A[:3, :3] @ B[:3, :3].T
    s = np.array([E[2, 1] - E[1, 2], E[0, 2] - E[2, 0], E[1, 0] - E[0, 1]])
    return math.degrees(math.atan2(0.5 * np.linalg.norm(s), 0.5 * (np.trace(E) - 1)))


def asmd_cases():
    T = synth.trajectory_pose(1.3)
    lid = synth.scan(synth.Corridor(), synth.Lidar(), T, synth.rng(8))
    g = np.random.default_rng(9)
    rnd = g.uniform(-40, 40, (3, 20001)).astype(np.float32)
    rnd[1, 7] = np.nan
    far = (g.uniform(30, 60, (3, 500)) * np.sign(g.uniform(-1, 1, (3, 500)))).astype(np.float32)
    return {"lidar_scan": (lid, T), "random_nonfinite": (rnd, np.eye(4)),
            "no_near_points": (far, np.eye(4)), "one_point": (np.zeros((3, 1), np.float32), T)}


@pytest.mark.parametrize("name", list(asmd_cases()))
def test_asmd_caps_bit_exact(orc, name):
    from paper_2606_26010_amd import far
    xs, T = asmd_cases()[name]
    xm = orc.transform(xs, T)
    oc, om = orc.asmd_caps(xs, xm, 1.0, 5, 20, 20.0, 120.0)
    gc, gm = far.far_asmd_caps(dev(xs), dev(xm), 1.0, 5, 20, 20.0, 120.0)
    say(f"asmd {name}: mean {om}, caps {np.bincount(oc).nonzero()[0].tolist()}")
    assert gm == om
    np.testing.assert_array_equal(host(gc), oc)


def test_evict_insert_sequence_matches_oracle(orc):
    from paper_2606_26010_amd import far
    c = synth.make_tiny(1)
    gm = far.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, 1 << 16, 0, c.k)
    om = orc.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.k,
                 point_capacity=1 << 16, voxel_capacity=1 << 16)
    steps = [("insert", 0), ("insert", 1), ("evict", ((3.0, -4.0, 1.0), 12.5)),
             ("insert", 2), ("insert", 3), ("evict", ((-10.0, 5.0, 0.0), 18.0)),
             ("insert", 4), ("evict", ((0.0, 0.0, 0.0), 1e6)), ("evict", ((50.0, 50.0, 0.0), 1.0)),
             ("insert", 5), ("insert", 6)]
    for what, arg in steps:
        if what == "insert":
            b = c.map_batches[arg]
            gs, ga = gm.insert(dev(b))
            orc_rc, oa, _ = om.insert(b, check=False)
            assert (gs, ga) == (orc_rc, oa), arg
        else:
            ctr, rad = arg
            assert gm.evict(ctr, rad) == om.evict(ctr, rad), arg
        gx, gc, gv = gm.export()
        ox, oc, ov = om.export()
        np.testing.assert_array_equal(host(gx), ox)
        np.testing.assert_array_equal(host(gv), ov)
        np.testing.assert_array_equal(host(gc), oc)   # carried over, never recomputed
        say(f"{what} {arg}: {om.size} points")
    # the rebuilt map: neighbour queries and a linearisation still match
    q = synth.random_cloud(6, 5000, extent=20.0)
    gi, gd, gn = gm.knn(dev(q), 5, 1.0)
    oi, od, on = om.knn(q, 5, 1.0)
    np.testing.assert_array_equal(host(gn), on)
    np.testing.assert_array_equal(host(gi), oi)
    cov, val = orc.scan_covariances(c.source, c.voxel_size, c.k)
    cov = cov.astype(np.float32)
    T = c.T_gt @ synth.random_offset(synth.rng(12), 0.1, 1.0)
    o = om.linearize(c.source, cov, val, T, c.tau, c.kappa, c=T[:3, 3], want_corr=True)
    g = gm.linearize(dev(c.source), dev(cov), dev(val), T, c.tau, c.kappa, c=T[:3, 3],
                     want_corr=True)
    np.testing.assert_array_equal(host(g["corr"]), o["corr"])
    assert np.linalg.norm(g["H"] - o["H"]) <= 1e-4 * np.linalg.norm(o["H"])


def test_evict_empty_and_all(orc):
    from paper_2606_26010_amd import far
    gm = far.Map(1.0, 20, -1.0, 1 << 12, 0, 5)
    assert gm.evict((0.0, 0.0, 0.0), 10.0) == 0
    b = synth.random_cloud(7, 3000, extent=10.0)
    gm.insert(dev(b))
    n = gm.stats()["n_points"]
    assert gm.evict((0.0, 0.0, 0.0), 0.0) == n
    s = gm.stats()
    assert s["n_points"] == 0 and s["n_voxels"] == 0
    gs, ga = gm.insert(dev(b))
    om = orc.Map(1.0, 20, 1.0 / math.sqrt(20.0), 5, point_capacity=1 << 12, voxel_capacity=1 << 12)
    assert (gs, ga) == om.insert(b, check=False)[:2]


@pytest.mark.timeout(900)
def test_sequence_with_asmd_and_eviction(orc):
    from paper_2606_26010_amd import far
    n = 60
    c = synth.make_sequence(2, n_scans=n)
    v1 = np.linalg.inv(c.poses[0]) @ c.poses[1]
    kw = dict(max_iters=10, eps=0.0)
    ref, om = orc.odometry(c.scans, c.poses[0], v1, c.voxel_size, c.max_pts_per_voxel,
                           c.min_spacing, c.k, c.map_capacity, c.downsample, c.sigma0, c.r_max,
                           asmd=True, r_near=20.0, evict_radius=150.0, **kw)
    gm = far.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.map_capacity,
                 c.map_capacity, c.k)
    od = far.Odometry(gm, c.poses[0], v1, downsample=c.downsample, sigma0=c.sigma0,
                      r_max=c.r_max, asmd=True, r_near=20.0, evict_radius=150.0, **kw)
    worst = (0.0, 0.0)
    evicted = 0
    for s, raw in enumerate(c.scans):
        T, st = od.step(dev(raw))
        r = ref[s]
        assert st["n_down"] == r["n"] and st["status"] == r["status"], s
        assert st["asmd_mean"] == pytest.approx(r["asmd_mean"], rel=1e-3), s
        dt = float(np.linalg.norm(T[:3, 3] - r["T"][:3, 3]))
        da = angle_deg(T, r["T"])
        worst = (max(worst[0], dt), max(worst[1], da))
        assert dt <= 1e-3 and da <= 1e-2, (s, dt, da)
        size = gm.stats()["n_points"]
        assert abs(size - r["map_points"]) <= 1e-3 * max(r["map_points"], 1), (s, size)
        evicted += st["n_evicted"]
    say(f"sequence asmd+evict: worst {worst[0]:.2e} m, {worst[1]:.2e} deg; evicted {evicted} "
        f"points; final map {gm.stats()['n_points']} (oracle {ref[-1]['map_points']})")
    assert evicted > 0
    od.close()
    gm.close()
