"""Motion undistortion (Sec. III-A.1) on the GPU against the oracle: every
output coordinate within one float32 ulp of the oracle's (both evaluate the
motion in FP64 and round once; the summation orders of the fit differ), the
reference time exact, points with non-finite times copied bit for bit; the
edge cases (empty scan, no usable samples, one sample, equal sample times,
non-finite samples, in place); the batched entry point identical to the
single-scan one; and a 64-scan batch of full racing scans."""
import math

import numpy as np
import pytest
import torch

from paper_2606_26010_amd import synth

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)


def assert_parity(g, o, what):
    """Within one float32 ulp per coordinate, and mostly bit-exact."""
    g, o = np.asarray(g), np.asarray(o)
    assert g.shape == o.shape
    same = (g == o) | (np.isnan(g) & np.isnan(o))
    fin = np.isfinite(o)
    assert np.array_equal(np.isfinite(g), fin), what
    d = np.abs(g[fin].astype(np.float64) - o[fin])
    assert np.all(d <= np.spacing(np.abs(o[fin]))), (what, float(d.max()))
    frac = same.mean() if same.size else 1.0
    say(f"{what}: {o.shape[-1]} points, bit-exact fraction {frac:.6f}")
    assert frac >= 0.99, what


def scatter(seed, n, r=100.0):
    g = np.random.default_rng(seed)
    d = g.normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0)
    return (d * g.uniform(1.0, r, n)).astype(np.float32), g.uniform(0, 0.1, n).astype(np.float32)


def cases():
    c = synth.make_deskew(6, n_scans=2)
    xs, ts = scatter(3, 9000)
    g = np.random.default_rng(4)
    vt = np.linspace(-0.01, 0.1, 23)
    big = np.array([5.0, -40.0, 3.0, 2.5, 1.0, -3.0]) + np.outer(vt, [20, 4, -3, 6, -2, 8])
    xn, tn = scatter(5, 4097)
    tn[[0, 17, 4096]] = [np.nan, np.inf, -np.inf]
    vn = big.copy()
    vn[3, 2] = np.nan
    vtn = vt.copy()
    vtn[7] = np.inf
    return {
        "racing_scan": (c.scans[1], c.times[1], c.vel_t[1], c.vel[1]),
        "large_motion": (xs, ts, vt, big),
        "nonfinite_times_and_samples": (xn, tn, vtn, vn),
        "no_samples": (xs[:, :1000], ts[:1000], np.zeros(0), np.zeros((0, 6))),
        "one_sample": (xs[:, :3000], ts[:3000], vt[:1], big[:1]),
        "equal_sample_times": (xs[:, :3000], ts[:3000], np.full(5, 0.05), big[:5]),
        "tiny_rotation": (xs[:, :2000], ts[:2000], vt, np.tile([30, 0, 0, 1e-7, 0, 2e-7], (23, 1))),
        "one_point": (xs[:, :1], ts[:1], vt, big),
        "ragged_257": (xs[:, :257], ts[:257], vt, big),
        "many_samples": (xs[:, :3000], ts[:3000], np.linspace(-0.01, 0.1, 300),
                         np.array([5.0, -40.0, 3.0, 2.5, 1.0, -3.0])
                         + np.outer(np.linspace(-0.01, 0.1, 300), [20, 4, -3, 6, -2, 8])
                         + g.normal(size=(300, 6))),
    }


@pytest.mark.parametrize("name", list(cases()))
def test_undistort_matches_oracle(orc, name):
    from paper_2606_26010_amd import far
    xyz, t, vt, v = cases()[name]
    say(f"undistort case {name}: n={xyz.shape[1]} m={vt.size}")
    o, otr = orc.undistort(xyz, t, vt, v)
    g, gtr = far.far_undistort(dev(xyz), dev(t), dev(vt.astype(np.float64)),
                               dev(v.astype(np.float64).reshape(-1, 6)))
    g = host(g)
    gtr = float(host(gtr)[0])
    assert (gtr == otr) or (math.isnan(gtr) and math.isnan(otr))
    assert_parity(g, o, name)
    bad = ~np.isfinite(t)
    np.testing.assert_array_equal(g[:, bad], xyz[:, bad])


def test_undistort_empty_in_place_and_all_nonfinite(orc):
    from paper_2606_26010_amd import far
    vt, v = dev(np.linspace(0, 0.1, 5)), dev(np.tile([10.0, 0, 0, 0, 0, 1.0], (5, 1)))
    e, tr = far.far_undistort(torch.zeros((3, 0), dtype=torch.float32).cuda(),
                              torch.zeros(0, dtype=torch.float32).cuda(), vt, v)
    assert e.shape == (3, 0) and math.isnan(float(host(tr)[0]))
    xyz, t = scatter(8, 5000)
    o, _ = orc.undistort(xyz, t, host(vt), host(v))
    x = dev(xyz)
    g, _ = far.far_undistort(x, dev(t), vt, v, out=x)        # in place
    assert g.data_ptr() == x.data_ptr()
    assert_parity(host(x), o, "in_place")
    tn = np.full(300, np.nan, np.float32)
    g, tr = far.far_undistort(dev(xyz[:, :300]), dev(tn), vt, v)
    assert math.isnan(float(host(tr)[0]))
    np.testing.assert_array_equal(host(g), xyz[:, :300])


def batch_of(scans, times, vts, vels):
    offs = np.concatenate([[0], np.cumsum([s.shape[1] for s in scans])]).astype(np.int64)
    voffs = np.concatenate([[0], np.cumsum([x.size for x in vts])]).astype(np.int64)
    xyz = np.concatenate(scans, 1) if offs[-1] else np.zeros((3, 0), np.float32)
    t = np.concatenate(times).astype(np.float32)
    vt = np.concatenate(vts).astype(np.float64) if voffs[-1] else np.zeros(1)
    v = np.concatenate([x.reshape(-1, 6) for x in vels]) if voffs[-1] else np.zeros((1, 6))
    return xyz, t, offs, vt, v, voffs


def test_undistort_batch_equals_single_and_oracle(orc):
    from paper_2606_26010_amd import far
    cs = cases()
    names = ["racing_scan", "no_samples", "large_motion", "one_point",
             "nonfinite_times_and_samples", "ragged_257", "equal_sample_times"]
    parts = [cs[n] for n in names]
    empty = (np.zeros((3, 0), np.float32), np.zeros(0, np.float32), np.linspace(0, 0.1, 3),
             np.ones((3, 6)))
    parts.insert(2, empty)                                     # an empty scan inside the batch
    xyz, t, offs, vt, v, voffs = batch_of(*zip(*parts))
    g, gtr = far.far_undistort_batch(dev(xyz), dev(t), dev(offs), dev(vt), dev(v), dev(voffs))
    g, gtr = host(g), host(gtr)
    for s, (px, pt, pvt, pv) in enumerate(parts):
        a, b = offs[s], offs[s + 1]
        o, otr = orc.undistort(px, pt, pvt, pv)
        assert (gtr[s] == otr) or (math.isnan(gtr[s]) and math.isnan(otr)), s
        single, _ = far.far_undistort(dev(px), dev(pt), dev(np.asarray(pvt, np.float64)),
                                      dev(np.asarray(pv, np.float64).reshape(-1, 6)))
        np.testing.assert_array_equal(g[:, a:b], host(single))
        if b > a:
            assert_parity(g[:, a:b], o, f"batch scan {s}")


def test_undistort_batch_many_tiny_scans(orc):
    """300 scans of 0..40 points: point chunks of the time reduction span
    dozens of scans (the per-lane fallback) and the apply blocks several."""
    from paper_2606_26010_amd import far
    g = np.random.default_rng(12)
    scans, times, vts, vels = [], [], [], []
    for s in range(300):
        n = int(g.integers(0, 41))
        x, t = scatter(1000 + s, n)
        t = (t - 0.05 * (s % 7)).astype(np.float32)      # negative times too
        m = int(g.integers(0, 4))
        vt = np.sort(g.uniform(-0.4, 0.1, m))
        scans.append(x)
        times.append(t)
        vts.append(vt)
        vels.append(g.normal(size=(m, 6)) * [10, 1, 1, 0.5, 0.5, 2])
    xyz, t, offs, vt, v, voffs = batch_of(scans, times, vts, vels)
    say(f"tiny scans: {xyz.shape[1]} points in 300 scans")
    g_, gtr = far.far_undistort_batch(dev(xyz), dev(t), dev(offs), dev(vt), dev(v), dev(voffs))
    g_, gtr = host(g_), host(gtr)
    o = np.empty_like(xyz)
    for s in range(300):
        a, b = offs[s], offs[s + 1]
        o[:, a:b], otr = orc.undistort(scans[s], times[s], vts[s], vels[s])
        assert (gtr[s] == otr) or (math.isnan(gtr[s]) and math.isnan(otr)), s
    assert_parity(g_, o, "tiny scans")


@pytest.mark.timeout(600)
def test_undistort_full_racing_batch(orc):
    """64 racing scans (8 distinct scans of about 80,000 points, each used
    eight times with its own time offset) in one launch sequence."""
    from paper_2606_26010_amd import far
    c = synth.make_deskew(6, n_scans=8)
    scans, times, vts, vels = [], [], [], []
    for r in range(8):
        for s in range(8):
            scans.append(c.scans[s])
            times.append(c.times[s] + np.float32(0.125 * r))
            vts.append(c.vel_t[s] + 0.125 * r)
            vels.append(c.vel[s])
    xyz, t, offs, vt, v, voffs = batch_of(scans, times, vts, vels)
    say(f"full racing batch: {xyz.shape[1]} points")
    g, gtr = far.far_undistort_batch(dev(xyz), dev(t), dev(offs), dev(vt), dev(v), dev(voffs))
    g, gtr = host(g), host(gtr)
    o = np.empty_like(xyz)
    for s in range(64):
        a, b = offs[s], offs[s + 1]
        o[:, a:b], otr = orc.undistort(scans[s], times[s], vts[s], vels[s])
        assert gtr[s] == otr, s
    assert_parity(g, o, "full racing batch")


def angle_deg(A, B):
    E = A[:3, :3] @ B[:3, :3].T
    s = np.array([E[2, 1] - E[1, 2], E[0, 2] - E[2, 0], E[1, 0] - E[0, 1]])
    return math.degrees(math.atan2(0.5 * np.linalg.norm(s), 0.5 * (np.trace(E) - 1)))


@pytest.mark.timeout(900)
def test_odometry_with_undistortion_matches_oracle(orc):
    """30 scans of the racing line through the odometry, each undistorted on
    the GPU first (far_odometry_step_timed): poses within the sequence bar
    of the oracle's, reference times exact; and the motion-undistortion
    ablation on the GPU (the same scans without it drift several times
    farther from the trajectory)."""
    from paper_2606_26010_amd import far
    n = 30
    c = synth.make_deskew(6, n_scans=n)
    v1 = np.linalg.inv(c.poses[0]) @ c.poses[1]
    kw = dict(max_iters=10, eps=0.0)
    ref, _ = orc.odometry(c.scans, c.poses[0], v1, c.voxel_size, c.max_pts_per_voxel,
                          c.min_spacing, c.k, c.map_capacity, c.downsample, c.sigma0, c.r_max,
                          times=c.times, vel_t=c.vel_t, vel=c.vel, **kw)
    drift = {}
    for deskew in (True, False):
        gm = far.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.map_capacity,
                     c.map_capacity, c.k)
        od = far.Odometry(gm, c.poses[0], v1, downsample=c.downsample, sigma0=c.sigma0,
                          r_max=c.r_max, **kw)
        worst = (0.0, 0.0)
        err = 0.0
        for s in range(n):
            if deskew:
                T, st = od.step(dev(c.scans[s]), times=dev(c.times[s]), vel_t=dev(c.vel_t[s]),
                                vel=dev(c.vel[s]))
                r = ref[s]
                assert st["t_ref"] == r["t_ref"], s
                assert st["n_down"] == r["n"] and st["status"] == r["status"], s
                dt = float(np.linalg.norm(T[:3, 3] - r["T"][:3, 3]))
                da = angle_deg(T, r["T"])
                worst = (max(worst[0], dt), max(worst[1], da))
                assert dt <= 1e-3 and da <= 1e-2, (s, dt, da)
            else:
                T, st = od.step(dev(c.scans[s]))
                assert math.isnan(st["t_ref"])
            err = max(err, float(np.linalg.norm(T[:3, 3] - c.poses[s][:3, 3])))
        drift[deskew] = err
        if deskew:
            say(f"odometry with undistortion vs oracle: worst {worst[0]:.2e} m, {worst[1]:.2e} deg")
        od.close()
        gm.close()
    say(f"drift from the trajectory: undistorted {drift[True]:.3f} m, raw {drift[False]:.3f} m")
    assert drift[True] <= 0.2 and drift[True] <= 0.25 * drift[False]
