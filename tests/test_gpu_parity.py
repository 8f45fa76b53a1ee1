"""GPU parity: the HIP library through its C ABI against the FP64 CPU oracle.

Bars: neighbour ids, map ids/coordinates, validity flags and correspondences
bit-exact; covariances to FP32 rounding (rtol 2e-6); H, b, cost to a relative
norm of 1e-4 (FP32 bulk) or 1e-9 (FP64 path); pose within 1e-3 m and 0.01 deg.
Sizes span several 256-point tiles with ragged tails; seeds are fixed.
"""
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


@pytest.fixture(scope="module")
def far():
    from paper_2606_26010_amd import far as F
    F.lib()
    assert torch.cuda.is_available()
    return F


def say(*a):
    print(*a, flush=True)


def build_pair(far, orc, batches, v, nmax, dmin, k, caps=None, point_cap=1 << 20,
               voxel_cap=0):
    gm = far.Map(v, nmax, dmin, point_cap, voxel_cap, k)
    om = orc.Map(v, nmax, dmin, k, point_capacity=point_cap,
                 voxel_capacity=voxel_cap if voxel_cap > 0 else point_cap)
    res = []
    for bi, b in enumerate(batches):
        c = None if caps is None else caps[bi]
        gs, ga = gm.insert(dev(b), None if c is None else dev(c))
        orc_rc, oa, _ = om.insert(b, c, check=False)
        res.append((gs, ga, orc_rc, oa))
    return gm, om, res


def assert_same_map(gm, om):
    gx, gc, gv = gm.export()
    ox, oc, ov = om.export()
    assert gx.shape == ox.shape, (gx.shape, ox.shape)
    np.testing.assert_array_equal(host(gx), ox)
    np.testing.assert_array_equal(host(gv), ov)
    np.testing.assert_allclose(host(gc), oc, rtol=2e-6, atol=1e-6)
    assert gm.stats()["n_voxels"] == om.n_voxels


# ---------------------------------------------------------------- insert
INSERT_CASES = {
    "tiny_scene": lambda: (synth.make_tiny(1).map_batches, 1.0, 20, 1 / math.sqrt(20), 5, None),
    "spacing_cap20": lambda: ([synth.random_cloud(s, 6000, extent=4.0) for s in (1, 2)],
                              1.0, 20, 0.3, 5, None),
    "cap3_nospacing_dups": lambda: ([synth.random_cloud(3, 9000, extent=2.0, dup_frac=0.2,
                                                        on_faces=0.3)], 0.5, 3, 0.0, 5, None),
    "cap1_downsample": lambda: ([synth.random_cloud(4, 20000, extent=6.0)], 0.5, 1, 0.0, 1, None),
    "non_pow2_voxel": lambda: ([synth.random_cloud(5, 7000, extent=3.0, on_faces=0.3, v=0.3)],
                               0.3, 10, 0.05, 8, None),
    "per_point_caps": lambda: ([synth.random_cloud(6, 5000, extent=2.0)], 1.0, 8, 0.1, 5,
                               [synth.rng(7).integers(-1, 10, 5000).astype(np.int32)]),
}


@pytest.mark.parametrize("case", sorted(INSERT_CASES))
def test_insert_parity(far, orc, case):
    batches, v, nmax, dmin, k, caps = INSERT_CASES[case]()
    say(f"insert case {case}: {sum(b.shape[1] for b in batches)} points")
    gm, om, res = build_pair(far, orc, batches, v, nmax, dmin, k, caps)
    for gs, ga, orc_rc, oa in res:
        assert gs == orc_rc and ga == oa
    assert_same_map(gm, om)
    gm.close()


def test_insert_nonfinite_and_duplicates_stress(far, orc):
    g = synth.rng(8)
    pts = np.repeat(np.array([[1.25], [-0.5], [3.75]], np.float32), 200_000, axis=1)
    pts = np.concatenate([pts, synth.random_cloud(9, 50_000, extent=3.0)], 1)
    pts = np.ascontiguousarray(pts[:, g.permutation(pts.shape[1])])
    pts[0, 17] = np.nan
    pts[2, 99] = np.inf
    gm, om, res = build_pair(far, orc, [pts], 1.0, 20, 0.0, 5)
    (gs, ga, orc_rc, oa), = res
    assert gs == orc_rc == 0 and ga == oa
    assert_same_map(gm, om)


def test_insert_capacity_parity(far, orc):
    pts = synth.random_cloud(10, 4000, extent=3.0)
    gm, om, res = build_pair(far, orc, [pts[:, :2000], pts[:, 2000:]], 1.0, 50, 0.0, 5,
                             point_cap=2500)
    assert res[0][0] == 0 and res[1][0] == 2 and res[1][2] == 2
    assert res[1][1] == res[1][3] == 500
    assert_same_map(gm, om)
    gm2, om2, res2 = build_pair(far, orc, [pts], 1.0, 50, 0.0, 5, voxel_cap=20)
    assert res2[0][0] == res2[0][2] == 2 and res2[0][1] == res2[0][3] == 0
    assert gm2.stats()["n_points"] == 0
    far_pt = np.array([[4.0e6], [0.0], [0.0]], np.float32)
    st, _ = far.far_map_insert(gm.h, dev(far_pt), raise_on=False)
    assert st == far.FAR_E_INVALID


# ---------------------------------------------------------------- knn
@pytest.mark.parametrize("k,r", [(1, 1.0), (5, 1.0), (8, 0.6), (17, 1.0), (32, 0.9)])
def test_knn_parity(far, orc, k, r):
    c = synth.make_tiny(2)
    gm, om, _ = build_pair(far, orc, c.map_batches, c.voxel_size, c.max_pts_per_voxel,
                           c.min_spacing, c.k)
    q = np.concatenate([synth.tiny_scene_samples(synth.rng(11), 3000),
                        synth.random_cloud(12, 1000, extent=20.0, on_faces=0.3)], 1)
    q[1, 5] = np.nan
    say(f"knn k={k} r={r}: {q.shape[1]} queries on {om.size} points")
    gi, gd, gc = gm.knn(dev(q), k, r)
    oi, od, oc = om.knn(q, k, r)
    np.testing.assert_array_equal(host(gc), oc)
    np.testing.assert_array_equal(host(gi), oi)
    np.testing.assert_array_equal(host(gd), np.where(oi >= 0, od, -1.0).astype(np.float32))
    gm.close()


# ---------------------------------------------------------------- scan covariances
@pytest.mark.parametrize("k,v", [(5, 1.0), (10, 1.0), (5, 0.5), (32, 2.0)])
def test_scan_covariances_parity(far, orc, k, v):
    c = synth.make_tiny(3)
    pts = np.concatenate([c.source, synth.random_cloud(13, 3001, extent=3.0, dup_frac=0.1,
                                                       on_faces=0.2, v=v)], 1)
    pts[0, 3] = np.inf
    pts = np.ascontiguousarray(pts)
    gcov, gval = far.far_scan_covariances(dev(pts), v, k)
    ocov, oval = orc.scan_covariances(pts, v, k)
    np.testing.assert_array_equal(host(gval), oval)
    np.testing.assert_allclose(host(gcov), ocov, rtol=2e-6, atol=1e-6)


# ---------------------------------------------------------------- linearize
def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def tiny_pair(far, orc):
    c = synth.make_tiny(4)
    gm, om, _ = build_pair(far, orc, c.map_batches, c.voxel_size, c.max_pts_per_voxel,
                           c.min_spacing, c.k)
    assert_same_map(gm, om)
    ocov, oval = orc.scan_covariances(c.source, c.voxel_size, c.k)
    yield c, gm, om, ocov.astype(np.float32), oval
    gm.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 1e-9)])
@pytest.mark.parametrize("pose", ["gt", "offset", "identity"])
def test_linearize_parity(far, orc, tiny_pair, prec, tol, pose):
    c, gm, om, ocov, oval = tiny_pair
    T = {"gt": c.T_gt, "identity": np.eye(4),
         "offset": c.T_gt @ synth.random_offset(synth.rng(14), 0.2, 1.5)}[pose]
    cen = T[:3, 3] + np.array([0.3, -0.2, 0.1])
    for tau in (c.tau, 0.4):
        g = gm.linearize(dev(c.source), dev(ocov), dev(oval), T, tau, c.kappa, c=cen,
                         precision=prec, want_corr=True)
        o = om.linearize(c.source, ocov, oval, T, tau, c.kappa, c=cen, want_corr=True)
        np.testing.assert_array_equal(host(g["corr"]), o["corr"])
        assert g["n_inliers"] == o["n_inliers"]
        eH, eb, ec = rel(g["H"], o["H"]), rel(g["b"], o["b"]), rel(g["cost"], o["cost"])
        say(f"linearize prec={prec} pose={pose} tau={tau}: relH {eH:.2e} relb {eb:.2e} "
            f"relcost {ec:.2e}")
        assert eH <= tol and eb <= tol and ec <= tol
        np.testing.assert_array_equal(g["H"], g["H"].T)


def test_linearize_ragged_sizes_and_sa(far, orc, tiny_pair):
    c, gm, om, ocov, oval = tiny_pair
    for n in (1, 255, 256, 257, 1023, 4999):
        src = np.ascontiguousarray(c.source[:, :n])
        cov = np.ascontiguousarray(ocov[:, :n])
        val = np.ascontiguousarray(oval[:n]).copy()
        val[::3] = 0                          # sparsity-aware (M = I) points
        g = gm.linearize(dev(src), dev(cov), dev(val), c.T_gt, c.tau, c.kappa,
                         want_corr=True)
        o = om.linearize(src, cov, val, c.T_gt, c.tau, c.kappa, want_corr=True)
        np.testing.assert_array_equal(host(g["corr"]), o["corr"])
        assert rel(g["H"], o["H"]) <= 1e-4 and rel(g["b"], o["b"]) <= 1e-4, n


# ---------------------------------------------------------------- align
def pose_err(A, B):
    E = A[:3, :3] @ B[:3, :3].T
    return (float(np.linalg.norm(A[:3, 3] - B[:3, 3])),
            math.degrees(math.acos(max(-1.0, min(1.0, (np.trace(E) - 1) / 2)))))


@pytest.mark.parametrize("prec", [0, 1])
def test_align_parity_full_pipeline(far, orc, prec):
    c = synth.make_tiny(5)
    gm, om, _ = build_pair(far, orc, c.map_batches, c.voxel_size, c.max_pts_per_voxel,
                           c.min_spacing, c.k)
    src = dev(c.source)
    gcov, gval = far.far_scan_covariances(src, c.voxel_size, c.k)
    ocov, oval = orc.scan_covariances(c.source, c.voxel_size, c.k)
    np.testing.assert_array_equal(host(gval), oval)
    for iters, eps in ((10, 0.0), (40, 1e-6)):
        prm = far.align_params(c.tau, c.kappa, max_iters=iters, eps=eps, precision=prec)
        st, T, stats = gm.align(src, gcov, gval, np.eye(4), prm)
        ref = om.align(c.source, ocov.astype(np.float32), oval, np.eye(4), c.tau, c.kappa,
                       max_iters=iters, eps=eps)
        dt, da = pose_err(T, ref["T"])
        say(f"align prec={prec} iters={iters} eps={eps}: gpu iters {stats['iters']} "
            f"oracle iters {ref['iters']} |dt| {dt:.2e} m angle {da:.2e} deg; "
            f"vs gt {pose_err(T, c.T_gt)}")
        assert st == ref["status"] == 0
        assert dt <= 1e-3 and da <= 1e-2
        if eps == 0.0:
            assert stats["iters"] == ref["iters"] == iters
    gm.close()


def test_align_batch_equals_single_and_oracle(far, orc, tiny_pair):
    c, gm, om, ocov, oval = tiny_pair
    g = synth.rng(15)
    sizes = [1, 300, 2500, 4999, 700, 5000]
    scans, covs, vals, T0s = [], [], [], []
    for s, n in enumerate(sizes):
        sel = np.sort(g.choice(c.source.shape[1], size=n, replace=False))
        scans.append(np.ascontiguousarray(c.source[:, sel]))
        covs.append(np.ascontiguousarray(ocov[:, sel]))
        vals.append(np.ascontiguousarray(oval[sel]))
        T0s.append(c.T_gt @ synth.random_offset(g, 0.1, 1.0, exact=False))
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    prm = far.align_params(c.tau, c.kappa, max_iters=8, eps=1e-7)
    T = dev(np.stack([t.reshape(16) for t in T0s]))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for rep in range(3):            # graph replays must agree with each other
            T.copy_(dev(np.stack([t.reshape(16) for t in T0s])))
            stats = gm.align_batch(dev(np.concatenate(scans, 1)), dev(offs),
                                   dev(np.concatenate(covs, 1)), dev(np.concatenate(vals)),
                                   T, prm)
            stream.synchronize()
            Tb = host(T).reshape(-1, 4, 4)
            sb = far.decode_stats(stats)
            if rep == 0:
                first = (Tb.copy(), sb.copy())
            else:
                np.testing.assert_array_equal(Tb, first[0])
    for s in range(len(sizes)):
        st, Ts, ss = gm.align(dev(scans[s]), dev(covs[s]), dev(vals[s]), T0s[s], prm)
        assert st == sb[s]["status"]
        np.testing.assert_array_equal(Ts, Tb[s])        # same kernels, same tiles
        assert ss["iters"] == sb[s]["iters"]
        ref = om.align(scans[s], covs[s], vals[s], T0s[s], c.tau, c.kappa, max_iters=8,
                       eps=1e-7)
        assert ref["status"] == st
        if st == 0:
            dt, da = pose_err(Tb[s], ref["T"])
            say(f"batch scan {s} n={sizes[s]}: iters {sb[s]['iters']}/{ref['iters']} "
                f"|dt| {dt:.2e} angle {da:.2e}")
            assert dt <= 1e-3 and da <= 1e-2


# ---------------------------------------------------------------- edge cases
def test_edge_cases(far, orc, tiny_pair):
    c, gm, om, ocov, oval = tiny_pair
    e = torch.empty((3, 0), dtype=torch.float32, device="cuda")
    assert far.far_map_insert(gm.h, e)[1] == 0
    i, d, n = gm.knn(e, 5, 1.0)
    assert i.numel() == 0
    cov, val = far.far_scan_covariances(e, 1.0, 5)
    assert cov.shape == (6, 0)
    # no correspondences: far away pose
    Tfar = np.eye(4)
    Tfar[:3, 3] = [800.0, 0.0, 0.0]
    prm = far.align_params(c.tau, c.kappa)
    st, T, stats = gm.align(dev(c.source), dev(ocov), dev(oval), Tfar, prm)
    ref = om.align(c.source, ocov, oval, Tfar, c.tau, c.kappa)
    assert st == ref["status"] == far.FAR_E_FEW_CORR
    np.testing.assert_array_equal(T, Tfar)
    # points on the x axis, linearised about the origin: the rotation about
    # that axis has an exactly zero Jacobian column, so H is singular
    line = np.zeros((3, 3000), np.float32)
    line[0] = np.linspace(-3.0, 3.0, 3000, dtype=np.float32)
    pm, pom, _ = build_pair(far, orc, [line], 1.0, 64, 0.0, 5)
    src = np.ascontiguousarray(line[:, ::2])
    z = np.zeros((6, src.shape[1]), np.float32)
    v0 = np.zeros(src.shape[1], np.uint8)
    st, T, _ = pm.align(dev(src), dev(z), dev(v0), np.eye(4), far.align_params(0.5, 1.0))
    ref = pom.align(src, z, v0, np.eye(4), 0.5, 1.0)
    assert st == ref["status"] == far.FAR_E_NOT_PD
    np.testing.assert_array_equal(T, np.eye(4))
    pm.close()
    # invalid arguments
    with pytest.raises(far.FarError):
        gm.knn(dev(c.source), 33, 1.0)
    with pytest.raises(far.FarError):
        gm.knn(dev(c.source), 5, 1.5)


def test_map_stats_probe_lengths(far, tiny_pair):
    c, gm, om, _, _ = tiny_pair
    s = gm.stats()
    say("map stats", s)
    assert s["n_points"] == om.size and s["n_voxels"] == om.n_voxels
    assert s["load_factor"] <= 0.5 and 1.0 <= s["mean_probe"] < 4.0


def test_scan_covariances_batch_parity(far, orc):
    # overlapping scans of one scene: a batched call must keep them apart
    scans = [synth.make_tiny(s, n_batches=1, n_source=n).source
             for s, n in ((6, 1), (7, 3000), (8, 257), (9, 5000), (10, 1024))]
    scans.insert(2, np.zeros((3, 0), np.float32))
    bad = synth.random_cloud(11, 700, extent=2.0)
    bad[0, ::50] = np.nan
    scans.append(bad)
    sizes = [s.shape[1] for s in scans]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cov, val = far.far_scan_covariances_batch(dev(np.concatenate(scans, 1)), dev(offs), 1.0, 5)
    cov, val = host(cov), host(val)
    for s, sc in enumerate(scans):
        if sc.shape[1] == 0:
            continue
        oc, ov = orc.scan_covariances(np.ascontiguousarray(sc), 1.0, 5)
        np.testing.assert_array_equal(val[offs[s]:offs[s + 1]], ov)
        np.testing.assert_allclose(cov[:, offs[s]:offs[s + 1]], oc, rtol=2e-6, atol=1e-6)


@pytest.mark.parametrize("k", [1, 5])
def test_knn_parity_far_from_origin(far, orc, k):
    # FP32 spacing at 1.2e5 m is ~8 mm: candidate screening in FP32 must still
    # leave every exact FP64 decision (and tie) to the FP64 comparison
    shift = np.array([[123456.5], [-65432.25], [1000.0]], np.float32)
    cloud = (synth.random_cloud(31, 6000, extent=3.0, dup_frac=0.05) + shift).astype(np.float32)
    q = np.concatenate([cloud[:, :500],
                        (synth.random_cloud(32, 800, extent=3.5) + shift).astype(np.float32)], 1)
    gm, om, _ = build_pair(far, orc, [cloud], 1.0, 32, 0.0, 5)
    gi, gd, gn = gm.knn(dev(q), k, 1.0)
    oi, od, on = om.knn(q, k, 1.0)
    np.testing.assert_array_equal(host(gn), on)
    np.testing.assert_array_equal(host(gi), oi)
    np.testing.assert_array_equal(host(gd), np.where(oi >= 0, od, -1.0).astype(np.float32))
    gm.close()


def test_linearize_parity_far_from_origin(far, orc):
    c = synth.make_tiny(7, n_batches=4, n_source=3000)
    shift = np.array([[98765.25], [43210.5], [-250.0]], np.float32)
    batches = [(b + shift).astype(np.float32) for b in c.map_batches]
    gm, om, _ = build_pair(far, orc, batches, 1.0, 20, c.min_spacing, 5)
    src = c.source
    T = c.T_gt.copy()
    T[:3, 3] += shift[:, 0]
    ocov, oval = orc.scan_covariances(src, 1.0, 5)
    ocov = ocov.astype(np.float32)
    for prec in (0, 1):
        g = gm.linearize(dev(src), dev(ocov), dev(oval), T, 1.0, 1 / 9, c=T[:3, 3],
                         precision=prec, want_corr=True)
        o = om.linearize(src, ocov, oval, T, 1.0, 1 / 9, c=T[:3, 3], want_corr=True)
        np.testing.assert_array_equal(host(g["corr"]), o["corr"])
        assert rel(g["H"], o["H"]) <= (1e-4 if prec == 0 else 1e-9)
    gm.close()


def test_linearize_parity_non_pow2_voxel(far, orc):
    # v = 0.75 m is not a power of two: the search falls back to the voxels
    c = synth.make_tiny(8, n_batches=4, n_source=3000)
    gm, om, _ = build_pair(far, orc, c.map_batches, 0.75, 20, 0.2, 5)
    ocov, oval = orc.scan_covariances(c.source, 0.75, 5)
    ocov = ocov.astype(np.float32)
    for tau in (0.75, 0.5):
        g = gm.linearize(dev(c.source), dev(ocov), dev(oval), c.T_gt, tau, 0.1, want_corr=True)
        o = om.linearize(c.source, ocov, oval, c.T_gt, tau, 0.1, want_corr=True)
        np.testing.assert_array_equal(host(g["corr"]), o["corr"])
        assert rel(g["H"], o["H"]) <= 1e-4 and rel(g["b"], o["b"]) <= 1e-4
    gm.close()


def test_linearize_after_insert_refreshes_search_index(far, orc):
    c = synth.make_tiny(9, n_batches=6, n_source=4000)
    gm, om, _ = build_pair(far, orc, c.map_batches[:2], c.voxel_size, 20, c.min_spacing, 5)
    ocov, oval = orc.scan_covariances(c.source, 1.0, 5)
    ocov = ocov.astype(np.float32)
    src, cov, val = dev(c.source), dev(ocov), dev(oval)
    for b in c.map_batches[2:]:
        g = gm.linearize(src, cov, val, c.T_gt, 1.0, 1 / 9, want_corr=True)
        o = om.linearize(c.source, ocov, oval, c.T_gt, 1.0, 1 / 9, want_corr=True)
        np.testing.assert_array_equal(host(g["corr"]), o["corr"])
        gm.insert(dev(b))
        om.insert(b)
    g = gm.linearize(src, cov, val, c.T_gt, 1.0, 1 / 9, want_corr=True)
    o = om.linearize(c.source, ocov, oval, c.T_gt, 1.0, 1 / 9, want_corr=True)
    np.testing.assert_array_equal(host(g["corr"]), o["corr"])
    assert rel(g["H"], o["H"]) <= 1e-4
    gm.close()
