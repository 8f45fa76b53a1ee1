"""The step's one sort: the covariance grid's order handed to the align.

far_scan_covariances_batch_order returns the (scan, 4 x 4 x 4 block of cells,
cell, x) order its grid sorted the points in; far_gicp_align_batch_ordered packs the source in
that order instead of sorting it again.  The order must be a permutation
that keeps each scan in its own range with each voxel's points adjacent and
each 4 x 4 x 4 block of voxels together; the covariances are the same bits as without it;
the ordered align lands on the oracle's poses (the order only changes the
rounding order of the sums) and repeats bit for bit."""
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


def angle_deg(A, B):
    E = A[:3, :3] @ B[:3, :3].T
    s = np.array([E[2, 1] - E[1, 2], E[0, 2] - E[2, 0], E[1, 0] - E[0, 1]])
    return math.degrees(math.atan2(0.5 * np.linalg.norm(s), 0.5 * (np.trace(E) - 1)))


@pytest.fixture(scope="module")
def batch(orc):
    from paper_2606_26010_amd import far
    c = synth.make_batch(11, n_scans=6, n_min=3000, n_max=40000, map_points=300_000,
                         map_batch=300_000, n_map_batches=2)
    gm = far.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.map_capacity,
                 c.map_capacity, c.k)
    om = orc.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.k,
                 point_capacity=c.map_capacity, voxel_capacity=c.map_capacity)
    for b in c.map_batches:
        gm.insert(dev(b))
        om.insert(b, check=False)
    scans = [s.copy() for s in c.scans]
    scans[2][:, ::97] = np.nan                    # non-finite points sort last in their scan
    sizes = np.array([s.shape[1] for s in scans])
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    yield far, c, gm, om, scans, offs
    gm.close()


def test_covariance_order_is_the_grid_order(batch):
    far, c, gm, om, scans, offs = batch
    pts = np.concatenate(scans, 1)
    n = pts.shape[1]
    cov0, val0 = far.far_scan_covariances_batch(dev(pts), dev(offs), c.voxel_size, c.k)
    order = torch.empty(n, dtype=torch.int32, device="cuda")
    cov1, val1 = far.far_scan_covariances_batch_order(dev(pts), dev(offs), c.voxel_size, c.k,
                                                      order)
    np.testing.assert_array_equal(host(cov1), host(cov0))
    np.testing.assert_array_equal(host(val1), host(val0))
    o = host(order).astype(np.int64)
    assert np.array_equal(np.sort(o), np.arange(n))                 # a permutation
    allk = np.floor(pts[:, np.isfinite(pts).all(0)].astype(np.float64) / c.voxel_size)
    kmin = allk.min(1).astype(np.int64)[:, None]     # blocks count from the batch's minima
    for s in range(len(scans)):
        a, b = offs[s], offs[s + 1]
        seg = o[a:b]
        assert seg.min() >= a and seg.max() < b                      # the scan's own range
        p = pts[:, seg].astype(np.float64)
        fin = np.isfinite(p).all(0)
        nf = int((~fin).sum())
        assert fin[:len(seg) - nf].all() and not fin[len(seg) - nf:].any()   # non-finite last
        k = np.floor(p[:, fin] / c.voxel_size).astype(np.int64)
        key = (k[0] << 42) + (k[1] << 21) + k[2]
        runs = 1 + int(np.count_nonzero(np.diff(key)))
        assert runs == np.unique(key).size                           # a voxel's points adjacent
        kb = (k - kmin) >> 2
        b4 = (kb[0] << 42) + (kb[1] << 21) + kb[2]
        assert 1 + int(np.count_nonzero(np.diff(b4))) == np.unique(b4).size   # and its block's
    print(f"order: a permutation of {n} points, scans in place, voxels and 4^3 blocks "
          f"contiguous", flush=True)


def test_ordered_align_matches_oracle_and_repeats(batch, orc):
    far, c, gm, om, scans, offs = batch
    pts = np.concatenate(scans, 1)
    n = pts.shape[1]
    order = torch.empty(n, dtype=torch.int32, device="cuda")
    cov, val = far.far_scan_covariances_batch_order(dev(pts), dev(offs), c.voxel_size, c.k,
                                                    order)
    T0 = dev(np.stack([t.reshape(16) for t in c.T0]))
    prm = far.align_params(c.tau, c.kappa, max_iters=c.max_iters, eps=0.0)
    src = dev(pts)
    stream = torch.cuda.Stream()
    res = []
    with torch.cuda.stream(stream):
        for k in range(4):              # direct launches, then the captured graph
            T = T0.clone()
            st = far.decode_stats(far.far_gicp_align_batch_ordered(gm.h, src, dev(offs), cov,
                                                                  val, order, T, prm))
            stream.synchronize()
            res.append((host(T), st))
        T_own = T0.clone()
        far.far_gicp_align_batch(gm.h, src, dev(offs), cov, val, T_own, prm)
        stream.synchronize()
    for T, st in res[1:]:
        np.testing.assert_array_equal(T, res[0][0])
        for key in ("iters", "status", "n_inliers", "cost"):
            np.testing.assert_array_equal(st[key], res[0][1][key])
    Tb = res[0][0].reshape(-1, 4, 4)
    To = host(T_own).reshape(-1, 4, 4)
    assert (res[0][1]["status"] == 0).all()
    for s in (0, 3):
        ocov, oval = orc.scan_covariances(scans[s], c.voxel_size, c.k)
        ref = om.align(scans[s], ocov.astype(np.float32), oval, c.T0[s], c.tau, c.kappa,
                       max_iters=c.max_iters, eps=0.0)
        assert ref["status"] == 0
        assert np.linalg.norm(Tb[s][:3, 3] - ref["T"][:3, 3]) <= 1e-3
        assert angle_deg(Tb[s], ref["T"]) <= 1e-2
    dt = max(float(np.linalg.norm(Tb[s][:3, 3] - To[s][:3, 3])) for s in range(len(scans)))
    assert dt <= 1e-4
    print(f"ordered align: 4 runs identical, own-sort align within {dt:.2e} m", flush=True)


def test_packed_source_equals_ordered_pack(batch):
    """far_scan_covariances_batch_packed writes the align's packed source in
    the grid's order; the align on it equals the ordered align bit for bit."""
    far, c, gm, om, scans, offs = batch
    pts = np.concatenate(scans, 1)
    n = pts.shape[1]
    order = torch.empty(n, dtype=torch.int32, device="cuda")
    cov, val = far.far_scan_covariances_batch_order(dev(pts), dev(offs), c.voxel_size, c.k,
                                                    order)
    packed = torch.empty(10 * n, dtype=torch.float32, device="cuda")
    cov_p, val_p = far.far_scan_covariances_batch_packed(dev(pts), dev(offs), c.voxel_size,
                                                         c.k, packed)
    np.testing.assert_array_equal(host(cov_p), host(cov))
    np.testing.assert_array_equal(host(val_p), host(val))
    o = host(order).astype(np.int64)
    pk = host(packed)
    A = pk[:4 * n].reshape(n, 4)
    B = pk[4 * n:8 * n].reshape(n, 4)
    Cc = pk[8 * n:].reshape(n, 2)
    np.testing.assert_array_equal(A[:, :3], pts[:, o].T)                   # x, y, z
    np.testing.assert_array_equal(A[:, 3].view(np.int32), o)              # index bits
    cv, vl = host(cov)[:, o], host(val)[o]
    np.testing.assert_array_equal(B[:, 0], np.where(vl != 0, cv[0], -1.0).astype(np.float32))
    np.testing.assert_array_equal(B[:, 1:], cv[1:4].T)
    np.testing.assert_array_equal(Cc, cv[4:6].T)
    T0 = dev(np.stack([t.reshape(16) for t in c.T0]))
    prm = far.align_params(c.tau, c.kappa, max_iters=c.max_iters, eps=0.0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        Ta = T0.clone()
        sa = far.decode_stats(far.far_gicp_align_batch_ordered(gm.h, dev(pts), dev(offs), cov,
                                                              val, order, Ta, prm))
        res = []
        for _ in range(3):              # a direct launch, then the captured graph
            Tp = T0.clone()
            sp = far.decode_stats(far.far_gicp_align_batch_packed(gm.h, packed, dev(offs), Tp,
                                                                 prm))
            stream.synchronize()
            res.append((host(Tp), sp))
    for Tp, sp in res:
        np.testing.assert_array_equal(Tp, host(Ta))
        for key in ("iters", "status", "n_inliers", "cost"):
            np.testing.assert_array_equal(sp[key], sa[key])
    print(f"packed source: {n} points, align identical to the ordered align", flush=True)


def test_packed_source_ragged_and_empty_scans(batch):
    """The packed path on a batch with an empty scan, a one-point scan and a
    scan of non-finite points between two ordinary ones, and on a batch of
    empty scans only: the packed words follow the grid's order, the align on
    them equals the ordered align bit for bit, and every scan's status is the
    one the align on the unsorted source gives."""
    far, c, gm, om, scans, offs = batch
    nan = np.full((3, 50), np.nan, np.float32)
    parts = [scans[0][:, :5000], np.zeros((3, 0), np.float32), scans[1][:, :1], nan,
             scans[3][:, :7000]]
    pts = np.ascontiguousarray(np.concatenate(parts, 1))
    off = np.concatenate([[0], np.cumsum([p.shape[1] for p in parts])]).astype(np.int64)
    n = pts.shape[1]
    S = len(parts)
    T0 = dev(np.stack([c.T0[s % len(c.T0)].reshape(16) for s in range(S)]))
    prm = far.align_params(c.tau, c.kappa, max_iters=c.max_iters, eps=0.0)
    order = torch.empty(n, dtype=torch.int32, device="cuda")
    cov, val = far.far_scan_covariances_batch_order(dev(pts), dev(off), c.voxel_size, c.k, order)
    packed = torch.empty(10 * n, dtype=torch.float32, device="cuda")
    cov_p, val_p = far.far_scan_covariances_batch_packed(dev(pts), dev(off), c.voxel_size, c.k,
                                                         packed)
    np.testing.assert_array_equal(host(cov_p), host(cov))
    np.testing.assert_array_equal(host(val_p), host(val))
    o = host(order).astype(np.int64)
    A = host(packed)[:4 * n].reshape(n, 4)
    np.testing.assert_array_equal(A[:, 3].view(np.int32), o)
    fin = np.isfinite(pts[:, o]).all(0)
    np.testing.assert_array_equal(A[fin, :3], pts[:, o].T[fin])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        To, Tu, Tp = T0.clone(), T0.clone(), T0.clone()
        so = far.decode_stats(far.far_gicp_align_batch_ordered(gm.h, dev(pts), dev(off), cov, val,
                                                              order, To, prm))
        su = far.decode_stats(far.far_gicp_align_batch(gm.h, dev(pts), dev(off), cov, val, Tu,
                                                      prm))
        sp = far.decode_stats(far.far_gicp_align_batch_packed(gm.h, packed, dev(off), Tp, prm))
        stream.synchronize()
    np.testing.assert_array_equal(host(Tp), host(To))
    for key in ("iters", "status", "n_inliers", "cost"):
        np.testing.assert_array_equal(sp[key], so[key])
    np.testing.assert_array_equal(sp["status"], su["status"])
    for s in (1, 2, 3):                                  # nothing to align: T untouched
        assert sp["status"][s] != 0
        np.testing.assert_array_equal(host(Tp)[s], host(T0)[s])
    # a batch of empty scans only
    off0 = dev(np.zeros(3, np.int64))
    empty = torch.empty(0, dtype=torch.float32, device="cuda")
    T2 = T0[:2].clone()
    far.far_scan_covariances_batch_packed(torch.empty((3, 0), dtype=torch.float32,
                                                      device="cuda"), off0, c.voxel_size, c.k,
                                          empty)
    s0 = far.decode_stats(far.far_gicp_align_batch_packed(gm.h, empty, off0, T2, prm))
    torch.cuda.synchronize()
    assert (s0["status"] != 0).all()
    np.testing.assert_array_equal(host(T2), host(T0[:2]))
    print(f"packed source, ragged batch of {n} points: statuses {[int(x) for x in sp['status']]}", flush=True)
