"""Full-size parity on the batched-scans workload, in the benchmark's launch
configuration: a 2,000,000-point map (v = 1 m, N_max = 20, spacing v/sqrt(20))
and 64 scans with 4.9M points.  The map is compared whole (bit-exact ids and
coordinates); neighbour queries, scan covariances and aligned poses on
samples the oracle computes one by one.
"""
import math

import numpy as np
import pytest
import torch

from paper_2606_26010_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def big(orc):
    from paper_2606_26010_amd import far
    c = synth.make_batch(3)
    say(f"fullsize: {len(c.scans)} scans, {sum(s.shape[1] for s in c.scans)} points")
    gm = far.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.map_capacity,
                 c.map_capacity, c.k)
    om = orc.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, c.k,
                 point_capacity=c.map_capacity, voxel_capacity=c.map_capacity)
    for b in c.map_batches:
        gs, ga = gm.insert(dev(b))
        orc_rc, oa, _ = om.insert(b, check=False)
        assert (gs, ga) == (orc_rc, oa)
        if om.size >= c.map_capacity:
            break
    say(f"fullsize map: {om.size} points, {om.n_voxels} voxels")
    yield far, c, gm, om
    gm.close()


def test_fullsize_map_identical(big):
    far, c, gm, om = big
    gx, gc, gv = gm.export()
    ox, oc, ov = om.export()
    assert ox.shape[1] == c.map_capacity
    np.testing.assert_array_equal(host(gx), ox)
    np.testing.assert_array_equal(host(gv), ov)
    np.testing.assert_allclose(host(gc), oc, rtol=2e-6, atol=1e-6)
    s = gm.stats()
    say("map stats", s)
    assert s["n_voxels"] == om.n_voxels


def test_fullsize_knn_sampled(big):
    far, c, gm, om = big
    g = synth.rng(21)
    q = np.concatenate([c.scene.surface_samples(g, 20000),
                        synth.apply(c.T_gt[0], c.scans[0][:, ::7])], 1)
    gi, gd, gn = gm.knn(dev(q), 5, 1.0)
    oi, od, on = om.knn(q, 5, 1.0)
    np.testing.assert_array_equal(host(gn), on)
    np.testing.assert_array_equal(host(gi), oi)


def test_fullsize_batched_covariances_and_align(big):
    far, c, gm, om = big
    S = len(c.scans)
    sizes = np.array([s.shape[1] for s in c.scans])
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    src = dev(np.concatenate(c.scans, 1))
    doffs = dev(offs)
    cov, val = far.far_scan_covariances_batch(src, doffs, c.voxel_size, c.k)
    T = dev(np.stack([t.reshape(16) for t in c.T0]))
    prm = far.align_params(c.tau, c.kappa, max_iters=c.max_iters, eps=0.0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        stats = gm.align_batch(src, doffs, cov, val, T, prm)
        stream.synchronize()
    st = far.decode_stats(stats)
    Tb = host(T).reshape(S, 4, 4)
    assert np.all(st["status"] == 0) and np.all(st["iters"] == c.max_iters)
    cov, val = host(cov), host(val)
    for s in (0, 17, S - 1):                      # sampled scans
        sl = slice(offs[s], offs[s + 1])
        oc, ov = orc_scan_cov(c.scans[s], c)
        np.testing.assert_array_equal(val[sl], ov)
        np.testing.assert_allclose(cov[:, sl], oc, rtol=2e-6, atol=1e-6)
        ref = om.align(c.scans[s], oc.astype(np.float32), ov, c.T0[s], c.tau, c.kappa,
                       max_iters=c.max_iters, eps=0.0)
        E = Tb[s][:3, :3] @ ref["T"][:3, :3].T
        dt = float(np.linalg.norm(Tb[s][:3, 3] - ref["T"][:3, 3]))
        da = math.degrees(math.acos(max(-1.0, min(1.0, (np.trace(E) - 1) / 2))))
        say(f"fullsize scan {s} n={sizes[s]}: |dt| {dt:.2e} m angle {da:.2e} deg; "
            f"gpu inliers {st['n_inliers'][s]} oracle {ref['n_inliers']}")
        assert ref["status"] == 0 and dt <= 1e-3 and da <= 1e-2


def orc_scan_cov(scan, c):
    from oracle import far_oracle
    return far_oracle.scan_covariances(scan, c.voxel_size, c.k)
