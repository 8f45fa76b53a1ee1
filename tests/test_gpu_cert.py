"""The correspondence search with nearest-neighbour certificates against the
oracle's 27-voxel search (Sec. III-A.2, closest map point within the
threshold, ties by id): correspondences bit-exact where many map points lie
at exactly the same distance (queries at the centres, face and edge
midpoints of an exact lattice, so the (d2, id) rule decides), where points
repeat more often than a certificate lists (rho 0: every query falls back to
the exact search), after inserts that put new points next to certified ones,
and after an eviction renumbers the map; and seeded iterations (the previous
match certified again, or walked from) agreeing with the oracle's align in
the FP64 path to 1e-9 m."""
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


@pytest.fixture(scope="module")
def far():
    from paper_2606_26010_amd import far as F
    F.lib()
    return F


def lattice(n=12, step=0.25, origin=(-1.5, -1.5, -1.5)):
    g = np.arange(n) * step
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    p = np.stack([x.ravel(), y.ravel(), z.ravel()]) + np.asarray(origin)[:, None]
    return np.ascontiguousarray(p.astype(np.float32))


def tie_queries(step=0.25, origin=(-1.5, -1.5, -1.5), n=11, seed=3):
    """Cell centres (8 map points at one distance), face centres (4) and edge
    midpoints (2), all exactly representable, plus random points."""
    o = np.asarray(origin)[:, None]
    g = np.arange(n) * step
    out = []
    for off in ((0.5, 0.5, 0.5), (0.5, 0.5, 0.0), (0.0, 0.5, 0.5), (0.5, 0.0, 0.0)):
        x, y, z = np.meshgrid(g + off[0] * step, g + off[1] * step, g + off[2] * step,
                              indexing="ij")
        out.append(np.stack([x.ravel(), y.ravel(), z.ravel()]) + o)
    r = np.random.default_rng(seed)
    out.append(r.uniform(-1.6, 1.3, size=(3, 2000)))
    q = np.concatenate(out, axis=1).astype(np.float32)
    return np.ascontiguousarray(q[:, r.permutation(q.shape[1])])


def pair(far, orc, batches, v=1.0, nmax=64, dmin=0.0, k=5, cap=1 << 16):
    gm = far.Map(v, nmax, dmin, cap, 0, k)
    om = orc.Map(v, nmax, dmin, k, point_capacity=cap, voxel_capacity=cap)
    for b in batches:
        gm.insert(dev(b))
        om.insert(b)
    return gm, om


def check_corr(gm, om, orc, q, T, tau, what, prec=0):
    cov, val = orc.scan_covariances(q, 1.0, 5)
    cov = cov.astype(np.float32)
    g = gm.linearize(dev(q), dev(cov), dev(val), T, tau, 1 / 9, precision=prec, want_corr=True)
    o = om.linearize(q, cov, val, T, tau, 1 / 9, want_corr=True)
    gc, oc = host(g["corr"]), o["corr"]
    bad = np.nonzero(gc != oc)[0]
    say(f"{what}: {q.shape[1]} queries, {int((oc >= 0).sum())} matched, "
        f"{bad.size} differ")
    np.testing.assert_array_equal(gc, oc)


def test_lattice_ties_resolved_by_id(far, orc):
    gm, om = pair(far, orc, [lattice()])
    q = tie_queries()
    for tau in (1.0, 0.2, 0.125):
        check_corr(gm, om, orc, q, np.eye(4), tau, f"lattice ties, tau {tau}")
    # the same ties seen through a pose whose products are exact
    T = np.eye(4)
    T[:3, 3] = [0.125, -0.25, 0.0]
    check_corr(gm, om, orc, q, T, 1.0, "lattice ties, translated")
    gm.close()


def test_repeated_points_fall_back_to_the_exact_search(far, orc):
    """Every location holds 12 copies: the 9th other point of a certificate
    lies at distance 0, so rho is 0 and no candidate certifies."""
    r = np.random.default_rng(7)
    base = r.uniform(-6, 6, size=(3, 400)).astype(np.float32)
    gm, om = pair(far, orc, [base] * 12)
    assert om.size == 12 * 400 and gm.stats()["n_points"] == om.size
    q = np.ascontiguousarray((base + r.normal(scale=0.05, size=base.shape)).astype(np.float32))
    q = np.concatenate([q, base], axis=1)
    check_corr(gm, om, orc, q, np.eye(4), 1.0, "12 copies per location")
    gm.close()


def test_inserts_and_eviction_refresh_certificates(far, orc):
    r = np.random.default_rng(11)
    q = r.uniform(-4, 4, size=(3, 6000)).astype(np.float32)
    gm, om = pair(far, orc, [], nmax=20, dmin=0.05)
    for b in range(5):
        # each batch densifies the same region: certificates of points next
        # to the new ones must shrink or change
        batch = r.uniform(-4, 4, size=(3, 3000)).astype(np.float32)
        gm.insert(dev(batch))
        om.insert(batch)
        check_corr(gm, om, orc, q, np.eye(4), 1.0, f"after insert {b}")
    for rad in (3.0, 2.0):
        ng = gm.evict(np.zeros(3), rad)
        no = om.evict(np.zeros(3), rad)
        say(f"evicted beyond {rad} m: {ng} / {no}")
        check_corr(gm, om, orc, q, np.eye(4), 1.0, f"after eviction at {rad} m")
    gm.close()


def test_seeded_iterations_match_the_oracle_align(far, orc):
    """Iterations after the first start from the previous match: FP64 aligns
    of 1..4 iterations equal the oracle's to 1e-9 m (a single different
    correspondence moves the pose far more)."""
    c = synth.make_tiny(5, n_batches=8, n_source=5000)
    gm, om = pair(far, orc, c.map_batches, nmax=c.max_pts_per_voxel, dmin=c.min_spacing)
    cov, val = orc.scan_covariances(c.source, c.voxel_size, c.k)
    cov = cov.astype(np.float32)
    T0 = c.T_gt @ synth.random_offset(synth.rng(3), 0.3, 2.0)
    for iters in (1, 2, 4):
        prm = far.align_params(c.tau, c.kappa, max_iters=iters, eps=0.0,
                               precision=far.FAR_PREC_FP64)
        st, T, stats = gm.align(dev(c.source), dev(cov), dev(val), T0, prm)
        ref = om.align(c.source, cov, val, T0, c.tau, c.kappa, max_iters=iters, eps=0.0)
        dt = float(np.linalg.norm(T[:3, 3] - ref["T"][:3, 3]))
        dr = float(np.abs(T[:3, :3] - ref["T"][:3, :3]).max())
        say(f"FP64 align, {iters} iterations: |dt| {dt:.2e} m, max |dR| {dr:.2e}")
        assert st == 0 and dt < 1e-9 and dr < 1e-9
    gm.close()


def test_queries_in_empty_voxels_next_to_the_map(far, orc):
    """Queries in empty voxels: next to an occupied one (their ghost's
    neighbour row lists the occupied neighbours), two or more voxels away
    (no ghost: nothing within v), and the same with the ghost table too small
    for the map (isolated voxels have 26 ghosts each), where the search
    probes the neighbours one by one."""
    r = np.random.default_rng(23)
    # isolated clusters of points 5 m apart, each within one voxel
    centres = np.stack(np.meshgrid(np.arange(4) * 5.0, np.arange(4) * 5.0, [0.0],
                                   indexing="ij")).reshape(3, -1) + 0.5
    pts = np.concatenate([c[:, None] + r.uniform(-0.45, 0.45, size=(3, 12))
                          for c in centres.T], axis=1).astype(np.float32)
    q = np.concatenate([c[:, None] + r.uniform(-2.0, 2.0, size=(3, 300))
                        for c in centres.T], axis=1).astype(np.float32)
    for voxel_cap, what in ((0, "ghosts held"), (16, "ghost table too small")):
        gm = far.Map(1.0, 20, 0.0, 1 << 12, voxel_cap, 5)
        om = orc.Map(1.0, 20, 0.0, 5, point_capacity=1 << 12, voxel_capacity=1 << 12)
        gm.insert(dev(pts))
        om.insert(pts)
        check_corr(gm, om, orc, q, np.eye(4), 1.0, what)
        gm.close()
