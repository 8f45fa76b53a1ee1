"""Scan covariances over runs sorted by x inside each voxel.

The scan grid sorts each (scan, voxel) run by x up to a quantum of 2^-fb
cells and ranks a run outward from the query's x, a side stopping once its
x gap (less twice the quantum) exceeds the current k-th bound.  These cases
put many points on the same x, on quantum boundaries and one float step off
them, in clusters one float step apart inside one quantum (met out of x
order), and in mirror pairs at equal distance on either side of a query
(ties decided by id).  Each must give the oracle's neighbours (validity bit-exact,
covariances to rtol 2e-6) and the same bits as the full-key sort path, whose
runs are not ordered by x and are ranked whole."""
import numpy as np
import pytest
import torch

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


def x_planes(seed, n):
    """Points on three planes x = 0.25, 0.5, 0.75 (and their negatives): whole
    runs share one x."""
    g = np.random.default_rng(seed)
    x = g.choice([0.25, 0.5, 0.75, -0.25, -0.5, -0.75], size=n)
    yz = g.uniform(-2.0, 2.0, size=(2, n))
    return np.ascontiguousarray(np.vstack([x, yz]).astype(np.float32))


def x_quanta(seed, n, fb=14):
    """x on multiples of 2^-fb and one float step either side of them, in a
    thin slab so that runs are long."""
    g = np.random.default_rng(seed)
    x = (g.integers(-2 << fb, 2 << fb, size=n) * 2.0 ** -fb).astype(np.float32)
    step = g.integers(-1, 2, size=n)
    x = np.where(step < 0, np.nextafter(x, np.float32(-np.inf)),
                 np.where(step > 0, np.nextafter(x, np.float32(np.inf)), x))
    y = g.uniform(-1.0, 1.0, size=n).astype(np.float32)
    z = g.uniform(0.0, 0.2, size=n).astype(np.float32)
    return np.ascontiguousarray(np.vstack([x, y, z]).astype(np.float32))


def mirror_pairs(seed, n):
    """Centres with pairs at c +- d along x (same y, z): equal distances on
    either side of the centre, some pairs straddling a voxel face."""
    g = np.random.default_rng(seed)
    m = n // 3
    c = np.round(g.uniform(-2.0, 2.0, size=(3, m)) * 64.0) / 64.0
    c[0, : m // 3] = np.round(c[0, : m // 3])          # centres on voxel faces
    d = np.round(g.uniform(0.01, 0.4, size=m) * 256.0) / 256.0
    a = c.copy()
    a[0] -= d
    b = c.copy()
    b[0] += d
    return np.ascontiguousarray(np.concatenate([c, a, b], 1).astype(np.float32))


def x_within_quantum(seed, n):
    """Clusters of 24 points one float step apart along x (all inside one sort
    quantum, so their order in the run is the input order, here descending
    x) with the same y and z: a query's nearest neighbours are its
    neighbours in x, which a run ranked in quantum order meets out of x
    order; plus scattered points around them."""
    g = np.random.default_rng(seed)
    out = []
    while sum(a.shape[1] for a in out) < n - 24:
        c = g.uniform(-2.0, 2.0, size=3).astype(np.float32)
        xs = [c[0]]
        for _ in range(23):
            xs.append(np.nextafter(xs[-1], np.float32(np.inf)))
        xs = np.array(xs[::-1], np.float32)                 # descending x in input order
        cl = np.vstack([xs, np.full(24, c[1], np.float32), np.full(24, c[2], np.float32)])
        out.append(cl)
        out.append(g.uniform(-2.0, 2.0, size=(3, 8)).astype(np.float32))
    return np.ascontiguousarray(np.concatenate(out, 1)[:, :n].astype(np.float32))


CASES = {"x_planes": x_planes, "x_quanta": x_quanta, "mirror_pairs": mirror_pairs,
         "x_within_quantum": x_within_quantum}


def far_corners(v):
    """Eight points near +-1e6 voxels of edge v: their keys (inside
    [-2^20, 2^20)) force the full-key sort path."""
    c = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)],
                 np.float64).T * 1.0e6 * v
    return np.ascontiguousarray(c.astype(np.float32))


@pytest.mark.parametrize("v", [1.0, 0.25, 0.3])
@pytest.mark.parametrize("case", sorted(CASES))
def test_x_ordered_runs_match_oracle_and_full_sort(far, orc, case, v):
    scans = [CASES[case](40 + s, n) for s, n in enumerate((3000, 1200, 4500))]
    sizes = [s.shape[1] for s in scans]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pts = np.concatenate(scans, 1)
    cov, val = far.far_scan_covariances_batch(dev(pts), dev(offs), v, 5)
    cov, val = host(cov), host(val)
    for s, sc in enumerate(scans):
        oc, ov = orc.scan_covariances(sc, v, 5)
        np.testing.assert_array_equal(val[offs[s]:offs[s + 1]], ov)
        np.testing.assert_allclose(cov[:, offs[s]:offs[s + 1]], oc, rtol=2e-6, atol=1e-6)
    # the same scans beside a scan whose keys need the full-key path: runs
    # ranked whole, the same neighbours, the same bits
    wide = scans + [far_corners(v)]
    woffs = np.concatenate([[0], np.cumsum([s.shape[1] for s in wide])]).astype(np.int64)
    cw, vw = far.far_scan_covariances_batch(dev(np.concatenate(wide, 1)), dev(woffs), v, 5)
    n = pts.shape[1]
    np.testing.assert_array_equal(host(vw)[:n], val)
    np.testing.assert_array_equal(host(cw)[:, :n], cov)
    print(f"{case} v={v}: {int(val.sum())} of {n} valid, x-ordered and full-sort identical",
          flush=True)
