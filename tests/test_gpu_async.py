"""The device-output linearisation (far_gicp_linearize_async) and the
workspace reservation (far_map_reserve) against far_gicp_linearize: the
result left on the device equals the host result bit for bit (H, b, cost,
inliers, correspondences), for several sizes within one reservation and for
an empty scan; and the call recorded in a captured graph (possible because
it neither synchronises nor allocates once the workspace is reserved)
replays to the same result every time, with eager work of the program
between the replays."""
import numpy as np
import pytest
import torch

from paper_2606_26010_amd import synth

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def setup(orc):
    from paper_2606_26010_amd import far
    c = synth.make_tiny(7, n_batches=6, n_source=6000)
    gm = far.Map(c.voxel_size, c.max_pts_per_voxel, c.min_spacing, 1 << 16, 0, c.k)
    for b in c.map_batches:
        gm.insert(dev(b))
    cov, val = orc.scan_covariances(c.source, c.voxel_size, c.k)
    yield far, c, gm, cov.astype(np.float32), val
    gm.close()


def same(a, b, what):
    for k in ("H", "b"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"{what}: {k}")
    assert a["cost"] == b["cost"] and a["n_inliers"] == b["n_inliers"], what


def test_async_equals_sync_within_a_reservation(setup):
    far, c, gm, cov, val = setup
    gm.reserve(6000, 1)
    T = c.T_gt @ synth.random_offset(synth.rng(2), 0.2, 1.5)
    out = torch.full((far.LIN_WORDS,), float("nan"), dtype=torch.float64, device="cuda")
    for n in (6000, 257, 1, 0):
        src, cv, vl = dev(c.source[:, :n]), dev(cov[:, :n]), dev(val[:n])
        ref = gm.linearize(src, cv, vl, T, c.tau, c.kappa, c=T[:3, 3], want_corr=True)
        corr = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
        gm.linearize_async(src, cv, vl, T, c.tau, c.kappa, out, c=T[:3, 3], corr=corr[:n])
        torch.cuda.synchronize()
        got = far.lin_from_words(out.cpu().numpy())
        same(got, ref, f"n={n}")
        if n:
            assert torch.equal(corr[:n], ref["corr"])
        say(f"async n={n}: {got['n_inliers']} inliers, equal to the synchronous call")


def test_async_replays_in_a_captured_graph(setup):
    far, c, gm, cov, val = setup
    gm.reserve(6000, 1)
    src, cv, vl = dev(c.source), dev(cov), dev(val)
    T = c.T_gt @ synth.random_offset(synth.rng(3), 0.1, 1.0)
    ref = gm.linearize(src, cv, vl, T, c.tau, c.kappa, c=T[:3, 3])
    out = torch.zeros(far.LIN_WORDS, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    # warm the call up on the capture stream (the workspace exists already)
    with torch.cuda.stream(s):
        gm.linearize_async(src, cv, vl, T, c.tau, c.kappa, out, c=T[:3, 3], stream=s)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        gm.linearize_async(src, cv, vl, T, c.tau, c.kappa, out, c=T[:3, 3], stream=s)
    for rep in range(4):
        out.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        same(far.lin_from_words(out.cpu().numpy()), ref, f"replay {rep}")
        assert torch.isfinite(junk)
    say("4 replays of the captured linearisation equal the synchronous call")
