"""The allocation-free batch undistortion (far_undistort_batch_noalloc)
through the C ABI against far_undistort_batch, the entry point whose kernels
it shares: outputs and reference times bit-identical on two calls in a row,
the second on a smaller batch (the fixed scratch then holds the first call's
larger contents), with the outputs starting as junk; the library's scratch
pool is not touched; sizes beyond the fixed scratch are rejected before
anything is enqueued."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2606_26010_amd import synth

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def say(*a):
    print(*a, flush=True)


def batch(c, idx):
    scans = [c.scans[i] for i in idx]
    offs = np.concatenate([[0], np.cumsum([s.shape[1] for s in scans])]).astype(np.int64)
    voffs = np.concatenate([[0], np.cumsum([c.vel_t[i].size for i in idx])]).astype(np.int64)
    xyz = np.concatenate(scans, 1)
    t = np.concatenate([c.times[i] for i in idx]).astype(np.float32)
    vt = np.concatenate([c.vel_t[i] for i in idx]).astype(np.float64)
    v = np.concatenate([c.vel[i] for i in idx]).astype(np.float64)
    return [dev(a) for a in (xyz, t, offs, vt, v, voffs)]


def test_noalloc_matches_batch_on_two_calls():
    from paper_2606_26010_amd import far
    c = synth.make_deskew(17, n_scans=7)
    big, small = batch(c, range(5)), batch(c, (5, 6))
    far.far_scratch_release()
    for what, (xyz, t, offs, vt, v, voffs) in (("5 scans", big), ("2 scans", small)):
        S, n = offs.shape[0] - 1, xyz.shape[1]
        say(f"no-alloc undistortion: {what}, {n} points", )
        ref, ref_tr = far.far_undistort_batch(xyz, t, offs, vt, v, voffs)
        torch.cuda.synchronize()
        reserved = far.far_scratch_reserved()
        out = torch.full_like(xyz, float("nan"))
        tr = torch.full((S,), -7.0, dtype=torch.float64, device=xyz.device)
        far.far_undistort_batch_noalloc(xyz, t, offs, vt, v, voffs, out, tr)
        torch.cuda.synchronize()
        assert far.far_scratch_reserved() == reserved, "the no-alloc call took pool memory"
        assert torch.equal(out, ref), what
        assert torch.equal(tr, ref_tr), what
        moved = (out - xyz).abs().max().item()
        say(f"  bit-identical to far_undistort_batch; largest correction {moved:.3f} m")
        assert moved > 0.1


def test_noalloc_rejects_sizes_beyond_its_scratch():
    from paper_2606_26010_amd import far
    lib = far.lib()
    xyz = torch.zeros((3, 8), dtype=torch.float32, device="cuda")
    t = torch.zeros(8, dtype=torch.float32, device="cuda")
    vt = torch.zeros(1, dtype=torch.float64, device="cuda")
    v = torch.zeros((1, 6), dtype=torch.float64, device="cuda")
    out = torch.empty_like(xyz)
    for S, n in ((4097, 8), (1, (1 << 28) + 1)):
        offs = torch.zeros(S + 1, dtype=torch.int64, device="cuda")
        tr = torch.empty(S, dtype=torch.float64, device="cuda")
        p = lambda x: C.c_void_p(x.data_ptr())
        rc = lib.far_undistort_batch_noalloc(p(xyz), p(t), p(offs), S, n, p(vt), p(v), p(offs),
                                             p(out), p(tr), None)
        assert rc == far.FAR_E_CAPACITY, (S, n, rc)
        assert b"fixed scratch" in far.lib().far_last_error()
    torch.cuda.synchronize()
