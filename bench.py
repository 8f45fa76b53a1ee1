#!/usr/bin/env python
"""Benchmark of the batched GICP linearize+kNN hot path on one MI355X.

Workload (the batched-scans configuration the throughput target is quoted on):
64 independent spinning-LiDAR scans of uneven size (U[8k, 130k] points,
clamped to each scan's ray hits) at random poses along a corridor, each with
its own initial offset (<= 0.5 m, <= 3 deg), registered against one prebuilt
2,000,000-point voxel map (v = 1 m, N_max = 20, spacing v/sqrt(20), k = 5).
All data is seeded and synthetic (the paper's datasets are not available).

One step = the whole per-batch hot path with inputs resident in HBM:
  1. regularised covariances of every scan against itself (one batched call),
     which also writes the align's packed source in the (scan, block of
     cells, cell, x) order its grid sorted the points in;
  2. batched Gauss-Newton align of all scans on that packed source (the step
     sorts and packs its points once): each iteration is one
     linearisation launch over all scans' point tiles plus one
     reduce-and-solve launch, the whole align replayed as one HIP graph.

value = linearize+kNN points/s = sum over scans of (GN iterations x points)
divided by the step time.  Also reported: scans/s, the one-scan-per-launch
path, the roofline of the linearisation (HIP-event timed inside the library:
the certified search, the exact search of its queue and the term pass of one
GN iteration) against the 8 TB/s HBM peak and a copy bandwidth measured
here, with the counter-derived traffic, L2 hit rate and VALU and LDS issue
fractions of the committed profile when it matches the kernel sources; the
covariance call on its own; the same batch run to convergence; pose error
against the oracle and ground truth; and the FP64 CPU oracle timed on a
bounded sample of the same workload at all host threads and at one.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CLOCK_GHZ = 2.4           # MI355X peak engine clock
N_SIMD = 1024             # 256 CUs x 4 SIMDs
LDS_BYTES_PER_CLK_CU = 128
KERNEL_SOURCES = ["paper_2606_26010_amd/csrc/far_gicp.hip", "paper_2606_26010_amd/csrc/far_knn.h",
                  "paper_2606_26010_amd/csrc/far_internal.h"]
COUNTERS_FILE = os.path.join(ROOT, "profiles", "linearize_batch64_counters.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_fingerprint():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pose_err(A, B):
    import numpy as np
    E = A[:3, :3] @ B[:3, :3].T
    ang = math.degrees(math.acos(max(-1.0, min(1.0, (np.trace(E) - 1) / 2))))
    return float(np.linalg.norm(A[:3, 3] - B[:3, 3])), ang


def touched_voxels(map_keys_counts, scan_xyz, T, v):
    """Distinct non-empty map voxels in the 27-neighbourhoods of a scan's
    transformed points, and the points they hold (host-side byte model)."""
    import numpy as np
    keys, counts = map_keys_counts
    p = T[:3, :3] @ scan_xyz.astype(np.float64) + T[:3, 3:4]
    k = np.floor(p / v).astype(np.int64)
    k = np.unique(k, axis=1)
    offs = np.array([[a, b, c] for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]).T
    nb = (k[:, :, None] + offs[:, None, :]).reshape(3, -1)
    packed = ((nb[0] + (1 << 20)) << 42) | ((nb[1] + (1 << 20)) << 21) | (nb[2] + (1 << 20))
    packed = np.unique(packed)
    idx = np.searchsorted(keys, packed)
    idx = np.clip(idx, 0, len(keys) - 1)
    hit = keys[idx] == packed
    return packed[hit], counts[idx[hit]]


def read_counters(fp, tile):
    """Per-linearisation counter totals from the committed rocprofv3 --pmc
    summary, if it was taken on the current kernel sources at this tile."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    # one section per tile, each starting with its kernel_sources_sha256_16 line
    sections, kv = [], None
    for line in open(COUNTERS_FILE):
        if "=" in line and not line.startswith("#"):
            a, b = (x.strip() for x in line.split("=", 1))
            if a == "kernel_sources_sha256_16":
                kv = {}
                sections.append(kv)
            if kv is not None:
                kv[a] = b
    for kv in sections:
        if kv.get("kernel_sources_sha256_16") == fp and kv.get("tile") == str(tile):
            try:
                return {k: float(v) for k, v in kv.items()
                        if k not in ("kernel_sources_sha256_16", "tile", "kernels")}
            except ValueError:
                return None
    return None


def copy_gbps(torch, dev, stream, reps=5):
    """Device-to-device copy bandwidth (read + write bytes per second) of a
    1 GiB buffer on the benchmark stream, from HIP events."""
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        b.copy_(a)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * (1 << 30) / (ms * 1e-3) / 1e9


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def lib_ms(far, kinds, fn, reps):
    """GPU time per call (ms) of fn() for each timing kind, from the events the
    library records on its launch stream around its own device work."""
    fn()
    for k in kinds:
        far.far_timing_read_kind(k, reset=True)
    far.far_timing_enable(True)
    try:
        for _ in range(reps):
            fn()
    finally:
        far.far_timing_enable(False)
    return [far.far_timing_read_kind(k, reset=True)[0] / reps for k in kinds]


def hbm_roofline(bytes_per_call, ms):
    gbs = bytes_per_call / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 5), "algorithmic_bytes": round(bytes_per_call)}


def next_rows(far, synth, np, torch, dev, stream, gm, case, T_fin, cov, val, seed):
    """Timings of the steps around the registration, each on its own input
    (HIP events the library records on its launch stream around each call's
    device work, averaged over repetitions):
      undistort  64 racing scans (8 distinct moving-LiDAR scans used 8 times,
                 each with its own time offset) in one batched call; per point
                 16 B read (xyz, time) and 12 B written;
      gradient   d cost / d (pose, points) of every scan of the batch at its
                 aligned pose in one batched call: the linearisation's bytes
                 plus 12 B per point written (and the largest scan alone);
      asmd_caps  adaptive density caps of the largest scan: 24 B read and 4 B
                 written per point (the hash set of near voxels aside);
      evict      removal of the voxels beyond 300, 150, then 60 m of the first
                 scan's pose from the map and the rebuild of its structures:
                 the sum of each call's device phases between its host
                 synchronisations; the 60 m call is the reported one (last:
                 it changes the map)."""
    rows = {}
    c = synth.make_deskew(seed + 3, n_scans=8)
    scans, times, vts, vels = [], [], [], []
    for r in range(8):
        for s in range(8):
            scans.append(c.scans[s])
            times.append(c.times[s] + np.float32(0.125 * r))
            vts.append(c.vel_t[s] + 0.125 * r)
            vels.append(c.vel[s])
    offs = np.concatenate([[0], np.cumsum([x.shape[1] for x in scans])]).astype(np.int64)
    voffs = np.concatenate([[0], np.cumsum([x.size for x in vts])]).astype(np.int64)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    x, t, o, vt, v, vo = (to(np.concatenate(scans, 1)), to(np.concatenate(times)), to(offs),
                          to(np.concatenate(vts)), to(np.concatenate(vels)), to(voffs))
    out = torch.empty_like(x)
    n = int(offs[-1])
    ms, ms_apply = lib_ms(far, (far.FAR_TIME_UNDISTORT, far.FAR_TIME_UNDISTORT_APPLY),
                          lambda: far.far_undistort_batch(x, t, o, vt, v, vo, out=out), 20)
    rows["undistort"] = {"scans": 64, "points": n, "ms": round(ms, 4),
                         "points_per_s": round(n / (ms * 1e-3), 1),
                         "roofline": hbm_roofline(28.0 * n + 56.0 * int(voffs[-1]), ms),
                         "apply_kernel": {"kernel": "k_ud_apply", "ms": round(ms_apply, 4),
                                          "roofline": hbm_roofline(28.0 * n, ms_apply)}}
    del x, t, o, vt, v, vo, out

    # gradient of the whole batch at the aligned poses (one batched call), and
    # of its largest scan alone
    mx, _, _ = gm.export()
    mk = np.floor(mx.cpu().numpy().astype(np.float64) / case.voxel_size).astype(np.int64)
    mp = ((mk[0] + (1 << 20)) << 42) | ((mk[1] + (1 << 20)) << 21) | (mk[2] + (1 << 20))
    keys_counts = np.unique(mp, return_counts=True)
    S = len(case.scans)
    sizes = np.array([sc.shape[1] for sc in case.scans], np.int64)
    offs_b = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    src_b, o_b = to(np.concatenate(case.scans, 1)), to(offs_b)
    T_b = to(np.stack([T_fin[k].reshape(16) for k in range(S)]))
    ctr_b = to(np.stack([T_fin[k][:3, 3] for k in range(S)]))
    res = {}

    def grad_batch():
        res["b"] = far.far_gicp_gradient_batch(gm.h, src_b, o_b, cov, val, T_b, case.tau,
                                               case.kappa, c=ctr_b)
    ms, = lib_ms(far, (far.FAR_TIME_GRADIENT,), grad_batch, 20)
    inl = int(res["b"]["n_inliers"].sum())
    vox = [touched_voxels(keys_counts, case.scans[k], T_fin[k], case.voxel_size)
           for k in range(S)]
    vk = np.concatenate([x[0] for x in vox])
    vc = np.concatenate([x[1] for x in vox])
    uk, ui = np.unique(vk, return_index=True)
    N = int(offs_b[-1])
    nb = 37.0 * N + 32.0 * inl + 20.0 * uk.size + 16.0 * vc[ui].sum() + 12.0 * N
    rows["gradient"] = {"scans": S, "points": N, "inliers": inl, "ms": round(ms, 4),
                        "points_per_s": round(N / (ms * 1e-3), 1),
                        "roofline": hbm_roofline(float(nb), ms)}

    s = int(np.argmax(sizes))
    a, n = int(offs_b[s]), int(sizes[s])
    src = to(case.scans[s])
    cv, vl = cov[:, a:a + n].contiguous(), val[a:a + n].contiguous()
    T = T_fin[s]

    def grad():
        res["g"] = far.far_gicp_gradient(gm.h, src, cv, vl, T, case.tau, case.kappa, c=T[:3, 3])
    ms1, = lib_ms(far, (far.FAR_TIME_GRADIENT,), grad, 20)
    rows["gradient_one_scan"] = {"points": n, "ms": round(ms1, 4),
                                 "points_per_s": round(n / (ms1 * 1e-3), 1)}

    moved = far.far_transform_points(src, T)
    ms, = lib_ms(far, (far.FAR_TIME_ASMD,),
                 lambda: far.far_asmd_caps(src, moved, case.voxel_size, case.k,
                                           case.max_pts_per_voxel, 20.0, 120.0), 20)
    rows["asmd_caps"] = {"points": n, "ms": round(ms, 4),
                         "points_per_s": round(n / (ms * 1e-3), 1),
                         "roofline": hbm_roofline(28.0 * n, ms)}

    ctr = case.T0[0][:3, 3]
    calls = []
    for radius in (300.0, 150.0, 60.0):         # the first two warm the rebuild path
        before = gm.stats()["n_points"]
        far.far_timing_read_kind(far.FAR_TIME_EVICT, reset=True)
        far.far_timing_enable(True)
        try:
            removed = gm.evict(ctr, radius)
        finally:
            far.far_timing_enable(False)
        ms = far.far_timing_read_kind(far.FAR_TIME_EVICT, reset=True)[0]
        calls.append({"radius_m": radius, "map_points_before": before, "removed": removed,
                      "ms": round(ms, 4)})
    last = calls[-1]
    rows["evict"] = dict(last, map_points_per_s=round(last["map_points_before"] /
                                                        (last["ms"] * 1e-3), 1),
                         calls=calls)
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--scans", type=int, default=64)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--eps", type=float, default=5e-3,
                    help="stop when |delta| <= eps (the paper's 5e-3; 0: always run --iters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single", action="store_true", help="skip the one-scan-per-launch path")
    ap.add_argument("--cpu-sample-scans", type=int, default=3)
    ap.add_argument("--no-pipelined", action="store_true",
                    help="skip the steps pipelined over two streams")
    ap.add_argument("--no-converged", action="store_true",
                    help="skip the secondary run of the same batch to convergence")
    ap.add_argument("--conv-iters", type=int, default=40)
    ap.add_argument("--conv-eps", type=float, default=1e-6)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default schedules instead of autotuning them on the batch")
    ap.add_argument("--tile", type=int, choices=(128, 256, 512), default=0,
                    help="linearisation tile (skips its autotuning; 0: autotuned)")
    ap.add_argument("--lin-grid", type=int, default=-1,
                    help="blocks per CU of a persistent launch of the tile passes (0: one "
                         "block per tile; -1: timed on the batch and the faster kept)")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the timings of undistortion, gradient, ASMD caps and eviction")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (PMC byte-counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_26010_amd import far, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    if args.copy_calib:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_per_copy": a.numel() * 4}))
        return

    t_gen = time.time()
    case = synth.make_batch(args.seed, n_scans=args.scans)
    log(f"[bench] generated {len(case.scans)} scans, {sum(s.shape[1] for s in case.scans)} points "
        f"in {time.time() - t_gen:.1f}s")
    S = len(case.scans)
    sizes = np.array([s.shape[1] for s in case.scans], np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    N = int(offsets[-1])

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        # ---------------- map build (not timed as part of the step)
        gm = far.Map(case.voxel_size, case.max_pts_per_voxel, case.min_spacing,
                     point_capacity=case.map_capacity, voxel_capacity=1 << 19,
                     k_cov=case.k)
        t0 = time.time()
        inserted = 0
        for b in case.map_batches:
            st, acc = gm.insert(torch.from_numpy(b).to(dev))
            inserted += b.shape[1]
            if st == far.FAR_E_CAPACITY:
                break
        stream.synchronize()
        t_map = time.time() - t0
        mstats = gm.stats()
        log(f"[bench] map: {mstats['n_points']} points in {mstats['n_voxels']} voxels, "
            f"{inserted} candidates, {t_map:.2f}s, load {mstats['load_factor']:.3f}, "
            f"mean probe {mstats['mean_probe']:.3f}")

        src = torch.from_numpy(np.ascontiguousarray(np.concatenate(case.scans, 1))).to(dev)
        offs = torch.from_numpy(offsets).to(dev)
        T0 = torch.from_numpy(np.stack([t.reshape(16) for t in case.T0])).to(dev)
        T = T0.clone()
        stats_buf = torch.empty(S * far.STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        prec = far.FAR_PREC_FP64 if args.precision == "fp64" else far.FAR_PREC_FP32
        prm = far.align_params(case.tau, case.kappa, max_iters=args.iters, eps=args.eps,
                               recenter=1, precision=prec)

        cov_buf = torch.empty((6, N), dtype=torch.float32, device=dev)
        val_buf = torch.empty(N, dtype=torch.uint8, device=dev)

        # ---------------- schedules (autotuned on this batch, outside the timed steps)
        schedule = {"tile": 256, "fine_cells": 0, "cov_dense_threshold":
                    far.far_get_covariance_schedule(), "autotuned": False}
        if not args.no_autotune:
            t_at = time.time()
            thr, thr_ms = far.far_autotune_covariances(src, offs, case.voxel_size, case.k, reps=2)
            cov, val = far.far_scan_covariances_batch(src, offs, case.voxel_size, case.k,
                                                      out=(cov_buf, val_buf))
            schedule = {"tile": 256, "fine_cells": 0, "cov_dense_threshold": thr,
                        "autotuned": True,
                        "cov_ms_by_threshold": {str(t): round(x, 3) for t, x in
                                                zip((0, 16, 32, 64, 128), thr_ms)}}
            if not args.tile:
                best, lin_ms_c = far.far_autotune(gm.h, src, offs, cov, val, T0, prm, reps=2)
                schedule.update({"tile": best["tile"], "fine_cells": best["fine_cells"],
                                 "align_ms_by_candidate": {
                                     f"tile{t}_{'fine' if f else 'voxel'}":
                                     round(lin_ms_c[2 * i + f], 3)
                                     for i, t in enumerate((128, 256, 512)) for f in (0, 1)}})
            stream.synchronize()
            log(f"[bench] autotune {time.time() - t_at:.1f}s: {schedule}")
        if args.tile:
            far.far_map_set_schedule(gm.h, args.tile, 0)
            schedule["tile"], schedule["fine_cells"] = args.tile, 0
            schedule["tile_forced"] = True
        tile = schedule["tile"]
        # launch of the tile passes: one block per tile or a persistent grid of
        # n blocks per CU taking tiles in turn (identical results); timed on
        # the align of this batch and the faster kept, unless forced
        schedule["lin_blocks_per_cu"] = args.lin_grid if args.lin_grid >= 0 else 0
        if args.lin_grid < 0 and not args.no_autotune:
            cov_g, val_g = far.far_scan_covariances_batch(src, offs, case.voxel_size, case.k,
                                                          out=(cov_buf, val_buf))
            grid_ms = {}
            for g in (0, 4, 8, 16):
                far.far_set_linearize_grid(g)
                T_g = T0.clone()
                far.far_gicp_align_batch(gm.h, src, offs, cov_g, val_g, T_g, prm, stats=stats_buf)
                stream.synchronize()
                t0 = time.perf_counter()
                for _ in range(3):
                    T_g.copy_(T0)
                    far.far_gicp_align_batch(gm.h, src, offs, cov_g, val_g, T_g, prm,
                                             stats=stats_buf)
                stream.synchronize()
                grid_ms[str(g)] = round((time.perf_counter() - t0) / 3 * 1e3, 3)
            best_g = min(grid_ms, key=lambda k: grid_ms[k])
            schedule["lin_blocks_per_cu"] = int(best_g)
            schedule["align_ms_by_lin_blocks_per_cu"] = grid_ms
            log(f"[bench] tile-pass launch: {grid_ms} ms per align, kept {best_g} blocks per CU")
        far.far_set_linearize_grid(schedule["lin_blocks_per_cu"])

        # The step sorts and packs its points once: the covariance call
        # writes the align's packed source in its grid's (scan, block of
        # cells, cell, x) order beside cov6 and valid, and the align reads it
        # as it is (no sort or pack of its own).
        packed_buf = torch.empty(10 * N, dtype=torch.float32, device=dev)

        def step():
            cov, val = far.far_scan_covariances_batch_packed(src, offs, case.voxel_size, case.k,
                                                             packed_buf, out=(cov_buf, val_buf))
            T.copy_(T0)
            far.far_gicp_align_batch_packed(gm.h, packed_buf, offs, T, prm, stats=stats_buf)
            return cov, val

        for _ in range(args.warmup):
            step()
        stream.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            cov, val = step()
        stream.synchronize()
        torch.cuda.synchronize()
        t_step = (time.perf_counter() - t0) / args.steps
        stats = far.decode_stats(stats_buf)
        T_gpu = T.cpu().numpy().reshape(S, 4, 4)

        iters = stats["iters"].astype(np.int64)
        failed = stats["status"] != 0
        lin_per_scan = iters + failed.astype(np.int64)   # a failing iteration still linearised
        point_lins = int(np.sum(lin_per_scan * sizes))
        log(f"[bench] step {t_step * 1e3:.3f} ms, iterations {iters.min()}..{iters.max()}, "
            f"status {np.bincount(stats['status'], minlength=6).tolist()}")

        # ---------------- the same steps pipelined over two streams: the
        # covariances of batch k+1 on one stream beside the align of batch k
        # on another (default priorities, double-buffered covariances); every
        # step still does all of its work.  Reported beside the headline.
        piped = None
        if not args.no_pipelined:
            s_al = torch.cuda.Stream()
            cov_b = [cov_buf, torch.empty_like(cov_buf)]
            val_b = [val_buf, torch.empty_like(val_buf)]
            pk_b = [packed_buf, torch.empty_like(packed_buf)]
            ev_cov = [torch.cuda.Event(), torch.cuda.Event()]
            ev_al = [torch.cuda.Event(), torch.cuda.Event()]
            for e in ev_al:
                e.record(s_al)

            def step_piped(k):
                b = k % 2
                stream.wait_event(ev_al[b])     # the align that read buffer b is done
                far.far_scan_covariances_batch_packed(src, offs, case.voxel_size, case.k,
                                                      pk_b[b], out=(cov_b[b], val_b[b]))
                ev_cov[b].record(stream)
                with torch.cuda.stream(s_al):
                    s_al.wait_event(ev_cov[b])
                    T.copy_(T0)
                    far.far_gicp_align_batch_packed(gm.h, pk_b[b], offs, T, prm,
                                                    stats=stats_buf)
                    ev_al[b].record(s_al)

            for k in range(max(args.warmup, 4)):   # both buffers' aligns captured
                step_piped(k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(args.steps):
                step_piped(k)
            torch.cuda.synchronize()
            t_piped = (time.perf_counter() - t0) / args.steps
            same = bool(np.array_equal(T.cpu().numpy().reshape(S, 4, 4), T_gpu))
            piped = {"ms_per_step": round(t_piped * 1e3, 4),
                     "value": round(point_lins / t_piped, 1),
                     "scans_per_s": round(S / t_piped, 2), "same_poses": same}
            log(f"[bench] pipelined over two streams: {t_piped * 1e3:.3f} ms per step, "
                f"poses {'identical' if same else 'DIFFER'}")

        # ---------------- roofline of the linearisation (event-timed launches)
        far.far_timing_read(reset=True)
        far.far_timing_read_kind(far.FAR_TIME_COVARIANCES, reset=True)
        far.far_timing_enable(True)
        n_timed = max(1, min(args.steps, 5))
        for _ in range(n_timed):
            step()
        stream.synchronize()
        lin_ms, lin_launches = far.far_timing_read(reset=True)
        cov_ms_tot, cov_calls = far.far_timing_read_kind(far.FAR_TIME_COVARIANCES, reset=True)
        far.far_timing_enable(False)
        stats_t = far.decode_stats(stats_buf)
        T_fin = T.cpu().numpy().reshape(S, 4, 4)
        # Algorithmic bytes of one linearisation (the byte model of the method,
        # per GN iteration and scan): every active source point's xyz, cov6 and
        # valid (37 B); each inlier's matched map covariance, valid flag and id
        # (29 B); per distinct map voxel in the 27-neighbourhoods of the scan's
        # points, its slot and count (16 B) and its points (12 B each); the
        # scan's 29 FP64 sums (232 B).  Voxels are counted per scan (each scan
        # must read its own neighbourhood); the union over the active scans
        # (a voxel read once per launch) is reported beside it.
        mx, _, _ = gm.export()
        mk = np.floor(mx.cpu().numpy().astype(np.float64) / case.voxel_size).astype(np.int64)
        mp = ((mk[0] + (1 << 20)) << 42) | ((mk[1] + (1 << 20)) << 21) | (mk[2] + (1 << 20))
        mkeys, mcounts = np.unique(mp, return_counts=True)
        per_scan_vox = [touched_voxels((mkeys, mcounts), case.scans[s], T_fin[s], case.voxel_size)
                        for s in range(S)]
        it_t = stats_t["iters"].astype(np.int64) + (stats_t["status"] != 0)
        n_inl = stats_t["n_inliers"].astype(np.int64)
        launches_per_step = args.iters
        bytes_step = bytes_union_step = 0.0
        for it in range(launches_per_step):
            active = np.nonzero(it_t > it)[0]
            if active.size == 0:
                continue
            per = sum(16.0 * per_scan_vox[s][0].size + 12.0 * per_scan_vox[s][1].sum()
                      for s in active)
            bytes_step += 37.0 * sizes[active].sum() + 29.0 * n_inl[active].sum() + per + \
                232.0 * active.size
            vk = np.concatenate([per_scan_vox[s][0] for s in active])
            vc = np.concatenate([per_scan_vox[s][1] for s in active])
            uk, ui = np.unique(vk, return_index=True)
            bytes_union_step += (37.0 * sizes[active].sum() + 29.0 * n_inl[active].sum()
                                 + 16.0 * uk.size + 12.0 * vc[ui].sum() + 232.0 * active.size)
        bytes_per_launch = bytes_step / launches_per_step
        bytes_union_per_launch = bytes_union_step / launches_per_step
        avg_launch_ms = lin_ms / max(lin_launches, 1)
        achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
        fp = kernel_fingerprint()
        ctr = read_counters(fp, tile)
        copy_bw = copy_gbps(torch, dev, stream)
        t_s = avg_launch_ms * 1e-3
        roof_extra = {"copy_gbps": round(copy_bw, 1),
                      "frac_of_copy": round(achieved / copy_bw, 5),
                      "traffic": None, "l2_hit": None, "valu_frac": None, "lds_frac": None}
        if ctr is not None:
            roof_extra["traffic"] = ctr["fabric_read_bytes"] + ctr["fabric_write_bytes"]
            roof_extra["l2_hit"] = round(ctr["tcc_hit"] / max(ctr["tcc_hit"] + ctr["tcc_miss"], 1), 4)
            # a wave64 VALU instruction occupies its SIMD for 2 cycles at the
            # chip's 32-bit rate (157.3 TFLOP/s = 256 CUs x 4 SIMDs x 32 lanes x
            # 2 x 2.4 GHz; FP64 instructions take 4, so this is a lower bound)
            roof_extra["valu_frac"] = round(2.0 * ctr["valu_insts"] / (N_SIMD * CLOCK_GHZ * 1e9 * t_s), 4)
            roof_extra["lds_frac"] = round(ctr["lds_insts"] * 64 * 4 /
                                           (LDS_BYTES_PER_CLK_CU * 256 * CLOCK_GHZ * 1e9 * t_s), 4)
            if "ta_ta_busy_sum" in ctr:   # texture-address units, one per CU
                roof_extra["ta_busy_frac"] = round(ctr["ta_ta_busy_sum"] /
                                                   (256 * CLOCK_GHZ * 1e9 * t_s), 4)
            if ctr.get("tcp_tcc_read_req_sum"):
                roof_extra["l2_read_latency_cycles"] = round(
                    ctr["tcp_tcc_read_req_latency_sum"] / ctr["tcp_tcc_read_req_sum"], 1)
        log(f"[bench] linearisation: {lin_launches} launches, avg {avg_launch_ms * 1e3:.1f} us, "
            f"{bytes_per_launch / 1e6:.1f} MB algorithmic per launch "
            f"({bytes_union_per_launch / 1e6:.1f} MB with voxels counted once), "
            f"{achieved:.0f} GB/s, copy {copy_bw:.0f} GB/s, counters "
            f"{'matched' if ctr else 'not matched'}")
        # the covariance call on its own: n (12 + 8 + 4 + 24 + 1) per point plus,
        # per occupied (scan, voxel) run, its slot (16 B) and its points (12 B each)
        cov_ms = cov_ms_tot / max(cov_calls, 1)
        runs = sum(np.unique(np.floor(sc / case.voxel_size).astype(np.int64), axis=1).shape[1]
                   for sc in case.scans)
        cov_bytes = 49.0 * N + 16.0 * runs + 12.0 * N
        cov_row = {"ms": round(cov_ms, 4), "points_per_s": round(N / (cov_ms * 1e-3), 1),
                   "runs": int(runs), "roofline": hbm_roofline(cov_bytes, cov_ms)}
        log(f"[bench] covariances: {cov_ms:.3f} ms per call, {runs} (scan, voxel) runs")

        # ---------------- one-scan-per-launch path (same work, per-scan calls)
        single = None
        if not args.no_single:
            scan_t = [torch.from_numpy(np.ascontiguousarray(s)).to(dev) for s in case.scans]
            prm1 = far.align_params(case.tau, case.kappa, max_iters=args.iters, eps=args.eps,
                                    recenter=1, precision=prec)

            def single_step():
                out = []
                for s in range(S):
                    c1, v1 = far.far_scan_covariances(scan_t[s], case.voxel_size, case.k)
                    out.append(far.far_gicp_align(gm.h, scan_t[s], c1, v1, case.T0[s], prm1))
                return out

            single_step()
            stream.synchronize()
            n_single = max(1, min(args.steps, 3))
            t0 = time.perf_counter()
            for _ in range(n_single):
                res1 = single_step()
            stream.synchronize()
            t_single = (time.perf_counter() - t0) / n_single
            dmax = max(pose_err(res1[s][1], T_gpu[s])[0] for s in range(S))
            single = {"ms_per_step": round(t_single * 1e3, 3),
                      "scans_per_s": round(S / t_single, 2),
                      "batched_speedup": round(t_single / t_step, 2),
                      "max_pose_diff_vs_batched_m": dmax}
            log(f"[bench] single-scan path {t_single * 1e3:.2f} ms/step")

        gt_err = [pose_err(T_gpu[s], case.T_gt[s]) for s in range(S)]

        # ---------------- the same batch run to convergence (secondary line)
        conv = None
        if not args.no_converged:
            prm_c = far.align_params(case.tau, case.kappa, max_iters=args.conv_iters,
                                     eps=args.conv_eps, recenter=1, precision=prec)

            def step_c():
                far.far_scan_covariances_batch_packed(src, offs, case.voxel_size, case.k,
                                                      packed_buf, out=(cov_buf, val_buf))
                T.copy_(T0)
                far.far_gicp_align_batch_packed(gm.h, packed_buf, offs, T, prm_c,
                                                stats=stats_buf)

            step_c()
            stream.synchronize()
            n_c = max(1, min(args.steps, 5))
            t0 = time.perf_counter()
            for _ in range(n_c):
                step_c()
            stream.synchronize()
            t_c = (time.perf_counter() - t0) / n_c
            st_c = far.decode_stats(stats_buf)
            T_c = T.cpu().numpy().reshape(S, 4, 4)
            it_c = st_c["iters"].astype(np.int64)
            lins_c = int(np.sum((it_c + (st_c["status"] != 0)) * sizes))
            e_c = [pose_err(T_c[s], case.T_gt[s]) for s in range(S)]
            conv = {"iters_max": args.conv_iters, "eps": args.conv_eps,
                    "ms_per_step": round(t_c * 1e3, 3), "scans_per_s": round(S / t_c, 2),
                    "points_per_s": round(lins_c / t_c, 1),
                    "iterations": {"min": int(it_c.min()), "median": float(np.median(it_c)),
                                   "max": int(it_c.max()),
                                   "converged": int(st_c["converged"].sum())},
                    "pose_err_vs_gt": {"median_m": float(np.median([e[0] for e in e_c])),
                                       "max_m": max(e[0] for e in e_c),
                                       "median_deg": float(np.median([e[1] for e in e_c])),
                                       "max_deg": max(e[1] for e in e_c),
                                       "scans_over_0.1m": int(sum(e[0] > 0.1 for e in e_c)),
                                       "scans_over_0.05m": int(sum(e[0] > 0.05 for e in e_c))}}
            log(f"[bench] converged run: {t_c * 1e3:.2f} ms/step, iterations "
                f"{it_c.min()}..{it_c.max()}, median GT error {conv['pose_err_vs_gt']['median_m']:.4f} m")

        rows = None
        if not args.no_rows:
            t_rows = time.time()
            rows = next_rows(far, synth, np, torch, dev, stream, gm, case, T_fin, cov, val,
                             args.seed)
            log(f"[bench] rows {time.time() - t_rows:.1f}s: {rows}")

        # ---------------- CPU oracle on a bounded sample of the same workload
        cpu = None
        oracle_err = None
        if not args.no_cpu_baseline:
            from oracle import far_oracle as O
            om = O.Map(case.voxel_size, case.max_pts_per_voxel, case.min_spacing, case.k,
                       point_capacity=case.map_capacity, voxel_capacity=case.map_capacity)
            t0 = time.time()
            for b in case.map_batches:
                om.insert(b, check=False)
                if om.size >= case.map_capacity:
                    break
            log(f"[bench] oracle map built in {time.time() - t0:.1f}s ({om.size} points)")
            ns = min(args.cpu_sample_scans, S)

            def oracle_sample():
                t0 = time.perf_counter()
                o_lins, o_res = 0, []
                for s in range(ns):
                    oc, ov = O.scan_covariances(case.scans[s], case.voxel_size, case.k)
                    r = om.align(case.scans[s], oc.astype(np.float32), ov, case.T0[s], case.tau,
                                 case.kappa, max_iters=args.iters, eps=args.eps)
                    o_res.append(r)
                    o_lins += (r["iters"] + (1 if r["status"] else 0)) * case.scans[s].shape[1]
                return o_lins, time.perf_counter() - t0, o_res

            threads = O.get_threads()
            o_lins, t_cpu, o_res = oracle_sample()
            O.set_threads(1)
            o_lins1, t_cpu1, _ = oracle_sample()
            O.set_threads(threads)
            cpu = {"value": round(o_lins / t_cpu, 1), "unit": "points/s", "cores": threads,
                   "kind": "oracle", "cpu_model": cpu_model(),
                   "sample": f"{ns} of {S} scans ({int(sizes[:ns].sum())} points): FP64 oracle "
                             f"scan covariances + align, {args.iters} GN iterations max, "
                             f"{t_cpu:.2f} s at {threads} threads, {t_cpu1:.2f} s at 1",
                   "one_core": {"value": round(o_lins1 / t_cpu1, 1), "cores": 1}}
            log(f"[bench] oracle: {t_cpu:.2f} s at {threads} threads, {t_cpu1:.2f} s at 1 "
                f"({cpu['cpu_model']})")
            oracle_err = [pose_err(T_gpu[s], o_res[s]["T"]) for s in range(ns)]

    result = {
        "metric": "GICP linearize+kNN points/s and scans/s on 1 MI355X; % HBM roofline; pose err",
        "value": round(point_lins / t_step, 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == far.FAR_PREC_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"batched uneven scans: {S} spinning-LiDAR scans "
                               f"({N} points, {int(sizes.min())}..{int(sizes.max())} per scan) "
                               f"vs a {mstats['n_points']}-point voxel map (v=1 m, N_max=20, k=5), "
                               f"{args.iters} GN iterations max, eps={args.eps}",
                   "scans": S, "points": N, "map_points": mstats["n_points"],
                   "map_voxels": mstats["n_voxels"], "iters": args.iters, "eps": args.eps,
                   "parallelism": "single GPU"},
        "scans_per_s": round(S / t_step, 2),
        "point_linearizations_per_step": point_lins,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": roof_extra["traffic"],
                     "kernel": "linearisation",
                     "avg_launch_us": round(avg_launch_ms * 1e3, 2),
                     "algorithmic_bytes_per_launch": round(bytes_per_launch),
                     "algorithmic_bytes_union_per_launch": round(bytes_union_per_launch),
                     "copy_gbps": roof_extra["copy_gbps"],
                     "frac_of_copy": roof_extra["frac_of_copy"],
                     "l2_hit": roof_extra["l2_hit"], "valu_frac": roof_extra["valu_frac"],
                     "lds_frac": roof_extra["lds_frac"],
                     "ta_busy_frac": roof_extra.get("ta_busy_frac"),
                     "l2_read_latency_cycles": roof_extra.get("l2_read_latency_cycles"),
                     "kernel_sources_sha256_16": fp},
        "covariances": cov_row,
        "pipelined_two_streams": piped,
        "converged": conv,
        "cpu_baseline": cpu,
        "single_scan_path": single,
        "pose_err_vs_gt": {"max_m": max(e[0] for e in gt_err),
                           "max_deg": max(e[1] for e in gt_err),
                           "median_m": float(np.median([e[0] for e in gt_err])),
                           "median_deg": float(np.median([e[1] for e in gt_err])),
                           "scans_over_0.1m": int(sum(e[0] > 0.1 for e in gt_err))},
        "pose_err_vs_oracle": None if oracle_err is None else
        {"max_m": max(e[0] for e in oracle_err), "max_deg": max(e[1] for e in oracle_err),
         "scans": len(oracle_err)},
        "schedule": schedule,
        "rows": rows,
        "map_build": {"seconds": round(t_map, 3), "candidates": inserted,
                      "mean_probe": mstats["mean_probe"], "max_probe": mstats["max_probe"],
                      "load_factor": mstats["load_factor"]},
    }
    result["roofline"]["kernel"] = (
        f"linearisation at tile {tile}: k_cert<{tile}> + k_search + "
        f"k_linearize<{'double' if prec == far.FAR_PREC_FP64 else 'float'}, false, {tile}, "
        f"false, false, false> (the first iteration: k_linearize<..., true> with its own search)")
    print(json.dumps(result), flush=True)
    gm.close()


if __name__ == "__main__":
    main()
