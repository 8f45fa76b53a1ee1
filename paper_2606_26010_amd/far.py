"""Thin ctypes binding of libfar.so, with the C ABI's names (include/far.h).

Argument marshalling only: torch CUDA tensors supply device pointers and the
current HIP stream; every step of the computation runs in the library's HIP
kernels.  The library is loaded on first use; if it is missing, every call
raises (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfar.so")
_lib = None

FAR_OK, FAR_E_INVALID, FAR_E_CAPACITY, FAR_E_HIP, FAR_E_NOT_PD, FAR_E_FEW_CORR, \
    FAR_E_UNSUPPORTED = range(7)
FAR_PREC_FP32, FAR_PREC_FP64 = 0, 1
FAR_OPT_NO_SA = 0x100


class far_map_params_t(C.Structure):
    _fields_ = [("voxel_size", C.c_double), ("max_pts_per_voxel", C.c_int32),
                ("min_spacing", C.c_double), ("point_capacity", C.c_int64),
                ("voxel_capacity", C.c_int64), ("k_cov", C.c_int32)]


class far_lin_t(C.Structure):
    _fields_ = [("H", C.c_double * 36), ("b", C.c_double * 6), ("cost", C.c_double),
                ("n_inliers", C.c_int64)]


class far_align_params_t(C.Structure):
    _fields_ = [("tau", C.c_double), ("kappa", C.c_double), ("max_iters", C.c_int32),
                ("eps", C.c_double), ("recenter", C.c_int32), ("precision", C.c_int32)]


class far_align_stats_t(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("status", C.c_int32),
                ("reserved", C.c_int32), ("last", far_lin_t)]


class far_map_stats_t(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("n_voxels", C.c_int64), ("table_slots", C.c_int64),
                ("load_factor", C.c_double), ("mean_probe", C.c_double),
                ("max_probe", C.c_int32), ("max_pts_per_voxel", C.c_int32),
                ("voxel_size", C.c_double), ("min_spacing", C.c_double),
                ("bytes_device", C.c_int64)]


class far_schedule_t(C.Structure):
    _fields_ = [("tile", C.c_int32), ("fine_cells", C.c_int32)]


class far_threshold_t(C.Structure):
    _fields_ = [("sigma0", C.c_double), ("r_max", C.c_double), ("min_motion", C.c_double),
                ("sse", C.c_double), ("n_samples", C.c_int64)]


class far_odometry_params_t(C.Structure):
    _fields_ = [("downsample", C.c_double), ("sigma0", C.c_double), ("r_max", C.c_double),
                ("min_motion", C.c_double), ("max_iters", C.c_int32), ("eps", C.c_double),
                ("precision", C.c_int32), ("asmd", C.c_int32), ("r_near", C.c_double),
                ("evict_radius", C.c_double)]


class far_odometry_stats_t(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("n_raw", C.c_int64),
                ("n_down", C.c_int64), ("n_inserted", C.c_int64), ("map_full", C.c_int32),
                ("reserved", C.c_int32), ("n_evicted", C.c_int64), ("asmd_mean", C.c_double),
                ("tau", C.c_double), ("kappa", C.c_double),
                ("deviation", C.c_double), ("T_pred", C.c_double * 16), ("last", far_lin_t),
                ("t_ref", C.c_double)]


STATS_DTYPE = np.dtype([("iters", np.int32), ("converged", np.int32), ("status", np.int32),
                        ("reserved", np.int32), ("H", np.float64, (36,)),
                        ("b", np.float64, (6,)), ("cost", np.float64),
                        ("n_inliers", np.int64)])
assert STATS_DTYPE.itemsize == C.sizeof(far_align_stats_t)

_P = C.c_void_p
_SIGS = {
    "far_map_create": (C.c_int, [C.POINTER(far_map_params_t), _P, C.POINTER(_P)]),
    "far_map_destroy": (C.c_int, [_P]),
    "far_map_insert": (C.c_int, [_P, _P, C.c_int64, _P, _P, C.POINTER(C.c_int64)]),
    "far_map_knn": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.c_double, _P, _P, _P, _P]),
    "far_scan_covariances": (C.c_int, [_P, C.c_int64, C.c_double, C.c_int32, _P, _P, _P]),
    "far_scan_covariances_batch": (C.c_int, [_P, _P, C.c_int32, C.c_int64, C.c_double,
                                             C.c_int32, _P, _P, _P]),
    "far_scan_covariances_batch_order": (C.c_int, [_P, _P, C.c_int32, C.c_int64, C.c_double,
                                                   C.c_int32, _P, _P, _P, _P]),
    "far_scan_covariances_batch_packed": (C.c_int, [_P, _P, C.c_int32, C.c_int64, C.c_double,
                                                    C.c_int32, _P, _P, _P, _P]),
    "far_set_covariance_regularisation": (C.c_int, [C.c_int32]),
    "far_get_covariance_regularisation": (C.c_int, [C.POINTER(C.c_int32)]),
    "far_timing_enable": (C.c_int, [C.c_int32]),
    "far_scratch_release": (C.c_int, []),
    "far_scratch_reserved": (C.c_int, [C.POINTER(C.c_int64)]),
    "far_timing_read": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]),
    "far_timing_read_kind": (C.c_int, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                       C.c_int32]),
    "far_gicp_linearize": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.POINTER(C.c_double),
                                     C.c_double, C.c_double, C.POINTER(C.c_double),
                                     C.c_int32, _P, C.POINTER(far_lin_t), _P]),
    "far_gicp_linearize_async": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.POINTER(C.c_double),
                                           C.c_double, C.c_double, C.POINTER(C.c_double),
                                           C.c_int32, _P, _P, _P]),
    "far_map_reserve": (C.c_int, [_P, C.c_int64, C.c_int32, _P]),
    "far_set_linearize_grid": (C.c_int, [C.c_int32]),
    "far_get_linearize_grid": (C.c_int, [C.POINTER(C.c_int32)]),
    "far_gicp_gradient": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.POINTER(C.c_double),
                                    C.c_double, C.c_double, C.POINTER(C.c_double), C.c_int32,
                                    C.POINTER(C.c_double), C.POINTER(C.c_double), _P,
                                    C.POINTER(C.c_double), C.POINTER(C.c_int64), _P]),
    "far_gicp_align": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.POINTER(C.c_double),
                                 C.POINTER(far_align_params_t), C.POINTER(C.c_double),
                                 C.POINTER(far_align_stats_t), _P]),
    "far_gicp_align_batch": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, _P, _P, _P,
                                       C.POINTER(far_align_params_t), _P, _P]),
    "far_gicp_align_batch_ordered": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, _P, _P, _P,
                                               _P, C.POINTER(far_align_params_t), _P, _P]),
    "far_gicp_align_batch_packed": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, _P,
                                              C.POINTER(far_align_params_t), _P, _P]),
    "far_map_stats": (C.c_int, [_P, C.POINTER(far_map_stats_t), _P]),
    "far_map_export": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.POINTER(C.c_int64), _P]),
    "far_voxel_downsample": (C.c_int, [_P, C.c_int64, C.c_double, _P, _P,
                                       C.POINTER(C.c_int64), _P]),
    "far_transform_points": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_double), _P, _P]),
    "far_gicp_gradient_batch": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, _P, _P, _P, _P,
                                          C.c_double, C.c_double, C.c_int32, _P, _P, _P, _P,
                                          _P, _P]),
    "far_undistort": (C.c_int, [_P, _P, C.c_int64, _P, _P, C.c_int32, _P, _P, _P]),
    "far_undistort_batch": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, _P, _P, _P, _P, _P,
                                      _P]),
    "far_undistort_batch_noalloc": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, _P, _P, _P,
                                              _P, _P, _P]),
    "far_threshold_init": (C.c_int, [C.POINTER(far_threshold_t), C.c_double, C.c_double,
                                     C.c_double]),
    "far_threshold_update": (C.c_int, [C.POINTER(far_threshold_t), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "far_threshold_get": (C.c_int, [C.POINTER(far_threshold_t), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]),
    "far_odometry_create": (C.c_int, [_P, C.POINTER(far_odometry_params_t),
                                      C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(_P)]),
    "far_odometry_step": (C.c_int, [_P, _P, C.c_int64, C.POINTER(C.c_double),
                                    C.POINTER(far_odometry_stats_t), _P]),
    "far_odometry_step_timed": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P, C.c_int32,
                                          C.POINTER(C.c_double), _P, _P]),
    "far_odometry_destroy": (C.c_int, [_P]),
    "far_map_get_schedule": (C.c_int, [_P, C.POINTER(far_schedule_t)]),
    "far_map_set_schedule": (C.c_int, [_P, C.POINTER(far_schedule_t)]),
    "far_autotune": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, _P, _P, _P,
                               C.POINTER(far_align_params_t), C.c_int32,
                               C.POINTER(far_schedule_t), C.POINTER(C.c_double), _P]),
    "far_set_covariance_schedule": (C.c_int, [C.c_int32]),
    "far_get_covariance_schedule": (C.c_int, [C.POINTER(C.c_int32)]),
    "far_autotune_covariances": (C.c_int, [_P, _P, C.c_int32, C.c_int64, C.c_double, C.c_int32,
                                           _P, _P, C.c_int32, C.POINTER(C.c_int32),
                                           C.POINTER(C.c_double), _P]),
    "far_asmd_caps": (C.c_int, [_P, _P, C.c_int64, C.c_double, C.c_int32, C.c_int32,
                                C.c_double, C.c_double, _P, C.POINTER(C.c_double), _P]),
    "far_map_evict": (C.c_int, [_P, C.POINTER(C.c_double), C.c_double, C.POINTER(C.c_int64),
                                _P]),
    "far_status_str": (C.c_char_p, [C.c_int]),
    "far_last_error": (C.c_char_p, []),
}


class FarError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().far_last_error().decode(errors="replace")
        super().__init__(f"{where}: {lib().far_status_str(status).decode()} ({status}): {msg}")
        self.status = status


def lib():
    """Load libfar.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2606_26010_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status, where, ok=(FAR_OK,)):
    if status not in ok:
        raise FarError(status, where)
    return status


def _dev(t: torch.Tensor | None, dtype, name):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous {dtype} tensor on the GPU")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _pts(t, name="xyz"):
    if t.dim() != 2 or t.shape[0] != 3:
        raise ValueError(f"{name} must be SoA [3, n]")
    return _dev(t, torch.float32, name), t.shape[1]


def _mat4(T):
    a = np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(16))
    return (C.c_double * 16)(*a)


# ---------------------------------------------------------------- functions
def far_map_create(voxel_size, max_pts_per_voxel, min_spacing=-1.0, point_capacity=1 << 20,
                   voxel_capacity=0, k_cov=5, stream=None):
    p = far_map_params_t(voxel_size, max_pts_per_voxel, min_spacing, point_capacity,
                         voxel_capacity, k_cov)
    h = C.c_void_p()
    _check(lib().far_map_create(C.byref(p), _stream(stream), C.byref(h)), "far_map_create")
    return h


def far_map_destroy(h):
    _check(lib().far_map_destroy(h), "far_map_destroy")


def far_map_insert(h, xyz, voxel_cap=None, stream=None, raise_on=True):
    """Returns (status, n_accepted); raises on errors other than capacity unless
    raise_on is False."""
    p, n = _pts(xyz)
    acc = C.c_int64(0)
    st = lib().far_map_insert(h, p, n, _dev(voxel_cap, torch.int32, "voxel_cap"),
                              _stream(stream), C.byref(acc))
    if raise_on:
        _check(st, "far_map_insert", ok=(FAR_OK, FAR_E_CAPACITY))
    return st, acc.value


def far_map_knn(h, q, k, radius, want_d2=True, stream=None):
    p, n = _pts(q, "q")
    dev = q.device
    idx = torch.empty((n, k), dtype=torch.int32, device=dev)
    d2 = torch.empty((n, k), dtype=torch.float32, device=dev) if want_d2 else None
    cnt = torch.empty(n, dtype=torch.int32, device=dev)
    _check(lib().far_map_knn(h, p, n, k, radius, _dev(idx, torch.int32, "idx"),
                             _dev(d2, torch.float32, "d2"), _dev(cnt, torch.int32, "count"),
                             _stream(stream)), "far_map_knn")
    return idx, d2, cnt


def far_scan_covariances(xyz, voxel_size, k, stream=None):
    p, n = _pts(xyz)
    cov = torch.empty((6, n), dtype=torch.float32, device=xyz.device)
    val = torch.empty(n, dtype=torch.uint8, device=xyz.device)
    _check(lib().far_scan_covariances(p, n, voxel_size, k, _dev(cov, torch.float32, "cov6"),
                                      _dev(val, torch.uint8, "valid"), _stream(stream)),
           "far_scan_covariances")
    return cov, val


def far_scan_covariances_batch(xyz, offsets, voxel_size, k, out=None, stream=None,
                               order=None):
    """order: an int32 tensor [n] on the GPU (far_scan_covariances_batch_order:
    it receives the grid's sorted order) or None."""
    p, n = _pts(xyz)
    S = offsets.shape[0] - 1
    if out is None:
        cov = torch.empty((6, n), dtype=torch.float32, device=xyz.device)
        val = torch.empty(n, dtype=torch.uint8, device=xyz.device)
    else:
        cov, val = out
    if order is None:
        _check(lib().far_scan_covariances_batch(p, _dev(offsets, torch.int64, "offsets"), S, n,
                                                voxel_size, k, _dev(cov, torch.float32, "cov6"),
                                                _dev(val, torch.uint8, "valid"), _stream(stream)),
               "far_scan_covariances_batch")
    else:
        if order.numel() != n:
            raise ValueError("order must hold one entry per point")
        _check(lib().far_scan_covariances_batch_order(
            p, _dev(offsets, torch.int64, "offsets"), S, n, voxel_size, k,
            _dev(cov, torch.float32, "cov6"), _dev(val, torch.uint8, "valid"),
            _dev(order, torch.int32, "order"), _stream(stream)),
            "far_scan_covariances_batch_order")
    return cov, val


def far_scan_covariances_batch_order(xyz, offsets, voxel_size, k, order, out=None,
                                     stream=None):
    """far_scan_covariances_batch that also fills order (int32 [n] on the GPU)
    with the grid's sorted order."""
    return far_scan_covariances_batch(xyz, offsets, voxel_size, k, out=out, stream=stream,
                                      order=order)


def far_scan_covariances_batch_packed(xyz, offsets, voxel_size, k, packed, out=None,
                                      stream=None):
    """far_scan_covariances_batch that also writes the align's packed source
    into packed (a float32 tensor of 10 n values on the GPU: A float4 [n],
    B float4 [n], C float2 [n] in the grid's order)."""
    p, n = _pts(xyz)
    S = offsets.shape[0] - 1
    if out is None:
        cov = torch.empty((6, n), dtype=torch.float32, device=xyz.device)
        val = torch.empty(n, dtype=torch.uint8, device=xyz.device)
    else:
        cov, val = out
    if packed.numel() != 10 * n:
        raise ValueError("packed must hold 10 floats per point")
    _check(lib().far_scan_covariances_batch_packed(
        p, _dev(offsets, torch.int64, "offsets"), S, n, voxel_size, k,
        _dev(cov, torch.float32, "cov6"), _dev(val, torch.uint8, "valid"),
        _dev(packed, torch.float32, "packed"), _stream(stream)),
        "far_scan_covariances_batch_packed")
    return cov, val


FAR_REG_EQ1, FAR_REG_PLANE = 0, 1


def far_set_covariance_regularisation(mode: int):
    _check(lib().far_set_covariance_regularisation(int(mode)),
           "far_set_covariance_regularisation")


def far_get_covariance_regularisation() -> int:
    v = C.c_int32(0)
    _check(lib().far_get_covariance_regularisation(C.byref(v)),
           "far_get_covariance_regularisation")
    return v.value


def far_scratch_release():
    _check(lib().far_scratch_release(), "far_scratch_release")


def far_scratch_reserved() -> int:
    """Bytes the current device's scratch pool holds."""
    v = C.c_int64(0)
    _check(lib().far_scratch_reserved(C.byref(v)), "far_scratch_reserved")
    return v.value


def far_timing_enable(on: bool):
    _check(lib().far_timing_enable(1 if on else 0), "far_timing_enable")


FAR_TIME_LINEARIZE, FAR_TIME_UNDISTORT, FAR_TIME_UNDISTORT_APPLY = 0, 1, 2
FAR_TIME_GRADIENT, FAR_TIME_ASMD, FAR_TIME_EVICT, FAR_TIME_COVARIANCES = 3, 4, 5, 6


def far_timing_read_kind(kind: int, reset: bool = False):
    """(summed ms, count) of the event-timed intervals of one kind."""
    ms, n = C.c_double(0), C.c_int64(0)
    _check(lib().far_timing_read_kind(kind, C.byref(ms), C.byref(n), 1 if reset else 0),
           "far_timing_read_kind")
    return ms.value, n.value


def far_timing_read(reset: bool = False):
    ms, n = C.c_double(0), C.c_int64(0)
    _check(lib().far_timing_read(C.byref(ms), C.byref(n), 1 if reset else 0),
           "far_timing_read")
    return ms.value, n.value


def _lin_dict(lin: far_lin_t):
    return dict(H=np.array(lin.H[:]).reshape(6, 6), b=np.array(lin.b[:]), cost=lin.cost,
                n_inliers=lin.n_inliers)


def far_gicp_linearize(h, src, cov6, valid, T, tau, kappa, c=None, precision=FAR_PREC_FP32,
                       want_corr=False, stream=None):
    p, n = _pts(src, "src")
    corr = torch.empty(n, dtype=torch.int32, device=src.device) if want_corr else None
    cc = None if c is None else (C.c_double * 3)(*[float(x) for x in c])
    out = far_lin_t()
    _check(lib().far_gicp_linearize(h, p, _dev(cov6, torch.float32, "cov6"),
                                    _dev(valid, torch.uint8, "valid"), n, _mat4(T), tau, kappa,
                                    cc, precision, _dev(corr, torch.int32, "corr"),
                                    C.byref(out), _stream(stream)), "far_gicp_linearize")
    d = _lin_dict(out)
    if want_corr:
        d["corr"] = corr
    return d


LIN_WORDS = C.sizeof(far_lin_t) // 8


def far_gicp_linearize_async(h, src, cov6, valid, T, tau, kappa, out, c=None,
                             precision=FAR_PREC_FP32, corr=None, stream=None):
    """far_gicp_linearize with the result written to out, a float64 device
    tensor of LIN_WORDS words (decode with lin_from_words); no host sync."""
    p, n = _pts(src, "src")
    if out.numel() < LIN_WORDS:
        raise ValueError(f"out must hold {LIN_WORDS} float64 words")
    cc = None if c is None else (C.c_double * 3)(*[float(x) for x in c])
    _check(lib().far_gicp_linearize_async(h, p, _dev(cov6, torch.float32, "cov6"),
                                          _dev(valid, torch.uint8, "valid"), n, _mat4(T), tau,
                                          kappa, cc, precision, _dev(corr, torch.int32, "corr"),
                                          _dev(out, torch.float64, "out"), _stream(stream)),
           "far_gicp_linearize_async")
    return out


def lin_from_words(words):
    """Decode a far_lin_t read back as LIN_WORDS float64 words."""
    buf = np.ascontiguousarray(np.asarray(words, dtype=np.float64)[:LIN_WORDS])
    out = far_lin_t.from_buffer_copy(buf.tobytes())
    return _lin_dict(out)


def far_set_linearize_grid(blocks_per_cu):
    _check(lib().far_set_linearize_grid(int(blocks_per_cu)), "far_set_linearize_grid")


def far_get_linearize_grid():
    v = C.c_int32(0)
    _check(lib().far_get_linearize_grid(C.byref(v)), "far_get_linearize_grid")
    return v.value


def far_map_reserve(h, max_points, max_scans=1, stream=None):
    _check(lib().far_map_reserve(h, int(max_points), int(max_scans), _stream(stream)),
           "far_map_reserve")


def far_gicp_gradient(h, src, cov6, valid, T, tau, kappa, c=None, precision=FAR_PREC_FP32,
                      want_src=True, stream=None):
    """dict(grad_T [3, 4], grad_twist [6], grad_src [3, n] device tensor or None,
    cost, n_inliers)."""
    p, n = _pts(src, "src")
    gs = torch.empty((3, max(n, 1)), dtype=torch.float32, device=src.device) if want_src else None
    gT, gw = (C.c_double * 12)(), (C.c_double * 6)()
    cost, cnt = C.c_double(0), C.c_int64(0)
    cc = None if c is None else (C.c_double * 3)(*[float(x) for x in c])
    _check(lib().far_gicp_gradient(h, p, _dev(cov6, torch.float32, "cov6"),
                                   _dev(valid, torch.uint8, "valid"), n, _mat4(T), tau, kappa,
                                   cc, precision, gT, gw, _dev(gs, torch.float32, "grad_src"),
                                   C.byref(cost), C.byref(cnt), _stream(stream)),
           "far_gicp_gradient")
    return dict(grad_T=np.array(gT[:]).reshape(3, 4), grad_twist=np.array(gw[:]),
                grad_src=None if gs is None else gs[:, :n], cost=cost.value,
                n_inliers=cnt.value)


def align_params(tau, kappa, max_iters=10, eps=1e-6, recenter=1, precision=FAR_PREC_FP32,
                 sa=True):
    """sa=False sets FAR_OPT_NO_SA (pairs lacking a covariance are dropped)."""
    return far_align_params_t(tau, kappa, max_iters, eps, recenter,
                              precision | (0 if sa else FAR_OPT_NO_SA))


def far_gicp_align(h, src, cov6, valid, T0, params: far_align_params_t, stream=None):
    """Returns (status, T (4x4 numpy), stats dict)."""
    p, n = _pts(src, "src")
    Tout = (C.c_double * 16)()
    st = far_align_stats_t()
    status = lib().far_gicp_align(h, p, _dev(cov6, torch.float32, "cov6"),
                                  _dev(valid, torch.uint8, "valid"), n, _mat4(T0),
                                  C.byref(params), Tout, C.byref(st), _stream(stream))
    _check(status, "far_gicp_align", ok=(FAR_OK, FAR_E_NOT_PD, FAR_E_FEW_CORR))
    d = dict(iters=st.iters, converged=st.converged, status=st.status, **_lin_dict(st.last))
    return status, np.array(Tout[:]).reshape(4, 4), d


def far_gicp_align_batch(h, src, offsets, cov6, valid, T, params: far_align_params_t,
                         stats=None, stream=None, order=None):
    """T: float64 [S, 16] on the GPU (in/out).  stats: uint8 [S * sizeof] buffer or
    None (allocated).  order: None (the align sorts the source itself) or an
    int32 tensor [n] on the GPU (far_gicp_align_batch_ordered), e.g. the one
    far_scan_covariances_batch(..., order=...) filled.  Asynchronous; returns
    the stats buffer (decode with decode_stats after synchronising)."""
    p, n = _pts(src, "src")
    S = offsets.shape[0] - 1
    if stats is None:
        stats = torch.empty(S * STATS_DTYPE.itemsize, dtype=torch.uint8, device=src.device)
    args = (_dev(offsets, torch.int64, "offsets"), S, n, _dev(cov6, torch.float32, "cov6"),
            _dev(valid, torch.uint8, "valid"))
    rest = (_dev(T, torch.float64, "T"), C.byref(params), _dev(stats, torch.uint8, "stats"),
            _stream(stream))
    if order is None:
        _check(lib().far_gicp_align_batch(h, p, *args, *rest), "far_gicp_align_batch")
    else:
        if order.numel() != n:
            raise ValueError("order must hold one entry per point")
        _check(lib().far_gicp_align_batch_ordered(h, p, *args, _dev(order, torch.int32, "order"),
                                                  *rest), "far_gicp_align_batch_ordered")
    return stats


def far_gicp_align_batch_ordered(h, src, offsets, cov6, valid, order, T,
                                 params: far_align_params_t, stats=None, stream=None):
    """far_gicp_align_batch with the source packed in the given order."""
    return far_gicp_align_batch(h, src, offsets, cov6, valid, T, params, stats=stats,
                                stream=stream, order=order)


def far_gicp_align_batch_packed(h, packed, offsets, T, params: far_align_params_t, stats=None,
                                stream=None):
    """far_gicp_align_batch on a source already packed by
    far_scan_covariances_batch_packed (packed: float32 [10 n] on the GPU)."""
    n = packed.numel() // 10
    S = offsets.shape[0] - 1
    if stats is None:
        stats = torch.empty(S * STATS_DTYPE.itemsize, dtype=torch.uint8, device=packed.device)
    _check(lib().far_gicp_align_batch_packed(h, _dev(packed, torch.float32, "packed"),
                                             _dev(offsets, torch.int64, "offsets"), S, n,
                                             _dev(T, torch.float64, "T"), C.byref(params),
                                             _dev(stats, torch.uint8, "stats"),
                                             _stream(stream)),
           "far_gicp_align_batch_packed")
    return stats


def decode_stats(stats: torch.Tensor):
    return np.frombuffer(stats.cpu().numpy().tobytes(), dtype=STATS_DTYPE)


def far_map_stats(h, stream=None):
    s = far_map_stats_t()
    _check(lib().far_map_stats(h, C.byref(s), _stream(stream)), "far_map_stats")
    return {f: getattr(s, f) for f, _ in far_map_stats_t._fields_}


def far_map_export(h, capacity=None, device="cuda", stream=None):
    n = far_map_stats(h, stream)["n_points"] if capacity is None else capacity
    xyz = torch.empty((3, max(n, 1)), dtype=torch.float32, device=device)
    cov = torch.empty((6, max(n, 1)), dtype=torch.float32, device=device)
    val = torch.empty(max(n, 1), dtype=torch.uint8, device=device)
    out = C.c_int64(0)
    _check(lib().far_map_export(h, _dev(xyz, torch.float32, "xyz"),
                                _dev(cov, torch.float32, "cov6"),
                                _dev(val, torch.uint8, "valid"), n, C.byref(out),
                                _stream(stream)), "far_map_export")
    N = out.value
    if N == 0:
        return xyz[:, :0], cov[:, :0], val[:0]
    # SoA rows were written with stride N
    return (xyz.view(-1)[:3 * N].view(3, N), cov.view(-1)[:6 * N].view(6, N), val[:N])


class Map:
    """Owning wrapper of a far_map_t."""

    def __init__(self, voxel_size, max_pts_per_voxel, min_spacing=-1.0,
                 point_capacity=1 << 20, voxel_capacity=0, k_cov=5, stream=None):
        self.h = far_map_create(voxel_size, max_pts_per_voxel, min_spacing, point_capacity,
                                voxel_capacity, k_cov, stream)
        self.voxel_size = voxel_size

    def close(self):
        if getattr(self, "h", None):
            far_map_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, xyz, voxel_cap=None, stream=None):
        return far_map_insert(self.h, xyz, voxel_cap, stream)

    def knn(self, q, k, radius, stream=None):
        return far_map_knn(self.h, q, k, radius, stream=stream)

    def linearize(self, *a, **kw):
        return far_gicp_linearize(self.h, *a, **kw)

    def linearize_async(self, *a, **kw):
        return far_gicp_linearize_async(self.h, *a, **kw)

    def reserve(self, max_points, max_scans=1, stream=None):
        return far_map_reserve(self.h, max_points, max_scans, stream)

    def evict(self, center, radius, stream=None):
        return far_map_evict(self.h, center, radius, stream)

    def gradient(self, *a, **kw):
        return far_gicp_gradient(self.h, *a, **kw)

    def gradient_batch(self, *a, **kw):
        return far_gicp_gradient_batch(self.h, *a, **kw)

    def align(self, *a, **kw):
        return far_gicp_align(self.h, *a, **kw)

    def align_batch(self, *a, **kw):
        return far_gicp_align_batch(self.h, *a, **kw)

    def stats(self, stream=None):
        return far_map_stats(self.h, stream)

    def export(self, stream=None):
        return far_map_export(self.h, stream=stream)


def far_asmd_caps(xyz_sensor, xyz_map, v, k, nmax, r_near=20.0, r_max=120.0, stream=None):
    """(caps int32 device tensor [n], mean near-range points per voxel)."""
    ps, n = _pts(xyz_sensor, "xyz_sensor")
    pm, n2 = _pts(xyz_map, "xyz_map")
    if n2 != n:
        raise ValueError("xyz_sensor and xyz_map differ in size")
    caps = torch.empty(max(n, 1), dtype=torch.int32, device=xyz_sensor.device)
    mean = C.c_double(0)
    _check(lib().far_asmd_caps(ps, pm, n, v, k, nmax, r_near, r_max,
                               _dev(caps, torch.int32, "caps"), C.byref(mean), _stream(stream)),
           "far_asmd_caps")
    return caps[:n], mean.value


def far_map_evict(h, center, radius, stream=None):
    out = C.c_int64(0)
    cc = (C.c_double * 3)(*[float(x) for x in center])
    _check(lib().far_map_evict(h, cc, radius, C.byref(out), _stream(stream)), "far_map_evict")
    return out.value


def far_map_get_schedule(h):
    sc = far_schedule_t()
    _check(lib().far_map_get_schedule(h, C.byref(sc)), "far_map_get_schedule")
    return dict(tile=sc.tile, fine_cells=sc.fine_cells)


def far_map_set_schedule(h, tile=256, fine_cells=0):
    sc = far_schedule_t(tile, fine_cells)
    _check(lib().far_map_set_schedule(h, C.byref(sc)), "far_map_set_schedule")


def far_autotune(h, src, offsets, cov6, valid, T, params: far_align_params_t, reps=3,
                 stream=None):
    """Returns (best schedule dict, times in ms per candidate: tiles 128, 256,
    512, each with the voxel search then the fine cells; -1 = not run)."""
    p, n = _pts(src, "src")
    S = offsets.shape[0] - 1
    best = far_schedule_t()
    ms = (C.c_double * 6)()
    _check(lib().far_autotune(h, p, _dev(offsets, torch.int64, "offsets"), S, n,
                              _dev(cov6, torch.float32, "cov6"), _dev(valid, torch.uint8, "valid"),
                              _dev(T, torch.float64, "T"), C.byref(params), reps, C.byref(best),
                              ms, _stream(stream)), "far_autotune")
    return dict(tile=best.tile, fine_cells=best.fine_cells), list(ms)


def far_set_covariance_schedule(dense_threshold):
    _check(lib().far_set_covariance_schedule(dense_threshold), "far_set_covariance_schedule")


def far_get_covariance_schedule():
    v = C.c_int32(0)
    _check(lib().far_get_covariance_schedule(C.byref(v)), "far_get_covariance_schedule")
    return v.value


def far_autotune_covariances(xyz, offsets, voxel_size, k, reps=3, stream=None):
    """Returns (best dense threshold, times in ms for 0, 16, 32, 64, 128)."""
    p, n = _pts(xyz, "xyz")
    S = offsets.shape[0] - 1
    cov = torch.empty((6, max(n, 1)), dtype=torch.float32, device=xyz.device)
    val = torch.empty(max(n, 1), dtype=torch.uint8, device=xyz.device)
    best = C.c_int32(0)
    ms = (C.c_double * 5)()
    _check(lib().far_autotune_covariances(p, _dev(offsets, torch.int64, "offsets"), S, n,
                                          voxel_size, k, _dev(cov, torch.float32, "cov6"),
                                          _dev(val, torch.uint8, "valid"), reps, C.byref(best),
                                          ms, _stream(stream)), "far_autotune_covariances")
    return best.value, list(ms)


def far_voxel_downsample(xyz, v, want_keep=False, stream=None):
    """Returns (points SoA [3, m] float32 on the device, kept indices or None)."""
    p, n = _pts(xyz, "xyz")
    out = torch.empty(3 * max(n, 1), dtype=torch.float32, device=xyz.device)
    keep = torch.empty(max(n, 1), dtype=torch.int32, device=xyz.device) if want_keep else None
    m = C.c_int64(0)
    _check(lib().far_voxel_downsample(p, n, v, _dev(out, torch.float32, "out"),
                                      _dev(keep, torch.int32, "keep"), C.byref(m),
                                      _stream(stream)), "far_voxel_downsample")
    m = m.value
    pts = out[:3 * m].view(3, m)
    return pts, (keep[:m] if want_keep else None)


def far_transform_points(xyz, T, out=None, stream=None):
    p, n = _pts(xyz, "xyz")
    if out is None:
        out = torch.empty_like(xyz)
    _check(lib().far_transform_points(p, n, _mat4(T), _dev(out, torch.float32, "out"),
                                      _stream(stream)), "far_transform_points")
    return out


def _samples(vel_t, vel):
    if vel_t.dim() != 1 or vel.dim() != 2 or vel.shape[1] != 6 or vel.shape[0] != vel_t.shape[0]:
        raise ValueError("vel_t must be [m] and vel [m, 6]")
    return (_dev(vel_t, torch.float64, "vel_t"), _dev(vel, torch.float64, "vel"),
            vel_t.shape[0])


def far_gicp_gradient_batch(h, src, offsets, cov6, valid, T, tau, kappa, c=None,
                            precision=FAR_PREC_FP32, want_src=True, stream=None):
    """Batched gradient, all on the device: dict(grad_T [S, 3, 4], grad_twist
    [S, 6], grad_src [3, n] or None, cost [S], n_inliers [S]) as tensors."""
    p, n = _pts(src, "src")
    S = offsets.shape[0] - 1
    if T.shape != (S, 16) and T.shape != (S, 4, 4):
        raise ValueError("T must be [S, 16] or [S, 4, 4]")
    dv = src.device
    gT = torch.empty((S, 12), dtype=torch.float64, device=dv)
    gw = torch.empty((S, 6), dtype=torch.float64, device=dv)
    cost = torch.empty(S, dtype=torch.float64, device=dv)
    cnt = torch.empty(S, dtype=torch.int64, device=dv)
    gs = torch.empty((3, max(n, 1)), dtype=torch.float32, device=dv) if want_src else None
    _check(lib().far_gicp_gradient_batch(
        h, p, _dev(offsets, torch.int64, "offsets"), S, n, _dev(cov6, torch.float32, "cov6"),
        _dev(valid, torch.uint8, "valid"), _dev(T, torch.float64, "T"),
        _dev(c, torch.float64, "c"), tau, kappa, precision, _dev(gT, torch.float64, "grad_T"),
        _dev(gw, torch.float64, "grad_twist"), _dev(gs, torch.float32, "grad_src"),
        _dev(cost, torch.float64, "cost"), _dev(cnt, torch.int64, "n_inliers"), _stream(stream)),
        "far_gicp_gradient_batch")
    return dict(grad_T=gT.view(S, 3, 4), grad_twist=gw, grad_src=None if gs is None else gs[:, :n],
                cost=cost, n_inliers=cnt)


def far_undistort(xyz, t, vel_t, vel, out=None, stream=None):
    """Motion undistortion of one scan: (points [3, n] in the frame of the
    scan's last point time, t_ref as a float64 device tensor [1])."""
    p, n = _pts(xyz, "xyz")
    if t.dim() != 1 or t.shape[0] != n:
        raise ValueError("t must be [n]")
    pt, pv, m = _samples(vel_t, vel)
    if out is None:
        out = torch.empty_like(xyz)
    t_ref = torch.empty(1, dtype=torch.float64, device=xyz.device)
    _check(lib().far_undistort(p, _dev(t, torch.float32, "t"), n, pt, pv, m,
                               _dev(out, torch.float32, "out"), _dev(t_ref, torch.float64, "t_ref"),
                               _stream(stream)), "far_undistort")
    return out, t_ref


def far_undistort_batch(xyz, t, offsets, vel_t, vel, vel_offsets, out=None, stream=None):
    """far_undistort over S scans: (points [3, n_total], t_ref [S])."""
    p, n = _pts(xyz, "xyz")
    if t.dim() != 1 or t.shape[0] != n:
        raise ValueError("t must be [n_total]")
    S = offsets.shape[0] - 1
    if vel_offsets.shape[0] != S + 1:
        raise ValueError("offsets and vel_offsets differ in scan count")
    pt, pv, _ = _samples(vel_t, vel)
    if out is None:
        out = torch.empty_like(xyz)
    t_ref = torch.empty(max(S, 1), dtype=torch.float64, device=xyz.device)
    _check(lib().far_undistort_batch(p, _dev(t, torch.float32, "t"),
                                     _dev(offsets, torch.int64, "offsets"), S, n, pt, pv,
                                     _dev(vel_offsets, torch.int64, "vel_offsets"),
                                     _dev(out, torch.float32, "out"),
                                     _dev(t_ref, torch.float64, "t_ref"), _stream(stream)),
           "far_undistort_batch")
    return out, t_ref[:S]


def far_undistort_batch_noalloc(xyz, t, offsets, vel_t, vel, vel_offsets, out, t_ref,
                                stream=None):
    """far_undistort_batch through the allocation-free entry point: the
    caller passes out [3, n_total] and t_ref [S] (float64); the library
    allocates nothing for the call."""
    p, n = _pts(xyz, "xyz")
    if t.dim() != 1 or t.shape[0] != n:
        raise ValueError("t must be [n_total]")
    S = offsets.shape[0] - 1
    if vel_offsets.shape[0] != S + 1:
        raise ValueError("offsets and vel_offsets differ in scan count")
    if out.shape != xyz.shape or t_ref.dim() != 1 or t_ref.shape[0] < S:
        raise ValueError("out must be [3, n_total] and t_ref [S]")
    pt, pv, _ = _samples(vel_t, vel)
    _check(lib().far_undistort_batch_noalloc(p, _dev(t, torch.float32, "t"),
                                             _dev(offsets, torch.int64, "offsets"), S, n, pt, pv,
                                             _dev(vel_offsets, torch.int64, "vel_offsets"),
                                             _dev(out, torch.float32, "out"),
                                             _dev(t_ref, torch.float64, "t_ref"),
                                             _stream(stream)),
           "far_undistort_batch_noalloc")
    return out, t_ref[:S]


def far_threshold_init(sigma0, r_max, min_motion=0.1):
    s = far_threshold_t()
    _check(lib().far_threshold_init(C.byref(s), sigma0, r_max, min_motion), "far_threshold_init")
    return s


def far_threshold_update(s: far_threshold_t, T_pred, T_est):
    d = C.c_double(0)
    _check(lib().far_threshold_update(C.byref(s), _mat4(T_pred), _mat4(T_est), C.byref(d)),
           "far_threshold_update")
    return d.value


def far_threshold_get(s: far_threshold_t):
    tau, kappa = C.c_double(0), C.c_double(0)
    _check(lib().far_threshold_get(C.byref(s), C.byref(tau), C.byref(kappa)), "far_threshold_get")
    return tau.value, kappa.value


def far_odometry_create(map_h, T_first, v_first=None, downsample=0.5, sigma0=1.0 / 3.0,
                        r_max=120.0, min_motion=0.1, max_iters=10, eps=5e-3,
                        precision=FAR_PREC_FP32, asmd=False, r_near=20.0, evict_radius=0.0):
    prm = far_odometry_params_t(downsample, sigma0, r_max, min_motion, max_iters, eps, precision,
                                1 if asmd else 0, r_near, evict_radius)
    h = C.c_void_p()
    _check(lib().far_odometry_create(map_h, C.byref(prm), _mat4(T_first),
                                     _mat4_or_none(v_first), C.byref(h)), "far_odometry_create")
    return h


def far_odometry_step(h, xyz, stream=None):
    """One scan [3, n] float32 on the device -> (T 4x4 numpy, stats dict)."""
    p, n = _pts(xyz, "xyz")
    T = (C.c_double * 16)()
    st = far_odometry_stats_t()
    _check(lib().far_odometry_step(h, p, n, T, C.byref(st), _stream(stream)),
           "far_odometry_step")
    return np.array(T[:]).reshape(4, 4), _odo_dict(st)


def far_odometry_step_timed(h, xyz, t, vel_t, vel, stream=None):
    """One raw scan [3, n] with point times t [n] and velocity samples
    (vel_t [m], vel [m, 6], float64), all on the device: undistorted, then
    as far_odometry_step -> (T, stats dict with t_ref)."""
    p, n = _pts(xyz, "xyz")
    if t.dim() != 1 or t.shape[0] != n:
        raise ValueError("t must be [n]")
    pt, pv, m = _samples(vel_t, vel)
    T = (C.c_double * 16)()
    st = far_odometry_stats_t()
    _check(lib().far_odometry_step_timed(h, p, _dev(t, torch.float32, "t"), n, pt, pv, m, T,
                                         C.byref(st), _stream(stream)),
           "far_odometry_step_timed")
    return np.array(T[:]).reshape(4, 4), _odo_dict(st)


def far_odometry_destroy(h):
    _check(lib().far_odometry_destroy(h), "far_odometry_destroy")


def _mat4_or_none(T):
    return None if T is None else _mat4(T)


class Threshold:
    """Adaptive threshold state (far_threshold_t), host-side."""

    def __init__(self, sigma0, r_max, min_motion=0.1):
        self.s = far_threshold_init(sigma0, r_max, min_motion)

    def update(self, T_pred, T_est):
        return far_threshold_update(self.s, T_pred, T_est)

    def get(self):
        return far_threshold_get(self.s)


def _odo_dict(st: far_odometry_stats_t):
    d = {f: getattr(st, f) for f, _ in far_odometry_stats_t._fields_
         if f not in ("T_pred", "last", "reserved")}
    d["T_pred"] = np.array(st.T_pred[:]).reshape(4, 4)
    d.update(_lin_dict(st.last))
    return d


class Odometry:
    """Owning wrapper of a far_odometry_t over a Map (which must outlive it)."""

    def __init__(self, map_, T_first, v_first=None, **kw):
        self.map = map_
        self._h = far_odometry_create(map_.h, T_first, v_first, **kw)

    def step(self, xyz, stream=None, times=None, vel_t=None, vel=None):
        """One scan; with per-point times and velocity samples it is
        undistorted first (far_odometry_step_timed)."""
        if times is not None:
            return far_odometry_step_timed(self._h, xyz, times, vel_t, vel, stream)
        return far_odometry_step(self._h, xyz, stream)

    def close(self):
        if getattr(self, "_h", None):
            far_odometry_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
