"""ctypes wrapper of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Every array crossing this wrapper is a C-contiguous numpy array; points are
SoA float32 [3, n], covariances SoA [6, n] (xx, xy, xz, yy, yz, zz), poses
row-major float64 [4, 4].
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None
_HERE = os.path.dirname(os.path.abspath(__file__))

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


def _opt(t):
    """Pointer argument that also accepts None."""
    class _P(C.c_void_p):
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return t.from_param(obj)
    return _P


class _ThresholdState(C.Structure):
    _fields_ = [("sigma0", C.c_double), ("r_max", C.c_double), ("min_motion", C.c_double),
                ("sse", C.c_double), ("n", C.c_int64)]


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(
                os.path.join(_HERE, "far_oracle.cpp")):
            _build.build()
        L = C.CDLL(path)
        L.orc_map_new.restype = C.c_void_p
        L.orc_map_new.argtypes = [C.c_double, C.c_int32, C.c_double, C.c_int32, C.c_int64, C.c_int64]
        L.orc_map_free.argtypes = [C.c_void_p]
        L.orc_map_size.restype = C.c_int64
        L.orc_map_size.argtypes = [C.c_void_p]
        L.orc_map_nvoxels.restype = C.c_int64
        L.orc_map_nvoxels.argtypes = [C.c_void_p]
        L.orc_map_insert.argtypes = [C.c_void_p, _f32p, C.c_int64, _opt(_i32p),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.orc_map_export.argtypes = [C.c_void_p, _opt(_f32p), _opt(_f32p), _opt(_u8p)]
        L.orc_map_knn.argtypes = [C.c_void_p, _f32p, C.c_int64, C.c_int32, C.c_double,
                                  _i32p, _opt(_f64p), _opt(_i32p)]
        L.orc_scan_covariances.argtypes = [_f32p, C.c_int64, C.c_double, C.c_int32, _f64p, _u8p]
        L.orc_linearize.argtypes = [C.c_void_p, _f32p, _f32p, _u8p, C.c_int64, _f64p,
                                    C.c_double, C.c_double, _opt(_f64p), _f64p, _f64p,
                                    C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                    _opt(_i32p), _opt(_f64p), C.c_int32]
        L.orc_align.argtypes = [C.c_void_p, _f32p, _f32p, _u8p, C.c_int64, _f64p,
                                C.c_double, C.c_double, C.c_int32, C.c_double, C.c_int32,
                                _f64p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                _f64p, _f64p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                C.c_int32]
        L.orc_voxel_keys.argtypes = [_f32p, C.c_int64, C.c_double, _i64p]
        L.orc_se3_exp.argtypes = [_f64p, _f64p]
        L.orc_cholesky_solve6.argtypes = [_f64p, _f64p, _f64p]
        L.orc_regularize_cov.argtypes = [_f64p, _f64p]
        L.orc_plane_cov.argtypes = [_f64p, _f64p]
        L.orc_jacobi3.argtypes = [_f64p, _f64p, _f64p]
        L.orc_set_cov_mode.argtypes = [C.c_int32]
        L.orc_touch_stats.argtypes = [C.c_void_p, _f32p, C.c_int64, _f64p,
                                      C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.orc_cost_fixed.argtypes = [C.c_void_p, _f64p, _f32p, _u8p, C.c_int64, _f64p,
                                     C.c_double, _i32p, C.POINTER(C.c_double)]
        L.orc_gradient.argtypes = [C.c_void_p, _f32p, _f32p, _u8p, C.c_int64, _f64p, C.c_double,
                                   C.c_double, _opt(_f64p), _f64p, _f64p, _opt(_f64p),
                                   C.POINTER(C.c_double), C.POINTER(C.c_int64), _opt(_i32p),
                                   C.c_int32]
        L.orc_asmd_caps.argtypes = [_f32p, _f32p, C.c_int64, C.c_double, C.c_int32, C.c_int32,
                                    C.c_double, C.c_double, _i32p, C.POINTER(C.c_double)]
        L.orc_map_evict.argtypes = [C.c_void_p, _f64p, C.c_double, C.POINTER(C.c_int64)]
        L.orc_fit_twist.argtypes = [_f64p, _f64p, C.c_int64, C.POINTER(C.c_double), _f64p,
                                    _f64p]
        L.orc_undistort.argtypes = [_f32p, _f32p, C.c_int64, _f64p, _f64p, C.c_int64, _f32p,
                                    C.POINTER(C.c_double)]
        L.orc_downsample.argtypes = [_f32p, C.c_int64, C.c_double, _i64p,
                                     C.POINTER(C.c_int64)]
        L.orc_transform.argtypes = [_f32p, C.c_int64, _f64p, _f32p]
        L.orc_threshold_init.argtypes = [C.POINTER(_ThresholdState), C.c_double, C.c_double,
                                         C.c_double]
        L.orc_threshold_update.restype = C.c_double
        L.orc_threshold_update.argtypes = [C.POINTER(_ThresholdState), _f64p, _f64p]
        L.orc_threshold_get.argtypes = [C.POINTER(_ThresholdState), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        _lib = L
    return _lib


def set_threads(n):
    """Threads of the oracle's OpenMP loops (timing only; results do not
    depend on it)."""
    lib().orc_set_threads(int(n))


def get_threads():
    return int(lib().orc_get_threads())


def _soa(xyz):
    a = np.ascontiguousarray(xyz, dtype=np.float32)
    assert a.ndim == 2 and a.shape[0] == 3, "points are SoA float32 [3, n]"
    return a


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


class Map:
    """Oracle voxel map (sequential capped insert, FP64 decisions)."""

    def __init__(self, voxel_size, max_pts_per_voxel, min_spacing, k_cov,
                 point_capacity=1 << 24, voxel_capacity=1 << 22):
        self._h = lib().orc_map_new(voxel_size, max_pts_per_voxel, min_spacing, k_cov,
                                    point_capacity, voxel_capacity)
        if not self._h:
            raise OracleError(1, "orc_map_new")
        self.voxel_size = voxel_size

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_map_free(self._h)
            self._h = None

    def insert(self, xyz, caps=None, check=True):
        a = _soa(xyz)
        n = a.shape[1]
        c = None if caps is None else np.ascontiguousarray(caps, dtype=np.int32)
        acc, skip = C.c_int64(0), C.c_int64(0)
        rc = lib().orc_map_insert(self._h, a, n, c, C.byref(acc), C.byref(skip))
        if check and rc != 0:
            raise OracleError(rc, "orc_map_insert")
        return (rc, acc.value, skip.value) if not check else acc.value

    @property
    def size(self):
        return lib().orc_map_size(self._h)

    @property
    def n_voxels(self):
        return lib().orc_map_nvoxels(self._h)

    def export(self):
        N = self.size
        xyz = np.zeros((3, N), np.float32)
        cov = np.zeros((6, N), np.float32)
        val = np.zeros(N, np.uint8)
        lib().orc_map_export(self._h, xyz, cov, val)
        return xyz, cov, val

    def knn(self, q, k, r):
        a = _soa(q)
        n = a.shape[1]
        idx = np.zeros((n, k), np.int32)
        d2 = np.zeros((n, k), np.float64)
        cnt = np.zeros(n, np.int32)
        rc = lib().orc_map_knn(self._h, a, n, k, r, idx, d2, cnt)
        if rc:
            raise OracleError(rc, "orc_map_knn")
        return idx, d2, cnt

    def linearize(self, src, cov6, valid, T, tau, kappa, c=None, want_corr=False,
                  want_detail=False, sa=True):
        """One linearisation; sa=False drops pairs lacking a covariance instead
        of the sparsity-aware point-to-point term."""
        a = _soa(src)
        n = a.shape[1]
        cov = np.ascontiguousarray(cov6, dtype=np.float32)
        val = np.ascontiguousarray(valid, dtype=np.uint8)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(16)
        cc = None if c is None else np.ascontiguousarray(c, dtype=np.float64)
        H = np.zeros(36); b = np.zeros(6)
        cost, cnt = C.c_double(0), C.c_int64(0)
        corr = np.zeros(n, np.int32) if want_corr else None
        det = np.zeros((n, 18)) if want_detail else None
        rc = lib().orc_linearize(self._h, a, cov, val, n, T, tau, kappa, cc, H, b,
                                 C.byref(cost), C.byref(cnt), corr, det, 1 if sa else 0)
        if rc:
            raise OracleError(rc, "orc_linearize")
        out = dict(H=H.reshape(6, 6), b=b, cost=cost.value, n_inliers=cnt.value)
        if want_corr:
            out["corr"] = corr
        if want_detail:
            out["detail"] = det
        return out

    def align(self, src, cov6, valid, T0, tau, kappa, max_iters=10, eps=1e-6, recenter=1,
              sa=True):
        a = _soa(src)
        n = a.shape[1]
        cov = np.ascontiguousarray(cov6, dtype=np.float32)
        val = np.ascontiguousarray(valid, dtype=np.uint8)
        T0 = np.ascontiguousarray(T0, dtype=np.float64).reshape(16)
        Tout = np.zeros(16)
        it, conv = C.c_int32(0), C.c_int32(0)
        H = np.zeros(36); b = np.zeros(6)
        cost, cnt = C.c_double(0), C.c_int64(0)
        rc = lib().orc_align(self._h, a, cov, val, n, T0, tau, kappa, max_iters, eps,
                             recenter, Tout, C.byref(it), C.byref(conv), H, b,
                             C.byref(cost), C.byref(cnt), 1 if sa else 0)
        return dict(status=rc, T=Tout.reshape(4, 4), iters=it.value, converged=conv.value,
                    H=H.reshape(6, 6), b=b, cost=cost.value, n_inliers=cnt.value)

    def cost_fixed(self, src64, cov6, valid, T, kappa, corr):
        """Cost at T (rotation block used as a free 3x3) with correspondences
        corr fixed and FP64 source points src64 [3, n]."""
        a = np.ascontiguousarray(src64, dtype=np.float64)
        n = a.shape[1]
        out = C.c_double(0)
        rc = lib().orc_cost_fixed(self._h, a, np.ascontiguousarray(cov6, dtype=np.float32),
                                  np.ascontiguousarray(valid, dtype=np.uint8), n,
                                  np.ascontiguousarray(T, dtype=np.float64).reshape(16), kappa,
                                  np.ascontiguousarray(corr, dtype=np.int32), C.byref(out))
        if rc:
            raise OracleError(rc, "orc_cost_fixed")
        return out.value

    def gradient(self, src, cov6, valid, T, tau, kappa, c=None, want_src=True, sa=True):
        """dict(grad_T [3, 4], grad_twist [6], grad_src [3, n] or None, cost,
        n_inliers, corr)."""
        a = _soa(src)
        n = a.shape[1]
        gT, gw = np.zeros(12), np.zeros(6)
        gs = np.zeros((3, n)) if want_src else None
        cost, cnt = C.c_double(0), C.c_int64(0)
        corr = np.zeros(n, np.int32)
        cc = None if c is None else np.ascontiguousarray(c, dtype=np.float64)
        rc = lib().orc_gradient(self._h, a, np.ascontiguousarray(cov6, dtype=np.float32),
                                np.ascontiguousarray(valid, dtype=np.uint8), n,
                                np.ascontiguousarray(T, dtype=np.float64).reshape(16), tau,
                                kappa, cc, gT, gw, gs, C.byref(cost), C.byref(cnt), corr,
                                1 if sa else 0)
        if rc:
            raise OracleError(rc, "orc_gradient")
        return dict(grad_T=gT.reshape(3, 4), grad_twist=gw, grad_src=gs, cost=cost.value,
                    n_inliers=cnt.value, corr=corr)

    def evict(self, center, radius):
        """Remove voxels whose centre is farther than radius from center;
        returns the number of points removed."""
        out = C.c_int64(0)
        rc = lib().orc_map_evict(self._h, np.ascontiguousarray(center, dtype=np.float64),
                                 radius, C.byref(out))
        if rc:
            raise OracleError(rc, "orc_map_evict")
        return out.value

    def touch_stats(self, src, T):
        a = _soa(src)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(16)
        u, p = C.c_int64(0), C.c_int64(0)
        lib().orc_touch_stats(self._h, a, a.shape[1], T, C.byref(u), C.byref(p))
        return u.value, p.value


def scan_covariances(xyz, voxel_size, k):
    a = _soa(xyz)
    n = a.shape[1]
    cov = np.zeros((6, n), np.float64)
    val = np.zeros(n, np.uint8)
    rc = lib().orc_scan_covariances(a, n, voxel_size, k, cov, val)
    if rc:
        raise OracleError(rc, "orc_scan_covariances")
    return cov, val


def voxel_keys(xyz, v):
    a = _soa(xyz)
    out = np.zeros((a.shape[1], 3), np.int64)
    lib().orc_voxel_keys(a, a.shape[1], v, out)
    return out


def se3_exp(delta):
    T = np.zeros(16)
    lib().orc_se3_exp(np.ascontiguousarray(delta, dtype=np.float64), T)
    return T.reshape(4, 4)


def cholesky_solve6(H, b):
    x = np.zeros(6)
    rc = lib().orc_cholesky_solve6(np.ascontiguousarray(H, dtype=np.float64).reshape(36),
                                   np.ascontiguousarray(b, dtype=np.float64), x)
    return rc, x


def regularize_cov(S):
    out = np.zeros(9)
    lib().orc_regularize_cov(np.ascontiguousarray(S, dtype=np.float64).reshape(9), out)
    return out.reshape(3, 3)


def plane_cov(S):
    """Plane-regularised covariance of a 3x3 sample covariance."""
    out = np.zeros(9)
    lib().orc_plane_cov(np.ascontiguousarray(S, dtype=np.float64).reshape(9), out)
    return out.reshape(3, 3)


def jacobi3(S):
    """(eigenvalues [3], eigenvectors as columns [3, 3]) by cyclic Jacobi."""
    ev, V = np.zeros(3), np.zeros(9)
    lib().orc_jacobi3(np.ascontiguousarray(S, dtype=np.float64).reshape(9), ev, V)
    return ev, V.reshape(3, 3)


def set_cov_mode(mode):
    """0: Eq. (1) (default); 1: plane regularisation.  Process-wide."""
    if lib().orc_set_cov_mode(int(mode)):
        raise OracleError(1, "orc_set_cov_mode")


def downsample(xyz, v):
    """Indices (increasing) of the first point of every voxel of edge v."""
    a = _soa(xyz)
    n = a.shape[1]
    keep = np.zeros(max(n, 1), np.int64)
    m = C.c_int64(0)
    rc = lib().orc_downsample(a, n, v, keep, C.byref(m))
    if rc:
        raise OracleError(rc, "orc_downsample")
    return keep[:m.value].copy()


def transform(xyz, T):
    a = _soa(xyz)
    out = np.zeros_like(a)
    lib().orc_transform(a, a.shape[1], np.ascontiguousarray(T, dtype=np.float64).reshape(16), out)
    return out


def _samples(ts, xi):
    ts = np.ascontiguousarray(ts, dtype=np.float64).reshape(-1)
    xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, 6)
    assert xi.shape[0] == ts.size
    return (ts if ts.size else np.zeros(1)), (xi if ts.size else np.zeros((1, 6))), ts.size


def fit_twist(ts, xi):
    """Least-squares line per component of the velocity samples xi [m, 6]
    (vx vy vz wx wy wz, body frame) at times ts [m]: (tbar, a, b) with
    xi_k(t) ~ a_k + b_k (t - tbar)."""
    ts, xi, m = _samples(ts, xi)
    tb = C.c_double(0)
    a, b = np.zeros(6), np.zeros(6)
    lib().orc_fit_twist(ts, xi, m, C.byref(tb), a, b)
    return tb.value, a, b


def undistort(xyz, t, ts, xi):
    """Points [3, n] taken at times t [n] moved into the sensor frame of the
    largest finite point time, with the motion fitted to (ts, xi); returns
    (points float32 [3, n], t_ref)."""
    a = _soa(xyz)
    n = a.shape[1]
    tt = np.ascontiguousarray(t, dtype=np.float32).reshape(-1)
    assert tt.size == n
    ts, xi, m = _samples(ts, xi)
    out = np.zeros_like(a)
    tr = C.c_double(0)
    lib().orc_undistort(a, tt if n else np.zeros(1, np.float32), n, ts, xi, m, out, C.byref(tr))
    return out, tr.value


class Threshold:
    """Adaptive correspondence threshold and Cauchy kappa (KISS-ICP rule)."""

    def __init__(self, sigma0, r_max, min_motion=0.1):
        self._s = _ThresholdState()
        lib().orc_threshold_init(C.byref(self._s), sigma0, r_max, min_motion)

    def update(self, T_pred, T_est):
        return lib().orc_threshold_update(
            C.byref(self._s), np.ascontiguousarray(T_pred, dtype=np.float64).reshape(16),
            np.ascontiguousarray(T_est, dtype=np.float64).reshape(16))

    def get(self):
        tau, kappa = C.c_double(0), C.c_double(0)
        lib().orc_threshold_get(C.byref(self._s), C.byref(tau), C.byref(kappa))
        return tau.value, kappa.value

    @property
    def samples(self):
        return self._s.n


def _inv(T):
    R, t = T[:3, :3], T[:3, 3]
    out = np.eye(4)
    out[:3, :3] = R.T
    out[:3, 3] = -R.T @ t
    return out


def _nearest_rotation(R):
    """Closest rotation matrix in the Frobenius norm (SVD polar factor)."""
    U, _, Vt = np.linalg.svd(R)
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(U @ Vt))])
    return U @ D @ Vt


def odometry(scans, T_first, v_first, voxel_size, max_pts_per_voxel, min_spacing, k,
             map_capacity, downsample_v, sigma0, r_max, min_motion=0.1, max_iters=10,
             eps=0.0, asmd=False, r_near=20.0, evict_radius=0.0, times=None, vel_t=None,
             vel=None):
    """Scan-to-submap odometry over a sequence (Sec. III-A: downsample, source
    covariances, registration against the capped submap, insertion of the
    registered scan), driven by the oracle's own steps.

    Readings: the first scan is inserted at T_first; the motion prediction is
    constant velocity, T_pred = T_prev (T_prev2^-1 T_prev) with its rotation
    projected back onto SO(3) (without the projection the rounding error of
    the rotation grows about 2.4x per scan through the predictor), and the
    relative motion v_first (the inertial prediction of the paper's filter)
    for the second scan; the threshold and kappa come from Threshold before each
    registration and the deviation of the estimate is added after it; the
    registered, downsampled scan is inserted (with the adaptive submap density
    caps of asmd_caps when asmd is set); once the map is full, inserting stops
    (the map keeps what fit); with evict_radius > 0 the voxels farther than it
    from the estimate's position are then removed (Sec. III-A.3).  With per-point
    times and velocity samples given (lists over the scans), each raw scan is
    first undistorted to its last point time (Sec. III-A.1), so every pose is the
    sensor's at that time.  Returns per-scan dicts with the pose, the prediction,
    tau, kappa, the align status and map sizes."""
    m = Map(voxel_size, max_pts_per_voxel, min_spacing, k, point_capacity=map_capacity,
            voxel_capacity=map_capacity)
    thr = Threshold(sigma0, r_max, min_motion)
    out, poses = [], []
    full = False
    for s, raw in enumerate(scans):
        rec = {}
        if times is not None:
            raw, rec["t_ref"] = undistort(raw, times[s], vel_t[s], vel[s])
        src = _soa(raw)[:, downsample(raw, downsample_v)]
        rec["n"] = src.shape[1]
        if s == 0:
            T = np.array(T_first, dtype=np.float64)
            rec.update(T_pred=T.copy(), tau=None, kappa=None, status=0, iters=0)
        else:
            motion = v_first if s == 1 else _inv(poses[-2]) @ poses[-1]
            T_pred = poses[-1] @ motion
            T_pred[:3, :3] = _nearest_rotation(T_pred[:3, :3])
            tau, kappa = thr.get()
            cov, val = scan_covariances(src, voxel_size, k)
            r = m.align(src, cov.astype(np.float32), val, T_pred, tau, kappa,
                        max_iters=max_iters, eps=eps)
            T = r["T"] if r["status"] == 0 else T_pred
            rec.update(T_pred=T_pred, tau=tau, kappa=kappa, status=r["status"],
                       iters=r["iters"], n_inliers=r["n_inliers"], cost=r["cost"],
                       deviation=thr.update(T_pred, T))
        poses.append(T)
        if not full:
            moved = transform(src, T)
            caps = None
            if asmd:
                caps, rec["asmd_mean"] = asmd_caps(src, moved, voxel_size, k, max_pts_per_voxel,
                                                   r_near, r_max)
            rc, acc, _ = m.insert(moved, caps, check=False)
            full = rc == 2
            rec["inserted"] = acc
        if evict_radius > 0:
            rec["evicted"] = m.evict(T[:3, 3], evict_radius)
        rec.update(T=T, map_points=m.size, map_voxels=m.n_voxels)
        out.append(rec)
    return out, m


def asmd_caps(xyz_sensor, xyz_map, v, k, nmax, r_near=20.0, r_max=120.0):
    """Per-point insert caps of the adaptive submap density; (caps, mean)."""
    a, b = _soa(xyz_sensor), _soa(xyz_map)
    n = a.shape[1]
    caps = np.zeros(max(n, 1), np.int32)
    mean = C.c_double(0)
    rc = lib().orc_asmd_caps(a, b, n, v, k, nmax, r_near, r_max, caps, C.byref(mean))
    if rc:
        raise OracleError(rc, "orc_asmd_caps")
    return caps[:n], mean.value
