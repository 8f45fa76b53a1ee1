// far_odom.hip -- scan-to-submap odometry over a sequence (Sec. III-A): the
// host-side loop that strings the device entry points together per scan
// (downsample, scan covariances, Gauss-Newton align, submap insert), the
// constant-velocity motion prediction and the adaptive threshold of
// Sec. III-A.2.  Only scalar 4x4 pose arithmetic runs on the host; every
// per-point step is a kernel of this library.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "far_internal.h"

namespace {

// Row-major 4x4 rigid transforms.
void mul4(const double A[16], const double B[16], double C[16]) {
  double t[16];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      t[i * 4 + j] = A[i * 4 + 0] * B[0 * 4 + j] + A[i * 4 + 1] * B[1 * 4 + j] +
                     A[i * 4 + 2] * B[2 * 4 + j] + A[i * 4 + 3] * B[3 * 4 + j];
  std::memcpy(C, t, sizeof(t));
}

// [R t]^-1 = [R^T  -R^T t]
void rigid_inverse(const double T[16], double out[16]) {
  double o[16] = {0};
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) o[i * 4 + j] = T[j * 4 + i];
    o[i * 4 + 3] = -(T[0 * 4 + i] * T[3] + T[1 * 4 + i] * T[7] + T[2 * 4 + i] * T[11]);
  }
  o[15] = 1.0;
  std::memcpy(out, o, sizeof(o));
}

// Projects the rotation block of T back onto SO(3) through its unit
// quaternion: the largest of |w|, |x|, |y|, |z| from the diagonal, the rest
// from the off-diagonal sums and differences, normalised, and rebuilt.
void reorthonormalise(double T[16]) {
  const double m00 = T[0], m01 = T[1], m02 = T[2];
  const double m10 = T[4], m11 = T[5], m12 = T[6];
  const double m20 = T[8], m21 = T[9], m22 = T[10];
  const double tr = m00 + m11 + m22;
  double w, x, y, z;
  if (tr > 0.0) {
    const double r = 2.0 * std::sqrt(1.0 + tr);
    w = 0.25 * r; x = (m21 - m12) / r; y = (m02 - m20) / r; z = (m10 - m01) / r;
  } else if (m00 > m11 && m00 > m22) {
    const double r = 2.0 * std::sqrt(1.0 + m00 - m11 - m22);
    w = (m21 - m12) / r; x = 0.25 * r; y = (m01 + m10) / r; z = (m02 + m20) / r;
  } else if (m11 > m22) {
    const double r = 2.0 * std::sqrt(1.0 + m11 - m00 - m22);
    w = (m02 - m20) / r; x = (m01 + m10) / r; y = 0.25 * r; z = (m12 + m21) / r;
  } else {
    const double r = 2.0 * std::sqrt(1.0 + m22 - m00 - m11);
    w = (m10 - m01) / r; x = (m02 + m20) / r; y = (m12 + m21) / r; z = 0.25 * r;
  }
  const double nrm = std::sqrt(w * w + x * x + y * y + z * z);
  w /= nrm; x /= nrm; y /= nrm; z /= nrm;
  T[0] = 1.0 - 2.0 * (y * y + z * z); T[1] = 2.0 * (x * y - w * z); T[2] = 2.0 * (x * z + w * y);
  T[4] = 2.0 * (x * y + w * z); T[5] = 1.0 - 2.0 * (x * x + z * z); T[6] = 2.0 * (y * z - w * x);
  T[8] = 2.0 * (x * z - w * y); T[9] = 2.0 * (y * z + w * x); T[10] = 1.0 - 2.0 * (x * x + y * y);
}

bool finite16(const double T[16]) {
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(T[i])) return false;
  return true;
}

const double kIdentity[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};

}  // namespace

struct far_odometry_s {
  far_map_t map = nullptr;
  far_odometry_params_t p{};
  far_threshold_t thr{};
  double T_first[16], v_first[16];
  double T_prev[16], T_prev2[16];
  int64_t steps = 0;
  bool full = false;
  int64_t cap = 0;           // points the buffers hold
  float* down = nullptr;     // downsampled scan, sensor frame, SoA [3][cap]
  float* moved = nullptr;    // the same points in the map frame
  float* cov = nullptr;      // SoA [6][cap]
  uint8_t* valid = nullptr;  // [cap]
  int32_t* caps = nullptr;   // ASMD caps [cap]
  int64_t raw_cap = 0;       // points the undistortion buffer holds
  float* raw = nullptr;      // undistorted raw scan, SoA [3][raw_cap]
  double* t_ref = nullptr;   // its reference time [1]
};

namespace {

void release(far_odometry_s* o) {
  void* ptrs[] = {o->down, o->moved, o->cov, o->valid, o->caps, o->raw, o->t_ref};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  o->down = o->moved = o->cov = nullptr;
  o->valid = nullptr;
  o->caps = nullptr;
  o->cap = 0;
  o->raw = nullptr;
  o->t_ref = nullptr;
  o->raw_cap = 0;
}

far_status_t reserve_raw(far_odometry_s* o, int64_t n, hipStream_t st) {
  if (n <= o->raw_cap && o->t_ref) return FAR_OK;
  FAR_HIP(hipStreamSynchronize(st));
  if (o->raw) (void)hipFree(o->raw);
  o->raw = nullptr;
  o->raw_cap = 0;
  const int64_t cap = std::max<int64_t>(n, 1024);
  FAR_HIP(hipMalloc(&o->raw, size_t(cap) * 3 * sizeof(float)));
  if (!o->t_ref) FAR_HIP(hipMalloc(&o->t_ref, sizeof(double)));
  o->raw_cap = cap;
  return FAR_OK;
}

far_status_t reserve(far_odometry_s* o, int64_t n, hipStream_t st) {
  if (n <= o->cap) return FAR_OK;
  FAR_HIP(hipStreamSynchronize(st));
  void* ptrs[] = {o->down, o->moved, o->cov, o->valid, o->caps};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  o->down = o->moved = o->cov = nullptr;
  o->valid = nullptr;
  o->caps = nullptr;
  o->cap = 0;
  int64_t cap = std::max<int64_t>(n, 1024);
  FAR_HIP(hipMalloc(&o->down, size_t(cap) * 3 * sizeof(float)));
  FAR_HIP(hipMalloc(&o->moved, size_t(cap) * 3 * sizeof(float)));
  FAR_HIP(hipMalloc(&o->cov, size_t(cap) * 6 * sizeof(float)));
  FAR_HIP(hipMalloc(&o->valid, size_t(cap)));
  FAR_HIP(hipMalloc(&o->caps, size_t(cap) * sizeof(int32_t)));
  o->cap = cap;
  return FAR_OK;
}

}  // namespace

extern "C" {

far_status_t far_threshold_init(far_threshold_t* s, double sigma0, double r_max,
                                double min_motion) {
  if (!s || !(sigma0 > 0.0) || !(r_max >= 0.0) || !(min_motion >= 0.0) ||
      !std::isfinite(sigma0) || !std::isfinite(r_max) || !std::isfinite(min_motion)) {
    far::set_error("far_threshold_init: need sigma0 > 0, r_max >= 0, min_motion >= 0");
    return FAR_E_INVALID;
  }
  s->sigma0 = sigma0;
  s->r_max = r_max;
  s->min_motion = min_motion;
  s->sse = 0.0;
  s->n_samples = 0;
  return FAR_OK;
}

far_status_t far_threshold_update(far_threshold_t* s, const double T_pred[16],
                                  const double T_est[16], double* deviation) {
  if (!s || !T_pred || !T_est || !finite16(T_pred) || !finite16(T_est)) {
    far::set_error("far_threshold_update: invalid argument");
    return FAR_E_INVALID;
  }
  double Pi[16], D[16];
  rigid_inverse(T_pred, Pi);
  mul4(Pi, T_est, D);
  // rotation angle from both the symmetric and the skew part of R_D, which
  // keeps small angles accurate
  double sx = D[9] - D[6], sy = D[2] - D[8], sz = D[4] - D[1];
  double theta = std::atan2(0.5 * std::sqrt(sx * sx + sy * sy + sz * sz),
                            0.5 * (D[0] + D[5] + D[10] - 1.0));
  double dt = std::sqrt(D[3] * D[3] + D[7] * D[7] + D[11] * D[11]);
  double dev = 2.0 * s->r_max * std::sin(0.5 * theta) + dt;
  if (dev > s->min_motion) {
    s->sse += dev * dev;
    s->n_samples += 1;
  }
  if (deviation) *deviation = dev;
  return FAR_OK;
}

far_status_t far_threshold_get(const far_threshold_t* s, double* tau, double* kappa) {
  if (!s || !tau || !kappa) {
    far::set_error("far_threshold_get: null argument");
    return FAR_E_INVALID;
  }
  double sigma = s->n_samples > 0 ? std::sqrt(s->sse / double(s->n_samples)) : s->sigma0;
  *tau = 3.0 * sigma;
  *kappa = sigma / 3.0;
  return FAR_OK;
}

far_status_t far_odometry_create(far_map_t map, const far_odometry_params_t* params,
                                 const double T_first[16], const double v_first[16],
                                 far_odometry_t* out) {
  if (out) *out = nullptr;
  if (!map || !params || !T_first || !out || !finite16(T_first) ||
      (v_first && !finite16(v_first)) || !(params->downsample > 0.0) ||
      !std::isfinite(params->downsample) || params->max_iters < 1 || params->max_iters > 64 ||
      !(params->eps >= 0.0) || !(params->r_near >= 0.0) || !(params->evict_radius >= 0.0) ||
      (params->asmd != 0 && params->asmd != 1) ||
      ((params->precision & ~int32_t(FAR_OPT_NO_SA)) != FAR_PREC_FP32 &&
       (params->precision & ~int32_t(FAR_OPT_NO_SA)) != FAR_PREC_FP64)) {
    far::set_error("far_odometry_create: invalid argument");
    return FAR_E_INVALID;
  }
  far_odometry_s* o = new far_odometry_s();
  o->map = map;
  o->p = *params;
  far_status_t s = far_threshold_init(&o->thr, params->sigma0, params->r_max,
                                      params->min_motion);
  if (s != FAR_OK) {
    delete o;
    return s;
  }
  std::memcpy(o->T_first, T_first, sizeof(o->T_first));
  std::memcpy(o->v_first, v_first ? v_first : kIdentity, sizeof(o->v_first));
  *out = o;
  return FAR_OK;
}

far_status_t far_odometry_step(far_odometry_t o, const float* xyz, int64_t n, double T_out[16],
                               far_odometry_stats_t* stats, far_stream_t stream) {
  if (!o || !T_out || n < 0 || n >= (int64_t(1) << 31) || (n > 0 && !xyz)) {
    far::set_error("far_odometry_step: invalid argument");
    return FAR_E_INVALID;
  }
  hipStream_t st = far::S(stream);
  far_odometry_stats_t sx;
  std::memset(&sx, 0, sizeof(sx));
  sx.n_raw = n;
  sx.t_ref = std::nan("");
  FAR_TRY(reserve(o, n, st));
  int64_t m = 0;
  if (n > 0) FAR_TRY(far_voxel_downsample(xyz, n, o->p.downsample, o->down, nullptr, &m, stream));
  sx.n_down = m;
  double T[16];
  if (o->steps == 0) {
    std::memcpy(T, o->T_first, sizeof(T));
    std::memcpy(sx.T_pred, T, sizeof(T));
  } else {
    double vel[16];
    if (o->steps == 1) {
      std::memcpy(vel, o->v_first, sizeof(vel));
    } else {
      double inv2[16];
      rigid_inverse(o->T_prev2, inv2);
      mul4(inv2, o->T_prev, vel);
    }
    mul4(o->T_prev, vel, sx.T_pred);
    // the predictor inverts a rotation by transposing it, which doubles any
    // loss of orthonormality: without this projection the rounding error of
    // the rotation grows about 2.4x per scan
    reorthonormalise(sx.T_pred);
    FAR_TRY(far_threshold_get(&o->thr, &sx.tau, &sx.kappa));
    const far_map_s* mp = o->map;
    if (m > 0)
      FAR_TRY(far_scan_covariances(o->down, m, mp->p.voxel_size, mp->p.k_cov, o->cov, o->valid,
                                   stream));
    far_align_params_t ap{sx.tau, sx.kappa, o->p.max_iters, o->p.eps, 1, o->p.precision};
    far_align_stats_t as;
    std::memset(&as, 0, sizeof(as));
    far_status_t a = far_gicp_align(o->map, o->down, o->cov, o->valid, m, sx.T_pred, &ap, T,
                                    &as, stream);
    if (a != FAR_OK && a != FAR_E_NOT_PD && a != FAR_E_FEW_CORR) return a;
    sx.status = a;
    sx.iters = as.iters;
    sx.last = as.last;
    if (a != FAR_OK) std::memcpy(T, sx.T_pred, sizeof(T));
    FAR_TRY(far_threshold_update(&o->thr, sx.T_pred, T, &sx.deviation));
  }
  if (!o->full && m > 0) {
    FAR_TRY(far_transform_points(o->down, m, T, o->moved, stream));
    const int32_t* caps = nullptr;
    if (o->p.asmd) {
      const far_map_s* mp = o->map;
      FAR_TRY(far_asmd_caps(o->down, o->moved, m, mp->p.voxel_size, mp->p.k_cov,
                            mp->p.max_pts_per_voxel, o->p.r_near, o->p.r_max, o->caps,
                            &sx.asmd_mean, stream));
      caps = o->caps;
    }
    int64_t acc = 0;
    far_status_t s = far_map_insert(o->map, o->moved, m, caps, stream, &acc);
    if (s == FAR_E_CAPACITY)
      o->full = true;
    else if (s != FAR_OK)
      return s;
    sx.n_inserted = acc;
  }
  if (o->p.evict_radius > 0.0) {
    const double c[3] = {T[3], T[7], T[11]};
    FAR_TRY(far_map_evict(o->map, c, o->p.evict_radius, &sx.n_evicted, stream));
  }
  sx.map_full = o->full ? 1 : 0;
  std::memcpy(o->T_prev2, o->T_prev, sizeof(T));
  std::memcpy(o->T_prev, T, sizeof(T));
  o->steps += 1;
  std::memcpy(T_out, T, sizeof(T));
  if (stats) *stats = sx;
  return FAR_OK;
}

far_status_t far_odometry_step_timed(far_odometry_t o, const float* xyz, const float* t,
                                     int64_t n, const double* vel_t, const double* vel,
                                     int32_t m, double T_out[16], far_odometry_stats_t* stats,
                                     far_stream_t stream) {
  if (!o || !T_out || n < 0 || n >= (int64_t(1) << 31) || (n > 0 && (!xyz || !t)) || m < 0 ||
      (m > 0 && (!vel_t || !vel))) {
    far::set_error("far_odometry_step_timed: invalid argument");
    return FAR_E_INVALID;
  }
  hipStream_t st = far::S(stream);
  FAR_TRY(reserve_raw(o, n, st));
  FAR_TRY(far_undistort(xyz, t, n, vel_t, vel, m, o->raw, o->t_ref, stream));
  far_odometry_stats_t sx;
  FAR_TRY(far_odometry_step(o, o->raw, n, T_out, &sx, stream));
  double tr = std::nan("");
  FAR_HIP(hipMemcpyAsync(&tr, o->t_ref, sizeof(tr), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipStreamSynchronize(st));
  sx.t_ref = tr;
  if (stats) *stats = sx;
  return FAR_OK;
}

far_status_t far_odometry_destroy(far_odometry_t o) {
  if (!o) return FAR_OK;
  hipError_t e = hipDeviceSynchronize();
  release(o);
  delete o;
  if (e != hipSuccess) return far::hip_fail(e, "hipDeviceSynchronize", __FILE__, __LINE__);
  return FAR_OK;
}

}  // extern "C"
