// far_knn.h -- device-side neighbour search and covariance helpers shared by
// the map, scan-covariance and GICP kernels (header-only device code).
#pragma once

#include <climits>

#include "far_internal.h"

namespace far {

// Sorted list of the K best (d2, id) candidates; pos is the candidate's slot
// in the point store it came from (used to gather its coordinates).
template <int K>
struct TopK {
  double d[K];
  int32_t id[K];
  int32_t pos[K];
  __device__ inline void init() {
#pragma unroll
    for (int s = 0; s < K; ++s) {
      d[s] = __builtin_inf();
      id[s] = INT_MAX;
      pos[s] = -1;
    }
  }
  __device__ inline double bound() const { return d[K - 1]; }
  __device__ inline void push(double dd, int32_t ii, int32_t pp) {
    if (!rank_less(dd, ii, d[K - 1], id[K - 1])) return;
    bool placed = false;
#pragma unroll
    for (int s = K - 1; s > 0; --s) {
      if (!placed) {
        if (rank_less(dd, ii, d[s - 1], id[s - 1])) {
          d[s] = d[s - 1];
          id[s] = id[s - 1];
          pos[s] = pos[s - 1];
        } else {
          d[s] = dd;
          id[s] = ii;
          pos[s] = pp;
          placed = true;
        }
      }
    }
    if (!placed) {
      d[0] = dd;
      id[0] = ii;
      pos[0] = pp;
    }
  }
  __device__ inline int found() const {
    int c = 0;
#pragma unroll
    for (int s = 0; s < K; ++s) c += (d[s] < __builtin_inf()) ? 1 : 0;
    return c;
  }
};

// Voxel index of a coordinate; false when outside [-2^20, 2^20).
__device__ inline bool voxel_index(double x, double v, int64_t* k) {
  double f = floor(x / v);
  if (!(f >= -double(kKeyBias) && f < double(kKeyBias))) return false;
  *k = int64_t(f);
  return true;
}

// Rank the cnt points stored at pts[base ...] against q.  Loads are issued
// four at a time so that they overlap instead of waiting one by one.
template <int K>
__device__ inline void scan_voxel_points(const float4* pts, int32_t base, int32_t cnt,
                                         double qx, double qy, double qz, double r2,
                                         TopK<K>& top) {
  for (int32_t j = 0; j < cnt; j += 4) {
    float4 p[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (j + u < cnt) p[u] = pts[base + j + u];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (j + u < cnt) {
        double d = dist2(double(p[u].x), double(p[u].y), double(p[u].z), qx, qy, qz);
        if (d <= r2) top.push(d, __float_as_int(p[u].w), base + j + u);
      }
  }
}

// K nearest map points within sqrt(r2) of q over the 27-voxel neighbourhood,
// skipping voxels whose conservative lower bound exceeds the current K-th
// best (own voxel first, so the bound tightens early).
template <int K>
__device__ inline void map_knn_query(const MapView& m, double qx, double qy, double qz,
                                     double r2, TopK<K>& top) {
  top.init();
  int64_t kx, ky, kz;
  if (!voxel_index(qx, m.v, &kx) || !voxel_index(qy, m.v, &ky) ||
      !voxel_index(qz, m.v, &kz))
    return;
  for (int t = 0; t < 27; ++t) {
    int code = kNbrOrder[t];
    int ox = code / 9 - 1, oy = (code / 3) % 3 - 1, oz = code % 3 - 1;
    double bnd = fmin(r2, top.bound());
    if (voxel_lb2(qx, qy, qz, kx, ky, kz, ox, oy, oz, m.v) > bnd) continue;
    int32_t cnt;
    int32_t vox = map_find(m, kx + ox, ky + oy, kz + oz, &cnt);
    if (vox < 0) continue;
    scan_voxel_points<K>(m.vox_pts, vox * m.nmax, cnt, qx, qy, qz, r2, top);
  }
}

// Regularised covariance (Eq. 1) of the first k entries of a neighbour list.
// Two-pass FP64 sample covariance with 1/k, C = S + 1e-3 I, and
// Sigma = (C^-1 / ||C^-1||_F)^-1 = ||C^-1||_F C, where ||C^-1||_F is the
// Frobenius norm of the cofactor matrix over |det C|.
template <int K, class Get>
__device__ inline void regularised_cov(const TopK<K>& top, int k, Get get, double out[6]) {
  double mx = 0.0, my = 0.0, mz = 0.0;
#pragma unroll
  for (int s = 0; s < K; ++s)
    if (s < k) {
      float4 p = get(top.pos[s]);
      mx += double(p.x);
      my += double(p.y);
      mz += double(p.z);
    }
  double inv_k = 1.0 / double(k);
  mx *= inv_k;
  my *= inv_k;
  mz *= inv_k;
  double sxx = 0, sxy = 0, sxz = 0, syy = 0, syz = 0, szz = 0;
#pragma unroll
  for (int s = 0; s < K; ++s)
    if (s < k) {
      float4 p = get(top.pos[s]);
      double dx = double(p.x) - mx, dy = double(p.y) - my, dz = double(p.z) - mz;
      sxx += dx * dx;
      sxy += dx * dy;
      sxz += dx * dz;
      syy += dy * dy;
      syz += dy * dz;
      szz += dz * dz;
    }
  double c00 = sxx * inv_k + 1e-3, c01 = sxy * inv_k, c02 = sxz * inv_k;
  double c11 = syy * inv_k + 1e-3, c12 = syz * inv_k, c22 = szz * inv_k + 1e-3;
  double a00 = c11 * c22 - c12 * c12;
  double a01 = c02 * c12 - c01 * c22;
  double a02 = c01 * c12 - c02 * c11;
  double a11 = c00 * c22 - c02 * c02;
  double a12 = c01 * c02 - c00 * c12;
  double a22 = c00 * c11 - c01 * c01;
  double det = c00 * a00 + c01 * a01 + c02 * a02;
  double fro2 = a00 * a00 + a11 * a11 + a22 * a22 + 2.0 * (a01 * a01 + a02 * a02 + a12 * a12);
  double s = sqrt(fro2) / fabs(det);
  out[0] = s * c00;
  out[1] = s * c01;
  out[2] = s * c02;
  out[3] = s * c11;
  out[4] = s * c12;
  out[5] = s * c22;
}

}  // namespace far
