// far_gicp.hip -- sparsity-aware GICP linearisation and the Gauss-Newton
// iteration (Sec. III-A.2, Eqs. (2)-(6)), for one scan or many scans per
// launch.
//
// Work decomposition: every scan is cut into tiles of 256 consecutive points;
// one 256-thread block linearises one tile (one point per thread) and writes
// 29 FP64 partial sums (21 upper-triangle H entries, 6 b entries, cost,
// inlier count).  A second kernel runs one block per scan: it sums the scan's
// tile partials in tile order (deterministic) and one lane solves the 6x6
// system in FP64 and updates the pose.  Finished scans skip their tiles.
// One iteration is therefore two launches whatever the number of scans; the
// whole align (state init + max_iters iterations) is captured once into a HIP
// graph per argument set and replayed.
#include <cmath>
#include <cstring>
#include <type_traits>

#include "far_knn.h"

namespace far {
namespace {

constexpr int kTile = 256;
constexpr int kVals = 29;     // 21 H + 6 b + cost + count
constexpr int kStride = 32;   // partial row stride (doubles)

struct Params {
  double r2;        // min(tau, v)^2
  double kappa2;
  double eps;
  int32_t max_iters;
  int32_t recenter;
};

// ---------------------------------------------------------------- tiles
__global__ __launch_bounds__(256) void k_build_tiles(const int64_t* offsets, int32_t S,
                                                     int64_t n_total, int64_t max_tiles,
                                                     int32_t* tile_scan, uint32_t* tile_lo,
                                                     uint32_t* tile_hi, int32_t* begin,
                                                     int32_t* bad) {
  __shared__ int32_t s_total;
  __shared__ int32_t s_bad;
  if (threadIdx.x == 0) {
    int32_t b = (offsets[0] != 0 || offsets[S] != n_total) ? 1 : 0;
    int64_t acc = 0;
    begin[0] = 0;
    for (int32_t s = 0; s < S; ++s) {
      int64_t len = offsets[s + 1] - offsets[s];
      if (len < 0) b = 1;
      acc += len > 0 ? (len + kTile - 1) / kTile : 0;
      begin[s + 1] = int32_t(acc);
    }
    if (acc > max_tiles) b = 1;
    if (b)
      for (int32_t s = 0; s <= S; ++s) begin[s] = 0;
    s_total = b ? 0 : int32_t(acc);
    s_bad = b;
    *bad = b;
  }
  __syncthreads();
  for (int64_t t = threadIdx.x; t < max_tiles; t += blockDim.x)
    if (t >= s_total) tile_scan[t] = -1;
  if (s_bad) return;
  for (int32_t s = threadIdx.x; s < S; s += blockDim.x) {
    int64_t lo = offsets[s], hi = offsets[s + 1];
    for (int32_t t = begin[s]; t < begin[s + 1]; ++t) {
      int64_t a = lo + int64_t(t - begin[s]) * kTile;
      int64_t b = a + kTile < hi ? a + kTile : hi;
      tile_scan[t] = s;
      tile_lo[t] = uint32_t(a);
      tile_hi[t] = uint32_t(b);
    }
  }
}

// Per-scan state reset: not done, zero stats, linearisation centre.
__global__ __launch_bounds__(256) void k_init(int32_t S, const double* T, const int32_t* bad,
                                              int32_t recenter, const double* c_fixed,
                                              far_align_stats_t* stats, int32_t* done,
                                              double* ctr) {
  int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  int32_t b = *bad;
  done[s] = b;
  far_align_stats_t st = {};
  st.status = b ? FAR_E_INVALID : FAR_OK;
  stats[s] = st;
  const double* Ts = T + 16 * int64_t(s);
  for (int a = 0; a < 3; ++a)
    ctr[3 * s + a] = c_fixed ? c_fixed[a] : (recenter ? Ts[4 * a + 3] : 0.0);
}

// ---------------------------------------------------------------- reduction
__device__ inline void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  float bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}

// Wave-wide sum of one value per lane; FP32 values are combined with TwoSum
// so the carried error terms make the wave sum nearly exact.
__device__ inline double wave_sum(float v) {
  float s = v, c = 0.0f;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    float so = __shfl_xor(s, o, 64);
    float co = __shfl_xor(c, o, 64);
    float t, e;
    two_sum(s, so, t, e);
    s = t;
    c = (c + co) + e;
  }
  return double(s) + double(c);
}
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------- linearise
// One GICP term per thread (Eqs. (3)-(5), sparsity-aware):
//   p = R s + t (FP64, ((R0 sx + R1 sy) + R2 sz) + t, no FMA)
//   j = nearest map point within min(tau, v), ranked by (d2, id)
//   d = r_j - p,  a = p - c
//   M = Sigma_r + R Sigma_s R^T if both covariances are valid, else I
//   W = M^-1, e2 = d^T W d, w = k2/(k2 + e2), rho = k2/2 ln(1 + e2/k2)
//   J = [[a]x, -I]: H += w J^T W J, b += w J^T W d, cost += rho, n += 1
template <class Real>
__global__ __launch_bounds__(kTile) void k_linearize(
    MapView m, const float* __restrict__ src, const float* __restrict__ cov6,
    const uint8_t* __restrict__ valid, int64_t n_total, const int32_t* __restrict__ tile_scan,
    const uint32_t* __restrict__ tile_lo, const uint32_t* __restrict__ tile_hi,
    int64_t n_tiles, const double* __restrict__ T, const double* __restrict__ ctr,
    const int32_t* __restrict__ done, Params prm, double* __restrict__ partial,
    int32_t* __restrict__ corr) {
  __shared__ double red[kTile / 64][kVals];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int32_t s = tile_scan[t];
    if (s < 0 || done[s]) continue;
    const double* Ts = T + 16 * int64_t(s);
    const double R00 = Ts[0], R01 = Ts[1], R02 = Ts[2], tx = Ts[3];
    const double R10 = Ts[4], R11 = Ts[5], R12 = Ts[6], ty = Ts[7];
    const double R20 = Ts[8], R21 = Ts[9], R22 = Ts[10], tz = Ts[11];
    const double cx = ctr[3 * s], cy = ctr[3 * s + 1], cz = ctr[3 * s + 2];
    const int64_t i = int64_t(tile_lo[t]) + threadIdx.x;

    Real acc[kVals];
#pragma unroll
    for (int v = 0; v < kVals; ++v) acc[v] = Real(0);
    int32_t match = -1;

    if (i < int64_t(tile_hi[t])) {
      const float sx = src[i], sy = src[n_total + i], sz = src[2 * n_total + i];
      if (isfinite(sx) && isfinite(sy) && isfinite(sz)) {
        const double dsx = sx, dsy = sy, dsz = sz;
        const double px = ((R00 * dsx + R01 * dsy) + R02 * dsz) + tx;
        const double py = ((R10 * dsx + R11 * dsy) + R12 * dsz) + ty;
        const double pz = ((R20 * dsx + R21 * dsy) + R22 * dsz) + tz;
        TopK<1> top;
        map_knn_query<1>(m, px, py, pz, prm.r2, top);
        if (top.pos[0] >= 0) {
          match = top.id[0];
          const float4 r = m.vox_pts[top.pos[0]];
          const float4 ca = m.cov[2 * int64_t(match)];
          const float4 cb = m.cov[2 * int64_t(match) + 1];
          const Real d0 = Real(double(r.x) - px), d1 = Real(double(r.y) - py),
                     d2 = Real(double(r.z) - pz);
          const Real a0 = Real(px - cx), a1 = Real(py - cy), a2 = Real(pz - cz);
          Real M00, M01, M02, M11, M12, M22;
          if (valid[i] && cb.z != 0.0f) {
            // R Sigma_s R^T
            const Real q00 = cov6[i], q01 = cov6[n_total + i], q02 = cov6[2 * n_total + i];
            const Real q11 = cov6[3 * n_total + i], q12 = cov6[4 * n_total + i],
                       q22 = cov6[5 * n_total + i];
            const Real r00 = Real(R00), r01 = Real(R01), r02 = Real(R02);
            const Real r10 = Real(R10), r11 = Real(R11), r12 = Real(R12);
            const Real r20 = Real(R20), r21 = Real(R21), r22 = Real(R22);
            // RS = R * Sigma_s (rows of R times the symmetric matrix)
            const Real u00 = r00 * q00 + r01 * q01 + r02 * q02;
            const Real u01 = r00 * q01 + r01 * q11 + r02 * q12;
            const Real u02 = r00 * q02 + r01 * q12 + r02 * q22;
            const Real u10 = r10 * q00 + r11 * q01 + r12 * q02;
            const Real u11 = r10 * q01 + r11 * q11 + r12 * q12;
            const Real u12 = r10 * q02 + r11 * q12 + r12 * q22;
            const Real u20 = r20 * q00 + r21 * q01 + r22 * q02;
            const Real u21 = r20 * q01 + r21 * q11 + r22 * q12;
            const Real u22 = r20 * q02 + r21 * q12 + r22 * q22;
            M00 = Real(ca.x) + (u00 * r00 + u01 * r01 + u02 * r02);
            M01 = Real(ca.y) + (u00 * r10 + u01 * r11 + u02 * r12);
            M02 = Real(ca.z) + (u00 * r20 + u01 * r21 + u02 * r22);
            M11 = Real(ca.w) + (u10 * r10 + u11 * r11 + u12 * r12);
            M12 = Real(cb.x) + (u10 * r20 + u11 * r21 + u12 * r22);
            M22 = Real(cb.y) + (u20 * r20 + u21 * r21 + u22 * r22);
          } else {
            M00 = Real(1); M01 = Real(0); M02 = Real(0);
            M11 = Real(1); M12 = Real(0); M22 = Real(1);
          }
          // W = M^-1 by the adjugate (M is symmetric positive definite)
          const Real A00 = M11 * M22 - M12 * M12;
          const Real A01 = M02 * M12 - M01 * M22;
          const Real A02 = M01 * M12 - M02 * M11;
          const Real A11 = M00 * M22 - M02 * M02;
          const Real A12 = M01 * M02 - M00 * M12;
          const Real A22 = M00 * M11 - M01 * M01;
          const Real inv_det = Real(1) / (M00 * A00 + M01 * A01 + M02 * A02);
          const Real W00 = A00 * inv_det, W01 = A01 * inv_det, W02 = A02 * inv_det;
          const Real W11 = A11 * inv_det, W12 = A12 * inv_det, W22 = A22 * inv_det;
          // Wd, Mahalanobis e2, Cauchy weight and cost
          const Real g0 = W00 * d0 + W01 * d1 + W02 * d2;
          const Real g1 = W01 * d0 + W11 * d1 + W12 * d2;
          const Real g2 = W02 * d0 + W12 * d1 + W22 * d2;
          const Real e2 = d0 * g0 + d1 * g1 + d2 * g2;
          const Real k2 = Real(prm.kappa2);
          const Real w = k2 / (k2 + e2);
          const Real rho = Real(0.5) * k2 * log1p(e2 / k2);
          // Columns of A = [a]x: A0 = (0, a2, -a1), A1 = (-a2, 0, a0), A2 = (a1, -a0, 0).
          // B = W A (column j = W A_j).
          const Real B00 = W01 * a2 - W02 * a1, B10 = W11 * a2 - W12 * a1, B20 = W12 * a2 - W22 * a1;
          const Real B01 = W02 * a0 - W00 * a2, B11 = W12 * a0 - W01 * a2, B21 = W22 * a0 - W02 * a2;
          const Real B02 = W00 * a1 - W01 * a0, B12 = W01 * a1 - W11 * a0, B22 = W02 * a1 - W12 * a0;
          // H_rr[p][q] = A_p . B_q ; H_rt[p][q] = -B[q][p] ; H_tt = W
          auto dotA0 = [&](Real x0, Real x1, Real x2) { return a2 * x1 - a1 * x2; };
          auto dotA1 = [&](Real x0, Real x1, Real x2) { return a0 * x2 - a2 * x0; };
          auto dotA2 = [&](Real x0, Real x1, Real x2) { return a1 * x0 - a0 * x1; };
          const Real h00 = dotA0(B00, B10, B20), h01 = dotA0(B01, B11, B21), h02 = dotA0(B02, B12, B22);
          const Real h11 = dotA1(B01, B11, B21), h12 = dotA1(B02, B12, B22);
          const Real h22 = dotA2(B02, B12, B22);
          int v = 0;
          acc[v++] = w * h00; acc[v++] = w * h01; acc[v++] = w * h02;
          acc[v++] = -w * B00; acc[v++] = -w * B10; acc[v++] = -w * B20;
          acc[v++] = w * h11; acc[v++] = w * h12;
          acc[v++] = -w * B01; acc[v++] = -w * B11; acc[v++] = -w * B21;
          acc[v++] = w * h22;
          acc[v++] = -w * B02; acc[v++] = -w * B12; acc[v++] = -w * B22;
          acc[v++] = w * W00; acc[v++] = w * W01; acc[v++] = w * W02;
          acc[v++] = w * W11; acc[v++] = w * W12;
          acc[v++] = w * W22;
          // b = w J^T W d: rotation part A_p . g, translation part -g
          acc[v++] = w * dotA0(g0, g1, g2);
          acc[v++] = w * dotA1(g0, g1, g2);
          acc[v++] = w * dotA2(g0, g1, g2);
          acc[v++] = -w * g0; acc[v++] = -w * g1; acc[v++] = -w * g2;
          acc[v++] = rho;
          acc[v++] = Real(1);
        }
      }
      if (corr) corr[i] = match;
    }
    // Wave sums (compensated in FP32), then the block's four waves in FP64.
#pragma unroll
    for (int v = 0; v < kVals; ++v) {
      double sv = wave_sum(acc[v]);
      if (lane == 0) red[wave][v] = sv;
    }
    __syncthreads();
    if (threadIdx.x < kVals) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < kTile / 64; ++w) sum += red[w][threadIdx.x];
      partial[t * kStride + threadIdx.x] = sum;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- solve
// One 64-lane block per scan: sum the scan's tile partials in tile order,
// then lane 0 solves H delta = -b by Cholesky (FP64) and applies
// T <- T_c Exp(delta) T_c^-1 T.
__device__ void se3_apply(const double* dl, const double* c, double* T) {
  const double wx = dl[0], wy = dl[1], wz = dl[2];
  const double th2 = wx * wx + wy * wy + wz * wz;
  const double th = sqrt(th2);
  double A, B, C;
  if (th < 1e-6) {
    A = 1.0 - th2 / 6.0;
    B = 0.5 - th2 / 24.0;
    C = 1.0 / 6.0 - th2 / 120.0;
  } else {
    double sn = sin(th), cs = cos(th);
    A = sn / th;
    B = (1.0 - cs) / th2;
    C = (th - sn) / (th2 * th);
  }
  // Rodrigues: R = I + A K + B K^2, V = I + B K + C K^2, K = [w]x,
  // K^2 = w w^T - th2 I.
  const double K[9] = {0.0, -wz, wy, wz, 0.0, -wx, -wy, wx, 0.0};
  const double w3[3] = {wx, wy, wz};
  double RE[9], V[9];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) {
      double k2 = w3[r] * w3[q] - (r == q ? th2 : 0.0);
      double id = (r == q) ? 1.0 : 0.0;
      RE[3 * r + q] = id + A * K[3 * r + q] + B * k2;
      V[3 * r + q] = id + B * K[3 * r + q] + C * k2;
    }
  double tE[3];
  for (int r = 0; r < 3; ++r) tE[r] = V[3 * r] * dl[3] + V[3 * r + 1] * dl[4] + V[3 * r + 2] * dl[5];
  // x -> c + RE (R x + t - c) + tE
  double Rn[9], tn[3];
  for (int r = 0; r < 3; ++r) {
    for (int q = 0; q < 3; ++q)
      Rn[3 * r + q] = RE[3 * r] * T[q] + RE[3 * r + 1] * T[4 + q] + RE[3 * r + 2] * T[8 + q];
    tn[r] = c[r] + tE[r] + RE[3 * r] * (T[3] - c[0]) + RE[3 * r + 1] * (T[7] - c[1]) +
            RE[3 * r + 2] * (T[11] - c[2]);
  }
  for (int r = 0; r < 3; ++r) {
    for (int q = 0; q < 3; ++q) T[4 * r + q] = Rn[3 * r + q];
    T[4 * r + 3] = tn[r];
  }
}

__global__ __launch_bounds__(64) void k_reduce_solve(int32_t S, const int32_t* begin,
                                                     const double* partial, double* T,
                                                     double* ctr, int32_t* done,
                                                     far_align_stats_t* stats, Params prm,
                                                     int32_t solve) {
  __shared__ double lin[kVals];
  const int32_t s = blockIdx.x;
  if (s >= S || done[s]) return;
  const int v = threadIdx.x;
  if (v < kVals) {
    double acc = 0.0;
    for (int32_t t = begin[s]; t < begin[s + 1]; ++t) acc += partial[int64_t(t) * kStride + v];
    lin[v] = acc;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  far_align_stats_t& st = stats[s];
  double H[36], b[6];
  int u = 0;
  for (int p = 0; p < 6; ++p)
    for (int q = p; q < 6; ++q) {
      H[6 * p + q] = lin[u];
      H[6 * q + p] = lin[u];
      ++u;
    }
  for (int p = 0; p < 6; ++p) b[p] = lin[21 + p];
  for (int p = 0; p < 36; ++p) st.last.H[p] = H[p];
  for (int p = 0; p < 6; ++p) st.last.b[p] = b[p];
  st.last.cost = lin[27];
  st.last.n_inliers = int64_t(lin[28]);
  if (!solve) {
    done[s] = 1;
    return;
  }
  if (lin[28] < 6.0) {
    st.status = FAR_E_FEW_CORR;
    done[s] = 1;
    return;
  }
  // Cholesky H = L L^T; a pivot not above 1e-12 max|H_ii| means not PD.
  double L[36];
  double dmax = 0.0;
  for (int p = 0; p < 6; ++p) dmax = fmax(dmax, fabs(H[7 * p]));
  for (int j = 0; j < 6; ++j) {
    double sd = H[7 * j];
    for (int l = 0; l < j; ++l) sd -= L[6 * j + l] * L[6 * j + l];
    if (!(sd > 1e-12 * dmax) || !isfinite(sd)) {
      st.status = FAR_E_NOT_PD;
      done[s] = 1;
      return;
    }
    double dj = sqrt(sd);
    L[7 * j] = dj;
    for (int i = j + 1; i < 6; ++i) {
      double x = H[6 * i + j];
      for (int l = 0; l < j; ++l) x -= L[6 * i + l] * L[6 * j + l];
      L[6 * i + j] = x / dj;
    }
  }
  double y[6], dl[6];
  for (int i = 0; i < 6; ++i) {
    double x = -b[i];
    for (int l = 0; l < i; ++l) x -= L[6 * i + l] * y[l];
    y[i] = x / L[7 * i];
  }
  for (int i = 5; i >= 0; --i) {
    double x = y[i];
    for (int l = i + 1; l < 6; ++l) x -= L[6 * l + i] * dl[l];
    dl[i] = x / L[7 * i];
  }
  double* Ts = T + 16 * int64_t(s);
  double* cs = ctr + 3 * s;
  se3_apply(dl, cs, Ts);
  st.iters += 1;
  double nrm = 0.0;
  for (int p = 0; p < 6; ++p) nrm += dl[p] * dl[p];
  if (sqrt(nrm) <= prm.eps) {
    st.converged = 1;
    done[s] = 1;
  } else if (st.iters >= prm.max_iters) {
    done[s] = 1;
  }
  if (prm.recenter) {
    cs[0] = Ts[3];
    cs[1] = Ts[7];
    cs[2] = Ts[11];
  }
}

}  // namespace

// Device workspace of the align driver, owned by the map and reused (with its
// captured graph) while the call arguments stay the same.
struct AlignWS {
  int32_t S = 0;
  int64_t max_tiles = 0;
  int32_t* tile_scan = nullptr;
  uint32_t* tile_lo = nullptr;
  uint32_t* tile_hi = nullptr;
  int32_t* begin = nullptr;
  int32_t* bad = nullptr;
  int32_t* done = nullptr;
  double* ctr = nullptr;
  double* partial = nullptr;
  int64_t* offsets = nullptr;   // single-scan path
  double* T = nullptr;          // single-scan path
  double* cfix = nullptr;       // fixed centre (linearize)
  far_align_stats_t* stats = nullptr;   // single-scan path
  hipGraphExec_t exec = nullptr;
  // argument set the graph was captured for
  const void* key[10] = {};
  int64_t key_n = -1;
  Params key_prm{};
  int32_t key_prec = -1;
  int32_t key_S = -1;
};

void free_ws(AlignWS* w) {
  if (!w) return;
  if (w->exec) (void)hipGraphExecDestroy(w->exec);
  void* ptrs[] = {w->tile_scan, w->tile_lo, w->tile_hi, w->begin, w->bad, w->done, w->ctr,
                  w->partial, w->offsets, w->T, w->cfix, w->stats};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete w;
}

namespace {

far_status_t ensure_ws(far_map_s* m, int32_t S, int64_t max_tiles, AlignWS** out) {
  AlignWS* w = m->ws;
  if (w && w->S >= S && w->max_tiles >= max_tiles) {
    *out = w;
    return FAR_OK;
  }
  if (w) {
    FAR_HIP(hipDeviceSynchronize());
    free_ws(w);
    m->ws = nullptr;
  }
  w = new AlignWS();
  m->ws = w;
  w->S = S < 64 ? 64 : S;
  w->max_tiles = max_tiles < 1024 ? 1024 : max_tiles;
  FAR_HIP(hipMalloc(&w->tile_scan, size_t(w->max_tiles) * sizeof(int32_t)));
  FAR_HIP(hipMalloc(&w->tile_lo, size_t(w->max_tiles) * sizeof(uint32_t)));
  FAR_HIP(hipMalloc(&w->tile_hi, size_t(w->max_tiles) * sizeof(uint32_t)));
  FAR_HIP(hipMalloc(&w->partial, size_t(w->max_tiles) * kStride * sizeof(double)));
  FAR_HIP(hipMalloc(&w->begin, size_t(w->S + 1) * sizeof(int32_t)));
  FAR_HIP(hipMalloc(&w->bad, sizeof(int32_t)));
  FAR_HIP(hipMalloc(&w->done, size_t(w->S) * sizeof(int32_t)));
  FAR_HIP(hipMalloc(&w->ctr, size_t(w->S) * 3 * sizeof(double)));
  FAR_HIP(hipMalloc(&w->offsets, 2 * sizeof(int64_t)));
  FAR_HIP(hipMalloc(&w->T, 16 * sizeof(double)));
  FAR_HIP(hipMalloc(&w->cfix, 3 * sizeof(double)));
  FAR_HIP(hipMalloc(&w->stats, sizeof(far_align_stats_t)));
  *out = w;
  return FAR_OK;
}

struct Job {
  const float* src;
  const int64_t* offsets;
  int32_t S;
  int64_t n_total;
  const float* cov6;
  const uint8_t* valid;
  double* T;
  far_align_stats_t* stats;
  const double* c_fixed;   // non-null: one linearisation about this centre, no solve
  int32_t* corr;
  Params prm;
  int32_t precision;
};

// Enqueue the whole job (init + iterations) on st.
far_status_t enqueue(far_map_s* m, AlignWS* w, const Job& j, int64_t max_tiles,
                     hipStream_t st) {
  MapView mv = m->view();
  k_build_tiles<<<1, 256, 0, st>>>(j.offsets, j.S, j.n_total, max_tiles, w->tile_scan,
                                   w->tile_lo, w->tile_hi, w->begin, w->bad);
  FAR_HIP(hipGetLastError());
  k_init<<<(j.S + 255) / 256, 256, 0, st>>>(j.S, j.T, w->bad, j.prm.recenter, j.c_fixed,
                                            j.stats, w->done, w->ctr);
  FAR_HIP(hipGetLastError());
  int64_t grid = max_tiles;
  int64_t cap = int64_t(device_cu_count()) * 16;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  const int iters = j.c_fixed ? 1 : j.prm.max_iters;
  for (int it = 0; it < iters; ++it) {
    if (j.precision == FAR_PREC_FP64)
      k_linearize<double><<<unsigned(grid), kTile, 0, st>>>(
          mv, j.src, j.cov6, j.valid, j.n_total, w->tile_scan, w->tile_lo, w->tile_hi,
          max_tiles, j.T, w->ctr, w->done, j.prm, w->partial, j.corr);
    else
      k_linearize<float><<<unsigned(grid), kTile, 0, st>>>(
          mv, j.src, j.cov6, j.valid, j.n_total, w->tile_scan, w->tile_lo, w->tile_hi,
          max_tiles, j.T, w->ctr, w->done, j.prm, w->partial, j.corr);
    FAR_HIP(hipGetLastError());
    k_reduce_solve<<<unsigned(j.S), 64, 0, st>>>(j.S, w->begin, w->partial, j.T, w->ctr,
                                                 w->done, j.stats, j.prm, j.c_fixed ? 0 : 1);
    FAR_HIP(hipGetLastError());
  }
  return FAR_OK;
}

// Run a job, through a cached graph when the stream allows capture.
far_status_t run_job(far_map_s* m, const Job& j, hipStream_t st, bool use_graph) {
  const int64_t max_tiles = (j.n_total + kTile - 1) / kTile + j.S;
  AlignWS* w = nullptr;
  FAR_TRY(ensure_ws(m, j.S, max_tiles, &w));
  (void)device_cu_count();   // query the device outside any capture
  if (!use_graph || st == nullptr) return enqueue(m, w, j, max_tiles, st);
  const void* key[10] = {j.src, j.offsets, j.cov6, j.valid, j.T, j.stats, j.c_fixed, j.corr,
                         m->vox_pts, nullptr};
  bool same = w->exec && w->key_n == j.n_total && w->key_S == j.S &&
              w->key_prec == j.precision && memcmp(w->key, key, sizeof(key)) == 0 &&
              memcmp(&w->key_prm, &j.prm, sizeof(Params)) == 0;
  if (!same) {
    if (w->exec) {
      FAR_HIP(hipGraphExecDestroy(w->exec));
      w->exec = nullptr;
    }
    hipGraph_t g = nullptr;
    FAR_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    far_status_t rs = enqueue(m, w, j, max_tiles, st);
    hipError_t e = hipStreamEndCapture(st, &g);
    if (rs != FAR_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rs;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
    e = hipGraphInstantiate(&w->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      w->exec = nullptr;
      return hip_fail(e, "hipGraphInstantiate", __FILE__, __LINE__);
    }
    memcpy(w->key, key, sizeof(key));
    w->key_n = j.n_total;
    w->key_S = j.S;
    w->key_prec = j.precision;
    w->key_prm = j.prm;
  }
  FAR_HIP(hipGraphLaunch(w->exec, st));
  return FAR_OK;
}

bool params_ok(const far_align_params_t* p) {
  return p && p->tau > 0.0 && std::isfinite(p->tau) && p->kappa > 0.0 &&
         std::isfinite(p->kappa) && p->max_iters >= 1 && p->max_iters <= 64 &&
         p->eps >= 0.0 && (p->precision == FAR_PREC_FP32 || p->precision == FAR_PREC_FP64);
}

Params make_params(const far_map_s* m, double tau, double kappa, double eps, int32_t max_iters,
                   int32_t recenter) {
  Params prm;
  double r = tau < m->p.voxel_size ? tau : m->p.voxel_size;
  prm.r2 = r * r;
  prm.kappa2 = kappa * kappa;
  prm.eps = eps;
  prm.max_iters = max_iters;
  prm.recenter = recenter ? 1 : 0;
  return prm;
}

void lin_from_stats(const far_align_stats_t& st, far_lin_t* out) { *out = st.last; }

}  // namespace
}  // namespace far

using namespace far;

extern "C" {

far_status_t far_gicp_linearize(far_map_t m, const float* src, const float* cov6,
                                const uint8_t* valid, int64_t n, const double T[16],
                                double tau, double kappa, const double c[3],
                                int32_t precision, int32_t* corr, far_lin_t* out,
                                far_stream_t stream) {
  if (!m || !T || !out || n < 0 || n >= (int64_t(1) << 31) || !(tau > 0.0) ||
      !(kappa > 0.0) || (n > 0 && (!src || !cov6 || !valid)) ||
      (precision != FAR_PREC_FP32 && precision != FAR_PREC_FP64)) {
    set_error("far_gicp_linearize: invalid argument");
    return FAR_E_INVALID;
  }
  memset(out, 0, sizeof(*out));
  if (n == 0) return FAR_OK;
  hipStream_t st = S(stream);
  AlignWS* w = nullptr;
  FAR_TRY(ensure_ws(m, 1, (n + kTile - 1) / kTile + 1, &w));
  int64_t offs[2] = {0, n};
  double cc[3] = {c ? c[0] : 0.0, c ? c[1] : 0.0, c ? c[2] : 0.0};
  FAR_HIP(hipMemcpyAsync(w->offsets, offs, sizeof(offs), hipMemcpyHostToDevice, st));
  FAR_HIP(hipMemcpyAsync(w->T, T, 16 * sizeof(double), hipMemcpyHostToDevice, st));
  FAR_HIP(hipMemcpyAsync(w->cfix, cc, sizeof(cc), hipMemcpyHostToDevice, st));
  Job j{src, w->offsets, 1, n, cov6, valid, w->T, w->stats, w->cfix, corr,
        make_params(m, tau, kappa, 0.0, 1, 0), precision};
  FAR_TRY(run_job(m, j, st, false));
  far_align_stats_t hs;
  FAR_HIP(hipMemcpyAsync(&hs, w->stats, sizeof(hs), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipStreamSynchronize(st));
  lin_from_stats(hs, out);
  return FAR_OK;
}

far_status_t far_gicp_align(far_map_t m, const float* src, const float* cov6,
                            const uint8_t* valid, int64_t n, const double T0[16],
                            const far_align_params_t* params, double T_out[16],
                            far_align_stats_t* stats, far_stream_t stream) {
  if (!m || !T0 || !T_out || !params_ok(params) || n < 0 || n >= (int64_t(1) << 31) ||
      (n > 0 && (!src || !cov6 || !valid))) {
    set_error("far_gicp_align: invalid argument");
    return FAR_E_INVALID;
  }
  far_align_stats_t hs;
  memset(&hs, 0, sizeof(hs));
  if (n == 0) {
    memcpy(T_out, T0, 16 * sizeof(double));
    hs.status = FAR_E_FEW_CORR;
    if (stats) *stats = hs;
    return FAR_E_FEW_CORR;
  }
  hipStream_t st = S(stream);
  AlignWS* w = nullptr;
  FAR_TRY(ensure_ws(m, 1, (n + kTile - 1) / kTile + 1, &w));
  int64_t offs[2] = {0, n};
  FAR_HIP(hipMemcpyAsync(w->offsets, offs, sizeof(offs), hipMemcpyHostToDevice, st));
  FAR_HIP(hipMemcpyAsync(w->T, T0, 16 * sizeof(double), hipMemcpyHostToDevice, st));
  Job j{src, w->offsets, 1, n, cov6, valid, w->T, w->stats, nullptr, nullptr,
        make_params(m, params->tau, params->kappa, params->eps, params->max_iters,
                    params->recenter),
        params->precision};
  FAR_TRY(run_job(m, j, st, true));
  FAR_HIP(hipMemcpyAsync(T_out, w->T, 16 * sizeof(double), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipMemcpyAsync(&hs, w->stats, sizeof(hs), hipMemcpyDeviceToHost, st));
  FAR_HIP(hipStreamSynchronize(st));
  if (stats) *stats = hs;
  return far_status_t(hs.status);
}

far_status_t far_gicp_align_batch(far_map_t m, const float* src, const int64_t* offsets,
                                  int32_t S_, int64_t n_total, const float* cov6,
                                  const uint8_t* valid, double* T,
                                  const far_align_params_t* params, far_align_stats_t* stats,
                                  far_stream_t stream) {
  if (!m || !offsets || !T || !stats || !params_ok(params) || S_ < 1 || n_total < 0 ||
      n_total >= (int64_t(1) << 31) || (n_total > 0 && (!src || !cov6 || !valid))) {
    set_error("far_gicp_align_batch: invalid argument");
    return FAR_E_INVALID;
  }
  hipStream_t st = S(stream);
  Job j{src, offsets, S_, n_total, cov6, valid, T, stats, nullptr, nullptr,
        make_params(m, params->tau, params->kappa, params->eps, params->max_iters,
                    params->recenter),
        params->precision};
  return run_job(m, j, st, true);
}

}  // extern "C"
