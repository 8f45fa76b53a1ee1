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

// A query with an FP32 screen.  Every candidate's squared distance is first
// formed in FP32 from the query rounded to FP32; only candidates whose FP32
// value is within the screen bound get the exact FP64 evaluation that decides.
//
// The screen is conservative: with D = q - fl32(p) exactly, |D - d| <= delta,
// delta = 2^-24 (|px| + |py| + |pz|) (rounding of p to FP32), and the FP32
// subtraction and fused sum of squares add at most a factor (1 + 2^-24)^5.
// So any candidate with exact d2 <= B has FP32 value
// <= (sqrt(B) + delta)^2 (1 + 2^-24)^5, which screen_bound over-estimates:
// it works in FP32 (no FP64 square root in the candidate loop), with margin
// m >= 2 delta and factors that outweigh every rounding on the way - the
// conversion of B and the square root (2^-23 each, covered by 1 + 2^-21
// twice), the sum and the square (2^-24 each) and the (1 + 2^-24)^5 above
// (all covered by 1 + 2^-19).  A floor of 2^-100 keeps distances that
// underflow FP32 inside the screen.
struct Query {
  double x, y, z;
  float fx, fy, fz;
  float m;
  float bound_f;
};

__device__ inline float screen_bound(double B, float m) {
  const float s = sqrtf(float(B) * (1.0f + 0x1p-21f)) * (1.0f + 0x1p-21f) + m;
  return fmaxf(s * s * (1.0f + 0x1p-19f), 0x1p-100f);
}

__device__ inline Query make_query(double x, double y, double z, double r2) {
  Query q;
  q.x = x;
  q.y = y;
  q.z = z;
  q.fx = float(x);
  q.fy = float(y);
  q.fz = float(z);
  q.m = float(0x1p-23 * (fabs(x) + fabs(y) + fabs(z)) + 1e-30) * (1.0f + 0x1p-21f);
  q.bound_f = screen_bound(r2, q.m);
  return q;
}

// Rank the cnt points stored at pts[base ...] against q.  Loads are issued
// kW at a time (4 by default) so that they overlap instead of waiting one by
// one.
template <int K, int kW = 4>
__device__ inline void scan_voxel_points(const float4* pts, int32_t base, int32_t cnt,
                                         Query& q, double r2, TopK<K>& top) {
  for (int32_t j = 0; j < cnt; j += kW) {
    float4 p[kW];
#pragma unroll
    for (int u = 0; u < kW; ++u)
      if (j + u < cnt) p[u] = pts[base + j + u];
#pragma unroll
    for (int u = 0; u < kW; ++u)
      if (j + u < cnt) {
        const float dx = p[u].x - q.fx, dy = p[u].y - q.fy, dz = p[u].z - q.fz;
        const float d2f = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
        if (d2f <= q.bound_f) {
          const double d = dist2(double(p[u].x), double(p[u].y), double(p[u].z), q.x, q.y, q.z);
          const int32_t id = __float_as_int(p[u].w);
          if (d <= r2 && rank_less(d, id, top.d[K - 1], top.id[K - 1])) {
            top.push(d, id, base + j + u);
            q.bound_f = screen_bound(fmin(r2, top.bound()), q.m);
          }
        }
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
  Query q = make_query(qx, qy, qz, r2);
  for (int t = 0; t < 27; ++t) {
    int code = kNbrOrder[t];
    int ox = code / 9 - 1, oy = (code / 3) % 3 - 1, oz = code % 3 - 1;
    double bnd = fmin(r2, top.bound());
    if (voxel_lb2(qx, qy, qz, kx, ky, kz, ox, oy, oz, m.v) > bnd) continue;
    int32_t cnt;
    int32_t vox = map_find(m, kx + ox, ky + oy, kz + oz, &cnt);
    if (vox < 0) continue;
    scan_voxel_points<K>(m.vox_pts, vox * m.nmax, cnt, q, r2, top);
  }
}

// Neighbour offsets in visiting order (faces, edges, corners), packed five
// bits per entry as code = (ox+1)*9 + (oy+1)*3 + (oz+1): ranks 1-12, 13-24,
// 25-26 in three words.
__device__ inline int nbr_code(int rank) {
  constexpr uint64_t w0 = (uint64_t(4) << 0) | (uint64_t(22) << 5) | (uint64_t(10) << 10) |
                          (uint64_t(16) << 15) | (uint64_t(12) << 20) | (uint64_t(14) << 25) |
                          (uint64_t(1) << 30) | (uint64_t(3) << 35) | (uint64_t(5) << 40) |
                          (uint64_t(7) << 45) | (uint64_t(9) << 50) | (uint64_t(11) << 55);
  constexpr uint64_t w1 = (uint64_t(15) << 0) | (uint64_t(17) << 5) | (uint64_t(19) << 10) |
                          (uint64_t(21) << 15) | (uint64_t(23) << 20) | (uint64_t(25) << 25) |
                          (uint64_t(0) << 30) | (uint64_t(2) << 35) | (uint64_t(6) << 40) |
                          (uint64_t(8) << 45) | (uint64_t(18) << 50) | (uint64_t(20) << 55);
  constexpr uint64_t w2 = (uint64_t(24) << 0) | (uint64_t(26) << 5);
  const int r = rank - 1;
  const uint64_t w = r < 12 ? w0 : (r < 24 ? w1 : w2);
  const int sh = 5 * (r < 12 ? r : (r < 24 ? r - 12 : r - 24));
  return int((w >> sh) & 31u);
}

__device__ inline double lb2_of(const double* gl2, const double* gh2, int code) {
  const int ox = code / 9 - 1, oy = (code / 3) % 3 - 1, oz = code % 3 - 1;
  return (ox < 0 ? gl2[0] : (ox > 0 ? gh2[0] : 0.0)) + (oy < 0 ? gl2[1] : (oy > 0 ? gh2[1] : 0.0)) +
         (oz < 0 ? gl2[2] : (oz > 0 ? gh2[2] : 0.0));
}

// Exact K nearest points within sqrt(r2) of p over a grid of cells of edge
// c, with r <= range * c (range 1 or 2): every such point lies within
// `range` cells per axis of p's own cell.  Visits the own cell, then the 26
// cells around it - each lane keeps the ones it still needs (lower bound <=
// current K-th best) as a bit mask and takes its own next one in lockstep -
// then, when range is 2 and the K-th best can still be beaten there, the 98
// cells two away.  find(kx, ky, kz, &cnt) gives the start of the cell's run
// in pts (or -1) and its length.
template <int K, class Find>
__device__ inline void knn_cells(double px, double py, double pz, double c, double inv_c,
                                 bool pow2, bool range2, double r2, const float4* pts,
                                 Find find, TopK<K>& top) {
  top.init();
  const double fx = floor(pow2 ? px * inv_c : px / c), fy = floor(pow2 ? py * inv_c : py / c),
               fz = floor(pow2 ? pz * inv_c : pz / c);
  const double lim = double(kKeyBias);
  if (!(fx >= -lim && fx < lim && fy >= -lim && fy < lim && fz >= -lim && fz < lim)) return;
  const int64_t kx = int64_t(fx), ky = int64_t(fy), kz = int64_t(fz);
  const double slack = 1e-7 * c;
  double gl[3], gh[3], gl2[3], gh2[3];
  gl[0] = fmax(px - fx * c - slack, 0.0); gh[0] = fmax((fx + 1.0) * c - px - slack, 0.0);
  gl[1] = fmax(py - fy * c - slack, 0.0); gh[1] = fmax((fy + 1.0) * c - py - slack, 0.0);
  gl[2] = fmax(pz - fz * c - slack, 0.0); gh[2] = fmax((fz + 1.0) * c - pz - slack, 0.0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    gl2[a] = gl[a] * gl[a];
    gh2[a] = gh[a] * gh[a];
  }
  Query q = make_query(px, py, pz, r2);
  int32_t cnt;
  int32_t st = find(kx, ky, kz, &cnt);
  if (st >= 0) scan_voxel_points<K>(pts, st, cnt, q, r2, top);
  uint32_t need = 0;
  {
    const double bnd = fmin(r2, top.bound());
#pragma unroll
    for (int rank = 1; rank < 27; ++rank)
      if (lb2_of(gl2, gh2, nbr_code(rank)) <= bnd) need |= 1u << rank;
  }
  while (need) {
    const int rank = __builtin_ctz(need);
    need &= need - 1;
    const int code = nbr_code(rank);
    if (lb2_of(gl2, gh2, code) > fmin(r2, top.bound())) continue;
    st = find(kx + code / 9 - 1, ky + (code / 3) % 3 - 1, kz + code % 3 - 1, &cnt);
    if (st >= 0) scan_voxel_points<K>(pts, st, cnt, q, r2, top);
  }
  if (!range2) return;
  // cells two away along some axis lie at least one cell beyond a face
  const double far_lb2 =
      fmin(fmin(fmin((gl[0] + c) * (gl[0] + c), (gh[0] + c) * (gh[0] + c)),
                fmin((gl[1] + c) * (gl[1] + c), (gh[1] + c) * (gh[1] + c))),
           fmin((gl[2] + c) * (gl[2] + c), (gh[2] + c) * (gh[2] + c)));
  if (far_lb2 > fmin(r2, top.bound())) return;
  for (int ox = -2; ox <= 2; ++ox)
    for (int oy = -2; oy <= 2; ++oy)
      for (int oz = -2; oz <= 2; ++oz) {
        if (ox > -2 && ox < 2 && oy > -2 && oy < 2 && oz > -2 && oz < 2) continue;
        const double g0 = ox < 0 ? gl[0] + (ox == -2 ? c : 0.0) : (ox > 0 ? gh[0] + (ox == 2 ? c : 0.0) : 0.0);
        const double g1 = oy < 0 ? gl[1] + (oy == -2 ? c : 0.0) : (oy > 0 ? gh[1] + (oy == 2 ? c : 0.0) : 0.0);
        const double g2 = oz < 0 ? gl[2] + (oz == -2 ? c : 0.0) : (oz > 0 ? gh[2] + (oz == 2 ? c : 0.0) : 0.0);
        if ((g0 * g0 + g1 * g1) + g2 * g2 > fmin(r2, top.bound())) continue;
        st = find(kx + ox, ky + oy, kz + oz, &cnt);
        if (st >= 0) scan_voxel_points<K>(pts, st, cnt, q, r2, top);
      }
}

// Smallest float not below d (d finite and non-negative): a float compared
// with it keeps every case the comparison with d keeps and adds at most the
// ties with the rounded value, which only adds visits to an exact search.
__device__ inline float f32_up(double d) {
  float f = float(d);
  if (double(f) < d) f = __uint_as_float(__float_as_uint(f) + 1u);
  return f;
}

// Squared face distance as a float that never exceeds the FP64 value:
// rounded down and shrunk by 2^-20 (which also covers the rounding of the
// float sums of up to three such terms).  Used only to skip cells.
__device__ inline float lb_down_sq(double g) {
  return __double2float_rd(g * g) * (1.0f - 0x1p-20f);
}

// Rank the cnt points of a run stored at pts[st ...] against q, taking them
// outward from position i0 (the right side from i0 up, the left side from
// i0 - 1 down), two per side at a time so that four loads are in flight.
// In a run sorted by x up to a quantum, no point after the last one taken on
// a side lies more than mx back towards the query along x than it, so the
// side stops once that point's x gap less mx exceeds the current bound on
// the distance (every later point is then strictly farther than the K-th
// best or the radius).  mx = infinity never stops: the whole run is ranked.
// The set ranked is a superset of the candidates that can enter, so the
// result is the K best by (d2, id) whatever i0 is.
template <int K>
__device__ inline void scan_run_x(const float4* pts, int32_t st, int32_t cnt, int32_t i0,
                                  Query& q, double r2, double mx, TopK<K>& top) {
  const int32_t e = st + cnt;
  int32_t r = i0, l = i0 - 1;
  bool ra = r < e, la = l >= st;
  while (ra || la) {
    const bool u0 = ra, u1 = ra && r + 1 < e, u2 = la, u3 = la && l - 1 >= st;
    // the four loads unconditional, at indices clamped into the run (the
    // loop runs only on a run of at least one point), so that they go out
    // together: loads under their own conditions were issued one after the
    // other, each waiting for the one before
    const float4 p0 = pts[min(r, e - 1)];
    const float4 p1 = pts[min(r + 1, e - 1)];
    const float4 p2 = pts[max(l, st)];
    const float4 p3 = pts[max(l - 1, st)];
    auto rank_one = [&](const float4& pp, int32_t at) {
      const float dx = pp.x - q.fx, dy = pp.y - q.fy, dz = pp.z - q.fz;
      const float d2f = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
      if (d2f <= q.bound_f) {
        const double d = dist2(double(pp.x), double(pp.y), double(pp.z), q.x, q.y, q.z);
        const int32_t id = __float_as_int(pp.w);
        if (d <= r2 && rank_less(d, id, top.d[K - 1], top.id[K - 1])) {
          top.push(d, id, at);
          q.bound_f = screen_bound(fmin(r2, top.bound()), q.m);
        }
      }
    };
    if (u0) rank_one(p0, r);
    if (u1) rank_one(p1, r + 1);
    if (u2) rank_one(p2, l);
    if (u3) rank_one(p3, l - 1);
    // a gap g beats the bound b when g > 0 and g^2 (shrunk by 2^-40 against
    // the rounding of the FP64 distances it stands for) exceeds b
    const double b = fmin(r2, top.bound());
    if (ra) {
      const double g = (double(u1 ? p1.x : p0.x) - q.x) - mx;
      r += u1 ? 2 : 1;
      ra = r < e && !(g > 0.0 && g * g * (1.0 - 0x1p-40) > b);
    }
    if (la) {
      const double g = (q.x - double(u3 ? p3.x : p2.x)) - mx;
      l -= u3 ? 2 : 1;
      la = l >= st && !(g > 0.0 && g * g * (1.0 - 0x1p-40) > b);
    }
  }
}

// Exact K nearest points within sqrt(r2) of p over a grid of cells of edge
// c >= sqrt(r2) (the 27 cells around p's own cell hold every candidate),
// with the visiting rule of knn_cells for range 1: own cell, then each
// neighbour cell whose conservative lower bound can still beat the current
// K-th best, taken in lockstep from a per-lane bit mask.  Bounds are kept as
// floats to save registers.  find(code, &cnt) gives the start of the run in
// the cell at offset code = (ox+1)*9 + (oy+1)*3 + oz+1 from p's own cell (or
// -1) and its length.  Each cell's
// run is ranked by scan_run_x from where p's x falls in it: p's own sorted
// position own in its own cell (own < 0: the run's start), the run's start
// or end for the cells beside or behind p's along x, and for the cells of
// p's own x layer the position that p's fraction of the cell width gives
// (exact for any start; near p's x when the run's points spread evenly).
template <int K, class Find>
__device__ inline void knn_cells27(double px, double py, double pz, double c, double inv_c,
                                   bool pow2, double r2, const float4* pts, int32_t own,
                                   double mx, Find find, TopK<K>& top) {
  top.init();
  const double tx = pow2 ? px * inv_c : px / c;
  const double fx = floor(tx), fy = floor(pow2 ? py * inv_c : py / c),
               fz = floor(pow2 ? pz * inv_c : pz / c);
  const double lim = double(kKeyBias);
  if (!(fx >= -lim && fx < lim && fy >= -lim && fy < lim && fz >= -lim && fz < lim)) return;
  const float ux = float(tx - fx);     // p's fraction of its cell along x, in [0, 1]
  const double slack = 1e-7 * c;
  float gl2[3], gh2[3];
  gl2[0] = lb_down_sq(fmax(px - fx * c - slack, 0.0)); gh2[0] = lb_down_sq(fmax((fx + 1.0) * c - px - slack, 0.0));
  gl2[1] = lb_down_sq(fmax(py - fy * c - slack, 0.0)); gh2[1] = lb_down_sq(fmax((fy + 1.0) * c - py - slack, 0.0));
  gl2[2] = lb_down_sq(fmax(pz - fz * c - slack, 0.0)); gh2[2] = lb_down_sq(fmax((fz + 1.0) * c - pz - slack, 0.0));
  Query q = make_query(px, py, pz, r2);
  int32_t cnt;
  int32_t st = find(13, &cnt);
  if (st >= 0) scan_run_x<K>(pts, st, cnt, own >= 0 ? own : st, q, r2, mx, top);
  // two plain selects per axis (a nested conditional compiles to divergent
  // branches for a run-time code); the value is the same
  auto gap = [](int o, float lo, float hi) {
    const float t = o < 0 ? lo : 0.0f;
    return o > 0 ? hi : t;
  };
  auto lb = [&](int code) {
    const int ox = code / 9 - 1, oy = (code / 3) % 3 - 1, oz = code % 3 - 1;
    return double((gap(ox, gl2[0], gh2[0]) + gap(oy, gl2[1], gh2[1])) +
                  gap(oz, gl2[2], gh2[2]));
  };
  uint32_t need = 0;
  {
    const float bnd = f32_up(fmin(r2, top.bound()));
#pragma unroll
    for (int rank = 1; rank < 27; ++rank) {
      const int code = nbr_code(rank);
      const int ox = code / 9 - 1, oy = (code / 3) % 3 - 1, oz = code % 3 - 1;
      const float s = (ox < 0 ? gl2[0] : (ox > 0 ? gh2[0] : 0.0f)) +
                      (oy < 0 ? gl2[1] : (oy > 0 ? gh2[1] : 0.0f)) +
                      (oz < 0 ? gl2[2] : (oz > 0 ? gh2[2] : 0.0f));
      if (s <= bnd) need |= 1u << rank;
    }
  }
  while (need) {
    const int rank = __builtin_ctz(need);
    need &= need - 1;
    const int code = nbr_code(rank);
    if (lb(code) > fmin(r2, top.bound())) continue;
    const int ox = code / 9 - 1;
    st = find(code, &cnt);
    if (st >= 0) {
      // start: cnt * (p's x position in cells from the cell's low face),
      // clamped to the run: its end for ox = -1, its start for ox = 1
      const float w = fminf(fmaxf(float(cnt) * (ux - float(ox)), 0.0f), float(cnt));
      scan_run_x<K>(pts, st, cnt, st + min(int32_t(w), cnt), q, r2, mx, top);
    }
  }
}

// Plane regularisation after Segal et al., beside Eq. (1): I + (eps - 1) n n^T
// with eps = 1e-3 and n the unit eigenvector of the smallest eigenvalue of the
// sample covariance S, in FP64.  The smallest eigenvalue comes from the
// trigonometric solution of the characteristic cubic of a symmetric 3x3; n is
// the longest cross product of two rows of S - lambda I.  Degenerate cases:
// S diagonal gives the axis of its smallest entry (ties: the lowest axis),
// as a diagonalisation with no rotation does; when S - lambda I has rank one
// or less (a double smallest eigenvalue) any unit vector orthogonal to its
// largest row is an eigenvector, and one is taken.
__device__ inline void plane_regularised(double s00, double s01, double s02, double s11,
                                         double s12, double s22, double out[6]) {
  double n0 = 1.0, n1 = 0.0, n2 = 0.0;
  const double p1 = (s01 * s01 + s02 * s02) + s12 * s12;
  if (p1 == 0.0) {
    int a = 0;
    double m = s00;
    if (s11 < m) { a = 1; m = s11; }
    if (s22 < m) a = 2;
    n0 = a == 0 ? 1.0 : 0.0;
    n1 = a == 1 ? 1.0 : 0.0;
    n2 = a == 2 ? 1.0 : 0.0;
  } else {
    const double q = (s00 + s11 + s22) / 3.0;
    const double b00 = s00 - q, b11 = s11 - q, b22 = s22 - q;
    const double p2 = (b00 * b00 + b11 * b11 + b22 * b22) + 2.0 * p1;
    const double p = sqrt(p2 / 6.0), ip = 1.0 / p;
    const double c00 = b00 * ip, c11 = b11 * ip, c22 = b22 * ip;
    const double c01 = s01 * ip, c02 = s02 * ip, c12 = s12 * ip;
    double r = 0.5 * ((c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02)) +
                      c02 * (c01 * c12 - c11 * c02));
    r = fmin(1.0, fmax(-1.0, r));
    // eigenvalues q + 2 p cos(phi + 2 pi j / 3), phi = acos(r) / 3: j = 1 is
    // the smallest
    const double lam = q + 2.0 * p * cos(acos(r) / 3.0 + 2.0943951023931957);
    // rows of S - lambda I and their pairwise cross products, selected with
    // scalar compares (no dynamic indexing: the arrays stay in registers)
    const double a0 = s00 - lam, a1 = s01, a2 = s02;
    const double b0 = s01, b1 = s11 - lam, b2 = s12;
    const double d0 = s02, d1 = s12, d2 = s22 - lam;
    const double x0 = a1 * b2 - a2 * b1, x1 = a2 * b0 - a0 * b2, x2 = a0 * b1 - a1 * b0;
    const double y0 = a1 * d2 - a2 * d1, y1 = a2 * d0 - a0 * d2, y2 = a0 * d1 - a1 * d0;
    const double z0 = b1 * d2 - b2 * d1, z1 = b2 * d0 - b0 * d2, z2 = b0 * d1 - b1 * d0;
    const double dx = (x0 * x0 + x1 * x1) + x2 * x2;
    const double dy = (y0 * y0 + y1 * y1) + y2 * y2;
    const double dz = (z0 * z0 + z1 * z1) + z2 * z2;
    double c0 = x0, c1 = x1, c2 = x2, dm = dx;
    if (dy > dm) { c0 = y0; c1 = y1; c2 = y2; dm = dy; }
    if (dz > dm) { c0 = z0; c1 = z1; c2 = z2; dm = dz; }
    const double f2 = (s00 * s00 + s11 * s11 + s22 * s22) + 2.0 * p1;   // |S|_F^2
    if (dm > 1e-30 * f2 * f2) {
      const double il = 1.0 / sqrt(dm);
      n0 = c0 * il;
      n1 = c1 * il;
      n2 = c2 * il;
    } else {
      // rank <= 1: a unit vector orthogonal to the largest row w, as w x e_a
      // with a the axis where |w| is smallest
      const double na = (a0 * a0 + a1 * a1) + a2 * a2;
      const double nb = (b0 * b0 + b1 * b1) + b2 * b2;
      const double nd = (d0 * d0 + d1 * d1) + d2 * d2;
      double w0 = a0, w1 = a1, w2 = a2, nw = na;
      if (nb > nw) { w0 = b0; w1 = b1; w2 = b2; nw = nb; }
      if (nd > nw) { w0 = d0; w1 = d1; w2 = d2; nw = nd; }
      if (nw > 0.0) {
        double t0, t1, t2;
        if (fabs(w0) <= fabs(w1) && fabs(w0) <= fabs(w2)) {        // w x e_x
          t0 = 0.0; t1 = w2; t2 = -w1;
        } else if (fabs(w1) <= fabs(w2)) {                          // w x e_y
          t0 = -w2; t1 = 0.0; t2 = w0;
        } else {                                                    // w x e_z
          t0 = w1; t1 = -w0; t2 = 0.0;
        }
        const double il = 1.0 / sqrt((t0 * t0 + t1 * t1) + t2 * t2);
        n0 = t0 * il;
        n1 = t1 * il;
        n2 = t2 * il;
      }
    }
  }
  const double e = 1e-3 - 1.0;
  out[0] = 1.0 + e * n0 * n0;
  out[1] = e * n0 * n1;
  out[2] = e * n0 * n2;
  out[3] = 1.0 + e * n1 * n1;
  out[4] = e * n1 * n2;
  out[5] = 1.0 + e * n2 * n2;
}

// Regularised covariance of the first k entries of a neighbour list:
// two-pass FP64 sample covariance with 1/k, then with reg = FAR_REG_EQ1
// Eq. (1): C = S + 1e-3 I and Sigma = (C^-1 / ||C^-1||_F)^-1 = ||C^-1||_F C,
// where ||C^-1||_F is the Frobenius norm of the cofactor matrix over
// |det C|; with reg = FAR_REG_PLANE the plane regularisation above.
template <int K, class Get>
__device__ inline void regularised_cov(const TopK<K>& top, int k, Get get, double out[6],
                                       int reg) {
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
  if (reg == FAR_REG_PLANE) {
    plane_regularised(sxx * inv_k, sxy * inv_k, sxz * inv_k, syy * inv_k, syz * inv_k,
                      szz * inv_k, out);
    return;
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
