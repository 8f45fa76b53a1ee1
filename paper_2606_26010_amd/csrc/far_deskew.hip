// far_deskew.hip -- motion undistortion of LiDAR scans (Sec. III-A.1).
//
// The velocity history of the sensor fusion is fitted per scan by a straight
// line per twist component (least squares, centred on the mean sample time),
// and every raw point is carried from the sensor frame of its own firing time
// t_i to the frame of the scan's reference time t_ref (its largest finite
// point time) by the SE(3) exponential of the fitted twist integrated over
// [t_ref, t_i]: for a twist linear in time that integral is
// (t_i - t_ref) * xi((t_i + t_ref) / 2).
//
// Two launches per call on the caller's stream, with no memset and no global
// atomic (so a caller may capture them in a graph):
//   k_ud_scan   fit blocks: one wave per scan, the three-pass least-squares
//               fit in FP64 with butterfly wave sums (fixed order,
//               deterministic), from the samples held in registers; chunk
//               blocks, in the same grid: the maximum finite point time of
//               every scan a chunk of kUdChunk points touches, as
//               order-preserving integer encodings of the float: per chunk
//               the maxima of its first and last scan, and for scans lying
//               wholly inside the chunk a plain store (no other block
//               touches them);
//   k_ud_apply  four points per lane: t_ref of the block's scan reduced from
//               the chunk maxima while its points load, then the FP64
//               exponential (Taylor series of its coefficients for rotations
//               up to 1/2 rad), rounded once to float on output; trailing
//               blocks write the reference times, one wave per scan.
// Each point costs 16 bytes read (xyz, t) and 12 written.

#include <cmath>
#include <mutex>

#include "far_internal.h"

namespace far {
namespace {

constexpr int kUdBlock = 256;
constexpr int kUdPerThread = 16;          // points per lane of a chunk block
constexpr int kUdChunk = kUdBlock * kUdPerThread;
constexpr int kUdCoef = 16;               // tbar, a[6], b[6], 3 spare
constexpr int kUdLdsOff = 1024;           // offsets searched in LDS up to this S
constexpr int kUdLdsScans = 1024;         // scans per round of a mixed chunk
constexpr int kUdSamples = 1;             // velocity samples per lane in registers

// Order-preserving map of finite floats to unsigned integers, 0 = no value.
__device__ inline uint32_t time_enc(float t) {
  uint32_t u = __float_as_uint(t);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline double time_dec(uint32_t e) {
  if (e == 0) return __longlong_as_double(0x7FF8000000000000ll);   // NaN
  uint32_t u = (e & 0x80000000u) ? (e ^ 0x80000000u) : ~e;
  return double(__uint_as_float(u));
}

// Scan of point i: the last s with off[s] <= i, searched in [lo, hi].
__device__ inline int scan_of(const int64_t* off, int lo, int hi, int64_t i) {
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Scan range [lo, hi] of the points [i0, i1] of a block (off NULL: one scan).
// The offsets go through LDS when they fit, so that the search costs one
// global round trip (all lanes load) instead of one per bisection step.
__device__ inline void block_scans(const int64_t* off, int S, int64_t i0, int64_t i1, int* lo,
                                   int* hi) {
  __shared__ int s_rng[2];
  __shared__ int64_t s_off[kUdLdsOff + 1];
  const bool lds = off && S <= kUdLdsOff;
  if (lds)
    for (int j = threadIdx.x; j <= S; j += blockDim.x) s_off[j] = off[j];
  __syncthreads();
  if (threadIdx.x == 0) {
    if (off) {
      const int64_t* o = lds ? s_off : off;
      s_rng[0] = scan_of(o, 0, S - 1, i0);
      s_rng[1] = scan_of(o, s_rng[0], S - 1, i1);
    } else {
      s_rng[0] = s_rng[1] = 0;
    }
  }
  __syncthreads();
  *lo = s_rng[0];
  *hi = s_rng[1];
}

// Maximum of m over the block, valid in thread 0.
__device__ inline uint32_t block_max(uint32_t m) {
  __shared__ uint32_t s_m[kUdBlock / 64];
  for (int d = 32; d >= 1; d >>= 1) m = max(m, uint32_t(__shfl_xor(int(m), d)));
  __syncthreads();                      // s_m free from a previous round
  if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < kUdBlock / 64; ++w) m = max(m, s_m[w]);
  return m;
}

__device__ inline double wave_sum(double x) {
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
  return x;
}

// Time maxima of one chunk: part[c] = {first scan, last scan, max over the
// chunk's points of its first scan, of its last scan}; mid[s] for scans
// strictly between them.
__device__ void chunk_times(const float* __restrict__ t, const int64_t* __restrict__ off, int S,
                            int64_t n, int64_t c, int4* __restrict__ part,
                            uint32_t* __restrict__ mid) {
  const int64_t base = c * kUdChunk;
  const int64_t last = min(base + kUdChunk, n) - 1;
  uint32_t e[kUdPerThread];
#pragma unroll
  for (int j = 0; j < kUdPerThread; ++j) {
    const int64_t i = base + j * kUdBlock + threadIdx.x;
    const float v = t[min(i, last)];
    e[j] = (i <= last && isfinite(v)) ? time_enc(v) : 0u;
  }
  int lo, hi;
  block_scans(off, S, base, last, &lo, &hi);
  if (lo == hi) {
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < kUdPerThread; ++j) m = max(m, e[j]);
    m = block_max(m);
    if (threadIdx.x == 0) part[c] = make_int4(lo, hi, int(m), int(m));
    return;
  }
  // several scans: per-scan maxima by LDS atomics, kUdLdsScans scans a round
  __shared__ uint32_t s_mx[kUdLdsScans];
  __shared__ uint32_t s_end[2];
  int sj[kUdPerThread];
#pragma unroll
  for (int j = 0; j < kUdPerThread; ++j)
    sj[j] = scan_of(off, lo, hi, min(base + j * kUdBlock + threadIdx.x, last));
  for (int r0 = lo; r0 <= hi; r0 += kUdLdsScans) {
    const int r1 = min(hi, r0 + kUdLdsScans - 1);
    for (int s = r0 + threadIdx.x; s <= r1; s += kUdBlock) s_mx[s - r0] = 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kUdPerThread; ++j)
      if (e[j] && sj[j] >= r0 && sj[j] <= r1) atomicMax(&s_mx[sj[j] - r0], e[j]);
    __syncthreads();
    for (int s = r0 + threadIdx.x; s <= r1; s += kUdBlock) {
      const uint32_t v = s_mx[s - r0];
      if (s == lo) s_end[0] = v;
      else if (s == hi) s_end[1] = v;
      else mid[s] = v;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[c] = make_int4(lo, hi, int(s_end[0]), int(s_end[1]));
}

// Fit of scan s by the first wave of its block: coef[s] = {tbar, a[6], b[6]};
// with no points at all also the NaN reference time.
__device__ void fit_scan(int s, const double* __restrict__ ts, const double* __restrict__ xi,
                         const int64_t* __restrict__ voff, int64_t m, double* __restrict__ coef,
                         double* __restrict__ t_ref_out, int no_points) {
  const int lane = threadIdx.x;
  const int64_t j0 = voff ? voff[s] : 0;
  const int64_t j1 = voff ? voff[s + 1] : m;
  // the first kUdSamples * 64 samples stay in registers over the three passes
  double rt[kUdSamples], rx[kUdSamples][6];
  bool ok[kUdSamples];
#pragma unroll
  for (int q = 0; q < kUdSamples; ++q) {
    const int64_t j = j0 + q * 64 + lane;
    ok[q] = j < j1;
    const int64_t jj = ok[q] ? j : j0;
    rt[q] = ok[q] ? ts[jj] : 0.0;
    for (int k = 0; k < 6; ++k) rx[q][k] = ok[q] ? xi[jj * 6 + k] : 0.0;
    bool fin = isfinite(rt[q]);
    for (int k = 0; k < 6; ++k) fin = fin && isfinite(rx[q][k]);
    ok[q] = ok[q] && fin;
  }
  auto usable = [&](int64_t j) {
    bool u = isfinite(ts[j]);
    for (int k = 0; k < 6; ++k) u = u && isfinite(xi[j * 6 + k]);
    return u;
  };
  const int64_t jr = j0 + kUdSamples * 64;    // samples beyond the registers
  double cnt = 0.0, st = 0.0;
#pragma unroll
  for (int q = 0; q < kUdSamples; ++q)
    if (ok[q]) { cnt += 1.0; st += rt[q]; }
  for (int64_t j = jr + lane; j < j1; j += 64)
    if (usable(j)) { cnt += 1.0; st += ts[j]; }
  cnt = wave_sum(cnt);
  st = wave_sum(st);
  double tb = 0.0, a[6] = {0, 0, 0, 0, 0, 0}, b[6] = {0, 0, 0, 0, 0, 0};
  if (cnt > 0.0) {
    tb = st / cnt;
    double stt = 0.0, sy[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < kUdSamples; ++q)
      if (ok[q]) {
        const double dt = rt[q] - tb;
        stt += dt * dt;
        for (int k = 0; k < 6; ++k) sy[k] += rx[q][k];
      }
    for (int64_t j = jr + lane; j < j1; j += 64)
      if (usable(j)) {
        const double dt = ts[j] - tb;
        stt += dt * dt;
        for (int k = 0; k < 6; ++k) sy[k] += xi[j * 6 + k];
      }
    stt = wave_sum(stt);
    for (int k = 0; k < 6; ++k) a[k] = wave_sum(sy[k]) / cnt;
    double sty[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < kUdSamples; ++q)
      if (ok[q]) {
        const double dt = rt[q] - tb;
        for (int k = 0; k < 6; ++k) sty[k] += dt * (rx[q][k] - a[k]);
      }
    for (int64_t j = jr + lane; j < j1; j += 64)
      if (usable(j)) {
        const double dt = ts[j] - tb;
        for (int k = 0; k < 6; ++k) sty[k] += dt * (xi[j * 6 + k] - a[k]);
      }
    for (int k = 0; k < 6; ++k) {
      const double v = wave_sum(sty[k]);
      b[k] = stt > 0.0 ? v / stt : 0.0;
    }
  }
  if (lane == 0) {
    double* c = coef + size_t(s) * kUdCoef;
    c[0] = tb;
    for (int k = 0; k < 6; ++k) { c[1 + k] = a[k]; c[7 + k] = b[k]; }
    if (t_ref_out && no_points) t_ref_out[s] = time_dec(0);
  }
}

// Blocks [0, S) fit one scan each (first, so that their latency-bound
// passes overlap the chunks), blocks [S, S + n_chunks) take the point chunks.
__global__ __launch_bounds__(kUdBlock) void k_ud_scan(
    const float* __restrict__ t, const int64_t* __restrict__ off, int S, int64_t n,
    int64_t n_chunks, int4* __restrict__ part, uint32_t* __restrict__ mid,
    const double* __restrict__ ts, const double* __restrict__ xi,
    const int64_t* __restrict__ voff, int64_t m, double* __restrict__ coef,
    double* __restrict__ t_ref_out) {
  const int64_t b = blockIdx.x;
  if (b >= S) {
    chunk_times(t, off, S, n, b - S, part, mid);
    return;
  }
  if (threadIdx.x >= 64) return;
  fit_scan(int(b), ts, xi, voff, m, coef, t_ref_out, n == 0 ? 1 : 0);
}

// Encoded time maximum of scan s over the chunks c_begin, c_begin + c_step,
// ... up to c_end (0: no finite time).
__device__ inline uint32_t scan_tmax(int s, const int4* part, const uint32_t* mid,
                                     int64_t c_begin, int64_t c_end, int64_t c_step) {
  uint32_t m = 0;
  for (int64_t c = c_begin; c <= c_end; c += c_step) {
    const int4 P = part[c];
    const uint32_t v = P.x == s ? uint32_t(P.z) : (P.y == s ? uint32_t(P.w) : mid[s]);
    m = max(m, v);
  }
  return m;
}

// Time maximum of scan s by one lane (0 for an empty scan).
__device__ inline uint32_t scan_tmax_lane(const int64_t* off, int s, int64_t n, const int4* part,
                                          const uint32_t* mid) {
  const int64_t p0 = off ? off[s] : 0;
  const int64_t p1 = off ? off[s + 1] : n;
  if (p1 <= p0) return 0;
  return scan_tmax(s, part, mid, p0 / kUdChunk, (p1 - 1) / kUdChunk, 1);
}

__device__ inline void cross(const double u[3], const double v[3], double out[3]) {
  out[0] = fma(u[1], v[2], -u[2] * v[1]);
  out[1] = fma(u[2], v[0], -u[0] * v[2]);
  out[2] = fma(u[0], v[1], -u[1] * v[0]);
}

// Point p taken at time ti, moved to the frame of time tr with the fitted
// twist c = {tbar, a[6], b[6]}, in FP64; written to o as floats.
__device__ inline void undistort_point(const double* c, double tr, double ti, double px,
                                       double py, double pz, float o[3]) {
  const double tau = ti - tr;
  const double mid = (ti + tr) * 0.5 - c[0];
  double rho[3], w[3];
  for (int k = 0; k < 3; ++k) {
    rho[k] = tau * fma(c[7 + k], mid, c[1 + k]);
    w[k] = tau * fma(c[10 + k], mid, c[4 + k]);
  }
  const double th2 = fma(w[2], w[2], fma(w[1], w[1], w[0] * w[0]));
  // R = I + A W + B W^2, V = I + B W + C W^2 with W = [w]x, theta = |w|:
  // A = sin(th)/th, B = (1 - cos th)/th^2, C = (th - sin th)/th^3.  Up to
  // theta = 1/2 (a scan's rotation is far smaller) their Taylor series in
  // theta^2 to degree 7, whose first omitted terms are below 2^-64 relative:
  // no sine, square root or division.  Beyond, the closed forms with the
  // half-angle B = 2 sin^2(th/2)/th^2.
  double A, B, C;
  if (th2 <= 0.25) {
    const double x = -th2;
    A = fma(x, 1.0 / 1307674368000.0, 1.0 / 6227020800.0);
    B = fma(x, 1.0 / 20922789888000.0, 1.0 / 87178291200.0);
    C = fma(x, 1.0 / 355687428096000.0, 1.0 / 1307674368000.0);
    A = fma(x, A, 1.0 / 39916800.0);   B = fma(x, B, 1.0 / 479001600.0);
    C = fma(x, C, 1.0 / 6227020800.0);
    A = fma(x, A, 1.0 / 362880.0);     B = fma(x, B, 1.0 / 3628800.0);
    C = fma(x, C, 1.0 / 39916800.0);
    A = fma(x, A, 1.0 / 5040.0);       B = fma(x, B, 1.0 / 40320.0);
    C = fma(x, C, 1.0 / 362880.0);
    A = fma(x, A, 1.0 / 120.0);        B = fma(x, B, 1.0 / 720.0);
    C = fma(x, C, 1.0 / 5040.0);
    A = fma(x, A, 1.0 / 6.0);          B = fma(x, B, 1.0 / 24.0);
    C = fma(x, C, 1.0 / 120.0);
    A = fma(x, A, 1.0);                B = fma(x, B, 0.5);
    C = fma(x, C, 1.0 / 6.0);
  } else {
    const double th = sqrt(th2);
    double sh, ch;
    sincos(0.5 * th, &sh, &ch);
    A = 2.0 * sh * ch / th;
    B = 2.0 * (sh * sh) / th2;
    C = (th - th * A) / (th2 * th);
  }
  // R p + V rho = p + rho + A (w x p) + B (w x (w x p) + w x rho) + C w x (w x rho)
  const double p[3] = {px, py, pz};
  double wp[3], wr[3], q[3], wq[3], wwr[3];
  cross(w, p, wp);
  cross(w, rho, wr);
  for (int k = 0; k < 3; ++k) q[k] = wp[k] + rho[k];
  cross(w, q, wq);                        // w x (w x p) + w x rho
  cross(w, wr, wwr);
  for (int k = 0; k < 3; ++k)
    o[k] = float((p[k] + rho[k]) + fma(A, wp[k], fma(B, wq[k], C * wwr[k])));
}

constexpr int kUdApplyPts = 4;            // points per lane in k_ud_apply
constexpr int kUdApply = kUdBlock * kUdApplyPts;

// Time maximum of scan s (decoded) reduced over the block: each lane loads
// every kUdBlock-th of the scan's chunk maxima.  Valid in thread 0.
__device__ inline double block_scan_tref(const int64_t* off, int s, int64_t n, const int4* part,
                                         const uint32_t* mid) {
  const int64_t p0 = off ? off[s] : 0;
  const int64_t p1 = off ? off[s + 1] : n;
  uint32_t m = p1 > p0 ? scan_tmax(s, part, mid, p0 / kUdChunk + threadIdx.x,
                                   (p1 - 1) / kUdChunk, kUdBlock)
                       : 0u;
  return time_dec(block_max(m));
}

// Blocks [0, n_apply) take kUdApply points each; with t_ref_out, the blocks
// after them write the reference times, one wave per scan.
__global__ __launch_bounds__(kUdBlock) void k_ud_apply(
    const float* xyz, const float* __restrict__ t, const int64_t* __restrict__ off, int S,
    int64_t n, int64_t n_apply, const double* __restrict__ coef, const int4* __restrict__ part,
    const uint32_t* __restrict__ mid, double* __restrict__ t_ref_out, float* out) {
  if (int64_t(blockIdx.x) >= n_apply) {
    const int s = int((int64_t(blockIdx.x) - n_apply) * (kUdBlock / 64) + (threadIdx.x >> 6));
    if (s >= S) return;
    const int lane = threadIdx.x & 63;
    const int64_t p0 = off ? off[s] : 0;
    const int64_t p1 = off ? off[s + 1] : n;
    uint32_t m = p1 > p0 ? scan_tmax(s, part, mid, p0 / kUdChunk + lane, (p1 - 1) / kUdChunk, 64)
                         : 0u;
    for (int d = 32; d >= 1; d >>= 1) m = max(m, uint32_t(__shfl_xor(int(m), d)));
    if (lane == 0) t_ref_out[s] = time_dec(m);
    return;
  }
  __shared__ double s_c[kUdCoef];
  __shared__ double s_t[2];
  const int64_t base = int64_t(blockIdx.x) * kUdApply;
  const int64_t last = min(base + kUdApply, n) - 1;
  float px[kUdApplyPts], py[kUdApplyPts], pz[kUdApplyPts], tf[kUdApplyPts];
#pragma unroll
  for (int q = 0; q < kUdApplyPts; ++q) {
    const int64_t i = min(base + q * kUdBlock + threadIdx.x, last);
    px[q] = xyz[i];
    py[q] = xyz[n + i];
    pz[q] = xyz[2 * n + i];
    tf[q] = t[i];
  }
  int lo, hi;
  block_scans(off, S, base, last, &lo, &hi);
  // reference times of the block's first and last scans; scans strictly
  // between them lie inside the block (two chunks at most) and are reduced
  // per lane
  if (lo == hi && threadIdx.x < kUdCoef) s_c[threadIdx.x] = coef[size_t(lo) * kUdCoef + threadIdx.x];
  double tr = block_scan_tref(off, lo, n, part, mid);
  if (threadIdx.x == 0) s_t[0] = tr;
  if (hi != lo) {
    tr = block_scan_tref(off, hi, n, part, mid);
    if (threadIdx.x == 0) s_t[1] = tr;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kUdApplyPts; ++q) {
    const int64_t i = base + q * kUdBlock + threadIdx.x;
    if (i > last) break;
    float o[3] = {px[q], py[q], pz[q]};
    if (isfinite(tf[q])) {
      if (lo == hi) {
        undistort_point(s_c, s_t[0], double(tf[q]), px[q], py[q], pz[q], o);
      } else {
        const int s = scan_of(off, lo, hi, i);
        const double r = s == lo ? s_t[0]
                                 : (s == hi ? s_t[1]
                                            : time_dec(scan_tmax_lane(off, s, n, part, mid)));
        undistort_point(coef + size_t(s) * kUdCoef, r, double(tf[q]), px[q], py[q], pz[q], o);
      }
    }
    out[i] = o[0];
    out[n + i] = o[1];
    out[2 * n + i] = o[2];
  }
}

// The two launches of an undistortion, on scratch the caller provides:
// part [ceil(n / kUdChunk)], mid [S], coef [S * kUdCoef].  Every entry the
// launches read is written by k_ud_scan first, so the scratch needs no
// clearing and may hold an earlier call's contents.
far_status_t undistort_launch(const float* xyz, const float* t, const int64_t* off, int32_t S,
                              int64_t n, const double* vel_t, const double* vel,
                              const int64_t* voff, int64_t m, float* out, double* t_ref,
                              int4* part, uint32_t* mid, double* coef, bool timed,
                              hipStream_t st) {
  const int64_t n_chunks = (n + kUdChunk - 1) / kUdChunk;
  {
    TimedScope ts(timed ? FAR_TIME_UNDISTORT : -1, st);
    hipLaunchKernelGGL(k_ud_scan, dim3(unsigned(n_chunks + S)), dim3(kUdBlock), 0, st, t, off,
                       S, n, n_chunks, part, mid, vel_t, vel, voff, m, coef, t_ref);
    FAR_HIP(hipGetLastError());
    if (n > 0) {
      const int64_t n_apply = (n + kUdApply - 1) / kUdApply;
      const int64_t n_tref = t_ref ? (S + kUdBlock / 64 - 1) / (kUdBlock / 64) : 0;
      TimedScope ta(timed ? FAR_TIME_UNDISTORT_APPLY : -1, st);
      hipLaunchKernelGGL(k_ud_apply, dim3(unsigned(n_apply + n_tref)), dim3(kUdBlock), 0, st,
                         xyz, t, off, S, n, n_apply, coef, part, mid, t_ref, out);
      FAR_HIP(hipGetLastError());
    }
  }
  return FAR_OK;
}

far_status_t undistort_impl(const float* xyz, const float* t, const int64_t* off, int32_t S,
                            int64_t n, const double* vel_t, const double* vel,
                            const int64_t* voff, int64_t m, float* out, double* t_ref,
                            hipStream_t st) {
  Scratch scr(st);
  const int64_t n_chunks = (n + kUdChunk - 1) / kUdChunk;
  int4* part;
  uint32_t* mid;
  double* coef;
  FAR_TRY(scr.get(&part, size_t(n_chunks)));
  FAR_TRY(scr.get(&mid, size_t(S)));
  FAR_TRY(scr.get(&coef, size_t(S) * kUdCoef));
  return undistort_launch(xyz, t, off, S, n, vel_t, vel, voff, m, out, t_ref, part, mid, coef,
                          true, st);
}

// ---------------------------------------------------------------- no-alloc
// Scratch of the allocation-free batch call: a fixed device array, one copy
// per GPU (each device that loads the library holds it until the process
// ends).  Its host-side name is not a device address: host code uses only
// the address hipGetSymbolAddress returns for the current device.
constexpr int64_t kUdFixedMaxPoints = int64_t(1) << 28;
constexpr int32_t kUdFixedMaxScans = 4096;
constexpr size_t kUdFixedPart = size_t(kUdFixedMaxPoints / kUdChunk) * sizeof(int4);
constexpr size_t kUdFixedMid = (size_t(kUdFixedMaxScans) * sizeof(uint32_t) + 255) & ~size_t(255);
constexpr size_t kUdFixedCoef = size_t(kUdFixedMaxScans) * kUdCoef * sizeof(double);
constexpr size_t kUdFixedBytes = kUdFixedPart + kUdFixedMid + kUdFixedCoef;
static_assert(kUdFixedPart % 256 == 0, "scratch pieces stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kUdFixedBytes];

constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
char* g_fixed_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, looked up once per
// device.
far_status_t fixed_scratch(char** out) {
  int dev = -1;
  FAR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("far_undistort_batch_noalloc: device %d beyond the %d the library tracks", dev,
              kMaxDevices);
    return FAR_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_fixed_mu);
  if (!g_fixed_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("far_undistort_batch_noalloc: hipGetSymbolAddress failed on device %d: %s", dev,
                hipGetErrorString(e));
      return FAR_E_HIP;
    }
    g_fixed_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_fixed_ptr[dev];
  return FAR_OK;
}

}  // namespace
}  // namespace far

extern "C" {

far_status_t far_undistort(const float* xyz, const float* t, int64_t n, const double* vel_t,
                           const double* vel, int32_t m, float* out, double* t_ref,
                           far_stream_t stream) {
  if (n < 0 || m < 0 || n >= (int64_t(1) << 40) || (n > 0 && (!xyz || !t || !out)) ||
      (m > 0 && (!vel_t || !vel))) {
    far::set_error("far_undistort: bad arguments (n %lld, m %d)", (long long)n, m);
    return FAR_E_INVALID;
  }
  return far::undistort_impl(xyz, t, nullptr, 1, n, vel_t, vel, nullptr, m, out, t_ref,
                             far::S(stream));
}

far_status_t far_undistort_batch(const float* xyz, const float* t, const int64_t* offsets,
                                 int32_t S, int64_t n_total, const double* vel_t,
                                 const double* vel, const int64_t* vel_offsets, float* out,
                                 double* t_ref, far_stream_t stream) {
  if (S <= 0 || n_total < 0 || n_total >= (int64_t(1) << 40) || !offsets || !vel_offsets ||
      (n_total > 0 && (!xyz || !t || !out))) {
    far::set_error("far_undistort_batch: bad arguments (S %d, n_total %lld)", S,
                   (long long)n_total);
    return FAR_E_INVALID;
  }
  return far::undistort_impl(xyz, t, offsets, S, n_total, vel_t, vel, vel_offsets, 0, out,
                             t_ref, far::S(stream));
}

far_status_t far_undistort_batch_noalloc(const float* xyz, const float* t,
                                         const int64_t* offsets, int32_t S, int64_t n_total,
                                         const double* vel_t, const double* vel,
                                         const int64_t* vel_offsets, float* out, double* t_ref,
                                         far_stream_t stream) {
  if (S <= 0 || n_total < 0 || !offsets || !vel_offsets ||
      (n_total > 0 && (!xyz || !t || !out))) {
    far::set_error("far_undistort_batch_noalloc: bad arguments (S %d, n_total %lld)", S,
                   (long long)n_total);
    return FAR_E_INVALID;
  }
  if (S > far::kUdFixedMaxScans || n_total > far::kUdFixedMaxPoints) {
    far::set_error("far_undistort_batch_noalloc: S %d, n_total %lld exceed the fixed scratch "
                   "(at most %d scans, %lld points)", S, (long long)n_total,
                   far::kUdFixedMaxScans, (long long)far::kUdFixedMaxPoints);
    return FAR_E_CAPACITY;
  }
  char* base = nullptr;
  FAR_TRY(far::fixed_scratch(&base));
  int4* part = reinterpret_cast<int4*>(base);
  uint32_t* mid = reinterpret_cast<uint32_t*>(base + far::kUdFixedPart);
  double* coef = reinterpret_cast<double*>(base + far::kUdFixedPart + far::kUdFixedMid);
  return far::undistort_launch(xyz, t, offsets, S, n_total, vel_t, vel, vel_offsets, 0, out,
                               t_ref, part, mid, coef, false, far::S(stream));
}

}  // extern "C"
