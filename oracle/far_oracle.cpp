// far_oracle.cpp -- TEST INFRASTRUCTURE ONLY (see far_oracle.h).
//
// A plain, deliberately unoptimised FP64 CPU implementation of the FAR-LIO
// registration hot path (arXiv 2606.26010, Sec. III-A).  Every function below
// names the passage of the paper it follows; where the paper is silent the
// reading taken is stated in the comment.  Build flags: -O2 -ffp-contract=off
// (no fused multiply-add, no fast-math), so every expression is evaluated
// exactly in the order written.
//
// OpenMP is used only across independent queries; every sum is taken
// sequentially in point order, so results do not depend on the thread count.

#include <omp.h>
#include "far_oracle.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <unordered_map>
#include <utility>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Voxel keys (Sec. III-A.2, the cuVoxelMap paragraph): a key is the triple of
// integer voxel indices floor(x / v) of a point.  Floor, not truncation, so
// that negative coordinates fall into the voxel below.  Keys are limited to
// [-2^20, 2^20) per axis (the library packs 21 bits per axis); a point outside
// that range is an invalid input.
// ---------------------------------------------------------------------------
const int64_t kKeyLimit = int64_t(1) << 20;

struct Key {
  int64_t x, y, z;
  bool operator==(const Key& o) const { return x == o.x && y == o.y && z == o.z; }
};
struct KeyHash {
  size_t operator()(const Key& k) const {
    // Any hash works: the oracle's results are defined without one.
    uint64_t h = uint64_t(k.x) * 0x9E3779B97F4A7C15ull;
    h ^= uint64_t(k.y) + 0x7F4A7C159E3779B9ull + (h << 6) + (h >> 2);
    h ^= uint64_t(k.z) + 0x94D049BB133111EBull + (h << 6) + (h >> 2);
    return size_t(h);
  }
};

Key key_of(double x, double y, double z, double v) {
  return Key{int64_t(std::floor(x / v)), int64_t(std::floor(y / v)),
             int64_t(std::floor(z / v))};
}
bool key_in_range(const Key& k) {
  return k.x >= -kKeyLimit && k.x < kKeyLimit && k.y >= -kKeyLimit &&
         k.y < kKeyLimit && k.z >= -kKeyLimit && k.z < kKeyLimit;
}

// Squared distance in FP64, evaluated as (dx*dx + dy*dy) + dz*dz with each
// difference formed from the FP64 values of the operands.  This fixed order is
// the ranking key of every neighbour decision.
double dist2(double ax, double ay, double az, double bx, double by, double bz) {
  double dx = ax - bx, dy = ay - by, dz = az - bz;
  return (dx * dx + dy * dy) + dz * dz;
}

struct Pt {
  double x, y, z;
};

// ---------------------------------------------------------------------------
// Covariance regularisation, Eq. (1): Sigma = (C^-1 / ||C^-1||_F)^-1 with
// C = Sigma_hat + 1e-3 I.  Written out literally: invert C, normalise the
// inverse by its Frobenius norm, invert again.  The 3x3 inverses use the
// adjugate over the determinant.
// ---------------------------------------------------------------------------
void inv3(const double A[9], double out[9]) {
  double c00 = A[4] * A[8] - A[5] * A[7];
  double c01 = A[5] * A[6] - A[3] * A[8];
  double c02 = A[3] * A[7] - A[4] * A[6];
  double c10 = A[2] * A[7] - A[1] * A[8];
  double c11 = A[0] * A[8] - A[2] * A[6];
  double c12 = A[1] * A[6] - A[0] * A[7];
  double c20 = A[1] * A[5] - A[2] * A[4];
  double c21 = A[2] * A[3] - A[0] * A[5];
  double c22 = A[0] * A[4] - A[1] * A[3];
  double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  // adj(A) is the transpose of the cofactor matrix
  out[0] = c00 / det; out[1] = c10 / det; out[2] = c20 / det;
  out[3] = c01 / det; out[4] = c11 / det; out[5] = c21 / det;
  out[6] = c02 / det; out[7] = c12 / det; out[8] = c22 / det;
}

void regularize(const double S_hat[9], double Sigma[9]) {
  double C[9];
  for (int i = 0; i < 9; ++i) C[i] = S_hat[i];
  C[0] += 1e-3; C[4] += 1e-3; C[8] += 1e-3;
  double Ci[9];
  inv3(C, Ci);
  double fro = 0.0;
  for (int i = 0; i < 9; ++i) fro += Ci[i] * Ci[i];
  fro = std::sqrt(fro);
  double Cn[9];
  for (int i = 0; i < 9; ++i) Cn[i] = Ci[i] / fro;
  inv3(Cn, Sigma);
}

// Plane regularisation after Segal et al. (the GICP paper the sparsity-aware
// case cites), offered beside Eq. (1): the sample covariance's eigenvector n
// of its smallest eigenvalue is taken as the surface normal and the point's
// covariance becomes that of a plane of thickness eps, U diag(eps, 1, 1) U^T
// = I + (eps - 1) n n^T, eps = 1e-3.  The eigenvectors come from the cyclic
// Jacobi method on the 3x3 matrix: plane rotations J chosen to zero one
// off-diagonal entry at a time, A <- J^T A J, V <- V J, until the
// off-diagonal part vanishes (to rounding) or 50 sweeps; ties between
// smallest eigenvalues take the lowest index.
const double kPlaneEps = 1e-3;
int g_cov_mode = 0;   // 0: Eq. (1); 1: plane regularisation

void mat3_mul(const double A[9], const double B[9], double C[9]) {
  double t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double x = 0.0;
      for (int l = 0; l < 3; ++l) x += A[i * 3 + l] * B[l * 3 + j];
      t[i * 3 + j] = x;
    }
  std::memcpy(C, t, sizeof(t));
}

void jacobi3(const double S[9], double evals[3], double V[9]) {
  double A[9];
  std::memcpy(A, S, sizeof(A));
  for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
  double fro = 0.0;
  for (int i = 0; i < 9; ++i) fro += A[i] * A[i];
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    if (off == 0.0 || off <= 1e-36 * fro) break;
    const int P[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (auto& pq : P) {
      const int p = pq[0], q = pq[1];
      const double apq = A[p * 3 + q];
      if (apq == 0.0) continue;
      // tan of the rotation angle, the smaller root (|angle| <= pi/4)
      const double theta = (A[q * 3 + q] - A[p * 3 + p]) / (2.0 * apq);
      const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
      const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
      double J[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
      J[p * 3 + p] = c; J[q * 3 + q] = c;
      J[p * 3 + q] = sn; J[q * 3 + p] = -sn;
      double Jt[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Jt[i * 3 + j] = J[j * 3 + i];
      double T1[9];
      mat3_mul(Jt, A, T1);
      mat3_mul(T1, J, A);
      A[p * 3 + q] = A[q * 3 + p] = 0.0;   // zero by construction
      mat3_mul(V, J, V);
    }
  }
  evals[0] = A[0]; evals[1] = A[4]; evals[2] = A[8];
}

void plane_regularize(const double S_hat[9], double Sigma[9]) {
  double ev[3], V[9];
  jacobi3(S_hat, ev, V);
  int m = 0;
  for (int i = 1; i < 3; ++i)
    if (ev[i] < ev[m]) m = i;
  double n[3] = {V[0 * 3 + m], V[1 * 3 + m], V[2 * 3 + m]};
  const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (double& x : n) x /= len;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      Sigma[i * 3 + j] = (i == j ? 1.0 : 0.0) + (kPlaneEps - 1.0) * n[i] * n[j];
}

// Sample covariance of k points, two passes (mean first, then the centred
// outer products), normalised by 1/k.  The neighbourhood includes the point
// itself (Sec. III-A.2: covariance from the k nearest neighbours).
void covariance_of(const std::vector<Pt>& nb, double S[9]) {
  double k = double(nb.size());
  double mx = 0, my = 0, mz = 0;
  for (const Pt& q : nb) { mx += q.x; my += q.y; mz += q.z; }
  mx /= k; my /= k; mz /= k;
  double sxx = 0, sxy = 0, sxz = 0, syy = 0, syz = 0, szz = 0;
  for (const Pt& q : nb) {
    double dx = q.x - mx, dy = q.y - my, dz = q.z - mz;
    sxx += dx * dx; sxy += dx * dy; sxz += dx * dz;
    syy += dy * dy; syz += dy * dz; szz += dz * dz;
  }
  S[0] = sxx / k; S[1] = sxy / k; S[2] = sxz / k;
  S[3] = sxy / k; S[4] = syy / k; S[5] = syz / k;
  S[6] = sxz / k; S[7] = syz / k; S[8] = szz / k;
}

// ---------------------------------------------------------------------------
// A voxel grid: voxel key -> ids of its points in insertion order.  Used both
// for the submap Q and for the per-scan cloud whose covariances are needed
// (Sec. III-A.2: the scan covariances use their own voxel-map instance).
// ---------------------------------------------------------------------------
struct Grid {
  double v = 1.0;
  std::unordered_map<Key, std::vector<int64_t>, KeyHash> vox;
  std::vector<Pt> pts;  // by id, FP64 copies of the stored FP32 values
};

// k nearest points of the grid within radius r of q, ranked by (d2, id).
// Candidates are every point of the 27 voxels around key(q).  For r <= v this
// equals the brute-force k nearest of the whole cloud within r: a point within
// r of q differs from q by at most v per axis, so its voxel index differs by
// at most one per axis.
void knn(const Grid& g, double qx, double qy, double qz, int k, double r,
         std::vector<std::pair<double, int64_t>>& out) {
  out.clear();
  double r2 = r * r;
  Key kq = key_of(qx, qy, qz, g.v);
  std::vector<std::pair<double, int64_t>> cand;
  for (int64_t dx = -1; dx <= 1; ++dx)
    for (int64_t dy = -1; dy <= 1; ++dy)
      for (int64_t dz = -1; dz <= 1; ++dz) {
        auto it = g.vox.find(Key{kq.x + dx, kq.y + dy, kq.z + dz});
        if (it == g.vox.end()) continue;
        for (int64_t id : it->second) {
          const Pt& p = g.pts[size_t(id)];
          double d2 = dist2(p.x, p.y, p.z, qx, qy, qz);
          if (d2 <= r2) cand.push_back({d2, id});
        }
      }
  std::sort(cand.begin(), cand.end());  // lexicographic (d2, id)
  size_t m = std::min(cand.size(), size_t(k));
  out.assign(cand.begin(), cand.begin() + m);
}

// Regularised covariance of point p of grid g, as six upper-triangle values.
// valid <=> exactly k neighbours within r = v (reading of "lacks sufficient
// neighbors", Sec. III-A.2, sparsity-aware GICP paragraph).
bool point_covariance(const Grid& g, const Pt& p, int k, double out6[6]) {
  std::vector<std::pair<double, int64_t>> nb;
  knn(g, p.x, p.y, p.z, k, g.v, nb);
  if (int(nb.size()) != k) {
    for (int i = 0; i < 6; ++i) out6[i] = 0.0;
    return false;
  }
  std::vector<Pt> pts;
  for (auto& e : nb) pts.push_back(g.pts[size_t(e.second)]);
  double S[9], Sig[9];
  covariance_of(pts, S);
  if (g_cov_mode == 1)
    plane_regularize(S, Sig);
  else
    regularize(S, Sig);
  out6[0] = Sig[0]; out6[1] = Sig[1]; out6[2] = Sig[2];
  out6[3] = Sig[4]; out6[4] = Sig[5]; out6[5] = Sig[8];
  return true;
}

bool finite3(double x, double y, double z) {
  return std::isfinite(x) && std::isfinite(y) && std::isfinite(z);
}

// 4x4 row-major helpers.
void matmul4(const double A[16], const double B[16], double C[16]) {
  double t[16];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      for (int l = 0; l < 4; ++l) s += A[i * 4 + l] * B[l * 4 + j];
      t[i * 4 + j] = s;
    }
  std::memcpy(C, t, sizeof(t));
}

}  // namespace

// ---------------------------------------------------------------------------
// The submap (Sec. III-A.3 "Adaptive, Local Submap", and the cuVoxelMap
// paragraph of Sec. III-A.2): voxels of edge v holding at most N_max points,
// each point carrying a regularised covariance computed when it is added.
// ---------------------------------------------------------------------------
struct orc_map {
  Grid g;
  int32_t nmax = 20;
  double dmin = 0.0;
  int32_t k_cov = 5;
  int64_t point_cap = 0, voxel_cap = 0;
  std::vector<float> fx, fy, fz;  // stored FP32 coordinates, by id
  std::vector<float> cov;         // 6 per id, FP32
  std::vector<uint8_t> valid;
};

extern "C" {

orc_map* orc_map_new(double v, int32_t nmax, double dmin, int32_t k_cov,
                     int64_t point_cap, int64_t voxel_cap) {
  if (!(v > 0.0) || nmax < 1 || k_cov < 1 || point_cap < 1 || voxel_cap < 1)
    return nullptr;
  orc_map* m = new orc_map();
  m->g.v = v;
  m->nmax = nmax;
  m->dmin = dmin;
  m->k_cov = k_cov;
  m->point_cap = point_cap;
  m->voxel_cap = voxel_cap;
  return m;
}

void orc_map_free(orc_map* m) { delete m; }
int64_t orc_map_size(const orc_map* m) { return int64_t(m->g.pts.size()); }
int64_t orc_map_nvoxels(const orc_map* m) { return int64_t(m->g.vox.size()); }

// Capped insert (Sec. III-A.3: a point enters its voxel only while the voxel
// holds fewer points than its cap; Sec. III-A.2: the points of a voxel keep
// a minimum spacing from each other).  Semantics, taken as sequential in
// input order:
//   for each finite point i in order, with K = key(p_i):
//     accept iff count(K) < cap_i and, when dmin > 0, every point already in
//     K (including points accepted earlier in this batch) is at squared
//     distance >= dmin^2;  an accepted point receives the next id.
// Then the covariances of the added points are computed on the updated map;
// existing points keep theirs (Sec. III-A.3, last paragraph).
// Capacity rules: keys of every finite batch point are added to the voxel set
// (a voxel may end up empty); if that would exceed voxel_cap the batch is
// refused unchanged.  An acceptance beyond point_cap stops the batch: the
// points accepted before it stay.
int orc_map_insert(orc_map* m, const float* xyz, int64_t n, const int32_t* caps,
                   int64_t* n_accepted, int64_t* n_skipped) {
  if (n < 0) return 1;
  const float* X = xyz;
  const float* Y = xyz + n;
  const float* Z = xyz + 2 * n;
  double v = m->g.v;
  // Range check and voxel-capacity check first; nothing changes on failure.
  std::unordered_map<Key, int, KeyHash> fresh;
  int64_t skipped = 0;
  for (int64_t i = 0; i < n; ++i) {
    double x = X[i], y = Y[i], z = Z[i];
    if (!finite3(x, y, z)) { ++skipped; continue; }
    Key K = key_of(x, y, z, v);
    if (!key_in_range(K)) return 1;
    if (m->g.vox.find(K) == m->g.vox.end()) fresh[K] = 1;
  }
  if (n_skipped) *n_skipped = skipped;
  if (int64_t(m->g.vox.size()) + int64_t(fresh.size()) > m->voxel_cap) {
    if (n_accepted) *n_accepted = 0;
    return 2;
  }
  for (auto& kv : fresh) m->g.vox[kv.first];  // create the (empty) voxels

  double dmin2 = m->dmin * m->dmin;
  int64_t first_new = int64_t(m->g.pts.size());
  int status = 0;
  for (int64_t i = 0; i < n; ++i) {
    double x = X[i], y = Y[i], z = Z[i];
    if (!finite3(x, y, z)) continue;
    Key K = key_of(x, y, z, v);
    std::vector<int64_t>& ids = m->g.vox[K];
    int64_t cap = m->nmax;
    if (caps) cap = std::min<int64_t>(caps[i], m->nmax);
    if (int64_t(ids.size()) >= cap) continue;
    bool spaced = true;
    if (m->dmin > 0.0) {
      for (int64_t id : ids) {
        const Pt& q = m->g.pts[size_t(id)];
        if (dist2(x, y, z, q.x, q.y, q.z) < dmin2) { spaced = false; break; }
      }
    }
    if (!spaced) continue;
    if (int64_t(m->g.pts.size()) >= m->point_cap) { status = 2; break; }
    int64_t id = int64_t(m->g.pts.size());
    ids.push_back(id);
    m->g.pts.push_back(Pt{x, y, z});
    m->fx.push_back(X[i]); m->fy.push_back(Y[i]); m->fz.push_back(Z[i]);
  }
  int64_t n_new = int64_t(m->g.pts.size()) - first_new;
  m->cov.resize(size_t(m->g.pts.size()) * 6, 0.0f);
  m->valid.resize(m->g.pts.size(), 0);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t j = 0; j < n_new; ++j) {
    int64_t id = first_new + j;
    double c6[6];
    bool ok = point_covariance(m->g, m->g.pts[size_t(id)], m->k_cov, c6);
    for (int t = 0; t < 6; ++t) m->cov[size_t(id) * 6 + t] = float(c6[t]);
    m->valid[size_t(id)] = ok ? 1 : 0;
  }
  if (n_accepted) *n_accepted = n_new;
  return status;
}

void orc_map_export(const orc_map* m, float* xyz, float* cov6, uint8_t* valid) {
  int64_t N = int64_t(m->g.pts.size());
  for (int64_t i = 0; i < N; ++i) {
    if (xyz) {
      xyz[i] = m->fx[size_t(i)];
      xyz[N + i] = m->fy[size_t(i)];
      xyz[2 * N + i] = m->fz[size_t(i)];
    }
    if (cov6)
      for (int t = 0; t < 6; ++t) cov6[t * N + i] = m->cov[size_t(i) * 6 + t];
    if (valid) valid[i] = m->valid[size_t(i)];
  }
}

int orc_map_knn(const orc_map* m, const float* q, int64_t n, int32_t k, double r,
                int32_t* idx, double* d2, int32_t* count) {
  if (n < 0 || k < 1 || !(r > 0.0) || r > m->g.v) return 1;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    double x = q[i], y = q[n + i], z = q[2 * n + i];
    std::vector<std::pair<double, int64_t>> nb;
    if (finite3(x, y, z) && key_in_range(key_of(x, y, z, m->g.v)))
      knn(m->g, x, y, z, k, r, nb);
    for (int32_t j = 0; j < k; ++j) {
      bool have = j < int32_t(nb.size());
      idx[i * k + j] = have ? int32_t(nb[size_t(j)].second) : -1;
      if (d2) d2[i * k + j] = have ? nb[size_t(j)].first : -1.0;
    }
    if (count) count[i] = int32_t(nb.size());
  }
  return 0;
}

// Covariances of a scan against itself (Sec. III-A.2: "computing the point
// covariances using an instance of the cuVoxelMap"): every point of the scan
// goes into the grid (no cap), then each point's covariance uses its k nearest
// scan points within r = v, itself included.
int orc_scan_covariances(const float* xyz, int64_t n, double v, int32_t k,
                         double* cov6, uint8_t* valid) {
  if (n < 0 || !(v > 0.0) || k < 1) return 1;
  Grid g;
  g.v = v;
  g.pts.resize(size_t(n));
  std::vector<char> ok(size_t(n), 0);
  for (int64_t i = 0; i < n; ++i) {
    double x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
    g.pts[size_t(i)] = Pt{x, y, z};
    if (!finite3(x, y, z)) continue;
    Key K = key_of(x, y, z, v);
    if (!key_in_range(K)) return 1;
    ok[size_t(i)] = 1;
    g.vox[K].push_back(i);
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    double c6[6] = {0, 0, 0, 0, 0, 0};
    bool good = ok[size_t(i)] && point_covariance(g, g.pts[size_t(i)], k, c6);
    for (int t = 0; t < 6; ++t) cov6[t * n + i] = good ? c6[t] : 0.0;
    valid[i] = good ? 1 : 0;
  }
  return 0;
}

void orc_regularize_cov(const double S[9], double out[9]) { regularize(S, out); }

void orc_plane_cov(const double S[9], double out[9]) { plane_regularize(S, out); }

void orc_jacobi3(const double S[9], double evals[3], double V[9]) { jacobi3(S, evals, V); }

int orc_set_cov_mode(int32_t mode) {
  if (mode != 0 && mode != 1) return 1;
  g_cov_mode = mode;
  return 0;
}

void orc_voxel_keys(const float* xyz, int64_t n, double v, int64_t* keys3) {
  for (int64_t i = 0; i < n; ++i) {
    Key K = key_of(xyz[i], xyz[n + i], xyz[2 * n + i], v);
    keys3[i * 3 + 0] = K.x;
    keys3[i * 3 + 1] = K.y;
    keys3[i * 3 + 2] = K.z;
  }
}

// ---------------------------------------------------------------------------
// SE(3) exponential of the twist delta = (omega, v): rotation by Rodrigues'
// formula, translation V v with V = I + B W + C W^2 (W = [omega]x).  Used for
// the left-multiplicative iterate update of Eq. (6).
// ---------------------------------------------------------------------------
void orc_se3_exp(const double d[6], double T[16]) {
  double wx = d[0], wy = d[1], wz = d[2];
  double th2 = wx * wx + wy * wy + wz * wz;
  double th = std::sqrt(th2);
  double A, B, C;
  if (th < 1e-6) {
    A = 1.0 - th2 / 6.0;
    B = 0.5 - th2 / 24.0;
    C = 1.0 / 6.0 - th2 / 120.0;
  } else {
    A = std::sin(th) / th;
    B = (1.0 - std::cos(th)) / th2;
    C = (th - std::sin(th)) / (th2 * th);
  }
  double W[9] = {0, -wz, wy, wz, 0, -wx, -wy, wx, 0};
  double W2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int l = 0; l < 3; ++l) s += W[i * 3 + l] * W[l * 3 + j];
      W2[i * 3 + j] = s;
    }
  double R[9], V[9];
  for (int i = 0; i < 9; ++i) {
    double I = (i % 4 == 0) ? 1.0 : 0.0;
    R[i] = I + A * W[i] + B * W2[i];
    V[i] = I + B * W[i] + C * W2[i];
  }
  for (int i = 0; i < 16; ++i) T[i] = 0.0;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) T[i * 4 + j] = R[i * 3 + j];
    T[i * 4 + 3] = V[i * 3 + 0] * d[3] + V[i * 3 + 1] * d[4] + V[i * 3 + 2] * d[5];
  }
  T[15] = 1.0;
}

// Cholesky factorisation H = L L^T and the solve H x = b.  A pivot that is not
// above 1e-12 times the largest diagonal entry (or not finite) means H is not
// positive definite: returns 4.
int orc_cholesky_solve6(const double H[36], const double b[6], double x[6]) {
  double L[36] = {0};
  double dmax = 0.0;
  for (int i = 0; i < 6; ++i) dmax = std::max(dmax, std::fabs(H[i * 7]));
  for (int j = 0; j < 6; ++j) {
    double s = H[j * 6 + j];
    for (int l = 0; l < j; ++l) s -= L[j * 6 + l] * L[j * 6 + l];
    if (!(s > 1e-12 * dmax) || !std::isfinite(s)) return 4;
    L[j * 6 + j] = std::sqrt(s);
    for (int i = j + 1; i < 6; ++i) {
      double t = H[i * 6 + j];
      for (int l = 0; l < j; ++l) t -= L[i * 6 + l] * L[j * 6 + l];
      L[i * 6 + j] = t / L[j * 6 + j];
    }
  }
  double y[6];
  for (int i = 0; i < 6; ++i) {
    double s = b[i];
    for (int l = 0; l < i; ++l) s -= L[i * 6 + l] * y[l];
    y[i] = s / L[i * 6 + i];
  }
  for (int i = 5; i >= 0; --i) {
    double s = y[i];
    for (int l = i + 1; l < 6; ++l) s -= L[l * 6 + i] * x[l];
    x[i] = s / L[i * 6 + i];
  }
  return 0;
}

// ---------------------------------------------------------------------------
// One linearisation of the GICP objective, Eq. (4), at pose T.
//  - Eq. (2)/(6): p_i = R s_i + t, in FP64 as ((R00 sx + R01 sy) + R02 sz) + tx.
//  - Correspondence: the nearest map point within min(tau, v) (Sec. III-A.2,
//    "closest Euclidean neighbor" plus the adaptive threshold); none = outlier.
//  - Eq. (3): d_i = r_i - p_i.
//  - Eq. (4): M = Sigma_r + R Sigma_s R^T, W = M^-1, e2 = d^T W d.
//    Sparsity-aware case: if either covariance is invalid, Sigma_r = I and
//    Sigma_s = 0, i.e. M = I (point-to-point).  With sparsity_aware = 0 (the
//    ablation of Table III, standard GICP) such a pair is dropped instead:
//    no correspondence, no term, not an inlier.
//  - Eq. (5), Cauchy kernel on the Mahalanobis norm e = sqrt(e2):
//    rho = kappa^2/2 ln(1 + e2/kappa^2), IRLS weight w = kappa^2/(kappa^2+e2).
//  - Jacobian of d with respect to a left perturbation about the centre c,
//    p(delta) = c + Exp(delta)(p - c), delta = (omega, v):
//    J = [ [p - c]x , -I ].
//  - H = sum w J^T W J, b = sum w J^T W d, cost = sum rho.
// ---------------------------------------------------------------------------
int orc_linearize(const orc_map* m, const float* src, const float* src_cov6,
                  const uint8_t* src_valid, int64_t n, const double T[16],
                  double tau, double kappa, const double c[3], double H[36],
                  double b[6], double* cost, int64_t* n_inliers, int32_t* corr,
                  double* detail, int32_t sparsity_aware) {
  if (n < 0 || !(tau > 0.0) || !(kappa > 0.0)) return 1;
  const double R00 = T[0], R01 = T[1], R02 = T[2], tx = T[3];
  const double R10 = T[4], R11 = T[5], R12 = T[6], ty = T[7];
  const double R20 = T[8], R21 = T[9], R22 = T[10], tz = T[11];
  const double cx = c ? c[0] : 0.0, cy = c ? c[1] : 0.0, cz = c ? c[2] : 0.0;
  const double r = std::min(tau, m->g.v);
  const double k2 = kappa * kappa;

  // Per-point contributions first (parallel), then sums in point order.
  std::vector<double> rowH(size_t(n) * 21, 0.0), rowb(size_t(n) * 6, 0.0);
  std::vector<double> rowrho(size_t(n), 0.0);
  std::vector<int32_t> rowj(size_t(n), -1);

#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    if (detail)
      for (int t = 0; t < 18; ++t) detail[i * 18 + t] = NAN;
    double sx = src[i], sy = src[n + i], sz = src[2 * n + i];
    if (!finite3(sx, sy, sz)) continue;
    double px = ((R00 * sx + R01 * sy) + R02 * sz) + tx;
    double py = ((R10 * sx + R11 * sy) + R12 * sz) + ty;
    double pz = ((R20 * sx + R21 * sy) + R22 * sz) + tz;
    if (!key_in_range(key_of(px, py, pz, m->g.v))) continue;
    std::vector<std::pair<double, int64_t>> nb;
    knn(m->g, px, py, pz, 1, r, nb);
    if (nb.empty()) continue;
    int64_t j = nb[0].second;
    if (!sparsity_aware && !(src_valid[i] != 0 && m->valid[size_t(j)] != 0)) continue;
    rowj[size_t(i)] = int32_t(j);
    const Pt& q = m->g.pts[size_t(j)];
    double d[3] = {q.x - px, q.y - py, q.z - pz};

    double M[9];
    bool vs = src_valid[i] != 0, vr = m->valid[size_t(j)] != 0;
    if (vs && vr) {
      const float* cr = &m->cov[size_t(j) * 6];
      double Sr[9] = {cr[0], cr[1], cr[2], cr[1], cr[3], cr[4], cr[2], cr[4], cr[5]};
      double cs[6];
      for (int t = 0; t < 6; ++t) cs[t] = src_cov6[t * n + i];
      double Ss[9] = {cs[0], cs[1], cs[2], cs[1], cs[3], cs[4], cs[2], cs[4], cs[5]};
      double R[9] = {R00, R01, R02, R10, R11, R12, R20, R21, R22};
      double RS[9], RSRt[9];
      for (int a = 0; a < 3; ++a)
        for (int bb = 0; bb < 3; ++bb) {
          double s = 0.0;
          for (int l = 0; l < 3; ++l) s += R[a * 3 + l] * Ss[l * 3 + bb];
          RS[a * 3 + bb] = s;
        }
      for (int a = 0; a < 3; ++a)
        for (int bb = 0; bb < 3; ++bb) {
          double s = 0.0;
          for (int l = 0; l < 3; ++l) s += RS[a * 3 + l] * R[bb * 3 + l];
          RSRt[a * 3 + bb] = s;
        }
      for (int t = 0; t < 9; ++t) M[t] = Sr[t] + RSRt[t];
    } else {
      for (int t = 0; t < 9; ++t) M[t] = (t % 4 == 0) ? 1.0 : 0.0;
    }
    double W[9];
    inv3(M, W);
    double Wd[3];
    for (int a = 0; a < 3; ++a)
      Wd[a] = W[a * 3 + 0] * d[0] + W[a * 3 + 1] * d[1] + W[a * 3 + 2] * d[2];
    double e2 = d[0] * Wd[0] + d[1] * Wd[1] + d[2] * Wd[2];
    double w = k2 / (k2 + e2);
    double rho = 0.5 * k2 * std::log1p(e2 / k2);

    // J (3x6) = [ [a]x , -I ], a = p - c.
    double ax = px - cx, ay = py - cy, az = pz - cz;
    double J[18] = {0.0, -az, ay, -1.0, 0.0, 0.0,
                    az, 0.0, -ax, 0.0, -1.0, 0.0,
                    -ay, ax, 0.0, 0.0, 0.0, -1.0};
    double WJ[18];
    for (int a = 0; a < 3; ++a)
      for (int col = 0; col < 6; ++col) {
        double s = 0.0;
        for (int l = 0; l < 3; ++l) s += W[a * 3 + l] * J[l * 6 + col];
        WJ[a * 6 + col] = s;
      }
    int t = 0;
    for (int a = 0; a < 6; ++a)
      for (int bcol = a; bcol < 6; ++bcol) {
        double s = 0.0;
        for (int l = 0; l < 3; ++l) s += J[l * 6 + a] * WJ[l * 6 + bcol];
        rowH[size_t(i) * 21 + t++] = w * s;
      }
    for (int a = 0; a < 6; ++a) {
      double s = 0.0;
      for (int l = 0; l < 3; ++l) s += J[l * 6 + a] * Wd[l];
      rowb[size_t(i) * 6 + a] = w * s;
    }
    rowrho[size_t(i)] = rho;
    if (detail) {
      double* D = &detail[i * 18];
      D[0] = px; D[1] = py; D[2] = pz;
      D[3] = q.x; D[4] = q.y; D[5] = q.z;
      for (int u = 0; u < 9; ++u) D[6 + u] = W[u];
      D[15] = w; D[16] = rho; D[17] = e2;
    }
  }

  double Hs[21] = {0}, bs[6] = {0}, cs = 0.0;
  int64_t cnt = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (corr) corr[i] = rowj[size_t(i)];
    if (rowj[size_t(i)] < 0) continue;
    for (int t = 0; t < 21; ++t) Hs[t] += rowH[size_t(i) * 21 + t];
    for (int t = 0; t < 6; ++t) bs[t] += rowb[size_t(i) * 6 + t];
    cs += rowrho[size_t(i)];
    ++cnt;
  }
  int t = 0;
  for (int a = 0; a < 6; ++a)
    for (int bcol = a; bcol < 6; ++bcol) {
      H[a * 6 + bcol] = Hs[t];
      H[bcol * 6 + a] = Hs[t];
      ++t;
    }
  for (int a = 0; a < 6; ++a) b[a] = bs[a];
  *cost = cs;
  *n_inliers = cnt;
  return 0;
}

// ---------------------------------------------------------------------------
// Gauss-Newton align (Sec. III-A.2, Eq. (6) and the stopping rule after it).
// Each iteration linearises about c (the current translation when recenter is
// set, else the origin), solves H delta = -b by Cholesky and applies
// T <- T_c Exp(delta) T_c^-1 T.  Stops when ||delta||_2 <= eps (reading of the
// garbled norm criterion as the norm of the increment's twist) or after
// max_iters iterations (replacing the wall-clock limit).  Fewer than six
// inliers or a non positive definite H stop the loop with T unchanged by that
// iteration.
// ---------------------------------------------------------------------------
int orc_align(const orc_map* m, const float* src, const float* src_cov6,
              const uint8_t* src_valid, int64_t n, const double T0[16],
              double tau, double kappa, int32_t max_iters, double eps,
              int32_t recenter, double T_out[16], int32_t* iters,
              int32_t* converged, double H[36], double b[6], double* cost,
              int64_t* n_inliers, int32_t sparsity_aware) {
  if (max_iters < 1) return 1;
  double T[16];
  std::memcpy(T, T0, sizeof(T));
  int status = 0;
  *iters = 0;
  *converged = 0;
  for (int it = 0; it < max_iters; ++it) {
    double c[3] = {0.0, 0.0, 0.0};
    if (recenter) { c[0] = T[3]; c[1] = T[7]; c[2] = T[11]; }
    int rc = orc_linearize(m, src, src_cov6, src_valid, n, T, tau, kappa, c, H,
                           b, cost, n_inliers, nullptr, nullptr, sparsity_aware);
    if (rc) { status = rc; break; }
    if (*n_inliers < 6) { status = 5; break; }
    double nb[6], delta[6];
    for (int a = 0; a < 6; ++a) nb[a] = -b[a];
    if (orc_cholesky_solve6(H, nb, delta)) { status = 4; break; }
    double E[16], Tc[16], Tci[16], A1[16], A2[16];
    orc_se3_exp(delta, E);
    for (int a = 0; a < 16; ++a) Tc[a] = Tci[a] = (a % 5 == 0) ? 1.0 : 0.0;
    Tc[3] = c[0]; Tc[7] = c[1]; Tc[11] = c[2];
    Tci[3] = -c[0]; Tci[7] = -c[1]; Tci[11] = -c[2];
    matmul4(Tci, T, A1);
    matmul4(E, A1, A2);
    matmul4(Tc, A2, T);
    *iters = it + 1;
    double nrm = 0.0;
    for (int a = 0; a < 6; ++a) nrm += delta[a] * delta[a];
    if (std::sqrt(nrm) <= eps) { *converged = 1; break; }
  }
  std::memcpy(T_out, T, sizeof(T));
  return status;
}

void orc_touch_stats(const orc_map* m, const float* src, int64_t n,
                     const double T[16], int64_t* n_voxels, int64_t* n_points) {
  std::unordered_map<Key, int, KeyHash> seen;
  for (int64_t i = 0; i < n; ++i) {
    double sx = src[i], sy = src[n + i], sz = src[2 * n + i];
    if (!finite3(sx, sy, sz)) continue;
    double px = ((T[0] * sx + T[1] * sy) + T[2] * sz) + T[3];
    double py = ((T[4] * sx + T[5] * sy) + T[6] * sz) + T[7];
    double pz = ((T[8] * sx + T[9] * sy) + T[10] * sz) + T[11];
    Key K = key_of(px, py, pz, m->g.v);
    for (int64_t dx = -1; dx <= 1; ++dx)
      for (int64_t dy = -1; dy <= 1; ++dy)
        for (int64_t dz = -1; dz <= 1; ++dz) {
          Key N{K.x + dx, K.y + dy, K.z + dz};
          auto it = m->g.vox.find(N);
          if (it != m->g.vox.end() && !it->second.empty()) seen[N] = 1;
        }
  }
  int64_t pts = 0;
  for (auto& kv : seen) pts += int64_t(m->g.vox.at(kv.first).size());
  *n_voxels = int64_t(seen.size());
  *n_points = pts;
}


// ---------------------------------------------------------------------------
// Scan downsampling (part of the preprocessing in the runtime breakdown of
// Sec. IV-B; the rule is not given, read as "first point in input order per
// voxel").  A voxel seen for the first time keeps its point.
// ---------------------------------------------------------------------------
int orc_downsample(const float* xyz, int64_t n, double v, int64_t* keep, int64_t* n_keep) {
  *n_keep = 0;
  if (n < 0 || !(v > 0.0)) return 1;
  for (int64_t i = 0; i < n; ++i) {
    double x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
    if (finite3(x, y, z) && !key_in_range(key_of(x, y, z, v))) return 1;
  }
  std::unordered_map<Key, int, KeyHash> seen;
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    double x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
    if (!finite3(x, y, z)) continue;
    if (seen.emplace(key_of(x, y, z, v), 1).second) keep[m++] = i;
  }
  *n_keep = m;
  return 0;
}

// Rigid transform of a point set by a row-major 4x4 pose; each coordinate is
// ((R_r0 sx + R_r1 sy) + R_r2 sz) + t_r in FP64, then rounded to float.
void orc_transform(const float* xyz, int64_t n, const double T[16], float* out) {
  for (int64_t i = 0; i < n; ++i) {
    double s[3] = {xyz[i], xyz[n + i], xyz[2 * n + i]};
    for (int r = 0; r < 3; ++r) {
      double p = ((T[r * 4 + 0] * s[0] + T[r * 4 + 1] * s[1]) + T[r * 4 + 2] * s[2]) +
                 T[r * 4 + 3];
      out[r * n + i] = float(p);
    }
  }
}

// ---------------------------------------------------------------------------
// Adaptive threshold (Sec. III-A.2 adapts the correspondence threshold and
// the robust kernel's kappa to the motion, "analogous to" KISS-ICP).  Read as
// the published KISS-ICP rule: the deviation of the estimate from the motion
// prediction, measured as the largest displacement it causes within range
// r_max (2 r_max sin(theta/2) for the rotation, plus the translation), is a
// sample when it exceeds min_motion; sigma is the root mean square of the
// samples (sigma0 before the first), the threshold 3 sigma and kappa sigma/3.
// ---------------------------------------------------------------------------
void orc_threshold_init(orc_threshold* s, double sigma0, double r_max, double min_motion) {
  s->sigma0 = sigma0;
  s->r_max = r_max;
  s->min_motion = min_motion;
  s->sse = 0.0;
  s->n = 0;
}

double orc_threshold_update(orc_threshold* s, const double P[16], const double E[16]) {
  // D = P^-1 E with P^-1 = [R^T, -R^T t]
  double Pi[16] = {0};
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) Pi[i * 4 + j] = P[j * 4 + i];
    Pi[i * 4 + 3] = -(P[0 * 4 + i] * P[3] + P[1 * 4 + i] * P[7] + P[2 * 4 + i] * P[11]);
  }
  Pi[15] = 1.0;
  double D[16];
  matmul4(Pi, E, D);
  // rotation angle of D from its unit quaternion (Shepperd's method: build
  // the largest of |w|, |x|, |y|, |z| from the diagonal, the rest from the
  // off-diagonal sums and differences), theta = 2 atan2(|(x, y, z)|, |w|);
  // unlike acos of the trace this keeps full precision for small angles
  double tr = D[0] + D[5] + D[10];
  double q[4];  // w, x, y, z
  double d4[4] = {1.0 + tr, 1.0 + 2.0 * D[0] - tr, 1.0 + 2.0 * D[5] - tr, 1.0 + 2.0 * D[10] - tr};
  int big = int(std::max_element(d4, d4 + 4) - d4);
  double r = std::sqrt(d4[big]);  // = 2 |q_big|
  if (big == 0) {
    q[0] = 0.5 * r;
    q[1] = (D[9] - D[6]) / (2.0 * r);
    q[2] = (D[2] - D[8]) / (2.0 * r);
    q[3] = (D[4] - D[1]) / (2.0 * r);
  } else if (big == 1) {
    q[1] = 0.5 * r;
    q[0] = (D[9] - D[6]) / (2.0 * r);
    q[2] = (D[1] + D[4]) / (2.0 * r);
    q[3] = (D[2] + D[8]) / (2.0 * r);
  } else if (big == 2) {
    q[2] = 0.5 * r;
    q[0] = (D[2] - D[8]) / (2.0 * r);
    q[1] = (D[1] + D[4]) / (2.0 * r);
    q[3] = (D[6] + D[9]) / (2.0 * r);
  } else {
    q[3] = 0.5 * r;
    q[0] = (D[4] - D[1]) / (2.0 * r);
    q[1] = (D[2] + D[8]) / (2.0 * r);
    q[2] = (D[6] + D[9]) / (2.0 * r);
  }
  double theta = 2.0 * std::atan2(std::sqrt(q[1] * q[1] + q[2] * q[2] + q[3] * q[3]),
                                  std::fabs(q[0]));
  double dt = std::sqrt(D[3] * D[3] + D[7] * D[7] + D[11] * D[11]);
  double dev = 2.0 * s->r_max * std::sin(theta / 2.0) + dt;
  if (dev > s->min_motion) {
    s->sse += dev * dev;
    s->n += 1;
  }
  return dev;
}

void orc_threshold_get(const orc_threshold* s, double* tau, double* kappa) {
  double sigma = s->n > 0 ? std::sqrt(s->sse / double(s->n)) : s->sigma0;
  *tau = 3.0 * sigma;
  *kappa = sigma / 3.0;
}


// ---------------------------------------------------------------------------
// Differentiation of the GICP cost.  The cost is Eq. (4) with the Cauchy rho
// of Eq. (5): sum_i rho(e2_i), e2_i = d_i^T M_i^-1 d_i, d_i = r_j(i) - p_i,
// p_i = R s_i + t, M_i = Sigma_r + R Sigma_s,i R^T (or I, sparsity-aware
// case).  Readings: the correspondences j(i) and Sigma_s are held fixed; R
// enters both p and M, so the pose gradient carries the d M / d R term.
// ---------------------------------------------------------------------------
namespace {

// M (both covariances valid) or I, and its inverse W.
void m_and_w(const orc_map* m, const float* src_cov6, const uint8_t* src_valid, int64_t n,
             int64_t i, int64_t j, const double R[9], double M[9], double W[9], double Ss[9],
             bool* both) {
  *both = src_valid[i] != 0 && m->valid[size_t(j)] != 0;
  for (int t = 0; t < 9; ++t) Ss[t] = 0.0;
  if (*both) {
    const float* cr = &m->cov[size_t(j) * 6];
    double Sr[9] = {cr[0], cr[1], cr[2], cr[1], cr[3], cr[4], cr[2], cr[4], cr[5]};
    double cs[6];
    for (int t = 0; t < 6; ++t) cs[t] = src_cov6[t * n + i];
    double S9[9] = {cs[0], cs[1], cs[2], cs[1], cs[3], cs[4], cs[2], cs[4], cs[5]};
    for (int t = 0; t < 9; ++t) Ss[t] = S9[t];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) s += R[a * 3 + k] * S9[k * 3 + l] * R[b * 3 + l];
        M[a * 3 + b] = Sr[a * 3 + b] + s;
      }
  } else {
    for (int t = 0; t < 9; ++t) M[t] = (t % 4 == 0) ? 1.0 : 0.0;
  }
  inv3(M, W);
}

}  // namespace

int orc_cost_fixed(const orc_map* m, const double* src, const float* src_cov6,
                   const uint8_t* src_valid, int64_t n, const double T[16], double kappa,
                   const int32_t* corr, double* cost) {
  if (n < 0 || !(kappa > 0.0)) return 1;
  const double R[9] = {T[0], T[1], T[2], T[4], T[5], T[6], T[8], T[9], T[10]};
  const double k2 = kappa * kappa;
  double total = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = corr[i];
    if (j < 0) continue;
    double s[3] = {src[i], src[n + i], src[2 * n + i]};
    double p[3];
    for (int a = 0; a < 3; ++a)
      p[a] = R[a * 3] * s[0] + R[a * 3 + 1] * s[1] + R[a * 3 + 2] * s[2] + T[a * 4 + 3];
    const Pt& q = m->g.pts[size_t(j)];
    double d[3] = {q.x - p[0], q.y - p[1], q.z - p[2]};
    double M[9], W[9], Ss[9];
    bool both;
    m_and_w(m, src_cov6, src_valid, n, i, j, R, M, W, Ss, &both);
    double e2 = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) e2 += d[a] * W[a * 3 + b] * d[b];
    total += 0.5 * k2 * std::log1p(e2 / k2);
  }
  *cost = total;
  return 0;
}

// Gradient by the chain rule, per inlier (rho'(e2) = w/2 with the IRLS
// weight w = kappa^2 / (kappa^2 + e2)):
//   d e2 / d p = -2 u,  d e2 / d M = -u u^T,  u = W d;
//   d cost / d t   = -w u
//   d cost / d R   = -w u s^T  -  w u u^T R Sigma_s      (second term: M)
//   d cost / d s_i = -w R^T u
//   twist: d d / d delta = J = [[p - c]x, -I] gives w J^T u; the rotation
//   part of delta also moves M by [e_k]x A - A [e_k]x (A = R Sigma_s R^T),
//   adding (w/2) tr(-u u^T ([e_k]x A - A [e_k]x)) to component k.
int orc_gradient(const orc_map* m, const float* src, const float* src_cov6,
                 const uint8_t* src_valid, int64_t n, const double T[16], double tau,
                 double kappa, const double c[3], double grad_T[12], double grad_twist[6],
                 double* grad_src, double* cost, int64_t* n_inliers, int32_t* corr,
                 int32_t sparsity_aware) {
  if (n < 0 || !(tau > 0.0) || !(kappa > 0.0)) return 1;
  std::vector<int32_t> cj(size_t(n), -1);
  {
    double H[36], b[6], cst;
    int64_t cnt;
    int rc = orc_linearize(m, src, src_cov6, src_valid, n, T, tau, kappa, c, H, b, &cst, &cnt,
                           cj.data(), nullptr, sparsity_aware);
    if (rc) return rc;
  }
  const double R[9] = {T[0], T[1], T[2], T[4], T[5], T[6], T[8], T[9], T[10]};
  const double cc[3] = {c ? c[0] : 0.0, c ? c[1] : 0.0, c ? c[2] : 0.0};
  const double k2 = kappa * kappa;
  std::vector<double> rows(size_t(n) * 19, 0.0);   // 12 grad_T, 6 twist, rho
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    if (grad_src)
      for (int a = 0; a < 3; ++a) grad_src[a * n + i] = 0.0;
    int64_t j = cj[size_t(i)];
    if (j < 0) continue;
    double s[3] = {src[i], src[n + i], src[2 * n + i]};
    double p[3];
    for (int a = 0; a < 3; ++a)
      p[a] = ((R[a * 3] * s[0] + R[a * 3 + 1] * s[1]) + R[a * 3 + 2] * s[2]) + T[a * 4 + 3];
    const Pt& q = m->g.pts[size_t(j)];
    double d[3] = {q.x - p[0], q.y - p[1], q.z - p[2]};
    double M[9], W[9], Ss[9];
    bool both;
    m_and_w(m, src_cov6, src_valid, n, i, j, R, M, W, Ss, &both);
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = W[a * 3] * d[0] + W[a * 3 + 1] * d[1] + W[a * 3 + 2] * d[2];
    double e2 = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
    double w = k2 / (k2 + e2);
    double* row = &rows[size_t(i) * 19];
    // d cost / d R and d cost / d t
    double RS[9] = {0};   // R Sigma_s
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int k = 0; k < 3; ++k) RS[a * 3 + b] += R[a * 3 + k] * Ss[k * 3 + b];
    double uRS[3] = {0};  // u^T R Sigma_s
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) uRS[b] += u[a] * RS[a * 3 + b];
    for (int a = 0; a < 3; ++a) {
      for (int b = 0; b < 3; ++b) row[a * 4 + b] = -w * u[a] * s[b] - w * u[a] * uRS[b];
      row[a * 4 + 3] = -w * u[a];
    }
    // twist: w J^T u, then the M term of the rotation part
    double ax = p[0] - cc[0], ay = p[1] - cc[1], az = p[2] - cc[2];
    double J[18] = {0.0, -az, ay, -1.0, 0.0, 0.0,
                    az, 0.0, -ax, 0.0, -1.0, 0.0,
                    -ay, ax, 0.0, 0.0, 0.0, -1.0};
    for (int k = 0; k < 6; ++k)
      row[12 + k] = w * (J[k] * u[0] + J[6 + k] * u[1] + J[12 + k] * u[2]);
    if (both) {
      double A[9] = {0};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          for (int k = 0; k < 3; ++k) A[a * 3 + b] += RS[a * 3 + k] * R[b * 3 + k];
      for (int k = 0; k < 3; ++k) {
        double E[9] = {0};   // [e_k]x
        if (k == 0) { E[5] = -1; E[7] = 1; }
        if (k == 1) { E[2] = 1; E[6] = -1; }
        if (k == 2) { E[1] = -1; E[3] = 1; }
        double dM[9];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            double x = 0.0;
            for (int l = 0; l < 3; ++l) x += E[a * 3 + l] * A[l * 3 + b] - A[a * 3 + l] * E[l * 3 + b];
            dM[a * 3 + b] = x;
          }
        double quad = 0.0;   // u^T dM u
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) quad += u[a] * dM[a * 3 + b] * u[b];
        row[12 + k] += 0.5 * w * (-quad);
      }
    }
    row[18] = 0.5 * k2 * std::log1p(e2 / k2);
    if (grad_src)
      for (int b = 0; b < 3; ++b)
        grad_src[b * n + i] = -w * (R[0 * 3 + b] * u[0] + R[1 * 3 + b] * u[1] + R[2 * 3 + b] * u[2]);
  }
  double gT[12] = {0}, gw[6] = {0}, cs = 0.0;
  int64_t cnt = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (corr) corr[i] = cj[size_t(i)];
    if (cj[size_t(i)] < 0) continue;
    const double* row = &rows[size_t(i) * 19];
    for (int t = 0; t < 12; ++t) gT[t] += row[t];
    for (int t = 0; t < 6; ++t) gw[t] += row[12 + t];
    cs += row[18];
    ++cnt;
  }
  for (int t = 0; t < 12; ++t) grad_T[t] = gT[t];
  for (int t = 0; t < 6; ++t) grad_twist[t] = gw[t];
  *cost = cs;
  *n_inliers = cnt;
  return 0;
}


// ---------------------------------------------------------------------------
// Adaptive submap density (Sec. III-A.3): the cap follows the density of the
// current scan near the sensor and decays linearly over range, never below
// the k points a covariance needs.  The near range, the decay length and the
// rounding are readings (the paper names none).
// ---------------------------------------------------------------------------
int orc_asmd_caps(const float* xs, const float* xm, int64_t n, double v, int32_t k,
                  int32_t nmax, double r_near, double r_max, int32_t* caps,
                  double* mean_near) {
  if (n < 0 || !(v > 0.0) || k < 1 || nmax < k || !(r_near >= 0.0) || !(r_max > 0.0)) return 1;
  std::unordered_map<Key, int, KeyHash> vox;
  int64_t near = 0;
  for (int64_t i = 0; i < n; ++i) {
    double sx = xs[i], sy = xs[n + i], sz = xs[2 * n + i];
    double mx = xm[i], my = xm[n + i], mz = xm[2 * n + i];
    if (!finite3(sx, sy, sz) || !finite3(mx, my, mz)) continue;
    if ((sx * sx + sy * sy) + sz * sz <= r_near * r_near) {
      Key K = key_of(mx, my, mz, v);
      if (!key_in_range(K)) return 1;
      vox[K] = 1;
      ++near;
    }
  }
  double mean = vox.empty() ? double(nmax) : double(near) / double(vox.size());
  if (mean_near) *mean_near = mean;
  for (int64_t i = 0; i < n; ++i) {
    double sx = xs[i], sy = xs[n + i], sz = xs[2 * n + i];
    int32_t cap = k;
    if (finite3(sx, sy, sz)) {
      double r = std::sqrt((sx * sx + sy * sy) + sz * sz);
      double c = std::floor(mean * (1.0 - r / r_max) + 0.5);
      cap = c < double(k) ? k : (c > double(nmax) ? nmax : int32_t(c));
    }
    caps[i] = cap;
  }
  return 0;
}

// Eviction (Sec. III-A.3): remove the voxels farther than `radius` from c,
// judged by the voxel centre, and rebuild the map from the surviving points
// in id order.
int orc_map_evict(orc_map* m, const double c[3], double radius, int64_t* n_removed) {
  if (!(radius >= 0.0)) return 1;
  const double v = m->g.v, r2 = radius * radius;
  const int64_t N = int64_t(m->g.pts.size());
  orc_map fresh;
  fresh.g.v = v;
  fresh.nmax = m->nmax;
  fresh.dmin = m->dmin;
  fresh.k_cov = m->k_cov;
  fresh.point_cap = m->point_cap;
  fresh.voxel_cap = m->voxel_cap;
  int64_t removed = 0;
  for (int64_t id = 0; id < N; ++id) {
    const Pt& p = m->g.pts[size_t(id)];
    Key K = key_of(p.x, p.y, p.z, v);
    double dx = (double(K.x) + 0.5) * v - c[0];
    double dy = (double(K.y) + 0.5) * v - c[1];
    double dz = (double(K.z) + 0.5) * v - c[2];
    if ((dx * dx + dy * dy) + dz * dz > r2) { ++removed; continue; }
    int64_t nid = int64_t(fresh.g.pts.size());
    fresh.g.vox[K].push_back(nid);
    fresh.g.pts.push_back(p);
    fresh.fx.push_back(m->fx[size_t(id)]);
    fresh.fy.push_back(m->fy[size_t(id)]);
    fresh.fz.push_back(m->fz[size_t(id)]);
    for (int t = 0; t < 6; ++t) fresh.cov.push_back(m->cov[size_t(id) * 6 + t]);
    fresh.valid.push_back(m->valid[size_t(id)]);
  }
  *m = std::move(fresh);
  if (n_removed) *n_removed = removed;
  return 0;
}

// ---------------------------------------------------------------------------
// Motion undistortion (Sec. III-A.1).  The velocity history is fitted by
// ordinary least squares per twist component, centred on the mean sample
// time; every point is then carried to the frame of the scan's last point
// time by the exponential of the fitted twist integrated over [t_ref, t_i].
// For a twist linear in time the integral is tau times its value at the
// midpoint (t_i + t_ref) / 2.
// ---------------------------------------------------------------------------
void orc_fit_twist(const double* ts, const double* xi, int64_t m, double* tbar, double a[6],
                   double b[6]) {
  std::vector<int64_t> use;
  for (int64_t j = 0; j < m; ++j) {
    bool ok = std::isfinite(ts[j]);
    for (int k = 0; k < 6; ++k) ok = ok && std::isfinite(xi[j * 6 + k]);
    if (ok) use.push_back(j);
  }
  for (int k = 0; k < 6; ++k) a[k] = b[k] = 0.0;
  *tbar = 0.0;
  if (use.empty()) return;
  double st = 0.0;
  for (int64_t j : use) st += ts[j];
  double tb = st / double(use.size());
  double stt = 0.0;
  for (int64_t j : use) stt += (ts[j] - tb) * (ts[j] - tb);
  for (int k = 0; k < 6; ++k) {
    double sy = 0.0;
    for (int64_t j : use) sy += xi[j * 6 + k];
    double mean = sy / double(use.size());
    double sty = 0.0;
    for (int64_t j : use) sty += (ts[j] - tb) * (xi[j * 6 + k] - mean);
    a[k] = mean;
    b[k] = stt > 0.0 ? sty / stt : 0.0;
  }
  *tbar = tb;
}

void orc_undistort(const float* xyz, const float* t, int64_t n, const double* ts,
                   const double* xi, int64_t m, float* out, double* t_ref) {
  double tb, a[6], b[6];
  orc_fit_twist(ts, xi, m, &tb, a, b);
  bool any = false;
  double tr = 0.0;
  for (int64_t i = 0; i < n; ++i)
    if (std::isfinite(t[i]) && (!any || double(t[i]) > tr)) { tr = t[i]; any = true; }
  *t_ref = any ? tr : std::nan("");
  const float* X = xyz;
  const float* Y = xyz + n;
  const float* Z = xyz + 2 * n;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(t[i])) {
      out[i] = X[i]; out[n + i] = Y[i]; out[2 * n + i] = Z[i];
      continue;
    }
    double tau = double(t[i]) - tr;
    double mid = (double(t[i]) + tr) / 2.0 - tb;
    double phi[6];
    for (int k = 0; k < 6; ++k) phi[k] = tau * (a[k] + b[k] * mid);
    // orc_se3_exp takes (rotation, translation)
    double d[6] = {phi[3], phi[4], phi[5], phi[0], phi[1], phi[2]};
    double T[16];
    orc_se3_exp(d, T);
    double p[3] = {X[i], Y[i], Z[i]};
    for (int r = 0; r < 3; ++r)
      out[r * n + i] = float(((T[r * 4 + 0] * p[0] + T[r * 4 + 1] * p[1]) + T[r * 4 + 2] * p[2]) +
                             T[r * 4 + 3]);
  }
}

}  // extern "C"

// Threads of the OpenMP loops (timing of the oracle at a stated core count;
// results do not depend on it).
extern "C" int orc_set_threads(int n) {
  if (n < 1) return 1;
  omp_set_num_threads(n);
  return 0;
}
extern "C" int orc_get_threads(void) { return omp_get_max_threads(); }
