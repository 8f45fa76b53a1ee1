/*
 * far_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU implementation of the FAR-LIO registration hot path
 * (arXiv 2606.26010, Sec. III-A "LiDAR Scan Pipeline"), written to check the
 * GPU library against.  It shares no code with the GPU library; only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load it.
 *
 * Layouts: every point array is SoA float32 [3][n] (x row, then y, then z);
 * every covariance array is SoA [6][n] holding the upper triangle in the order
 * xx, xy, xz, yy, yz, zz.  Poses are row-major 4x4 doubles (map <- sensor).
 *
 * Return codes mirror the library's status values:
 *   0 ok, 1 invalid argument, 2 capacity, 4 not positive definite,
 *   5 too few correspondences.
 */
#ifndef FAR_ORACLE_H
#define FAR_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_map orc_map;

/* Map with voxel edge v, per-voxel cap nmax, insert spacing dmin (0 = off),
 * k_cov neighbours for covariances, fixed point / voxel capacities. */
orc_map* orc_map_new(double v, int32_t nmax, double dmin, int32_t k_cov,
                     int64_t point_cap, int64_t voxel_cap);
void     orc_map_free(orc_map* m);
int64_t  orc_map_size(const orc_map* m);      /* points held */
int64_t  orc_map_nvoxels(const orc_map* m);   /* voxel keys held */

/* Sequential capped insert (input order), then covariances of the added
 * points on the updated map.  caps: per-point cap or NULL (= nmax). */
int orc_map_insert(orc_map* m, const float* xyz, int64_t n, const int32_t* caps,
                   int64_t* n_accepted, int64_t* n_skipped);

/* Export in ID order: xyz [3][N], cov6 [6][N] (float), valid [N]. */
void orc_map_export(const orc_map* m, float* xyz, float* cov6, uint8_t* valid);

/* k nearest map points within radius r (r <= v) of each query.
 * idx [n][k] (-1 pad), d2 [n][k] (FP64, -1 pad), count [n]. */
int orc_map_knn(const orc_map* m, const float* q, int64_t n, int32_t k, double r,
                int32_t* idx, double* d2, int32_t* count);

/* Per-point regularised covariances of a cloud against itself (no cap). */
int orc_scan_covariances(const float* xyz, int64_t n, double v, int32_t k,
                         double* cov6, uint8_t* valid);

/* One linearisation at pose T about centre c (NULL = origin).
 * src_cov6 is float SoA [6][n] (the stored precision).
 * Outputs: H [36] row-major, b [6], cost, inlier count; optional per-point
 * correspondence ids corr [n] (-1 = none) and per-point detail rows
 * detail [n][18] = (p[3], r[3], W[9], w, rho, e2), NaN for a point without
 * a correspondence, or NULL.
 * sparsity_aware: 1 = a pair lacking a covariance enters with M = I
 * (Sec. III-A.2), 0 = such a pair is dropped (standard GICP). */
int orc_linearize(const orc_map* m, const float* src, const float* src_cov6,
                  const uint8_t* src_valid, int64_t n, const double T[16],
                  double tau, double kappa, const double c[3],
                  double H[36], double b[6], double* cost, int64_t* n_inliers,
                  int32_t* corr, double* detail, int32_t sparsity_aware);

/* Gauss-Newton align.  Returns status; writes T_out, iterations, converged and
 * the last linearisation. */
int orc_align(const orc_map* m, const float* src, const float* src_cov6,
              const uint8_t* src_valid, int64_t n, const double T0[16],
              double tau, double kappa, int32_t max_iters, double eps,
              int32_t recenter, double T_out[16], int32_t* iters,
              int32_t* converged, double H[36], double b[6], double* cost,
              int64_t* n_inliers, int32_t sparsity_aware);

/* Covariance regularisation used by every covariance computed afterwards
 * (map inserts and scan covariances): 0 = Eq. (1) (default), 1 = plane
 * regularisation after Segal et al., I + (1e-3 - 1) n n^T with n the
 * eigenvector of the smallest eigenvalue of the sample covariance (cyclic
 * Jacobi, FP64).  Returns 1 on another mode.  Process-wide. */
int orc_set_cov_mode(int32_t mode);
void orc_plane_cov(const double S[9], double out[9]);
/* Eigenvalues (diagonal order) and eigenvectors (columns of V) by cyclic
 * Jacobi. */
void orc_jacobi3(const double S[9], double evals[3], double V[9]);

/* Building blocks exposed for pinning. */
void orc_voxel_keys(const float* xyz, int64_t n, double v, int64_t* keys3);
void orc_se3_exp(const double delta[6], double T[16]);
int  orc_cholesky_solve6(const double H[36], const double b[6], double x[6]);
void orc_regularize_cov(const double S[9], double out[9]);

/* Map-side work counters of one linearisation at pose T: number of distinct
 * non-empty map voxels in the 27-neighbourhoods of the transformed queries and
 * the number of points they hold (used for the algorithmic byte model). */
void orc_touch_stats(const orc_map* m, const float* src, int64_t n,
                     const double T[16], int64_t* n_voxels, int64_t* n_points);

/* Voxel downsampling of a scan (the preprocessing named in the runtime
 * breakdown of Sec. IV-B; reading: keep, for every voxel of edge v, the
 * first point in input order).  keep [n] receives the kept input indices in
 * increasing order and *n_keep their number; non-finite points are dropped.
 * Returns 1 (and keeps nothing) when a finite point's key is out of range. */
int orc_downsample(const float* xyz, int64_t n, double v, int64_t* keep, int64_t* n_keep);

/* out = R s + t for every point, in FP64 with the fixed evaluation order
 * ((R00 sx + R01 sy) + R02 sz) + tx, rounded to float.  SoA in and out. */
void orc_transform(const float* xyz, int64_t n, const double T[16], float* out);

/* Adaptive correspondence threshold (Sec. III-A.2: the outlier threshold and
 * the Cauchy kappa adapt to the motion, following Vizzo et al., KISS-ICP).
 * State: sum of squared model deviations above min_motion and their count. */
typedef struct {
  double sigma0, r_max, min_motion, sse;
  int64_t n;
} orc_threshold;
void orc_threshold_init(orc_threshold* s, double sigma0, double r_max, double min_motion);
/* Model deviation of T_est against T_pred: 2 r_max sin(theta/2) + |dt| of
 * T_pred^-1 T_est; returns it and adds its square when above min_motion. */
double orc_threshold_update(orc_threshold* s, const double T_pred[16], const double T_est[16]);
/* sigma = sqrt(sse / n), or sigma0 before the first sample; tau = 3 sigma,
 * kappa = sigma / 3. */
void orc_threshold_get(const orc_threshold* s, double* tau, double* kappa);

/* GICP cost (Eq. 4 with the Cauchy rho of Eq. 5) at pose T [16] for given
 * correspondences corr [n] (-1 = none), with FP64 source points
 * src [3][n] double; the rotation block of T is used as a free 3x3 matrix in
 * p = R s + t and M = Sigma_r + R Sigma_s R^T (used for finite differences). */
int orc_cost_fixed(const orc_map* m, const double* src, const float* src_cov6,
                   const uint8_t* src_valid, int64_t n, const double T[16], double kappa,
                   const int32_t* corr, double* cost);

/* Gradient of the GICP cost at T, correspondences (nearest map point within
 * min(tau, v), as orc_linearize) and Sigma_s held fixed:
 *   grad_T [12]     d cost / d [R | t], row-major 3x4 (R as a free 3x3);
 *   grad_twist [6]  d cost / d delta at delta = 0 for
 *                   T(delta) = T_c Exp(delta) T_c^-1 T, delta = (omega, v);
 *   grad_src [3][n] d cost / d s_i (double, or NULL);
 *   cost, n_inliers; corr [n] or NULL receives the correspondences. */
int orc_gradient(const orc_map* m, const float* src, const float* src_cov6,
                 const uint8_t* src_valid, int64_t n, const double T[16], double tau,
                 double kappa, const double c[3], double grad_T[12], double grad_twist[6],
                 double* grad_src, double* cost, int64_t* n_inliers, int32_t* corr,
                 int32_t sparsity_aware);

/* Adaptive submap density (Sec. III-A.3, ASMD).  Reading (the paper gives
 * no constants): the mean number of points per voxel of edge v over the
 * finite points within r_near of the sensor, counted on their map-frame voxel
 * keys (xyz_map), or nmax when there are none; each point's cap is
 * clamp(floor(mean (1 - r_i / r_max) + 0.5), k, nmax), r_i its sensor range
 * (xyz_sensor), in FP64 evaluated in that order.  caps [n]; *mean_near.
 * Returns 1 on a bad argument. */
int orc_asmd_caps(const float* xyz_sensor, const float* xyz_map, int64_t n, double v,
                  int32_t k, int32_t nmax, double r_near, double r_max, int32_t* caps,
                  double* mean_near);

/* Submap eviction (Sec. III-A.3, last step): voxels whose centre
 * ((key + 1/2) v) is farther than radius from c are removed, with their
 * points; the surviving points keep their coordinates, covariances and
 * relative order and are renumbered consecutively; voxels are rebuilt from
 * the surviving points (empty voxels do not survive). */
int orc_map_evict(orc_map* m, const double c[3], double radius, int64_t* n_removed);

/* Motion model of a scan (Sec. III-A.1: a linear regression over the
 * velocity history of the sensor fusion).  Reading: samples are body-frame
 * twists xi = (vx, vy, vz, wx, wy, wz) at times ts; each component is fitted
 * by least squares as a_k + b_k (t - tbar), tbar the mean sample time.
 * Samples with a non-finite time or component are left out; with no sample
 * left a = b = 0, with all times equal b = 0.  xi [m x 6, row-major]. */
void orc_fit_twist(const double* ts, const double* xi, int64_t m, double* tbar, double a[6],
                   double b[6]);

/* Undistortion of a scan (Sec. III-A.1): every point is moved from the
 * sensor frame of its own time t_i to that of the frame reference time
 * t_ref = the largest finite point time.  Reading: the pose of the frame at
 * t_i relative to the frame at t_ref is the SE(3) exponential of the fitted
 * twist integrated from t_ref to t_i, tau (a + b ((t_i + t_ref) / 2 - tbar))
 * with tau = t_i - t_ref (exact for a constant twist and for twists that
 * keep one screw axis; otherwise the first term of its Magnus expansion).
 * Points with a non-finite time are copied unchanged.  xyz, out [SoA 3 x n];
 * t [n]; *t_ref (NaN when no time is finite). */
void orc_undistort(const float* xyz, const float* t, int64_t n, const double* ts,
                   const double* xi, int64_t m, float* out, double* t_ref);


/* Threads of the OpenMP loops (n >= 1; returns 1 for n < 1), and the current
 * maximum.  Only the timing depends on it. */
int orc_set_threads(int n);
int orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
