/*
 * far.h -- C ABI of the MI355X (gfx950) FAR-LIO registration hot path.
 *
 * FAR-LIO (arXiv 2606.26010) registers each LiDAR scan P* to a local submap Q
 * with a sparsity-aware GICP (Sec. III-A.2) on top of a GPU voxel hash map
 * with a per-voxel point cap (Sec. III-A.2 cuVoxelMap paragraph, Sec. III-A.3).
 * This library implements that hot path in hand-written HIP: the capped map
 * insert with per-point regularised covariances (Eq. 1), the 27-voxel
 * neighbour search, the per-point GICP term (Eqs. 3-5) reduced into a 6x6 H,
 * a 6-vector b and a cost, and the Gauss-Newton iteration (Eq. 6), for one
 * scan or for many scans in one launch.
 *
 * Conventions shared by every entry point
 *  - [dev]  pointer to HIP device memory owned by the caller; the call only
 *           borrows it for the stream-ordered work it enqueues on `stream`.
 *    [host] pointer to host memory, read or written before the call returns.
 *  - Points are SoA float32 [3][n]: n x values, then n y values, then n z.
 *  - Covariances are SoA float32 [6][n] holding the upper triangle of the
 *    symmetric 3x3 matrix in the order xx, xy, xz, yy, yz, zz.
 *  - Poses are row-major double[16] 4x4 rigid transforms, map <- sensor.
 *  - `stream` is a hipStream_t (NULL = the null stream).
 *  - Every function returns a far_status_t and never throws; on failure
 *    far_last_error() gives a thread-local message.  Arguments are checked
 *    before any work is enqueued (FAR_E_INVALID).  A HIP runtime failure is
 *    FAR_E_HIP.
 *  - Calls on one map must be ordered: issue them on one stream, or
 *    synchronise between streams yourself.
 *  - Every neighbour decision (voxel key, squared distance, radius test,
 *    ranking, spacing test) is taken in FP64 with the squared distance
 *    evaluated as (dx*dx + dy*dy) + dz*dz without fused multiply-add, and
 *    ties ranked by point id, so neighbour sets are reproducible bit for bit.
 */
#ifndef FAR_H
#define FAR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* far_stream_t;                /* a hipStream_t */
typedef struct far_map_s* far_map_t;       /* opaque; owns its device storage */

typedef enum {
  FAR_OK = 0,
  FAR_E_INVALID = 1,      /* bad argument or out-of-range coordinates       */
  FAR_E_CAPACITY = 2,     /* point or voxel capacity of the map exceeded     */
  FAR_E_HIP = 3,          /* HIP runtime error                               */
  FAR_E_NOT_PD = 4,       /* H not positive definite (degenerate geometry)  */
  FAR_E_FEW_CORR = 5,     /* fewer than 6 correspondences                    */
  FAR_E_UNSUPPORTED = 6   /* no usable gfx950 device / feature unavailable   */
} far_status_t;

typedef enum {
  FAR_PREC_FP32 = 0,      /* FP32 per-point term, FP64 sums                  */
  FAR_PREC_FP64 = 1       /* every per-point term and sum in FP64            */
} far_precision_t;

/* Option bit OR-ed into a precision argument (far_gicp_linearize,
 * far_gicp_gradient, far_gicp_gradient_batch) or field (far_align_params_t,
 * far_odometry_params_t).  FAR_OPT_NO_SA turns the sparsity-aware case of
 * Sec. III-A.2 off: a correspondence whose source or map covariance is
 * invalid is dropped like an outlier (no term, not an inlier, corr -1)
 * instead of entering as a point-to-point term with M = I; the ablation the
 * paper reports in Table III. */
enum { FAR_OPT_NO_SA = 0x100 };

/* Map parameters (Sec. III-A.2: voxel edge v, at most N_max "regularly
 * spaced" points per voxel; covariances from k neighbours).  Capacities are
 * fixed at create; the map never grows. */
typedef struct {
  double voxel_size;          /* v > 0, metres                                */
  int32_t max_pts_per_voxel;  /* N_max in [1, 64]                             */
  double min_spacing;         /* < 0: v / sqrt(N_max); 0: off; > 0: metres    */
  int64_t point_capacity;     /* >= 1, < 2^31                                 */
  int64_t voxel_capacity;     /* < 2^25; <= 0: min(point_capacity, 2^25 - 1)  */
  int32_t k_cov;              /* neighbours per covariance, [1, 32]           */
} far_map_params_t;

/* One linearisation: H = sum w J^T W J (row-major 6x6, symmetric),
 * b = sum w J^T W d, cost = sum rho, over n_inliers correspondences, with the
 * twist ordered (omega, v). */
typedef struct {
  double H[36];
  double b[6];
  double cost;
  int64_t n_inliers;
} far_lin_t;

/* Gauss-Newton parameters.  tau: correspondence threshold (the search radius
 * is min(tau, v)); kappa: Cauchy scale (Eq. 5); eps: stop when the norm of
 * the increment twist is <= eps; recenter: linearise about the current
 * translation (1) or the origin (0); precision: far_precision_t. */
typedef struct {
  double tau;
  double kappa;
  int32_t max_iters;          /* [1, 64] */
  double eps;
  int32_t recenter;
  int32_t precision;
} far_align_params_t;

typedef struct {
  int32_t iters;              /* Gauss-Newton updates applied                 */
  int32_t converged;          /* 1 if the last increment was <= eps           */
  int32_t status;             /* far_status_t of this scan                    */
  int32_t reserved;
  far_lin_t last;             /* linearisation of the last iteration          */
} far_align_stats_t;

typedef struct {
  int64_t n_points;
  int64_t n_voxels;           /* voxel keys held (a voxel may be empty)       */
  int64_t table_slots;        /* open-addressing slots (power of two)         */
  double load_factor;         /* n_voxels / table_slots                       */
  double mean_probe;          /* mean slots inspected to find a held key      */
  int32_t max_probe;          /* longest such probe                           */
  int32_t max_pts_per_voxel;
  double voxel_size;
  double min_spacing;         /* resolved spacing, metres                     */
  int64_t bytes_device;       /* device memory owned by the map               */
} far_map_stats_t;

/* Create an empty map (all storage allocated here, sized by the
 * capacities).  *out receives the handle.  FAR_E_INVALID on bad params. */
far_status_t far_map_create(const far_map_params_t* params /* [host] */,
                            far_stream_t stream, far_map_t* out /* [host] */);

/* Release the map and its device storage (synchronises the device). */
far_status_t far_map_destroy(far_map_t map);

/* Capped insert of n points xyz [dev, SoA 3 x n, map frame]
 * (Sec. III-A.3).  Result equals inserting the points one at a time in input
 * order: point i enters voxel K = floor(p_i / v) iff the voxel holds fewer
 * than cap_i = min(voxel_cap[i], N_max) points (N_max when voxel_cap is NULL)
 * and, when spacing is on, every point already in K is at least min_spacing
 * away.  Accepted points get consecutive ids.  Afterwards the regularised
 * covariance (Eq. 1, k_cov neighbours within v, the point itself included;
 * valid iff exactly k_cov exist) of every added point is computed on the
 * updated map; existing points keep theirs.
 * Non-finite points are skipped.  Keys outside [-2^20, 2^20) per axis:
 * FAR_E_INVALID with the map unchanged.  More new voxels than the voxel
 * capacity allows: FAR_E_CAPACITY with the map unchanged.  More accepted
 * points than the point capacity allows: FAR_E_CAPACITY, the points accepted
 * before the overflow are kept.  Synchronises `stream`.
 * voxel_cap: [dev] int32 per point, or NULL.  n_accepted: [host] or NULL. */
far_status_t far_map_insert(far_map_t map, const float* xyz, int64_t n,
                            const int32_t* voxel_cap, far_stream_t stream,
                            int64_t* n_accepted);

/* k nearest map points (k in [1, 32]) within radius (0 < radius <= v) of each
 * query q [dev, SoA 3 x n], searched over the 27 voxels around the query's
 * voxel (Sec. III-A.2, Fig. 3), ranked by (squared distance, id).
 * idx [dev, n x k] receives ids, padded with -1; d2 [dev, n x k, or NULL] the
 * squared distances rounded to float (-1 pad); count [dev, n, or NULL] the
 * number found.  Asynchronous. */
far_status_t far_map_knn(far_map_t map, const float* q, int64_t n, int32_t k,
                         double radius, int32_t* idx, float* d2, int32_t* count,
                         far_stream_t stream);

/* Regularised covariances of a scan against itself (Sec. III-A.2: the scan's
 * covariances come from its own voxel map, no cap): for each point, Eq. 1 on
 * its k nearest scan points within r = voxel_size (itself included).
 * xyz [dev, SoA 3 x n, sensor frame]; cov6 [dev, SoA 6 x n] (zero where
 * invalid); valid [dev, n] = 1 iff exactly k neighbours exist.  Keys outside
 * [-2^20, 2^20): FAR_E_INVALID.  Asynchronous apart from one small copy. */
far_status_t far_scan_covariances(const float* xyz, int64_t n, double voxel_size,
                                  int32_t k, float* cov6, uint8_t* valid,
                                  far_stream_t stream);

/* Covariances of S scans in one pass: scan s holds points
 * [offsets[s], offsets[s+1]) of xyz [dev, SoA 3 x n_total]; each point's
 * covariance uses only points of its own scan (as far_scan_covariances does
 * for one scan).  offsets [dev, S+1] int64, non-decreasing, offsets[0] = 0,
 * offsets[S] = n_total.  cov6 [dev, SoA 6 x n_total], valid [dev, n_total]. */
far_status_t far_scan_covariances_batch(const float* xyz, const int64_t* offsets, int32_t S,
                                        int64_t n_total, double voxel_size, int32_t k,
                                        float* cov6, uint8_t* valid, far_stream_t stream);

/* far_scan_covariances_batch that also returns the order its grid sorted the
 * points in: order [dev, n_total] uint32 receives, for each position j of
 * the (scan, 4 x 4 x 4 block of cells, cell, x) order, the index of the
 * point there.  Each scan's points keep the scan's own index range, the
 * points of one voxel and of one block are adjacent, so the order is a
 * spatially compact layout of every scan; the align below takes it in place
 * of sorting the source itself.  Ownership:
 * order is the caller's; it is written in full (n_total entries).  Errors as
 * far_scan_covariances_batch, and FAR_E_INVALID when order is null. */
far_status_t far_scan_covariances_batch_order(const float* xyz, const int64_t* offsets,
                                              int32_t S, int64_t n_total, double voxel_size,
                                              int32_t k, float* cov6, uint8_t* valid,
                                              uint32_t* order, far_stream_t stream);

/* far_scan_covariances_batch that also writes the source in the packed form
 * the batched align reads, in the grid's order (as for
 * far_scan_covariances_batch_order), so that the align neither sorts nor
 * packs: packed [dev, 40 x n_total bytes, 16-byte aligned] receives A float4
 * [n_total] (x, y, z, the point's index as int32 bits), then B float4
 * [n_total] (xx, or -1 when the covariance is invalid, xy, xz, yy), then C
 * float2 [n_total] (yz, zz), the covariance words as written to cov6.
 * Ownership: packed is the caller's.  Errors as far_scan_covariances_batch,
 * and FAR_E_INVALID when packed is null or misaligned. */
far_status_t far_scan_covariances_batch_packed(const float* xyz, const int64_t* offsets,
                                               int32_t S, int64_t n_total, double voxel_size,
                                               int32_t k, float* cov6, uint8_t* valid,
                                               void* packed, far_stream_t stream);

/* One GICP linearisation (Eqs. 3-5, sparsity-aware) of the scan src
 * [dev, SoA 3 x n] with covariances cov6 [dev, SoA 6 x n] and valid [dev, n]
 * against the map at pose T [host]: p = R s + t in FP64; correspondence = the
 * nearest map point within min(tau, v), none = outlier; d = r - p;
 * M = Sigma_r + R Sigma_s R^T (M = I unless both covariances are valid);
 * e2 = d^T M^-1 d; Cauchy weight w = kappa^2/(kappa^2 + e2) and cost
 * rho = kappa^2/2 ln(1 + e2/kappa^2); J = [[p - c]x, -I] for the perturbation
 * p -> c + Exp(delta)(p - c).  c [host, 3] or NULL for the origin.
 * corr [dev, n] or NULL receives each point's correspondence id (-1 none).
 * Synchronises `stream`; out [host]. */
far_status_t far_gicp_linearize(far_map_t map, const float* src, const float* cov6,
                                const uint8_t* valid, int64_t n, const double T[16],
                                double tau, double kappa, const double c[3],
                                int32_t precision, int32_t* corr, far_lin_t* out,
                                far_stream_t stream);

/* far_gicp_linearize with its result left on the device: out [dev, one
 * far_lin_t] is written stream-ordered; no host synchronisation, so the call
 * can be recorded in a graph (after far_map_reserve covers n, it allocates
 * nothing).  n == 0 writes a zero result. */
far_status_t far_gicp_linearize_async(far_map_t map, const float* src, const float* cov6,
                                      const uint8_t* valid, int64_t n, const double T[16],
                                      double tau, double kappa, const double c[3],
                                      int32_t precision, int32_t* corr, far_lin_t* out,
                                      far_stream_t stream);

/* Launch of the linearisation's tile passes (process-wide): blocks_per_cu 0
 * (the default) launches one block per tile; n > 0 launches a persistent grid
 * of n blocks per CU (rounded to a multiple of 8) in which each block takes
 * tiles in turn, every tile staying on the XCD it has in the one-block-per-
 * tile launch.  Results are identical for every setting; far_get_* reads it. */
far_status_t far_set_linearize_grid(int32_t blocks_per_cu);
far_status_t far_get_linearize_grid(int32_t* blocks_per_cu);

/* Reserves the map's registration workspace (packed source, tile tables,
 * search queue, partial sums, sort buffers) for scans or batches of up to
 * max_points points and max_scans scans (the paper preallocates its GPU
 * memory, Sec. IV-B).  Linearize, align and gradient calls within these
 * limits then allocate no workspace and never synchronise the device to grow
 * it; larger calls grow it (device synchronisation, reallocation).  Owned by
 * the map, freed by far_map_destroy.  Synchronises the device when the
 * workspace grows. */
far_status_t far_map_reserve(far_map_t map, int64_t max_points, int32_t max_scans,
                             far_stream_t stream);

/* Gradient of the GICP cost (Eq. 4 with the Cauchy rho of Eq. 5) at pose T
 * [host], with each point's correspondence (nearest map point within
 * min(tau, v), searched again here) and the source covariances held fixed;
 * R enters both p = R s + t and M = Sigma_r + R Sigma_s R^T.
 *   grad_T [host, 12]    d cost / d [R | t], row-major 3 x 4, R taken as a
 *                        free 3 x 3 matrix;
 *   grad_twist [host, 6] d cost / d delta at delta = 0 for the perturbation
 *                        T(delta) = T_c Exp(delta) T_c^-1 T about c [host, 3]
 *                        (NULL = origin), delta = (omega, v);
 *   grad_src [dev, SoA 3 x n, or NULL]  d cost / d s_i (0 for outliers);
 *   cost, n_inliers [host, or NULL].
 * precision as for far_gicp_linearize.  Synchronises `stream`. */
far_status_t far_gicp_gradient(far_map_t map, const float* src, const float* cov6,
                               const uint8_t* valid, int64_t n, const double T[16],
                               double tau, double kappa, const double c[3], int32_t precision,
                               double grad_T[12], double grad_twist[6], float* grad_src,
                               double* cost, int64_t* n_inliers, far_stream_t stream);

/* far_gicp_gradient for S scans in one pass: scan s holds points
 * [offsets[s], offsets[s+1]) of src [dev, SoA 3 x n_total], cov6 [dev, SoA
 * 6 x n_total] and valid [dev, n_total] (offsets [dev, S+1] int64,
 * non-decreasing, offsets[0] = 0, offsets[S] = n_total) at pose T [dev,
 * S x 16]; c [dev, S x 3, or NULL = origins] the twist centres.  Outputs
 * [dev]: grad_T [S x 12], grad_twist [S x 6], grad_src [SoA 3 x n_total, or
 * NULL], cost [S, or NULL], n_inliers [S, or NULL].  Each scan's values are
 * the bits far_gicp_gradient gives for it alone when the tile schedule
 * matches.  Malformed offsets give zero outputs.  Asynchronous. */
far_status_t far_gicp_gradient_batch(far_map_t map, const float* src, const int64_t* offsets,
                                     int32_t S, int64_t n_total, const float* cov6,
                                     const uint8_t* valid, const double* T, const double* c,
                                     double tau, double kappa, int32_t precision,
                                     double* grad_T, double* grad_twist, float* grad_src,
                                     double* cost, int64_t* n_inliers, far_stream_t stream);

/* Gauss-Newton align of one scan (Eq. 6): up to max_iters iterations of
 * linearise, solve H delta = -b by FP64 Cholesky, T <- T_c Exp(delta) T_c^-1 T
 * (T_c = translation by the linearisation centre), stopping when
 * ||delta|| <= eps.  Fewer than 6 inliers (FAR_E_FEW_CORR) or a non positive
 * definite H (FAR_E_NOT_PD) stop the loop leaving T as it was.  The solve runs
 * on the GPU; the host sees only the final copy.  T0, T_out, stats: [host].
 * Returns the scan's status. */
far_status_t far_gicp_align(far_map_t map, const float* src, const float* cov6,
                            const uint8_t* valid, int64_t n, const double T0[16],
                            const far_align_params_t* params, double T_out[16],
                            far_align_stats_t* stats, far_stream_t stream);

/* Gauss-Newton align of S scans in one pass per iteration: scan s holds
 * points [offsets[s], offsets[s+1]) of src [dev, SoA 3 x n_total], cov6
 * [dev, SoA 6 x n_total] and valid [dev, n_total]; offsets [dev, S+1] int64,
 * non-decreasing, offsets[0] = 0, offsets[S] = n_total.  T [dev, S x 16] holds
 * the initial poses and receives the results; stats [dev, S].  Each
 * iteration is one linearisation launch over all scans' point tiles, one
 * reduction-and-solve launch with a block per scan, captured in a HIP graph
 * and replayed; finished scans skip their tiles.  No host synchronisation. */
far_status_t far_gicp_align_batch(far_map_t map, const float* src, const int64_t* offsets,
                                  int32_t S, int64_t n_total, const float* cov6,
                                  const uint8_t* valid, double* T,
                                  const far_align_params_t* params,
                                  far_align_stats_t* stats, far_stream_t stream);

/* far_gicp_align_batch with the source packed in the caller's order instead
 * of its own locality sort (a sort by scan and Morton code of the
 * sensor-frame voxel): order [dev, n_total] uint32 must be a permutation
 * that keeps every scan's points in the scan's own index range, such as the
 * one far_scan_covariances_batch_order returns for the same batch, so the
 * step sorts its points once.  The order changes only the rounding order of
 * the FP64 sums.  An order that is not such a permutation gives meaningless
 * poses (entries out of range are skipped, nothing is written out of
 * bounds).  FAR_E_INVALID when order is null and n_total > 0. */
far_status_t far_gicp_align_batch_ordered(far_map_t map, const float* src,
                                          const int64_t* offsets, int32_t S, int64_t n_total,
                                          const float* cov6, const uint8_t* valid,
                                          const uint32_t* order, double* T,
                                          const far_align_params_t* params,
                                          far_align_stats_t* stats, far_stream_t stream);

/* far_gicp_align_batch on a source packed by
 * far_scan_covariances_batch_packed (packed [dev, 40 x n_total bytes] as
 * described there; offsets and the rest as for far_gicp_align_batch).  The
 * packed order must keep each scan's points in the scan's own range, as
 * the grid's order does; the results equal far_gicp_align_batch_ordered's
 * with that order, bit for bit.  FAR_E_INVALID when packed is null or not
 * 16-byte aligned. */
far_status_t far_gicp_align_batch_packed(far_map_t map, const void* packed,
                                         const int64_t* offsets, int32_t S, int64_t n_total,
                                         double* T, const far_align_params_t* params,
                                         far_align_stats_t* stats, far_stream_t stream);

/* Launch schedule of the linearisation on a map (the tile and probe schedule
 * of the batched iteration).  tile: points per block and tile, 128, 256
 * (default) or 512.  fine_cells: 1 = correspondence search over cells of
 * v/2 through a second hash index of the map (built lazily after inserts;
 * power-of-two v only, else ignored), 0 = over the 27 voxels (default).
 * Both searches are exact; the tile changes only the rounding order of the
 * FP64 sums.  A job with fewer tiles than two per compute unit at the map's
 * tile (a single scan of about 100k points) runs at tile 128. */
typedef struct {
  int32_t tile;
  int32_t fine_cells;
} far_schedule_t;

far_status_t far_map_get_schedule(far_map_t map, far_schedule_t* out);
far_status_t far_map_set_schedule(far_map_t map, const far_schedule_t* schedule);

/* Autotuner: times far_gicp_align_batch on the caller's batch (same
 * arguments; T [dev, S x 16] is read, never modified) under every schedule
 * candidate - tiles 128, 256, 512, each with the 27-voxel search and, for a
 * power-of-two v, the fine cells - taking the fastest of `reps` timed runs
 * (after one untimed run) of each.  The fastest schedule is set on the map
 * (the schedule already set stays unless a candidate is more than 2 % faster)
 * and written to best [host]; ms [host, 6 entries, or NULL] receives each
 * candidate's time in the order listed (tile-major, voxel search first;
 * -1 for a candidate not run).  Synchronises `stream`. */
far_status_t far_autotune(far_map_t map, const float* src, const int64_t* offsets, int32_t S,
                          int64_t n_total, const float* cov6, const uint8_t* valid,
                          const double* T, const far_align_params_t* params, int32_t reps,
                          far_schedule_t* best, double* ms, far_stream_t stream);

/* Covariance regularisation of every covariance computed afterwards (map
 * inserts and scan covariances; process-wide, default FAR_REG_EQ1).
 * FAR_REG_EQ1: Eq. (1) of Sec. III-A.2.  FAR_REG_PLANE: the plane
 * regularisation of Segal et al. (cited by the sparsity-aware paragraph),
 * Sigma = I + (1e-3 - 1) n n^T with n the unit eigenvector of the smallest
 * eigenvalue of the k-neighbour sample covariance (FP64 closed-form 3x3
 * eigen-solve on the GPU; when the smallest eigenvalue is double, any unit
 * vector of its eigenspace).  Validity (k neighbours within v) is the same
 * in both modes.  Another mode: FAR_E_INVALID. */
typedef enum { FAR_REG_EQ1 = 0, FAR_REG_PLANE = 1 } far_cov_reg_t;
far_status_t far_set_covariance_regularisation(int32_t mode);
far_status_t far_get_covariance_regularisation(int32_t* mode);

/* Schedule of the scan covariance search (process-wide).  The points of a
 * voxel holding at least dense_threshold of its scan's points are searched
 * by one wave per voxel (the voxel's points share one 27-voxel
 * neighbourhood, walked once at wave-uniform addresses), the others one
 * lane per point over the 27 voxels; 0 = one lane per point everywhere.
 * Default 0 (measured fastest on the batched workload).  Results are
 * identical for every setting. */
far_status_t far_set_covariance_schedule(int32_t dense_threshold);
far_status_t far_get_covariance_schedule(int32_t* dense_threshold);

/* Covariance autotuner: times far_scan_covariances_batch on the caller's
 * batch for dense thresholds 0, 16, 32, 64 and 128 (fastest of `reps`
 * timed runs after one untimed run each), sets the fastest (the threshold
 * already set stays unless a candidate is more than 2 % faster) and returns
 * it in best [host]; ms [host, 5 entries, or NULL] the times.  cov6 and valid
 * receive the covariances.  Synchronises `stream`. */
far_status_t far_autotune_covariances(const float* xyz, const int64_t* offsets, int32_t S,
                                      int64_t n_total, double voxel_size, int32_t k,
                                      float* cov6, uint8_t* valid, int32_t reps, int32_t* best,
                                      double* ms, far_stream_t stream);

/* Occupancy and probe statistics of the map's hash table.  Synchronises. */
far_status_t far_map_stats(far_map_t map, far_map_stats_t* out, far_stream_t stream);

/* Copy the map out in id order: xyz [dev, SoA 3 x N], cov6 [dev, SoA 6 x N],
 * valid [dev, N] (any may be NULL); N = the map's point count, written to
 * n_out [host].  The buffers must hold `capacity` points; FAR_E_CAPACITY if
 * N exceeds it (nothing written).  Synchronises. */
far_status_t far_map_export(far_map_t map, float* xyz, float* cov6, uint8_t* valid,
                            int64_t capacity, int64_t* n_out, far_stream_t stream);

/* ------------------------------------------------------------------------
 * Scan-to-submap odometry over a sequence (Sec. III-A: preprocessing,
 * registration against the capped submap, insertion of the registered scan
 * into the submap), with the adaptive threshold of Sec. III-A.2.
 * ---------------------------------------------------------------------- */

/* Voxel downsampling of a scan (the preprocessing of the runtime breakdown of
 * Sec. IV-B; the rule is not given and is read as: for every voxel of edge v
 * keep the first point in input order).  xyz [dev, SoA 3 x n]; out [dev, room
 * for 3 x n floats, not aliasing xyz] receives the kept points in input order,
 * SoA with row stride n_out; keep [dev, n, or NULL] their input indices;
 * n_out [host].  Non-finite points are dropped.  Keys outside [-2^20, 2^20):
 * FAR_E_INVALID, nothing written.  Synchronises `stream`. */
far_status_t far_voxel_downsample(const float* xyz, int64_t n, double v, float* out,
                                  int32_t* keep, int64_t* n_out, far_stream_t stream);

/* Rigid transform of xyz [dev, SoA 3 x n] by T [host]: each coordinate is
 * ((R_r0 x + R_r1 y) + R_r2 z) + t_r in FP64 without fused multiply-add,
 * rounded to float, into out [dev, SoA 3 x n] (may alias xyz).  Asynchronous. */
far_status_t far_transform_points(const float* xyz, int64_t n, const double T[16],
                                  float* out, far_stream_t stream);

/* Motion undistortion of one scan (Sec. III-A.1: the sensor's motion during
 * the sweep is modelled by a linear regression over the velocity history of
 * the sensor fusion, and each raw point is moved to the frame of the scan's
 * final point time).  Readings: the velocity samples are body-frame twists
 * vel [dev, m x 6 row-major: vx vy vz wx wy wz] at times vel_t [dev, m]
 * (seconds, the clock of t); each component is fitted by least squares as
 * a_k + b_k (time - tbar), tbar the mean sample time, leaving out samples with
 * a non-finite entry (none left: no motion; one time only: b = 0).  The
 * frame reference t_ref is the largest finite point time; point i at time
 * t[i] is moved by the SE(3) exponential of the fitted twist integrated over
 * [t_ref, t[i]], (t[i] - t_ref) xi((t[i] + t_ref) / 2), evaluated in FP64 and
 * rounded to float.  Points with a non-finite time are copied unchanged.
 * xyz, out [dev, SoA 3 x n; out may alias xyz]; t [dev, n, float seconds,
 * e.g. relative to the scan start]; t_ref [dev, 1, or NULL] receives the
 * reference time (NaN when no time is finite).  Asynchronous; no memset, so
 * the launches may be captured in a graph. */
far_status_t far_undistort(const float* xyz, const float* t, int64_t n, const double* vel_t,
                           const double* vel, int32_t m, float* out, double* t_ref,
                           far_stream_t stream);

/* far_undistort for S scans in one pass: scan s holds points
 * [offsets[s], offsets[s+1]) of xyz, t and out (SoA 3 x n_total) and
 * velocity samples [vel_offsets[s], vel_offsets[s+1]) of vel_t and vel;
 * offsets and vel_offsets [dev, S+1] int64, non-decreasing from 0, with
 * offsets[S] = n_total; t_ref [dev, S, or NULL]. */
far_status_t far_undistort_batch(const float* xyz, const float* t, const int64_t* offsets,
                                 int32_t S, int64_t n_total, const double* vel_t,
                                 const double* vel, const int64_t* vel_offsets, float* out,
                                 double* t_ref, far_stream_t stream);

/* far_undistort_batch for callers that cannot allocate device memory: code
 * recorded under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, kernels and results as
 * far_undistort_batch; it calls no hipMalloc, hipFree or allocating routine.
 * Its scratch (per-chunk time maxima and per-scan fit coefficients) is a
 * fixed device array of about 1.6 MB inside the library, one copy per GPU,
 * held until the process ends; its address is looked up on the first call
 * on each device.  Limits: S <= 4096 scans and n_total <= 2^28 points, else
 * FAR_E_CAPACITY with nothing enqueued.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller.  Not timed by
 * far_timing_*.  Asynchronous. */
far_status_t far_undistort_batch_noalloc(const float* xyz, const float* t,
                                         const int64_t* offsets, int32_t S, int64_t n_total,
                                         const double* vel_t, const double* vel,
                                         const int64_t* vel_offsets, float* out, double* t_ref,
                                         far_stream_t stream);

/* Adaptive submap density (Sec. III-A.3, ASMD): per-point insert caps that
 * follow the current scan's density near the sensor and decay over range
 * (the paper gives no constants; reading): mean = points per voxel of edge v
 * over the finite points within r_near of the sensor, counted on their
 * map-frame voxels (nmax when there are none); cap_i = clamp(floor(mean
 * (1 - r_i / r_max) + 0.5), k, nmax) with r_i the point's sensor range, in
 * FP64 in that order.  xyz_sensor and xyz_map [dev, SoA 3 x n] are the same
 * points in the sensor and the map frame; caps [dev, n] (non-finite points:
 * k), to pass to far_map_insert; mean_near [host, or NULL].  Near keys
 * outside [-2^20, 2^20): FAR_E_INVALID.  Synchronises `stream`. */
far_status_t far_asmd_caps(const float* xyz_sensor, const float* xyz_map, int64_t n, double v,
                           int32_t k, int32_t nmax, double r_near, double r_max, int32_t* caps,
                           double* mean_near, far_stream_t stream);

/* Submap eviction (Sec. III-A.3, last step): removes every voxel whose centre
 * ((key + 1/2) v per axis) is farther than radius from c [host, 3], with its
 * points; the surviving points keep their coordinates, covariances (not
 * recomputed) and relative order and are renumbered 0..N'-1; the voxel
 * structures are rebuilt from them (voxels left empty do not survive).
 * n_removed [host, or NULL].  Synchronises `stream`. */
far_status_t far_map_evict(far_map_t map, const double c[3], double radius,
                           int64_t* n_removed, far_stream_t stream);

/* Adaptive correspondence threshold tau and Cauchy scale kappa (Sec. III-A.2
 * adapts both to the motion following Vizzo et al., KISS-ICP; read as its
 * published rule).  The deviation of an estimate T_est from its motion
 * prediction T_pred is the largest displacement D = T_pred^-1 T_est causes
 * within range r_max: 2 r_max sin(theta/2) + |t_D| (theta = rotation angle
 * of D).  Deviations above min_motion are samples; sigma = their root mean
 * square (sigma0 before the first); tau = 3 sigma, kappa = sigma / 3.
 * Host-only state, plain C, no device work. */
typedef struct {
  double sigma0, r_max, min_motion;
  double sse;             /* sum of squared samples */
  int64_t n_samples;
} far_threshold_t;

far_status_t far_threshold_init(far_threshold_t* s, double sigma0, double r_max,
                                double min_motion);
/* Adds the deviation of T_est [host] from T_pred [host] when above
 * min_motion; deviation [host, or NULL] receives it. */
far_status_t far_threshold_update(far_threshold_t* s, const double T_pred[16],
                                  const double T_est[16], double* deviation);
far_status_t far_threshold_get(const far_threshold_t* s, double* tau, double* kappa);

typedef struct far_odometry_s* far_odometry_t;   /* opaque; owns scan buffers */

typedef struct {
  double downsample;      /* voxel edge of the scan downsample, > 0          */
  double sigma0;          /* threshold sigma before the first sample          */
  double r_max;           /* range of the deviation model (sensor max range)  */
  double min_motion;      /* smallest deviation taken as a sample             */
  int32_t max_iters;      /* Gauss-Newton iterations per scan, 1..64          */
  double eps;             /* stop when ||delta|| <= eps                       */
  int32_t precision;      /* far_precision_t                                  */
  int32_t asmd;           /* 1: insert with far_asmd_caps caps (ASMD)         */
  double r_near;          /* ASMD near range, metres                          */
  double evict_radius;    /* > 0: far_map_evict around the pose after insert  */
} far_odometry_params_t;

typedef struct {
  int32_t status;         /* align status of the scan (FAR_OK for the first) */
  int32_t iters;          /* Gauss-Newton iterations run                      */
  int64_t n_raw;          /* points passed in                                 */
  int64_t n_down;         /* points after the downsample                      */
  int64_t n_inserted;     /* points the map accepted                          */
  int32_t map_full;       /* the map reached its point capacity               */
  int32_t reserved;
  int64_t n_evicted;      /* map points removed by the eviction               */
  double asmd_mean;       /* ASMD near-range mean points per voxel (0: off)   */
  double tau, kappa;      /* threshold and Cauchy scale used (0 for the first)*/
  double deviation;       /* deviation of the estimate from the prediction    */
  double T_pred[16];      /* motion prediction (the initial guess)            */
  far_lin_t last;         /* last linearisation of the align                  */
  double t_ref;           /* reference time of the undistorted scan (NaN: none)*/
} far_odometry_stats_t;

/* An odometry over `map` (borrowed; it must outlive the odometry), whose
 * voxel size and k_cov are used for the scan covariances.  The first scan is
 * placed at T_first [host]; the second is predicted with the relative motion
 * v_first [host] (NULL = identity: the inertial prediction of the paper's
 * filter stands behind it), later ones with constant velocity
 * T_pred = T_prev (T_prev2^-1 T_prev), its rotation projected back onto
 * SO(3). */
far_status_t far_odometry_create(far_map_t map, const far_odometry_params_t* params,
                                 const double T_first[16], const double v_first[16],
                                 far_odometry_t* out);
/* One scan xyz [dev, SoA 3 x n, sensor frame]: downsample; for every scan but
 * the first, covariances of the downsampled scan, tau and kappa from the
 * threshold, align from T_pred, and the deviation added to the threshold (a
 * failed align keeps T_pred and is reported in stats->status); then the
 * downsampled scan, moved by the estimate, is inserted into the map (with
 * ASMD caps when params.asmd is set) until the map is full, and with
 * params.evict_radius > 0 the voxels farther than it from the estimate's
 * position are removed (Sec. III-A.3).  T_out [host] receives the estimate; stats [host, or NULL].
 * Returns FAR_OK unless an argument, a key range or the HIP runtime fails.
 * Synchronises `stream`. */
far_status_t far_odometry_step(far_odometry_t od, const float* xyz, int64_t n,
                               double T_out[16], far_odometry_stats_t* stats,
                               far_stream_t stream);
/* far_odometry_step on a raw scan taken while moving (Sec. III-A.1): the
 * scan xyz [dev, SoA 3 x n] with per-point times t [dev, n] is first
 * undistorted by far_undistort with the velocity samples vel_t [dev, m] and
 * vel [dev, m x 6] into a buffer the odometry owns, so every pose is the
 * sensor's at the scan's reference time (stats->t_ref).  Synchronises
 * `stream`. */
far_status_t far_odometry_step_timed(far_odometry_t od, const float* xyz, const float* t,
                                     int64_t n, const double* vel_t, const double* vel,
                                     int32_t m, double T_out[16], far_odometry_stats_t* stats,
                                     far_stream_t stream);
far_status_t far_odometry_destroy(far_odometry_t od);

/* Instrumentation.  With timing on, the device work of each kind below is
 * bracketed by HIP events recorded on the stream it runs on (before any host
 * synchronisation of the call), and the align entry points launch their
 * kernels directly instead of through a graph.  far_timing_read_kind waits
 * for the recorded intervals of one kind and returns their summed time (ms)
 * and count since the last reset (reset != 0 clears them after reading);
 * far_timing_read is the linearisation kind.  Process-wide; not meant for
 * concurrent use from several threads. */
typedef enum {
  FAR_TIME_LINEARIZE = 0,        /* each linearisation launch of an align    */
  FAR_TIME_UNDISTORT = 1,        /* each far_undistort(_batch) call          */
  FAR_TIME_UNDISTORT_APPLY = 2,  /* its per-point kernel alone               */
  FAR_TIME_GRADIENT = 3,         /* each far_gicp_gradient call              */
  FAR_TIME_ASMD = 4,             /* each far_asmd_caps call                  */
  FAR_TIME_EVICT = 5,            /* each far_map_evict call                  */
  FAR_TIME_COVARIANCES = 6,      /* each far_scan_covariances(_batch) call   */
  FAR_TIME_KINDS = 7
} far_time_kind_t;

far_status_t far_timing_enable(int32_t on);
far_status_t far_timing_read_kind(int32_t kind, double* ms, int64_t* count, int32_t reset);
far_status_t far_timing_read(double* linearize_ms, int64_t* launches, int32_t reset);

/* Scratch memory.  The temporary device buffers of every call (sort
 * buffers, grids, partial sums) come from one stream-ordered pool per device
 * that keeps freed memory for the next call instead of returning it to the
 * driver, so repeated calls map no new memory; the pool grows to the largest
 * scratch a single call has needed.  far_scratch_release returns the unused
 * part of every device's pool to the driver (buffers of calls still running
 * stay); far_scratch_reserved gives the bytes the current device's pool
 * holds (0 before its first use).  Both are safe at any time. */
far_status_t far_scratch_release(void);
far_status_t far_scratch_reserved(int64_t* bytes /* [host] */);

const char* far_status_str(far_status_t s);
const char* far_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FAR_H */
