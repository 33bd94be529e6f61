/* vgicp.h - C ABI of the MI355X (gfx950) VGICP matching-cost library.
 *
 * The library evaluates and linearizes the voxelized-GICP matching-cost factor of Koide et
 * al., "Globally Consistent and Tightly Coupled 3D LiDAR Inertial Mapping" (ICRA 2022):
 *
 *   Sec. III-A:  each point p_k is a Gaussian (mu_k, C_k); the target cloud P_j is cut into
 *                voxels, each holding a Gaussian aggregated from the means and covariances of
 *                the points inside it (the voxel map).
 *   Eq. (2):     e^M(P_i, P_j, T_i, T_j) = sum over p_k in P_i of e^D2D(p_k, T_ij).
 *   Eq. (3):     e^D2D = d_k^T (C'_k + R C_k R^T)^-1 d_k,  d_k = mu'_k - T_ij mu_k, where
 *                (mu'_k, C'_k) is the voxel of P_j that the transformed point falls in.
 *   Sec. III-A:  a Hessian factor (H, b, e) is re-formed from the derivatives of Eq. (2) at
 *                the current linearization point in every optimizer iteration.
 *   Sec. III-D:  the overlap rate of P_i on P_j is the fraction of points of P_i that fall in
 *                a voxel of P_j (inliers / n from vgicp_evaluate).
 *   Secs. III-D to III-F: unary factors (fixed keyframe pose, odometry), binary factors
 *                (two free poses, odometry / local / global mapping), thousands of factors per
 *                global-mapping iteration, optimized with Levenberg-Marquardt (Sec. III-F).
 *   Sec. III-B:  the IMU preintegration factor (Eqs. (4)-(9)) between two states.
 *   Sec. III-C:  preprocessing of a sweep: voxel-grid filter, k nearest neighbours, and the
 *                point covariances C_k of Sec. III-A from those neighbours.
 *
 * CONVENTIONS
 *   Clouds     device memory, FP32, structure of arrays: xyz = [3][n] (all x, then all y,
 *              then all z); cov = [6][n] holding xx, xy, xz, yy, yz, zz. The library never
 *              takes ownership of caller memory.
 *   Poses      world-from-local, FP64, row-major 3x4 [R | t] (12 doubles).
 *   Relative   T_ts = T_target^-1 T_source maps source-local points into the target's local
 *              frame, where the target's voxel map lives.
 *   Tangent    xi = [omega; rho] (rotation first), right perturbation T <- T Exp(xi).
 *   Factor     e(xi) ~= e + 2 b^T xi + xi^T H xi with H = sum J^T Omega J, b = sum J^T Omega d,
 *              Omega = (C'_k + R C_k R^T)^-1 frozen at the linearization point (Gauss-Newton);
 *              the Gauss-Newton step solves H dxi = -b. Unary: 6x6, the free variable is the
 *              source pose. Binary: 12x12 in the order [source | target]. H is row-major and
 *              symmetric (both triangles written).
 *   Voxels     coordinate k = floor(v / res) per axis in FP64 (v in the map's frame); a map
 *              point needs |k| < 2^20. Voxel ids are the rank of the key among the distinct
 *              keys in ascending (x, y, z) lexicographic order, so they do not depend on the
 *              point order or the hash layout. A source point whose voxel is absent
 *              contributes nothing and is not an inlier; its correspondence is -1.
 *   Streams    vgicp_stream is a hipStream_t (NULL = the default stream). Calls that take a
 *              stream are asynchronous on it unless stated otherwise.
 *
 * ERRORS
 *   Every call returns a vgicp_status. Argument errors found on the host return at once and
 *   enqueue nothing. Errors that only the GPU can see (a non-finite transformed point or a
 *   fused covariance that is not positive definite: VGICP_E_NONFINITE) set a sticky per-device
 *   word that vgicp_sync_status() reports (and clears); outputs of the affected call are then
 *   undefined. vgicp_last_error() returns a message for the calling thread's last failure.
 */
#ifndef VGICP_H
#define VGICP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VGICP_API __attribute__((visibility("default")))

typedef void* vgicp_stream; /* a hipStream_t */

typedef enum {
  VGICP_OK = 0,
  VGICP_E_INVALID_ARG = 1, /* null/negative/mismatched argument, bad resolution, bad ids */
  VGICP_E_NONFINITE = 2,   /* NaN/Inf input, or a fused covariance not positive definite */
  VGICP_E_KEY_RANGE = 3,   /* a map point's voxel coordinate has |k| >= 2^20 */
  VGICP_E_CAPACITY = 4,    /* a size exceeds what the library's index types can hold */
  VGICP_E_OOM = 5,         /* device allocation failed */
  VGICP_E_HIP = 6          /* any other HIP runtime error */
} vgicp_status;

/* Arithmetic of the per-point work. Voxel coordinates, the relative pose and the
 * transformed point are always FP64 (they decide which voxel a point falls in), except in
 * VGICP_NAIVE_WORLD_FP32; the fused covariance and its inverse are always FP64 (they lose
 * ~1e-4 relative in FP32 for plane-like covariances). */
typedef enum {
  VGICP_ACC_FP64 = 0,         /* FP64 fused covariance and inverse; FP32 Gauss-Newton terms;
                                 FP32 partial sums per lane over at most 32 of its points,
                                 FP64 for every sum above (default) */
  VGICP_ACC_KAHAN_FP32 = 1,   /* as VGICP_ACC_FP64 with Kahan-compensated FP32 lane sums */
  VGICP_NAIVE_WORLD_FP32 = 2, /* source point taken to world and back to the target frame in
                                 FP32 (FP32 keys), FP64 accumulation; a precision baseline */
  VGICP_MATH_FP64 = 3         /* FP64 per-point math and accumulation */
} vgicp_precision;

/* Lookup structure of a voxel map (which voxel, if any, holds a transformed source point).
 * Both give the same ids; they differ in memory and speed. */
typedef enum {
  VGICP_LAYOUT_AUTO = 0, /* grid when it needs at most 2^23 bricks or 32 bricks per voxel
                            (and at most 2^24), else hash */
  VGICP_LAYOUT_HASH = 1, /* open-addressing table of {key, id} slots, capacity a power of two
                            >= 4 V, linear probing: 32 V to 64 V bytes */
  VGICP_LAYOUT_GRID = 2  /* occupancy bricks of 4 x 4 x 2 voxels over the map's voxel bounding
                            box (a 32-bit mask and a record offset, 8 bytes per brick) plus a
                            copy of the voxel records in brick order: one 8-byte load per
                            lookup; E_CAPACITY above 2^24 bricks */
} vgicp_layout;

typedef struct vgicp_voxelmap_s* vgicp_voxelmap; /* opaque; owns its device memory */
typedef struct vgicp_batch_s* vgicp_batch;       /* opaque; owns its device memory */

/* A source cloud for batched calls: device pointers, layout as above. */
typedef struct {
  const float* xyz;
  const float* cov;
  int64_t n;
} vgicp_cloud;

/* One factor of a batch: indices into the batch's maps, clouds and pose array. binary = 0:
 * unary (target pose fixed, 6x6 result in the leading block of the 12x12 output, zeros
 * elsewhere); binary = 1: 12x12 [source | target]. */
typedef struct {
  int32_t target_map;
  int32_t source_cloud;
  int32_t target_pose;
  int32_t source_pose;
  int32_t binary;
} vgicp_factor;

/* Launch schedule of the batched kernel (chosen by vgicp_batch_autotune or set by hand).
 * block: threads per block (256 or 512); tile: source points per work item (a multiple of
 * block, at most 32 * block); blocks_per_cu: blocks per compute unit in the persistent grid;
 * lookahead: source points each lane resolves together in the lookup phase (2, 4 or 8: more
 * memory requests in flight per wave, more registers per wave). */
typedef struct {
  int32_t block;
  int32_t tile;
  int32_t blocks_per_cu;
  int32_t lookahead;
} vgicp_schedule;

/* ---------------------------------------------------------------------------- preprocessing */

/* Voxel-grid filter of Sec. III-C: every point goes to the cell floor(p / resolution) per axis
 * (FP64, |cell| < 2^20, as the voxel map) and each voxel becomes one point, the FP64 mean of
 * its members' positions rounded to FP32.
 *   xyz [3][n] device FP32 (the input cloud, e.g. a raw sweep in the sensor frame);
 *   t   [n] device FP32 per-point timestamps, or NULL. With timestamps, a cell's points are
 *       taken in ascending (t, index) order and a point whose timestamp differs from the running
 *       mean timestamp of the cell's current voxel by more than scan_duration / 10 starts a new
 *       voxel of that cell (the first and last points of a sweep do not fuse); the voxel's
 *       timestamp is the mean of its members'. Without timestamps a cell is one voxel, summed in
 *       point index order; scan_duration is then ignored (with timestamps it must be > 0).
 *   Output order: ascending cell in (x, y, z) lexicographic order, then creation order within
 *   the cell. xyz_out is written as [3][m] in its first 3 m floats (capacity >= m points);
 *   t_out (may be NULL) receives the m voxel timestamps when t is given. *n_out = m.
 * Synchronises the stream (twice: after the range checks and to learn m). Errors:
 * E_INVALID_ARG, E_NONFINITE (NaN/Inf position or timestamp), E_KEY_RANGE (|cell| >= 2^20),
 * E_CAPACITY (m > capacity: *n_out holds m, nothing is written; or n >= 2^30). */
VGICP_API vgicp_status vgicp_downsample(const float* xyz, const float* t, int64_t n,
                                        double resolution, double scan_duration, float* xyz_out,
                                        float* t_out, int64_t capacity, int64_t* n_out,
                                        vgicp_stream stream);

/* The k nearest neighbours of every point of a cloud (Sec. III-C: found once per sweep and
 * reused for the covariances of Sec. III-A). Exact: the k points with the smallest squared
 * distance (dx*dx + dy*dy) + dz*dz in FP64 from the FP32 coordinates, ties broken by the lower
 * point index; the point itself is included. neighbors is [k][n] device int32: column i holds
 * point i's neighbours, nearest first; -1 fills the entries beyond n when n < k.
 * 1 <= k <= 32. cell is the edge of the search grid, rounded up to a power of two, or 0 to
 * derive it from the cloud (the median distance, over 64 sampled points, within which k points
 * lie); it only affects speed. Synchronises the stream. Errors: E_INVALID_ARG, E_NONFINITE,
 * E_CAPACITY (n >= 2^30). */
VGICP_API vgicp_status vgicp_knn(const float* xyz, int64_t n, int32_t k, double cell,
                                 int32_t* neighbors, vgicp_stream stream);

/* Point covariances C_k (Sec. III-A: computed from each point's neighbouring points; Sec.
 * III-C: from the precomputed neighbour lists, after deskewing). For point i, S is the
 * scatter sum (p - m)(p - m)^T over its listed neighbours (entries -1 skipped) about their mean
 * m, in FP64. With scale > 0 the covariance is plane-regularized as in GICP: with u the unit
 * eigenvector of the smallest eigenvalue of S (cyclic Jacobi, FP64),
 * C = scale * (I - (1 - eps) u u^T), i.e. eigenvalues scale * (1, 1, eps). scale = 0 gives the
 * sample covariance S / m instead. xyz [3][n], neighbors [k][n] (as vgicp_knn writes them),
 * cov [6][n] FP32 xx, xy, xz, yy, yz, zz, all device memory; 1 <= k <= 32. Asynchronous; a
 * neighbour index outside [-1, n) sets the sticky error word (E_INVALID_ARG from
 * vgicp_sync_status) and is skipped. */
VGICP_API vgicp_status vgicp_point_covariances(const float* xyz, int64_t n,
                                               const int32_t* neighbors, int32_t k,
                                               double scale, double eps, float* cov,
                                               vgicp_stream stream);

/* ---------------------------------------------------------------------------- IMU factor */

/* IMU preintegration (Sec. III-B, Eqs. (4)-(6) integrated from the body frame of time i, as in
 * the on-manifold preintegration the section cites), batched over factors, FP64. Factor f owns
 * the samples seg[f] .. seg[f+1]-1 of the n_samples rows of imu, each 7 doubles (gyro w,
 * accelerometer a, interval dt > 0), and the fixed biases bias[f] = (b_a, b_w):
 *   dR <- dR Exp((w - b_w) dt),  dv <- dv + dR (a - b_a) dt,
 *   dp <- dp + dv dt + dR (a - b_a) dt^2 / 2,
 * with the 9x9 covariance of the preintegration noise (dphi, dv, dp) propagated to first order
 * from white gyro / accelerometer noise of densities gyro_sigma, acc_sigma (discrete variance
 * sigma^2 / dt). preint[f] = dR (row-major 9), dv (3), dp (3), total dt (1): [F][16];
 * cov [F][81] row-major. All arrays device memory; seg is int64 [F + 1]. An empty segment
 * gives the identity and a zero covariance. Asynchronous; a segment outside [0, n_samples] or
 * with seg[f+1] < seg[f] sets E_INVALID_ARG (the factor is skipped), a non-positive or
 * non-finite dt E_NONFINITE in the sticky error word. */
VGICP_API vgicp_status vgicp_imu_preintegrate(const double* imu, int64_t n_samples,
                                              const int64_t* seg, int32_t n_factors,
                                              const double* bias,
                                              double gyro_sigma, double acc_sigma,
                                              double* preint, double* cov, vgicp_stream stream);

/* Gauss-Newton blocks of IMU preintegration factors (Eqs. (7)-(9) as constraints between the
 * states i, j; the biases held at the preintegration's): residual
 *   r = [Log(dR^T R_i^T R_j); R_i^T (v_j - v_i - g dt) - dv; R_i^T (t_j - t_i - v_i dt - g dt^2/2) - dp],
 * e = r^T cov^-1 r, and over the unknowns [xi_i (6), v_i (3), xi_j (6), v_j (3)] (poses perturbed
 * on the right as T Exp(xi), xi = [omega; rho]; velocities additively, world frame)
 * H = J^T cov^-1 J (18x18 row-major), b = J^T cov^-1 r; e(d) ~= e + 2 b^T d + d^T H d.
 * states [F][2] int32 (i, j) index poses [P][12] (world-from-body [R | t]) and velocities [P][3];
 * gravity is a host array of 3 doubles (world frame). Device arrays: preint [F][16] and cov
 * [F][81] as vgicp_imu_preintegrate writes them, H [F][324], b [F][18], err [F]. Asynchronous;
 * a state index outside [0, P) sets E_INVALID_ARG, a covariance that is not positive definite
 * to working precision (a Cholesky pivot below 1e-13 of its diagonal entry: e.g. a factor of a
 * single sample, whose accelerometer noise moves dv and dp along one direction) E_NONFINITE in
 * the sticky error word. */
VGICP_API vgicp_status vgicp_imu_linearize(const double* preint, const double* cov,
                                           const int32_t* states, int32_t n_factors,
                                           const double* poses, const double* velocities,
                                           int32_t n_states, const double* gravity, double* H,
                                           double* b, double* err, vgicp_stream stream);

/* vgicp_imu_preintegrate and, in bias_jac [F][9][6] (device, row-major), the first-order
 * derivatives of the preintegrated values (rows dphi (3), dv (3), dp (3)) with respect to the
 * biases they were computed with (columns b_a (3), b_w (3); the rotation does not depend on b_a),
 * propagated sample by sample as in the preintegration the paper cites. Same errors. */
VGICP_API vgicp_status vgicp_imu_preintegrate_bias(const double* imu, int64_t n_samples,
                                                   const int64_t* seg, int32_t n_factors,
                                                   const double* bias, double gyro_sigma,
                                                   double acc_sigma, double* preint,
                                                   double* cov, double* bias_jac,
                                                   vgicp_stream stream);

/* The IMU factor with bias states (the state of Eq. (1) is pose, velocity and biases
 * b = [b_a, b_w]). With db = b_i - b0 (b0 = preint_bias[f], the biases the factor was
 * preintegrated with) the preintegrated values are corrected to first order,
 *   dR Exp(J_R,w db_w), dv + J_v db, dp + J_p db  (J = bias_jac[f]),
 * the residual of vgicp_imu_linearize uses them, and the bias random walk r_b = b_j - b_i with
 * covariance diag(bias_walk_acc^2 I, bias_walk_gyro^2 I) dt joins it: 15 residuals, weighted by
 * blockdiag(cov^-1, random-walk covariance^-1), over the 30 unknowns
 * [xi_i (6), v_i (3), b_i (6), xi_j (6), v_j (3), b_j (6)] (biases additively). Device arrays:
 * preint [F][16], cov [F][81], bias_jac [F][54], preint_bias [F][6], states [F][2] int32,
 * poses [P][12], velocities [P][3], biases [P][6]; outputs H [F][900] (30 x 30 row-major),
 * b [F][30], err [F]; e(d) ~= e + 2 b^T d + d^T H d. gravity: host, 3 doubles. Errors as
 * vgicp_imu_linearize; random-walk densities must be positive (E_INVALID_ARG). */
VGICP_API vgicp_status vgicp_imu_linearize_bias(
    const double* preint, const double* cov, const double* bias_jac, const double* preint_bias,
    const int32_t* states, int32_t n_factors, const double* poses, const double* velocities,
    const double* biases, int32_t n_states, const double* gravity, double bias_walk_acc,
    double bias_walk_gyro, double* H, double* b, double* err, vgicp_stream stream);

/* ---------------------------------------------------------------------------- voxel map */

/* Builds the voxel map of one target cloud (Sec. III-A: per voxel, the arithmetic mean of
 * the member points' means and of their covariances, summed in FP64 in increasing point
 * index; no minimum count). xyz/cov: device, [3][n] / [6][n], read during the call only;
 * n >= 0; resolution > 0 and finite. Runs on `stream` and synchronises it once (the voxel
 * count sizes the table). On success *out owns the map: release it with
 * vgicp_destroy_voxelmap. Errors: E_INVALID_ARG, E_NONFINITE (NaN/Inf point),
 * E_KEY_RANGE, E_OOM, E_HIP; *out is then NULL. */
VGICP_API vgicp_status vgicp_build_voxelmap(const float* xyz, const float* cov, int64_t n,
                                            double resolution, vgicp_stream stream,
                                            vgicp_voxelmap* out);

/* As vgicp_build_voxelmap with an explicit lookup structure (vgicp_layout; the plain call
 * uses VGICP_LAYOUT_AUTO). The voxels, their ids and every result computed with the map are
 * the same for every layout. Errors: as vgicp_build_voxelmap, E_INVALID_ARG for an unknown
 * layout, E_CAPACITY for a grid above 2^24 bricks. */
VGICP_API vgicp_status vgicp_build_voxelmap_layout(const float* xyz, const float* cov,
                                                   int64_t n, double resolution,
                                                   int32_t layout, vgicp_stream stream,
                                                   vgicp_voxelmap* out);

/* Number of voxels V and size of the lookup structure of a map: hash slots, or bricks for
 * the grid layout (host outputs, either may be NULL). */
VGICP_API vgicp_status vgicp_voxelmap_size(vgicp_voxelmap map, int64_t* num_voxels,
                                           int64_t* capacity);

/* Lookup structure a map was built with: VGICP_LAYOUT_HASH or VGICP_LAYOUT_GRID (host
 * output). */
VGICP_API vgicp_status vgicp_voxelmap_layout(vgicp_voxelmap map, int32_t* layout);

/* Copies the map in voxel-id order to caller device memory (any pointer may be NULL):
 * keys [V] (packed ((kx+2^20)<<42)|((ky+2^20)<<21)|(kz+2^20)), mean [3][V] FP64,
 * cov [6][V] FP64, count [V]. Asynchronous on `stream`. */
VGICP_API vgicp_status vgicp_voxelmap_export(vgicp_voxelmap map, int64_t* keys, double* mean,
                                             double* cov, int32_t* count, vgicp_stream stream);

/* Frees a map (waits for the device to finish with it). NULL is accepted. */
VGICP_API vgicp_status vgicp_destroy_voxelmap(vgicp_voxelmap map);

/* ---------------------------------------------------------------------------- one factor */

/* Linearizes one matching-cost factor (Eqs. (2)-(3) and their Gauss-Newton derivatives).
 * map: the target's voxel map. xyz/cov/n: the source cloud (device). T_target/T_source:
 * HOST arrays of 12 doubles. binary: 0 = unary (6x6, source pose free), 1 = binary (12x12,
 * [source | target]). Outputs (device): H [36] or [144], b [6] or [12], err [1] (the cost
 * e), inliers [1], corr [n] (voxel id per source point or -1; may be NULL). Results are
 * deterministic: repeated calls give bitwise-equal outputs. n = 0 or no inlier gives zeros. */
VGICP_API vgicp_status vgicp_linearize(vgicp_voxelmap map, const float* xyz, const float* cov,
                                       int64_t n, const double* T_target,
                                       const double* T_source, int32_t binary,
                                       vgicp_precision precision, double* H, double* b,
                                       double* err, int64_t* inliers, int32_t* corr,
                                       vgicp_stream stream);

/* Allocation-free form of vgicp_linearize, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc). Same
 * arguments, kernels and results (bitwise) as vgicp_linearize; the per-tile partial sums live
 * in a static device array of the library (950,272 bytes per device, held until the process
 * ends) instead of a stream-ordered allocation, and the call makes no allocation of any kind.
 * Limit: at most 4,096 tiles, i.e. n <= 33,554,432 points on a 256-CU device; larger n returns
 * VGICP_E_CAPACITY before any launch. Every call on one device shares that array: calls whose
 * work overlaps on the device (different streams without ordering) race and give wrong
 * results; calls on one stream, or otherwise ordered, are safe. Nothing in the array needs
 * clearing (every tile writes its whole record before the final sum reads it). */
VGICP_API vgicp_status vgicp_linearize_noalloc(vgicp_voxelmap map, const float* xyz,
                                               const float* cov, int64_t n,
                                               const double* T_target, const double* T_source,
                                               int32_t binary, vgicp_precision precision,
                                               double* H, double* b, double* err,
                                               int64_t* inliers, int32_t* corr,
                                               vgicp_stream stream);

/* Eq. (2) only: the cost err [1], inliers [1] and optional corr [n] (device outputs).
 * inliers / n is the overlap rate of Sec. III-D. */
VGICP_API vgicp_status vgicp_evaluate(vgicp_voxelmap map, const float* xyz, const float* cov,
                                      int64_t n, const double* T_target,
                                      const double* T_source, vgicp_precision precision,
                                      double* err, int64_t* inliers, int32_t* corr,
                                      vgicp_stream stream);

/* Exact gradient of Eq. (2) with the correspondences `corr` (device [n], from
 * vgicp_evaluate or vgicp_linearize at the same poses) held fixed and the inverse fused
 * covariance NOT held fixed. With w_k = R^T Omega_k d_k (R = rotation of T_ts):
 *   de/domega_s = sum 2 w_k x (mu_k + C_k w_k),  de/drho_s = -2 sum w_k,  de/dmu_k = -2 w_k,
 *   de/dxi_t = -Ad(T_st)^T de/dxi_s  (Ad(R, t) = [[R, 0], [[t]x R, R]], T_st = T_ts^-1).
 * grad_err: device [1], the upstream gradient g; outputs are scaled by it. grad_xi: device
 * [6] (unary) or [12] (binary, [source | target]). grad_xyz: device [3][n] or NULL.
 * precision: VGICP_ACC_FP64 or VGICP_MATH_FP64 (others: E_INVALID_ARG). */
VGICP_API vgicp_status vgicp_backward(vgicp_voxelmap map, const float* xyz, const float* cov,
                                      int64_t n, const double* T_target,
                                      const double* T_source, int32_t binary,
                                      const int32_t* corr, const double* grad_err,
                                      vgicp_precision precision, double* grad_xi,
                                      float* grad_xyz, vgicp_stream stream);

/* vgicp_backward at the poses T_source Exp(xi_source) and T_target Exp(xi_target) (right
 * perturbation, xi = [omega; rho]), returning the gradient in those tangent coordinates:
 * grad_xi = J_r(xi)^T g, with g the right-perturbation gradient of vgicp_backward at the moved
 * poses and J_r the right Jacobian of SE(3) (vgicp_se3_right_jacobian). This is the gradient of
 * the cost with respect to the tangent vectors themselves (the torch.autograd.Function passes
 * its xi tensors here). xi_source, xi_target: HOST arrays of 6 doubles, NULL = zero (xi_target
 * is ignored for a unary factor); |xi| must be below 3 (E_INVALID_ARG), non-finite values give
 * E_NONFINITE. corr must come from vgicp_evaluate / vgicp_linearize at the moved poses. Other
 * arguments, outputs and errors as vgicp_backward; the point gradients are unchanged by the
 * tangent map. */
VGICP_API vgicp_status vgicp_backward_tangent(vgicp_voxelmap map, const float* xyz,
                                              const float* cov, int64_t n,
                                              const double* T_target, const double* T_source,
                                              const double* xi_target, const double* xi_source,
                                              int32_t binary, const int32_t* corr,
                                              const double* grad_err,
                                              vgicp_precision precision, double* grad_xi,
                                              float* grad_xyz, vgicp_stream stream);

/* ---------------------------------------------------------------------------- batches */

/* Prepares a batch of factors (Sec. III-F: one factor per submap pair, re-linearized in
 * every iteration). maps [n_maps], clouds [n_clouds], factors [n_factors] are HOST arrays
 * copied during the call; the maps and the cloud memory they name must outlive the batch.
 * n_poses is the length of the pose array later passed to vgicp_batch_linearize. The batch
 * splits every factor's source into tiles and orders the work so that factors sharing a
 * target run together on one XCD (its L2 keeps the target's voxel table). At creation the
 * batch copies every source cloud (36 bytes per point) in a spatial order - the Morton order of
 * its cells at the finest resolution of the maps it is matched against - with interleaved
 * covariances: neighbouring points then read neighbouring bricks and voxel records, and an
 * inlier touches one 24-byte record instead of six planes. The per-factor results are the
 * same sums in another order (deterministic). Call vgicp_batch_refresh after changing the
 * clouds' points or covariances. Synchronises the null stream.
 * Calls on one batch share its scratch (relative poses, work queues, partial sums, the LM
 * system) and are ordered: each call's stream first waits for the batch's previous call (an
 * event recorded at the end of every call), so calls issued on different streams run one after
 * another instead of racing. */
VGICP_API vgicp_status vgicp_batch_create(const vgicp_voxelmap* maps, int32_t n_maps,
                                          const vgicp_cloud* clouds, int32_t n_clouds,
                                          const vgicp_factor* factors, int32_t n_factors,
                                          int32_t n_poses, vgicp_batch* out);

/* Re-copies the clouds (positions and covariances, spatially ordered) into the batch, for
 * callers that changed them since vgicp_batch_create. Synchronises `stream`. */
VGICP_API vgicp_status vgicp_batch_refresh(vgicp_batch batch, vgicp_stream stream);

/* Sets the batch's launch schedule (host struct). E_INVALID_ARG if unsupported. */
VGICP_API vgicp_status vgicp_batch_set_schedule(vgicp_batch batch,
                                                const vgicp_schedule* schedule);

/* Current schedule of the batch (host output). */
VGICP_API vgicp_status vgicp_batch_get_schedule(vgicp_batch batch, vgicp_schedule* schedule);

/* Times the candidate schedules (block {256, 512} x points per thread {8, 16, 32} x blocks
 * per CU {1, 2, 3, 4, 8} x lookahead {2, 4, 8}) on this batch at `poses` (device
 * [n_poses][12]) with HIP events: every candidate by the median of 3 launches, the six fastest
 * again by the median of 31; keeps the fastest. The result is also returned in *chosen (may be
 * NULL). If
 * cache_path is not NULL the choice is looked up in / stored to that JSON file, keyed by
 * device, precision and batch shape. Synchronises `stream`. */
VGICP_API vgicp_status vgicp_batch_autotune(vgicp_batch batch, const double* poses,
                                            vgicp_precision precision, const char* cache_path,
                                            vgicp_schedule* chosen, vgicp_stream stream);

/* Linearizes every factor of the batch in one persistent launch, replayed from a captured
 * HIP graph (captured on first use for each (precision, pointer set, schedule); a batch keeps
 * the 16 most recent, and synchronises the device when it drops one). poses:
 * device [n_poses][12]; the graph reads them at replay, so updating the pose buffer between
 * iterations needs no new capture. Outputs (device): H [F][144], b [F][12], err [F],
 * inliers [F]. Bitwise deterministic. */
VGICP_API vgicp_status vgicp_batch_linearize(vgicp_batch batch, const double* poses,
                                             vgicp_precision precision, double* H, double* b,
                                             double* err, int64_t* inliers,
                                             vgicp_stream stream);

/* Cost and inliers of every factor (device outputs err [F], inliers [F]). */
VGICP_API vgicp_status vgicp_batch_evaluate(vgicp_batch batch, const double* poses,
                                            vgicp_precision precision, double* err,
                                            int64_t* inliers, vgicp_stream stream);

/* Overlap rates (Sec. III-D and III-F: the fraction of a source submap's points that fall in a
 * voxel of the target's map; keyframes and global factors are created above a threshold). For
 * every factor of the batch at `poses` (device [n_poses][12]): rates [F] FP64 = inliers / n
 * (0 for an empty source) and inliers [F] int64, both device. Keys as in every other form (FP64,
 * bit-exact); no covariance, inverse or residual work, so it runs at the lookup phase's speed.
 * The unary/binary flag of a factor is ignored. Asynchronous on `stream`. */
VGICP_API vgicp_status vgicp_batch_overlap(vgicp_batch batch, const double* poses,
                                           double* rates, int64_t* inliers,
                                           vgicp_stream stream);

/* Backward of the batch (the differentiation form of Eq. (2) over a factor list): at `poses`
 * (device [P][12]) the gradient of L = sum_f grad_err[f] e_f with every factor's
 * correspondences held at those the forward pass finds at the same poses (recomputed: keys are
 * exact, so they are the same) and the inverse fused covariances NOT held, as vgicp_backward.
 * grad_err: device [F]. Outputs (device): grad_poses [P][6], the right-perturbation gradient
 * of every pose ([omega; rho]; a pose no factor reaches gets zeros; a unary factor gives its
 * target pose nothing), each the sum of its factors' contributions in factor order;
 * grad_factors [F][12] (may be NULL): per factor [source | target] (target half zero for a unary
 * factor); grad_points (may be NULL): a HOST array of n_clouds device pointers, entry c being
 * the caller's [3][n_c] FP32 array for cloud c in the cloud's own point order (NULL entries are
 * skipped; a cloud no factor reads gets zeros), each point's gradient summed over the factors
 * that read it in factor order. Deterministic. precision: VGICP_ACC_FP64 or VGICP_MATH_FP64.
 * The first call allocates the backward's buffers (12 bytes per factor source point). Calls on
 * a batch are ordered (see vgicp_batch_create); when the grad_points pointers differ from the
 * previous call's the host waits for the batch's previous call before uploading them. */
VGICP_API vgicp_status vgicp_batch_backward(vgicp_batch batch, const double* poses,
                                            vgicp_precision precision,
                                            const double* grad_err, double* grad_poses,
                                            double* grad_factors, float* const* grad_points,
                                            vgicp_stream stream);

/* One Levenberg-Marquardt step of the pose graph the batch's factors form (Sec. III-F: the
 * global mapping graph over submap poses is optimized with LM; each factor contributes its
 * Gauss-Newton blocks of Eq. (2)). At `poses` (device [P][12]) the call linearizes every factor
 * with `precision`, assembles the 6P x 6P system (6x6 blocks [omega; rho] per pose, summed in
 * factor order: deterministic), damps it as H + lambda diag(H), solves
 * (H + lambda diag H) delta = -b by an FP64 Cholesky factorization, and retracts every pose:
 * poses_new[i] = poses[i] Exp(delta_i) (right perturbation). A pose that no factor reaches, and
 * fixed_pose when >= 0 (the gauge), get delta = 0. Outputs (device): poses_new [P][12];
 * delta [P][6] (may be NULL); cost [2] = {sum of factor costs at poses, the same at poses_new,
 * both from linearizations with `precision`}. The caller accepts the step (and lowers lambda)
 * when cost[1] < cost[0]. Solver: at its first LM call the batch orders the poses to reduce the
 * bandwidth of the system (reverse Cuthill-McKee from several starts and a spectral order, the
 * narrowest kept); when the half-bandwidth w is at most 131 unknowns (21 poses) the banded
 * system is factored in LDS. When at least 16 poses lie outside a separator of (w + 1) / 6
 * consecutive poses in the order, it is eliminated from both ends at once (two workgroups: the
 * poses before the separator forward, the poses after it in reverse order), then the
 * separator's system (the sum of the two Schur complements) is solved and the two ends are
 * substituted back side by side; this needs 6 m + 18 (w + 1) <= 18,221 for the longer end's m
 * poses (separator included: up to 5,665 poses at w = 65, 5,258 at w = 131); otherwise one
 * workgroup solves it in one sweep if 6P + 18 (w + 1) <= 18,221. Other graphs use a dense
 * blocked factorization (288 P^2 bytes, P <= 5,460). Asynchronous on `stream`; the first call
 * allocates the step's buffers. Errors: E_INVALID_ARG, E_CAPACITY (dense system beyond 5,460 poses); a damped
 * system that is not positive definite sets the device error word (E_NONFINITE at the next
 * sync). */
VGICP_API vgicp_status vgicp_batch_lm_step(vgicp_batch batch, const double* poses,
                                           vgicp_precision precision, double lambda,
                                           int32_t fixed_pose, double* poses_new, double* delta,
                                           double* cost, vgicp_stream stream);

/* `iterations` Levenberg-Marquardt iterations with every decision on the device (no host
 * synchronisation): each iteration solves the damped system of the linearization at the current
 * poses, retracts, linearizes at the candidate poses, and takes the step when the candidate's
 * cost is finite and lower (poses <- candidate, the candidate's linearization becomes the
 * current one, lambda / 10), otherwise keeps the poses and multiplies lambda by 10 (lambda
 * stays within [1e-12, 1e12]). The linearization at the current poses is reused, so an
 * iteration costs one linearization and one solve. poses: device [P][12], updated in place;
 * lambda: device [1], in/out; cost: device [iterations + 1], the cost at the start and after
 * every iteration. Same solver, precision, gauge and errors as vgicp_batch_lm_step. */
VGICP_API vgicp_status vgicp_batch_lm_iterate(vgicp_batch batch, double* poses,
                                              vgicp_precision precision, double* lambda,
                                              int32_t fixed_pose, int32_t iterations,
                                              double* cost, vgicp_stream stream);

/* Solver of the batch's LM calls: 0 = automatic (banded when the ordered graph allows it, from
 * both ends when it is long enough; the default), 1 = dense, 2 = banded in one sweep when the
 * graph allows it and fits one sweep (else dense). Synchronises the device and drops the LM
 * buffers (rebuilt at the next LM call). */
VGICP_API vgicp_status vgicp_batch_lm_solver(vgicp_batch batch, int32_t solver);

/* Host outputs (either may be NULL): banded = 0 when the LM calls use the dense solver, 1 the
 * banded one in one sweep, 2 the banded one from both ends; and the half-bandwidth (in
 * unknowns) of the ordered system. Prepares the LM structure if needed. */
VGICP_API vgicp_status vgicp_batch_lm_info(vgicp_batch batch, int32_t* banded,
                                           int32_t* half_bandwidth);

/* Host only, no device call: the pose order that the LM calls use for the banded solve, for an
 * undirected graph of P poses with n_links links (links [n_links][2] of pose indices; repeated
 * links and self-links are ignored). pos (host [P], written) = position of every pose, a
 * permutation of 0 .. P - 1; bandwidth (host, may be NULL) = the largest position difference
 * of two linked poses. The order is the narrowest of the identity, reverse Cuthill-McKee from a
 * pseudo-peripheral pose (repeated breadth-first search) and from the four lowest-degree poses,
 * and the spectral order (poses sorted by the graph Laplacian's second eigenvector, by power
 * iteration); ties keep the earlier. The banded system's half-bandwidth is 6 bandwidth + 5
 * unknowns (Sec. III-F: LM over the global graph). Errors: E_INVALID_ARG (a negative count, a
 * NULL array with a nonzero count, a pose index out of range). */
VGICP_API vgicp_status vgicp_pose_order(int32_t P, const int32_t* links, int32_t n_links,
                                        int32_t* pos, int32_t* bandwidth);

/* Frees a batch (waits for the device). NULL is accepted. */
VGICP_API vgicp_status vgicp_batch_destroy(vgicp_batch batch);

/* One-shot form: create, linearize, destroy. Synchronises `stream` before returning. */
VGICP_API vgicp_status vgicp_linearize_batched(const vgicp_voxelmap* maps, int32_t n_maps,
                                               const vgicp_cloud* clouds, int32_t n_clouds,
                                               const double* poses, int32_t n_poses,
                                               const vgicp_factor* factors, int32_t n_factors,
                                               vgicp_precision precision, double* H, double* b,
                                               double* err, int64_t* inliers,
                                               vgicp_stream stream);

/* ---------------------------------------------------------------------------- utilities */

/* Synchronises `stream` and returns (and clears) the sticky device-side error of the
 * current device, or the HIP error of the synchronisation. */
VGICP_API vgicp_status vgicp_sync_status(vgicp_stream stream);

/* Message of the calling thread's last failed call ("" if none). Valid until the next call
 * on the same thread. */
VGICP_API const char* vgicp_last_error(void);

/* T_ts = T_target^-1 T_source in the fixed FP64 evaluation order the kernels use
 *   R_ts[r][c] = (Rt[0][r] Rs[0][c] + Rt[1][r] Rs[1][c]) + Rt[2][r] Rs[2][c],
 *   t_ts[r]    = (Rt[0][r] dt0 + Rt[1][r] dt1) + Rt[2][r] dt2,  dt = t_s - t_t,
 * without fused multiply-adds. Host arrays of 12 doubles. */
VGICP_API vgicp_status vgicp_relative_pose(const double* T_target, const double* T_source,
                                           double* T_ts);

/* Right perturbation out = T Exp(xi), xi = [omega; rho], host FP64 (12 / 6 / 12 doubles). */
VGICP_API vgicp_status vgicp_se3_retract(const double* T, const double* xi, double* out);

/* Right Jacobian of SE(3) at xi: Exp(xi + delta) = Exp(xi) Exp(J delta + O(|delta|^2)), as the
 * series sum_k (-ad_xi)^k / (k+1)! with ad_xi = [[omega^, 0], [rho^, omega^]]. J is a host
 * row-major 6x6. The gradient of a cost f(T Exp(xi)) with respect to xi is J^T g, g being
 * the right-perturbation gradient at T Exp(xi). |xi| must be below 3 (E_INVALID_ARG). */
VGICP_API vgicp_status vgicp_se3_right_jacobian(const double* xi, double* J);

/* Library version string. */
VGICP_API const char* vgicp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VGICP_H */
