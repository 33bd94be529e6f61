// Host-side internals shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/vgicp.h"
#include "common.h"

// The opaque voxel map handle of the C ABI.
struct vgicp_voxelmap_s {
  int device = 0;
  double res = 0.0;
  double inv_res = 0.0;
  int pow2 = 0;
  int64_t V = 0;
  int64_t cap = 0;
  int lo[3] = {0, 0, 0};
  int ext[3] = {0, 0, 0};
  int by = 0, bz = 0;
  bool key32 = true;
  int layout = vgicp::kLayoutHash32;  // the lookup structure the kernels use
  vgicp::Brick* bricks = nullptr;    // [nbricks] occupancy bricks, for the grid layout
  int64_t nbricks = 0;
  int gby = 0, gbz = 0;
  vgicp::VoxelData* voxb = nullptr;  // [V] records in brick order (grid layout)
  int* rec_id = nullptr;             // [V] voxel id of each brick-ordered record
  uint2* slots32 = nullptr;          // [cap] {relative key, id}, when key32
  longlong2* slots64 = nullptr;      // [cap] {packed key, id}, otherwise
  vgicp::VoxelData* vox = nullptr;   // [V] canonical order
  int64_t* keys = nullptr;           // [V] canonical order
  double* mean = nullptr;            // [3][V]
  double* cov = nullptr;             // [6][V]
  int32_t* count = nullptr;          // [V]

  vgicp::MapView view() const {
    vgicp::MapView m;
    const bool g = layout == vgicp::kLayoutGrid;
    m.bricks = g ? bricks : nullptr;
    m.brick_bytes = g ? (unsigned)(nbricks * (int64_t)sizeof(vgicp::Brick)) : 0u;
    m.rec = g ? voxb : vox;
    m.rec_id = g ? rec_id : nullptr;
    m.slots32 = layout == vgicp::kLayoutHash32 ? slots32 : nullptr;
    m.slots64 = layout == vgicp::kLayoutHash64 ? slots64 : nullptr;
    m.gby = gby;
    m.gbz = gbz;
    m.mask = (unsigned)(cap - 1);
    m.pow2 = pow2;
    m.res = res;
    m.inv_res = inv_res;
    for (int a = 0; a < 3; ++a) {
      m.lo[a] = lo[a];
      m.ext[a] = ext[a];
    }
    m.by = by;
    m.bz = bz;
    m.vox = vox;
    m.V = V;
    return m;
  }
};

namespace vgicp {

constexpr unsigned kFlagBadIndex = 8u;  // device flag: a neighbour index outside [-1, n)
constexpr int kMaxNeighbors = 32;       // k of the neighbour search

// Thread-local error reporting.
vgicp_status fail(vgicp_status st, const std::string& msg);
vgicp_status hip_fail(hipError_t e, const char* what);
void clear_error();

// Per-device sticky error word (device memory, lazily allocated).
unsigned* device_flags(int device);
vgicp_status flags_to_status(unsigned flags);
int device_cu_count(int device);
double* device_scratch(int device);

// Host FP64 relative pose in the kernels' fixed evaluation order, plus the FP32 forms.
void relative_pose(const double* Tt, const double* Ts, double* Tts);
RelPose make_rel_pose(const double* Tt, const double* Ts, double inv_res);

// Device buffers owned by one host call, freed (hipFree synchronises) when it returns.
struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  hipError_t alloc(T** p, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, (count > 0 ? count : 1) * sizeof(T));
    if (e == hipSuccess) ptrs.push_back(q);
    *p = static_cast<T*>(q);
    return e;
  }
};

// Device-wide primitives (voxelmap.hip), enqueued on s. Exclusive scan of n ints (in and out
// may alias). Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the keys,
// 8 bits per pass: the sorted pairs end in (*k, *v) - the pointers swap with the temporaries
// (*kt, *vt) as the passes go. A scatter outside [0, n) sets kFlagInternal in flags.
hipError_t scan_exclusive(const int* in, int* out, long long n, hipStream_t s, Scratch& sc);
hipError_t radix_sort_pairs(unsigned long long** k, int** v, unsigned long long** kt, int** vt,
                            long long n, int bits, unsigned* flags, hipStream_t s, Scratch& sc);

// Voxel map build (voxelmap.hip).
vgicp_status build_voxelmap(const float* xyz, const float* cov, int64_t n, double res,
                            int layout, hipStream_t s, vgicp_voxelmap* out);
void destroy_voxelmap(vgicp_voxelmap m);
// A cloud in the spatial order of the Morton codes of its cells of size `cell` (stable):
// positions [3][n] and interleaved covariances [n][6], and its bounding box (host, 6 floats:
// lo, hi; infinite when a coordinate is not finite, empty when n = 0) (voxelmap.hip).
// Synchronises s.
// perm_out (device [n], may be NULL) receives the permutation: spatial index -> original index.
vgicp_status spatial_copy(const float* xyz, const float* cov, int64_t n, double cell,
                          float* xyz_out, float* cov6_out, float* box, int* perm_out,
                          hipStream_t s);

// Preprocessing (preprocess.hip). downsample and knn synchronise s; the covariance kernel is
// enqueued only and reports a neighbour index outside [-1, n) through flags.
vgicp_status downsample(const float* xyz, const float* t, int64_t n, double res, double d_scan,
                        float* xyz_out, float* t_out, int64_t capacity, int64_t* n_out,
                        hipStream_t s);
vgicp_status knn(const float* xyz, int64_t n, int k, double cell, int32_t* nbr, hipStream_t s);
void launch_point_covariances(const float* xyz, int64_t n, const int32_t* nbr, int k,
                              double scale, double eps, float* cov, unsigned* flags,
                              hipStream_t s);

// IMU preintegration factor (imu.hip). Enqueue only; bad indices and non-positive intervals or
// covariances are reported through flags.
void launch_imu_preintegrate(const double* imu, int64_t m, const int64_t* seg, int F,
                             const double* bias,
                             double sigma_g, double sigma_a, double* pre, double* cov,
                             double* jac, unsigned* flags, hipStream_t s);
void launch_imu_linearize_bias(const double* pre, const double* cov, const double* jac,
                               const double* bias0, const int32_t* idx, int F,
                               const double* poses, const double* vel, const double* biases,
                               int P, const double g[3], double sigma_ba, double sigma_bw,
                               double* H, double* b, double* err, unsigned* flags,
                               hipStream_t s);
void launch_imu_linearize(const double* pre, const double* cov, const int32_t* idx, int F,
                          const double* poses, const double* vel, int P, const double g[3],
                          double* H, double* b, double* err, unsigned* flags, hipStream_t s);

// Single-factor kernels (kernels.hip). Enqueue only; partials must hold ntiles * stride doubles.
int plain_tile(int precision);
void launch_plain(const MapView& m, const RelPose& T, const float* xyz, const float* cov6,
                  int64_t n, int binary, int precision, bool linearize, double* partials,
                  int ntiles, int tile, int32_t* corr, unsigned* flags, double* H, double* b,
                  double* err, int64_t* inliers, hipStream_t s);
void launch_backward(const MapView& m, const RelPose& T, const TangentMap& J, const float* xyz,
                     const float* cov, int64_t n, int binary, int precision,
                     const int32_t* corr, const double* grad_err, double* partials, int ntiles,
                     int tile, double* grad_xi, float* grad_xyz, hipStream_t s);

// Batched kernels (kernels.hip).
struct BatchLaunch {
  const FactorView* factors;
  const float* boxes;        // [clouds][6] source bounding boxes (lo, hi), local frames
  RelPose* rel;              // [F], written by the prep kernel
  const double* poses;       // [P][12]
  const WorkItem* items;     // schedule order, per-XCD segments
  const int* seg;            // [kNumXcd + 1]
  unsigned long long* heads; // [kNumXcd] items taken: from the head (low 32 bits), from the tail (high)
  double* partials;          // [total tiles][kPartialStride], canonical order
  unsigned* flags;
  int F;
  int grid;
  int block;
  int tile;
  int lookahead;
  int precision;
  bool linearize;
  double* H;
  double* b;
  double* err;
  int64_t* inliers;
};
void launch_batched(const BatchLaunch& L, hipStream_t s);

// Batched backward (kernels.hip): the batch kernel in its gradient mode (the queue of inliers
// carries the gradient terms), then per factor, per pose and per source point sums.
struct BatchGrad {
  const double* grad_err;    // [F] upstream gradient of every factor's cost
  float* gpts;               // [sum of factor sizes][3] per factor and point (spatial order)
  double* gf;                // [F][12] per factor [source | target]
  double* grad_poses;        // [P][6]
  const int* bptr;           // [P + 1] contributions per pose ((factor << 1) | half)
  const int* bcontrib;
  int P;
  const int* cptr;           // [clouds + 1] factors reading each cloud as a source
  const int* cfac;           // factor indices, in factor order
  const long long* cloud_n;  // [clouds]
  const long long* cloud_off;// [clouds] first point of the cloud in the batch's copies
  const int* perm;           // [points] spatial index -> the caller's index, per cloud
  float* const* out;         // [clouds] the caller's [3][n] gradient arrays (NULL: skip)
  int n_clouds;
  long long max_n;
};
void launch_batched_backward(const BatchLaunch& L, const BatchGrad& G, hipStream_t s);

// Levenberg-Marquardt step of a batch's pose graph (lm.hip).
struct LmBlock {
  int row, col;     // pose indices of a nonzero 6x6 block
  int first, count; // its contributions in LmStructure::contrib
};
struct LmStructure {  // host: built once per batch, in factor order
  std::vector<LmBlock> blocks;
  std::vector<int> contrib;   // (factor << 2) | (a << 1) | b: 6x6 sub-block (a, b) of H_f
  std::vector<int> bptr;      // [P + 1]
  std::vector<int> bcontrib;  // (factor << 1) | half of b_f
  int n_real = 0, n = 0;      // 6P, padded to the Cholesky block
  std::vector<int> pos;       // [P] position of every pose in the bandwidth-reducing order
  int pose_bw = 0;            // largest position difference of two linked poses
  int w = 0;                  // half-bandwidth of the permuted system, 6 pose_bw + 5
  bool band = false;          // the banded solver applies (w and 6P within its limits)
  bool one_sweep = false;     // the banded system also fits one sweep on one workgroup
  // banded, from both ends: blocks 0 .. m_top - 1 (top end) and the last m_bot blocks (bottom
  // end, eliminated in reverse order) are eliminated side by side; the pose_bw + 1 blocks
  // between them (w + 1 unknowns) form the separator, which couples the two
  bool split = false;
  int m_top = 0, m_bot = 0;
};
struct LmDevice {  // device buffers of the LM step
  const LmBlock* blocks;
  int nblocks;
  const int* contrib;
  const int* bptr;
  const int* bcontrib;
  const double* Hf;  // [F][144] linearization at the current poses
  const double* bf;  // [F][12]
  double* A;         // [n][n]
  double* diag_raw;  // [n]
  double* x;         // [n + 64] right-hand side, then the step (64 spare values)
  double* Dinv;      // dense: [n][64] inverses of the diagonal blocks (the banded solver has none)
  int n, n_real;
  const double* lambda;  // [1] damping (device)
  int band;              // 1: banded solve (Ab, pos, w), 0: dense (A)
  double* Ab;            // [6P + 6][w + 1] (+ 64) band rows of the permuted system, then of its factor; spare rows
  const int* pos;        // [P]
  int w;
  // split banded solve (LmStructure::split): top end in Ab and x (rows 0 .. 6 m_top + w), the
  // bottom end in reverse order in Ab_bot [6 m_bot + w + 7][w + 1] (+ 64) and x_bot
  // [6 m_bot + w + 1 + 64], the separator's system in Ab_sep [w + 7][w + 1] (+ 64) and x_sep
  // [w + 1 + 64]
  int split, m_top, m_bot;
  double *Ab_bot, *Ab_sep, *x_bot, *x_sep;
};
void build_lm_structure(const std::vector<FactorView>& hf, int P, LmStructure& s);
// A bandwidth-reducing order of the poses of an undirected graph (adj: the neighbours of every
// pose, no self-links): pos[p] = position of pose p, bw = largest position difference of two
// linked poses. Host only.
void order_poses(const std::vector<std::vector<int>>& adj, std::vector<int>& pos, int& bw);
// Solves the damped system of the linearization (Hf, bf) and writes the retracted poses. x holds
// the solution in the solver's order.
void launch_lm_solve(const LmDevice& d, int P, int fixed, const double* poses, double* poses_new,
                     double* delta, unsigned* flags, hipStream_t s);
void launch_lm_cost(const double* e0, const double* e1, int F, double* cost, hipStream_t s);
void launch_lm_set(double* p, double v, hipStream_t s);
void launch_lm_decide(const double* e_cur, const double* e_cand, int F, double* lambda,
                      int* accept, double* cost_first, double* cost_out, hipStream_t s);
void launch_lm_commit(const int* accept, int P, int F, const double* cand, double* poses,
                      const double* Hc, const double* bc, const double* ec, double* H, double* b,
                      double* e, hipStream_t s);

}  // namespace vgicp
