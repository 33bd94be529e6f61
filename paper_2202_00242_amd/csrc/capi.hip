// C ABI of the VGICP library: argument validation, error reporting, single-factor calls,
// batches (persistent kernel replayed from a captured HIP graph) and the schedule autotuner.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "device_math.h"
#include "internal.h"

namespace vgicp {

// Per-device static memory of the library (zero at load, held until the process ends; every
// device the library runs on has its own copy at its own address, taken once per device with
// hipGetSymbolAddress - in host code the names below are not device addresses):
//   error_word - the sticky device-side error flags (kFlag*), set by kernels with atomicOr;
//   scratch    - per-tile partial sums of vgicp_linearize_noalloc, at most kNoAllocMaxTiles
//                tiles of kPartialStride doubles (950,272 bytes). Each tile writes its whole
//                record before the finalize reads it, so nothing needs clearing between calls.
static __device__ unsigned error_word;
static __device__ __align__(256) double scratch[(size_t)kNoAllocMaxTiles * kPartialStride];

namespace {
thread_local std::string g_last_error;
std::mutex g_dev_mutex;
struct DevState {
  unsigned* flags = nullptr;
  double* scratch = nullptr;
  int cus = 0;
  std::string arch;
};
std::map<int, DevState> g_dev;

DevState* dev_state(int device) {
  std::lock_guard<std::mutex> lk(g_dev_mutex);
  DevState& d = g_dev[device];
  if (!d.flags) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != device) (void)hipSetDevice(device);
    void* p = nullptr;
    void* q = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(error_word)) == hipSuccess &&
        hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) == hipSuccess) {
      d.flags = static_cast<unsigned*>(p);
      d.scratch = static_cast<double*>(q);
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
      d.cus = prop.multiProcessorCount;
      d.arch = prop.gcnArchName;
    }
    if (cur != device) (void)hipSetDevice(cur);
  }
  return d.flags ? &d : nullptr;
}
}  // namespace

vgicp_status fail(vgicp_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

vgicp_status hip_fail(hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return fail(VGICP_E_OOM, m);
  return fail(VGICP_E_HIP, m);
}

void clear_error() { g_last_error.clear(); }

unsigned* device_flags(int device) {
  DevState* d = dev_state(device);
  return d ? d->flags : nullptr;
}

double* device_scratch(int device) {
  DevState* d = dev_state(device);
  return d ? d->scratch : nullptr;
}

int device_cu_count(int device) {
  DevState* d = dev_state(device);
  return d && d->cus > 0 ? d->cus : 256;
}

vgicp_status flags_to_status(unsigned f) {
  if (f & kFlagNonFinite)
    return fail(VGICP_E_NONFINITE,
                "non-finite transformed point or fused covariance not positive definite");
  if (f & kFlagKeyRange) return fail(VGICP_E_KEY_RANGE, "voxel coordinate out of range");
  if (f & kFlagBadIndex)
    return fail(VGICP_E_INVALID_ARG, "index out of range (neighbour list, IMU segment or state)");
  return VGICP_OK;
}

}  // namespace vgicp

using namespace vgicp;

namespace {

bool finite12(const double* T) {
  for (int i = 0; i < 12; ++i)
    if (!std::isfinite(T[i])) return false;
  return true;
}

hipStream_t stream_of(vgicp_stream s) { return reinterpret_cast<hipStream_t>(s); }

bool valid_precision(int p) { return p >= 0 && p <= 3; }

// Tile of the single-factor kernels: about two blocks per CU for mid-size clouds.
int plain_tile_for(int64_t n, int cus) {
  const int64_t want = (n + 2LL * cus - 1) / (2LL * cus);
  int64_t t = ((want + 255) / 256) * 256;
  return (int)std::min<int64_t>(std::max<int64_t>(t, 256), kMaxPointsPerLane * 256);
}

vgicp_status check_map(vgicp_voxelmap map) {
  if (!map) return fail(VGICP_E_INVALID_ARG, "voxel map is NULL");
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || cur != map->device)
    return fail(VGICP_E_INVALID_ARG, "voxel map lives on another device than the current one");
  return VGICP_OK;
}

vgicp_status check_cloud(const float* xyz, const float* cov, int64_t n) {
  if (n < 0) return fail(VGICP_E_INVALID_ARG, "negative point count");
  if (n > 0 && (!xyz || !cov)) return fail(VGICP_E_INVALID_ARG, "cloud pointer is NULL");
  if (n >= kMaxCloudPoints) return fail(VGICP_E_CAPACITY, "cloud of 2^30 points or more");
  return VGICP_OK;
}

}  // namespace

// Right Jacobian of SE(3) at xi (row-major 6x6); false when |xi| >= 3.
static bool right_jacobian(const double* xi, double* J) {
  double nrm = 0.0;
  for (int i = 0; i < 6; ++i) nrm += xi[i] * xi[i];
  if (!(std::sqrt(nrm) < 3.0)) return false;
  // ad_xi = [[w^, 0], [rho^, w^]]
  double ad[36] = {0};
  const double* w = xi;
  const double* r = xi + 3;
  const double W[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
  const double P[9] = {0, -r[2], r[1], r[2], 0, -r[0], -r[1], r[0], 0};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      ad[6 * a + b] = W[3 * a + b];
      ad[6 * (a + 3) + b + 3] = W[3 * a + b];
      ad[6 * (a + 3) + b] = P[3 * a + b];
    }
  double term[36] = {0}, out[36] = {0};
  for (int i = 0; i < 6; ++i) term[7 * i] = 1.0;  // (-ad)^0 / 1!
  for (int i = 0; i < 36; ++i) out[i] = term[i];
  for (int k = 1; k < 60; ++k) {
    double nt[36];
    double mx = 0.0;
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b) {
        double s = 0.0;
        for (int c = 0; c < 6; ++c) s += term[6 * a + c] * (-ad[6 * c + b]);
        nt[6 * a + b] = s / (double)(k + 1);
        mx = std::max(mx, std::fabs(nt[6 * a + b]));
      }
    for (int i = 0; i < 36; ++i) {
      term[i] = nt[i];
      out[i] += nt[i];
    }
    if (mx < 1e-18) break;
  }
  std::memcpy(J, out, sizeof(out));
  return true;
}

extern "C" {

VGICP_API const char* vgicp_version(void) { return "vgicp-gfx950 1.0"; }

VGICP_API const char* vgicp_last_error(void) { return g_last_error.c_str(); }

VGICP_API vgicp_status vgicp_relative_pose(const double* T_target, const double* T_source,
                                           double* T_ts) {
  if (!T_target || !T_source || !T_ts) return fail(VGICP_E_INVALID_ARG, "NULL pose");
  relative_pose(T_target, T_source, T_ts);
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_se3_retract(const double* T, const double* xi, double* out) {
  if (!T || !xi || !out) return fail(VGICP_E_INVALID_ARG, "NULL argument");
  double o[12];
  se3_retract(T, xi, o);
  std::memcpy(out, o, sizeof(o));
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_se3_right_jacobian(const double* xi, double* J) {
  if (!xi || !J) return fail(VGICP_E_INVALID_ARG, "NULL argument");
  if (!right_jacobian(xi, J)) return fail(VGICP_E_INVALID_ARG, "|xi| must be below 3");
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_sync_status(vgicp_stream stream) {
  hipError_t e = hipStreamSynchronize(stream_of(stream));
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
  unsigned* f = device_flags(dev);
  if (!f) return fail(VGICP_E_HIP, "device error word address");
  unsigned h = 0;
  if ((e = hipMemcpy(&h, f, sizeof(h), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "read device error word");
  if (h) {
    if ((e = hipMemset(f, 0, sizeof(unsigned))) != hipSuccess)
      return hip_fail(e, "clear device error word");
    return flags_to_status(h);
  }
  return VGICP_OK;
}

// ------------------------------------------------------------------------ preprocessing

VGICP_API vgicp_status vgicp_downsample(const float* xyz, const float* t, int64_t n,
                                        double resolution, double scan_duration, float* xyz_out,
                                        float* t_out, int64_t capacity, int64_t* n_out,
                                        vgicp_stream stream) {
  if (!n_out) return fail(VGICP_E_INVALID_ARG, "n_out is NULL");
  *n_out = 0;
  if (n < 0 || capacity < 0) return fail(VGICP_E_INVALID_ARG, "negative size");
  if (n > 0 && !xyz) return fail(VGICP_E_INVALID_ARG, "cloud pointer is NULL");
  if (capacity > 0 && !xyz_out) return fail(VGICP_E_INVALID_ARG, "output pointer is NULL");
  if (n >= kMaxCloudPoints) return fail(VGICP_E_CAPACITY, "cloud of 2^30 points or more");
  if (!(resolution > 0.0) || !std::isfinite(resolution))
    return fail(VGICP_E_INVALID_ARG, "resolution must be positive and finite");
  if (t && (!(scan_duration > 0.0) || !std::isfinite(scan_duration)))
    return fail(VGICP_E_INVALID_ARG, "timestamps need a positive, finite scan duration");
  return downsample(xyz, t, n, resolution, scan_duration, xyz_out, t ? t_out : nullptr,
                    capacity, n_out, stream_of(stream));
}

VGICP_API vgicp_status vgicp_knn(const float* xyz, int64_t n, int32_t k, double cell,
                                 int32_t* neighbors, vgicp_stream stream) {
  if (n < 0) return fail(VGICP_E_INVALID_ARG, "negative point count");
  if (n > 0 && (!xyz || !neighbors)) return fail(VGICP_E_INVALID_ARG, "pointer is NULL");
  if (k < 1 || k > kMaxNeighbors) return fail(VGICP_E_INVALID_ARG, "k must be in [1, 32]");
  if (!(cell >= 0.0) || !std::isfinite(cell))
    return fail(VGICP_E_INVALID_ARG, "cell must be 0 (automatic) or positive and finite");
  if (n >= kMaxCloudPoints) return fail(VGICP_E_CAPACITY, "cloud of 2^30 points or more");
  return knn(xyz, n, k, cell, neighbors, stream_of(stream));
}

VGICP_API vgicp_status vgicp_point_covariances(const float* xyz, int64_t n,
                                               const int32_t* neighbors, int32_t k,
                                               double scale, double eps, float* cov,
                                               vgicp_stream stream) {
  if (n < 0) return fail(VGICP_E_INVALID_ARG, "negative point count");
  if (n > 0 && (!xyz || !neighbors || !cov)) return fail(VGICP_E_INVALID_ARG, "pointer is NULL");
  if (k < 1 || k > kMaxNeighbors) return fail(VGICP_E_INVALID_ARG, "k must be in [1, 32]");
  if (!(scale >= 0.0) || !std::isfinite(scale) || !(eps >= 0.0) || !std::isfinite(eps))
    return fail(VGICP_E_INVALID_ARG, "scale and eps must be finite and non-negative");
  if (n >= kMaxCloudPoints) return fail(VGICP_E_CAPACITY, "cloud of 2^30 points or more");
  if (n == 0) return VGICP_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  unsigned* flags = device_flags(dev);
  if (!flags) return fail(VGICP_E_HIP, "device error word address");
  launch_point_covariances(xyz, n, neighbors, k, scale, eps, cov, flags, stream_of(stream));
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "point covariance launch");
  return VGICP_OK;
}

// ------------------------------------------------------------------------ IMU factor

static vgicp_status imu_preintegrate(const double* imu, int64_t n_samples, const int64_t* seg,
                                     int32_t n_factors, const double* bias, double gyro_sigma,
                                     double acc_sigma, double* preint, double* cov,
                                     double* bias_jac, vgicp_stream stream) {
  if (n_factors < 0 || n_samples < 0) return fail(VGICP_E_INVALID_ARG, "negative count");
  if (n_factors > 0 && ((n_samples > 0 && !imu) || !seg || !bias || !preint || !cov))
    return fail(VGICP_E_INVALID_ARG, "pointer is NULL");
  if (!(gyro_sigma > 0.0) || !(acc_sigma > 0.0) || !std::isfinite(gyro_sigma) ||
      !std::isfinite(acc_sigma))
    return fail(VGICP_E_INVALID_ARG, "noise densities must be positive and finite");
  if (n_factors == 0) return VGICP_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  unsigned* flags = device_flags(dev);
  if (!flags) return fail(VGICP_E_HIP, "device error word address");
  launch_imu_preintegrate(imu, n_samples, seg, n_factors, bias, gyro_sigma, acc_sigma, preint,
                          cov, bias_jac, flags, stream_of(stream));
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "imu preintegration launch");
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_imu_preintegrate(const double* imu, int64_t n_samples,
                                              const int64_t* seg, int32_t n_factors,
                                              const double* bias,
                                              double gyro_sigma, double acc_sigma,
                                              double* preint, double* cov, vgicp_stream stream) {
  return imu_preintegrate(imu, n_samples, seg, n_factors, bias, gyro_sigma, acc_sigma, preint,
                          cov, nullptr, stream);
}

VGICP_API vgicp_status vgicp_imu_preintegrate_bias(const double* imu, int64_t n_samples,
                                                   const int64_t* seg, int32_t n_factors,
                                                   const double* bias, double gyro_sigma,
                                                   double acc_sigma, double* preint,
                                                   double* cov, double* bias_jac,
                                                   vgicp_stream stream) {
  if (n_factors > 0 && !bias_jac) return fail(VGICP_E_INVALID_ARG, "bias_jac is NULL");
  return imu_preintegrate(imu, n_samples, seg, n_factors, bias, gyro_sigma, acc_sigma, preint,
                          cov, bias_jac, stream);
}

VGICP_API vgicp_status vgicp_imu_linearize_bias(
    const double* preint, const double* cov, const double* bias_jac, const double* preint_bias,
    const int32_t* states, int32_t n_factors, const double* poses, const double* velocities,
    const double* biases, int32_t n_states, const double* gravity, double bias_walk_acc,
    double bias_walk_gyro, double* H, double* b, double* err, vgicp_stream stream) {
  if (n_factors < 0 || n_states < 0) return fail(VGICP_E_INVALID_ARG, "negative count");
  if (!gravity) return fail(VGICP_E_INVALID_ARG, "gravity is NULL");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(gravity[a])) return fail(VGICP_E_INVALID_ARG, "gravity is not finite");
  if (!(bias_walk_acc > 0.0) || !(bias_walk_gyro > 0.0) || !std::isfinite(bias_walk_acc) ||
      !std::isfinite(bias_walk_gyro))
    return fail(VGICP_E_INVALID_ARG, "bias random-walk densities must be positive and finite");
  if (n_factors > 0 && (!preint || !cov || !bias_jac || !preint_bias || !states || !poses ||
                        !velocities || !biases || !H || !b || !err))
    return fail(VGICP_E_INVALID_ARG, "pointer is NULL");
  if (n_factors == 0) return VGICP_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  unsigned* flags = device_flags(dev);
  if (!flags) return fail(VGICP_E_HIP, "device error word address");
  launch_imu_linearize_bias(preint, cov, bias_jac, preint_bias, states, n_factors, poses,
                            velocities, biases, n_states, gravity, bias_walk_acc,
                            bias_walk_gyro, H, b, err, flags, stream_of(stream));
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "imu linearization launch");
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_imu_linearize(const double* preint, const double* cov,
                                           const int32_t* states, int32_t n_factors,
                                           const double* poses, const double* velocities,
                                           int32_t n_states, const double* gravity, double* H,
                                           double* b, double* err, vgicp_stream stream) {
  if (n_factors < 0 || n_states < 0) return fail(VGICP_E_INVALID_ARG, "negative count");
  if (!gravity) return fail(VGICP_E_INVALID_ARG, "gravity is NULL");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(gravity[a])) return fail(VGICP_E_INVALID_ARG, "gravity is not finite");
  if (n_factors > 0 && (!preint || !cov || !states || !poses || !velocities || !H || !b || !err))
    return fail(VGICP_E_INVALID_ARG, "pointer is NULL");
  if (n_factors == 0) return VGICP_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  unsigned* flags = device_flags(dev);
  if (!flags) return fail(VGICP_E_HIP, "device error word address");
  launch_imu_linearize(preint, cov, states, n_factors, poses, velocities, n_states, gravity, H, b,
                       err, flags, stream_of(stream));
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "imu linearization launch");
  return VGICP_OK;
}

// ------------------------------------------------------------------------ voxel maps

VGICP_API vgicp_status vgicp_build_voxelmap(const float* xyz, const float* cov, int64_t n,
                                            double resolution, vgicp_stream stream,
                                            vgicp_voxelmap* out) {
  if (!out) return fail(VGICP_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  vgicp_status st = check_cloud(xyz, cov, n);
  if (st != VGICP_OK) return st;
  if (!(resolution > 0.0) || !std::isfinite(resolution))
    return fail(VGICP_E_INVALID_ARG, "resolution must be positive and finite");
  return build_voxelmap(xyz, cov, n, resolution, VGICP_LAYOUT_AUTO, stream_of(stream), out);
}

VGICP_API vgicp_status vgicp_build_voxelmap_layout(const float* xyz, const float* cov,
                                                   int64_t n, double resolution,
                                                   int32_t layout, vgicp_stream stream,
                                                   vgicp_voxelmap* out) {
  if (!out) return fail(VGICP_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (layout != VGICP_LAYOUT_AUTO && layout != VGICP_LAYOUT_HASH && layout != VGICP_LAYOUT_GRID)
    return fail(VGICP_E_INVALID_ARG, "unknown voxel map layout");
  vgicp_status st = check_cloud(xyz, cov, n);
  if (st != VGICP_OK) return st;
  if (!(resolution > 0.0) || !std::isfinite(resolution))
    return fail(VGICP_E_INVALID_ARG, "resolution must be positive and finite");
  return build_voxelmap(xyz, cov, n, resolution, layout, stream_of(stream), out);
}

VGICP_API vgicp_status vgicp_voxelmap_size(vgicp_voxelmap map, int64_t* num_voxels,
                                           int64_t* capacity) {
  if (!map) return fail(VGICP_E_INVALID_ARG, "voxel map is NULL");
  if (num_voxels) *num_voxels = map->V;
  if (capacity) *capacity = map->layout == kLayoutGrid ? map->nbricks : map->cap;
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_voxelmap_layout(vgicp_voxelmap map, int32_t* layout) {
  if (!map) return fail(VGICP_E_INVALID_ARG, "voxel map is NULL");
  if (!layout) return fail(VGICP_E_INVALID_ARG, "layout is NULL");
  *layout = map->layout == kLayoutGrid ? VGICP_LAYOUT_GRID : VGICP_LAYOUT_HASH;
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_voxelmap_export(vgicp_voxelmap map, int64_t* keys, double* mean,
                                             double* cov, int32_t* count, vgicp_stream stream) {
  vgicp_status st = check_map(map);
  if (st != VGICP_OK) return st;
  const size_t V = (size_t)map->V;
  hipStream_t s = stream_of(stream);
  hipError_t e = hipSuccess;
  if (V == 0) return VGICP_OK;
  if (keys && (e = hipMemcpyAsync(keys, map->keys, V * 8, hipMemcpyDeviceToDevice, s)))
    return hip_fail(e, "export keys");
  if (mean && (e = hipMemcpyAsync(mean, map->mean, 3 * V * 8, hipMemcpyDeviceToDevice, s)))
    return hip_fail(e, "export means");
  if (cov && (e = hipMemcpyAsync(cov, map->cov, 6 * V * 8, hipMemcpyDeviceToDevice, s)))
    return hip_fail(e, "export covariances");
  if (count && (e = hipMemcpyAsync(count, map->count, V * 4, hipMemcpyDeviceToDevice, s)))
    return hip_fail(e, "export counts");
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_destroy_voxelmap(vgicp_voxelmap map) {
  destroy_voxelmap(map);
  return VGICP_OK;
}

// ------------------------------------------------------------------------ one factor

static vgicp_status single_factor(vgicp_voxelmap map, const float* xyz, const float* cov,
                                  int64_t n, const double* T_target, const double* T_source,
                                  int32_t binary, int precision, bool linearize, double* H,
                                  double* b, double* err, int64_t* inliers, int32_t* corr,
                                  vgicp_stream stream, bool noalloc = false) {
  vgicp_status st = check_map(map);
  if (st != VGICP_OK) return st;
  if ((st = check_cloud(xyz, cov, n)) != VGICP_OK) return st;
  if (!T_target || !T_source) return fail(VGICP_E_INVALID_ARG, "NULL pose");
  if (!finite12(T_target) || !finite12(T_source)) return fail(VGICP_E_NONFINITE, "non-finite pose");
  if (binary != 0 && binary != 1) return fail(VGICP_E_INVALID_ARG, "binary must be 0 or 1");
  if (!valid_precision(precision)) return fail(VGICP_E_INVALID_ARG, "unknown precision");
  if (!err || !inliers || (linearize && (!H || !b)))
    return fail(VGICP_E_INVALID_ARG, "NULL output");
  unsigned* flags = device_flags(map->device);
  if (!flags) return fail(VGICP_E_HIP, "device error word address");
  hipStream_t s = stream_of(stream);
  const RelPose T = make_rel_pose(T_target, T_source, map->inv_res);
  const int tile = plain_tile_for(n, device_cu_count(map->device));
  const int ntiles = (int)((n + tile - 1) / tile);
  double* partials = nullptr;
  hipError_t e;
  if (noalloc) {
    if (ntiles > kNoAllocMaxTiles)
      return fail(VGICP_E_CAPACITY, "vgicp_linearize_noalloc: " + std::to_string(n) +
                                        " points need " + std::to_string(ntiles) +
                                        " tiles, the static scratch holds " +
                                        std::to_string(kNoAllocMaxTiles));
    if (!(partials = device_scratch(map->device)))
      return fail(VGICP_E_HIP, "static scratch address");
  } else if ((e = hipMallocAsync(reinterpret_cast<void**>(&partials),
                                 (size_t)std::max(ntiles, 1) * kPartialStride * sizeof(double),
                                 s)) != hipSuccess) {
    return hip_fail(e, "hipMallocAsync (partials)");
  }
  launch_plain(map->view(), T, xyz, cov, n, binary, precision, linearize, partials, ntiles, tile,
               corr, flags, H, b, err, inliers, s);
  e = hipGetLastError();
  if (!noalloc) (void)hipFreeAsync(partials, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_linearize(vgicp_voxelmap map, const float* xyz, const float* cov,
                                       int64_t n, const double* T_target,
                                       const double* T_source, int32_t binary,
                                       vgicp_precision precision, double* H, double* b,
                                       double* err, int64_t* inliers, int32_t* corr,
                                       vgicp_stream stream) {
  return single_factor(map, xyz, cov, n, T_target, T_source, binary, (int)precision, true, H, b,
                       err, inliers, corr, stream);
}

VGICP_API vgicp_status vgicp_linearize_noalloc(vgicp_voxelmap map, const float* xyz,
                                               const float* cov, int64_t n,
                                               const double* T_target, const double* T_source,
                                               int32_t binary, vgicp_precision precision,
                                               double* H, double* b, double* err,
                                               int64_t* inliers, int32_t* corr,
                                               vgicp_stream stream) {
  return single_factor(map, xyz, cov, n, T_target, T_source, binary, (int)precision, true, H, b,
                       err, inliers, corr, stream, true);
}

VGICP_API vgicp_status vgicp_evaluate(vgicp_voxelmap map, const float* xyz, const float* cov,
                                      int64_t n, const double* T_target,
                                      const double* T_source, vgicp_precision precision,
                                      double* err, int64_t* inliers, int32_t* corr,
                                      vgicp_stream stream) {
  return single_factor(map, xyz, cov, n, T_target, T_source, 0, (int)precision, false, nullptr,
                       nullptr, err, inliers, corr, stream);
}

static vgicp_status backward_impl(vgicp_voxelmap map, const float* xyz, const float* cov,
                                  int64_t n, const double* T_target, const double* T_source,
                                  const double* xi_target, const double* xi_source,
                                  int32_t binary, const int32_t* corr, const double* grad_err,
                                  int precision, double* grad_xi, float* grad_xyz,
                                  vgicp_stream stream) {
  vgicp_status st = check_map(map);
  if (st != VGICP_OK) return st;
  if ((st = check_cloud(xyz, cov, n)) != VGICP_OK) return st;
  if (!T_target || !T_source) return fail(VGICP_E_INVALID_ARG, "NULL pose");
  if (!finite12(T_target) || !finite12(T_source)) return fail(VGICP_E_NONFINITE, "non-finite pose");
  if (binary != 0 && binary != 1) return fail(VGICP_E_INVALID_ARG, "binary must be 0 or 1");
  if (precision != VGICP_ACC_FP64 && precision != VGICP_MATH_FP64)
    return fail(VGICP_E_INVALID_ARG, "backward supports VGICP_ACC_FP64 and VGICP_MATH_FP64");
  if ((n > 0 && !corr) || !grad_err || !grad_xi)
    return fail(VGICP_E_INVALID_ARG, "NULL argument");
  // the poses at which the cost is differentiated, and the tangent maps
  TangentMap J{};
  double Tt[12], Ts[12];
  std::memcpy(Tt, T_target, sizeof(Tt));
  std::memcpy(Ts, T_source, sizeof(Ts));
  const double zero[6] = {0, 0, 0, 0, 0, 0};
  if (xi_source || (binary && xi_target)) {
    const double* xs = xi_source ? xi_source : zero;
    const double* xt = (binary && xi_target) ? xi_target : zero;
    for (int i = 0; i < 6; ++i)
      if (!std::isfinite(xs[i]) || !std::isfinite(xt[i]))
        return fail(VGICP_E_NONFINITE, "non-finite tangent");
    if (!right_jacobian(xs, J.Js) || !right_jacobian(xt, J.Jt))
      return fail(VGICP_E_INVALID_ARG, "|xi| must be below 3");
    se3_retract(T_source, xs, Ts);
    se3_retract(T_target, xt, Tt);
    J.use = 1;
  }
  hipStream_t s = stream_of(stream);
  const RelPose T = make_rel_pose(Tt, Ts, map->inv_res);
  const int tile = plain_tile_for(n, device_cu_count(map->device));
  const int ntiles = (int)((n + tile - 1) / tile);
  double* partials = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&partials),
                                (size_t)std::max(ntiles, 1) * 6 * sizeof(double), s);
  if (e != hipSuccess) return hip_fail(e, "hipMallocAsync (partials)");
  launch_backward(map->view(), T, J, xyz, cov, n, binary, precision, corr, grad_err, partials,
                  ntiles, tile, grad_xi, grad_xyz, s);
  e = hipGetLastError();
  (void)hipFreeAsync(partials, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_backward(vgicp_voxelmap map, const float* xyz, const float* cov,
                                      int64_t n, const double* T_target,
                                      const double* T_source, int32_t binary,
                                      const int32_t* corr, const double* grad_err,
                                      vgicp_precision precision, double* grad_xi,
                                      float* grad_xyz, vgicp_stream stream) {
  return backward_impl(map, xyz, cov, n, T_target, T_source, nullptr, nullptr, binary, corr,
                       grad_err, (int)precision, grad_xi, grad_xyz, stream);
}

VGICP_API vgicp_status vgicp_backward_tangent(vgicp_voxelmap map, const float* xyz,
                                              const float* cov, int64_t n,
                                              const double* T_target, const double* T_source,
                                              const double* xi_target, const double* xi_source,
                                              int32_t binary, const int32_t* corr,
                                              const double* grad_err,
                                              vgicp_precision precision, double* grad_xi,
                                              float* grad_xyz, vgicp_stream stream) {
  return backward_impl(map, xyz, cov, n, T_target, T_source, xi_target, xi_source, binary, corr,
                       grad_err, (int)precision, grad_xi, grad_xyz, stream);
}

}  // extern "C"

// ------------------------------------------------------------------------ batches

struct vgicp_batch_s {
  int device = 0;
  int F = 0, P = 0;
  std::vector<FactorView> hf;       // host copy (tile_base/ntiles follow the schedule)
  std::vector<int> target_of;       // map index per factor
  std::vector<vgicp_cloud> clouds;  // the caller's clouds (source of the batch's copies)
  std::vector<int64_t> cov6_offset; // per cloud: first point in the copies
  std::vector<double> cloud_cell;   // per cloud: cell of its spatial order (finest target res)
  std::vector<float> boxes;         // per cloud: bounding box lo, hi (local frame)
  float* d_boxes = nullptr;
  float* d_xyz = nullptr;           // every cloud's positions in spatial order, [3][n] each
  float* d_cov6 = nullptr;          // and its covariances, interleaved [n][6]
  int* d_perm = nullptr;            // and its order: spatial index -> the caller's index
  int64_t gpts_total = 0;           // sum of the factors' source sizes
  // backward (allocated on first use)
  bool grad_ready = false;
  float* d_gpts = nullptr;          // [gpts_total][3] per factor and point
  double* d_gf = nullptr;           // [F][12]
  int *d_gbptr = nullptr, *d_gbcontrib = nullptr, *d_cptr = nullptr, *d_cfac = nullptr;
  long long *d_cloud_n = nullptr, *d_cloud_off = nullptr;
  float** d_gout = nullptr;         // [clouds] the caller's point-gradient arrays
  float** h_gout = nullptr;         // pinned staging of the same
  std::vector<float*> gout_last;    // last uploaded contents
  long long max_cloud_n = 0;
  // Levenberg-Marquardt step (allocated on first use)
  bool lm_ready = false;
  int lm_solver = 0;               // vgicp_batch_lm_solver: 0 automatic, 1 dense, 2 one sweep
  LmStructure lm;
  LmBlock* d_lm_blocks = nullptr;
  int *d_lm_contrib = nullptr, *d_lm_bptr = nullptr, *d_lm_bcontrib = nullptr;
  double *d_lm_H = nullptr, *d_lm_b = nullptr, *d_lm_e0 = nullptr, *d_lm_e1 = nullptr;
  int64_t *d_lm_n0 = nullptr, *d_lm_n1 = nullptr;
  double *d_lm_A = nullptr, *d_lm_diag = nullptr, *d_lm_x = nullptr, *d_lm_dinv = nullptr;
  double *d_lm_Hc = nullptr, *d_lm_bc = nullptr, *d_lm_cand = nullptr, *d_lm_lambda = nullptr;
  int *d_lm_pos = nullptr, *d_lm_accept = nullptr;
  vgicp_schedule sched{256, 8192, 2, 4};
  FactorView* d_factors = nullptr;
  RelPose* d_rel = nullptr;
  WorkItem* d_items = nullptr;
  int* d_seg = nullptr;
  unsigned long long* d_heads = nullptr;
  double* d_partials = nullptr;
  size_t items_cap = 0, partials_cap = 0;
  int total_tiles = 0;
  int grid = 0;
  int64_t total_points = 0;
  hipStream_t capture_stream = nullptr;
  // Every call on the batch uses the scratch above (relative poses, queue heads, partial sums,
  // the LM system); each call's stream waits for the previous call's work, whatever stream
  // that ran on, so calls on different streams are ordered instead of racing.
  hipEvent_t done = nullptr;
  bool done_recorded = false;
  hipStream_t last_stream = nullptr;  // stream of the previous call (its end is `done`)
  struct Graph {
    std::array<uintptr_t, 8> key;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;

  void drop_graphs() {
    for (auto& g : graphs) {
      (void)hipGraphExecDestroy(g.exec);
      (void)hipGraphDestroy(g.graph);
    }
    graphs.clear();
  }
};

namespace {

// Orders a call on the batch after the previous one (see vgicp_batch_s::done).
vgicp_status batch_begin(vgicp_batch b, hipStream_t s) {
  hipError_t e;
  if (!b->done && (e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming)))
    return hip_fail(e, "hipEventCreate");
  // the same stream orders the calls by itself; only a change of stream needs the wait
  if (b->done_recorded && s != b->last_stream && (e = hipStreamWaitEvent(s, b->done, 0)))
    return hip_fail(e, "hipStreamWaitEvent");
  return VGICP_OK;
}

vgicp_status batch_end(vgicp_batch b, hipStream_t s, vgicp_status st) {
  if (!b->done) return st;
  const hipError_t e = hipEventRecord(b->done, s);
  if (e != hipSuccess) return st == VGICP_OK ? hip_fail(e, "hipEventRecord") : st;
  b->done_recorded = true;
  b->last_stream = s;
  return st;
}

bool valid_schedule(const vgicp_schedule& s) {
  return (s.block == 256 || s.block == 512) && s.tile >= s.block && s.tile % s.block == 0 &&
         s.tile <= kMaxPointsPerLane * s.block && s.blocks_per_cu >= 1 &&
         s.blocks_per_cu <= 16 && (s.lookahead == 2 || s.lookahead == 4 || s.lookahead == 8);
}

// Splits every factor into tiles and orders the work: factors are grouped by target map, the
// groups are dealt to the XCD queues by decreasing size onto the least-loaded queue (LPT), and
// inside a queue the tiles of a group are consecutive.
vgicp_status apply_schedule(vgicp_batch b, const vgicp_schedule& sc) {
  const int tile = sc.tile;
  std::vector<int> ntiles(b->F), base(b->F);
  int64_t total = 0;
  for (int f = 0; f < b->F; ++f) {
    const int64_t nt = (b->hf[f].n + tile - 1) / tile;
    if (total + nt >= (1LL << 31) / kPartialStride)
      return fail(VGICP_E_CAPACITY, "too many work items for this tile size");
    ntiles[f] = (int)nt;
    base[f] = (int)total;
    total += nt;
  }
  std::map<int, std::vector<int>> groups;
  for (int f = 0; f < b->F; ++f) groups[b->target_of[f]].push_back(f);
  std::vector<std::pair<int64_t, int>> gsz;
  for (auto& kv : groups) {
    int64_t pts = 0;
    for (int f : kv.second) pts += b->hf[f].n;
    gsz.push_back({pts, kv.first});
  }
  std::stable_sort(gsz.begin(), gsz.end(),
                   [](const std::pair<int64_t, int>& a, const std::pair<int64_t, int>& c) {
                     return a.first > c.first;
                   });
  std::array<int64_t, kNumXcd> load{};
  std::array<std::vector<int>, kNumXcd> xg;
  for (auto& g : gsz) {
    int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[x] += g.first;
    xg[x].push_back(g.second);
  }
  std::vector<WorkItem> items;
  items.reserve((size_t)total);
  std::vector<int> seg(kNumXcd + 1, 0);
  for (int x = 0; x < kNumXcd; ++x) {
    seg[x] = (int)items.size();
    std::sort(xg[x].begin(), xg[x].end());
    for (int g : xg[x])
      for (int f : groups[g])
        for (int t = 0; t < ntiles[f]; ++t) items.push_back({f, t});
  }
  seg[kNumXcd] = (int)items.size();
  for (int f = 0; f < b->F; ++f) {
    b->hf[f].tile_base = base[f];
    b->hf[f].ntiles = ntiles[f];
  }
  hipError_t e;
  if (items.size() > b->items_cap) {
    (void)hipFree(b->d_items);
    b->d_items = nullptr;
    if ((e = hipMalloc(&b->d_items, std::max<size_t>(items.size(), 1) * sizeof(WorkItem))))
      return hip_fail(e, "hipMalloc (work items)");
    b->items_cap = items.size();
  }
  const size_t np = (size_t)std::max<int64_t>(total, 1) * kPartialStride;
  if (np > b->partials_cap) {
    (void)hipFree(b->d_partials);
    b->d_partials = nullptr;
    if ((e = hipMalloc(&b->d_partials, np * sizeof(double))))
      return hip_fail(e, "hipMalloc (partials)");
    b->partials_cap = np;
  }
  if ((!items.empty() && (e = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(WorkItem),
                                         hipMemcpyHostToDevice))) ||
      (e = hipMemcpy(b->d_seg, seg.data(), seg.size() * sizeof(int), hipMemcpyHostToDevice)) ||
      (b->F > 0 && (e = hipMemcpy(b->d_factors, b->hf.data(), b->hf.size() * sizeof(FactorView),
                                  hipMemcpyHostToDevice))))
    return hip_fail(e, "upload schedule");
  b->total_tiles = (int)total;
  const int cus = device_cu_count(b->device);
  b->grid = ((cus * sc.blocks_per_cu + kNumXcd - 1) / kNumXcd) * kNumXcd;
  b->sched = sc;
  b->drop_graphs();
  return VGICP_OK;
}

BatchLaunch make_launch(vgicp_batch b, const double* poses, int precision, bool lin, double* H,
                        double* bb, double* err, int64_t* inliers) {
  BatchLaunch L;
  L.factors = b->d_factors;
  L.boxes = b->d_boxes;
  L.rel = b->d_rel;
  L.poses = poses;
  L.items = b->d_items;
  L.seg = b->d_seg;
  L.heads = b->d_heads;
  L.partials = b->d_partials;
  L.flags = device_flags(b->device);
  L.F = b->F;
  L.grid = b->grid;
  L.block = b->sched.block;
  L.tile = b->sched.tile;
  L.lookahead = b->sched.lookahead;
  L.precision = precision;
  L.linearize = lin;
  L.H = H;
  L.b = bb;
  L.err = err;
  L.inliers = inliers;
  return L;
}

vgicp_status check_batch_call(vgicp_batch b, const double* poses, int precision) {
  if (!b) return fail(VGICP_E_INVALID_ARG, "batch is NULL");
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || cur != b->device)
    return fail(VGICP_E_INVALID_ARG, "batch lives on another device than the current one");
  if (!poses && b->F > 0) return fail(VGICP_E_INVALID_ARG, "poses is NULL");
  if (!valid_precision(precision)) return fail(VGICP_E_INVALID_ARG, "unknown precision");
  if (!device_flags(b->device)) return fail(VGICP_E_HIP, "device error word address");
  return VGICP_OK;
}

// Runs the batch through a captured graph (capture on the batch's private stream, launch on
// the caller's). One graph per (precision, mode, pointer set, grid), at most kMaxGraphs.
constexpr size_t kMaxGraphs = 16;
vgicp_status run_batch(vgicp_batch b, const double* poses, int precision, bool lin, double* H,
                       double* bb, double* err, int64_t* inliers, hipStream_t s) {
  if (b->F == 0) return VGICP_OK;
  const std::array<uintptr_t, 8> key = {(uintptr_t)precision, (uintptr_t)lin, (uintptr_t)poses,
                                        (uintptr_t)H, (uintptr_t)bb, (uintptr_t)err,
                                        (uintptr_t)inliers, (uintptr_t)b->grid};
  hipError_t e;
  for (auto& g : b->graphs)
    if (g.key == key) {
      if ((e = hipGraphLaunch(g.exec, s))) return hip_fail(e, "hipGraphLaunch");
      return VGICP_OK;
    }
  if (!b->capture_stream &&
      (e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking)))
    return hip_fail(e, "hipStreamCreate");
  if (b->graphs.size() >= kMaxGraphs) {  // bounded cache: drop the oldest capture
    if ((e = hipDeviceSynchronize())) return hip_fail(e, "hipDeviceSynchronize");
    (void)hipGraphExecDestroy(b->graphs.front().exec);
    (void)hipGraphDestroy(b->graphs.front().graph);
    b->graphs.erase(b->graphs.begin());
  }
  const BatchLaunch L = make_launch(b, poses, precision, lin, H, bb, err, inliers);
  if ((e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeRelaxed)))
    return hip_fail(e, "hipStreamBeginCapture");
  launch_batched(L, b->capture_stream);
  vgicp_batch_s::Graph g;
  g.key = key;
  e = hipStreamEndCapture(b->capture_stream, &g.graph);
  if (e) return hip_fail(e, "hipStreamEndCapture");
  if ((e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0))) {
    (void)hipGraphDestroy(g.graph);
    return hip_fail(e, "hipGraphInstantiate");
  }
  b->graphs.push_back(g);
  if ((e = hipGraphLaunch(g.exec, s))) return hip_fail(e, "hipGraphLaunch");
  return VGICP_OK;
}

std::string tune_key(vgicp_batch b, int precision) {
  std::ostringstream os;
  DevState* d = nullptr;
  (void)d;
  int dev = b->device;
  hipDeviceProp_t prop;
  std::string arch = "gpu";
  int cus = device_cu_count(dev);
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == '"' || c == ':') c = '_';
  os << arch << "/cu" << cus << "/p" << precision << "/F" << b->F << "/N" << b->total_points;
  return os.str();
}

// Minimal reader/writer of {"key": [block, tile, blocks_per_cu, lookahead], ...}.
std::map<std::string, std::array<int, 4>> read_cache(const char* path) {
  std::map<std::string, std::array<int, 4>> m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t p = 0;
  while ((p = s.find('"', p)) != std::string::npos) {
    const size_t q = s.find('"', p + 1);
    if (q == std::string::npos) break;
    const std::string k = s.substr(p + 1, q - p - 1);
    const size_t lb = s.find('[', q), rb = s.find(']', q);
    if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
    std::array<int, 4> v{0, 0, 0, 0};
    if (std::sscanf(s.substr(lb + 1, rb - lb - 1).c_str(), "%d , %d , %d , %d", &v[0], &v[1],
                    &v[2], &v[3]) == 4)
      m[k] = v;
    p = rb + 1;
  }
  return m;
}

void write_cache(const char* path, const std::map<std::string, std::array<int, 4>>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t i = 0;
    for (auto& kv : m) {
      f << "  \"" << kv.first << "\": [" << kv.second[0] << ", " << kv.second[1] << ", "
        << kv.second[2] << ", " << kv.second[3] << "]" << (++i < m.size() ? "," : "") << "\n";
    }
    f << "}\n";
  }
  std::rename(tmp.c_str(), path);
}

}  // namespace

extern "C" {

VGICP_API vgicp_status vgicp_batch_create(const vgicp_voxelmap* maps, int32_t n_maps,
                                          const vgicp_cloud* clouds, int32_t n_clouds,
                                          const vgicp_factor* factors, int32_t n_factors,
                                          int32_t n_poses, vgicp_batch* out) {
  if (!out) return fail(VGICP_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n_maps < 0 || n_clouds < 0 || n_factors < 0 || n_poses < 0)
    return fail(VGICP_E_INVALID_ARG, "negative count");
  if ((n_maps && !maps) || (n_clouds && !clouds) || (n_factors && !factors))
    return fail(VGICP_E_INVALID_ARG, "NULL array");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e) return hip_fail(e, "hipGetDevice");
  for (int i = 0; i < n_maps; ++i) {
    if (!maps[i]) return fail(VGICP_E_INVALID_ARG, "NULL voxel map in batch");
    if (maps[i]->device != dev) return fail(VGICP_E_INVALID_ARG, "voxel map on another device");
  }
  for (int i = 0; i < n_clouds; ++i) {
    vgicp_status st = check_cloud(clouds[i].xyz, clouds[i].cov, clouds[i].n);
    if (st != VGICP_OK) return st;
  }
  auto* b = new vgicp_batch_s;
  b->device = dev;
  b->F = n_factors;
  b->P = n_poses;
  b->hf.resize(n_factors);
  b->target_of.resize(n_factors);
  b->clouds.assign(clouds, clouds + n_clouds);
  b->cov6_offset.resize(n_clouds);
  int64_t cov6_points = 0;
  for (int i = 0; i < n_clouds; ++i) {
    b->cov6_offset[i] = cov6_points;
    cov6_points += clouds[i].n;
  }
  b->cloud_cell.assign(n_clouds, 0.0);
  if ((e = hipMalloc(&b->d_cov6, (size_t)std::max<int64_t>(cov6_points, 1) * 24)) ||
      (e = hipMalloc(&b->d_xyz, (size_t)std::max<int64_t>(cov6_points, 1) * 12)) ||
      (e = hipMalloc(&b->d_perm, (size_t)std::max<int64_t>(cov6_points, 1) * 4)) ||
      (e = hipMalloc(&b->d_boxes, (size_t)std::max(n_clouds, 1) * 6 * sizeof(float)))) {
    (void)hipFree(b->d_cov6);
    (void)hipFree(b->d_xyz);
    (void)hipFree(b->d_perm);
    delete b;
    return hip_fail(e, "hipMalloc (cloud copy)");
  }
  for (int f = 0; f < n_factors; ++f) {
    const vgicp_factor& fc = factors[f];
    if (fc.target_map < 0 || fc.target_map >= n_maps || fc.source_cloud < 0 ||
        fc.source_cloud >= n_clouds || fc.target_pose < 0 || fc.target_pose >= n_poses ||
        fc.source_pose < 0 || fc.source_pose >= n_poses || (fc.binary != 0 && fc.binary != 1)) {
      vgicp_batch_destroy(b);
      return fail(VGICP_E_INVALID_ARG, "factor " + std::to_string(f) + " has an invalid index");
    }
    FactorView v;
    v.map = maps[fc.target_map]->view();
    v.xyz = b->d_xyz + 3 * b->cov6_offset[fc.source_cloud];
    v.cov6 = b->d_cov6 + 6 * b->cov6_offset[fc.source_cloud];
    double& cell = b->cloud_cell[fc.source_cloud];
    cell = cell > 0.0 ? std::min(cell, maps[fc.target_map]->res) : maps[fc.target_map]->res;
    v.n = clouds[fc.source_cloud].n;
    v.binary = fc.binary;
    v.tile_base = 0;
    v.ntiles = 0;
    v.target_pose = fc.target_pose;
    v.source_pose = fc.source_pose;
    v.source_cloud = fc.source_cloud;
    v.gbase = b->gpts_total;
    b->gpts_total += v.n;
    b->hf[f] = v;
    b->target_of[f] = fc.target_map;
    b->total_points += v.n;
  }
  const size_t F1 = (size_t)std::max(n_factors, 1);
  if ((e = hipMalloc(&b->d_factors, F1 * sizeof(FactorView))) ||
      (e = hipMalloc(&b->d_rel, F1 * sizeof(RelPose))) ||
      (e = hipMalloc(&b->d_seg, (kNumXcd + 1) * sizeof(int))) ||
      (e = hipMalloc(&b->d_heads, kNumXcd * sizeof(unsigned long long)))) {
    vgicp_batch_destroy(b);
    return hip_fail(e, "hipMalloc (batch)");
  }
  vgicp_status st = apply_schedule(b, b->sched);
  if (st == VGICP_OK) st = vgicp_batch_refresh(b, nullptr);
  if (st == VGICP_OK && (e = hipStreamSynchronize(nullptr))) st = hip_fail(e, "batch setup");
  if (st != VGICP_OK) {
    vgicp_batch_destroy(b);
    return st;
  }
  *out = b;
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_batch_refresh(vgicp_batch batch, vgicp_stream stream) {
  if (!batch) return fail(VGICP_E_INVALID_ARG, "batch is NULL");
  hipStream_t s = stream_of(stream);
  vgicp_status st0 = batch_begin(batch, s);
  if (st0 != VGICP_OK) return st0;
  batch->boxes.assign(6 * std::max<size_t>(batch->clouds.size(), 1), 0.0f);
  for (size_t i = 0; i < batch->clouds.size(); ++i) {
    float* box = batch->boxes.data() + 6 * i;
    if (batch->cloud_cell[i] <= 0.0) continue;  // no factor reads this cloud
    const int64_t o = batch->cov6_offset[i];
    vgicp_status st = spatial_copy(batch->clouds[i].xyz, batch->clouds[i].cov, batch->clouds[i].n,
                                   batch->cloud_cell[i], batch->d_xyz + 3 * o,
                                   batch->d_cov6 + 6 * o, box, batch->d_perm + o, s);
    if (st != VGICP_OK) return batch_end(batch, s, st);
  }
  hipError_t e = hipMemcpy(batch->d_boxes, batch->boxes.data(),
                           batch->boxes.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return batch_end(batch, s, hip_fail(e, "upload bounding boxes"));
  return batch_end(batch, s, VGICP_OK);
}

VGICP_API vgicp_status vgicp_batch_set_schedule(vgicp_batch batch,
                                                const vgicp_schedule* schedule) {
  if (!batch || !schedule) return fail(VGICP_E_INVALID_ARG, "NULL argument");
  if (!valid_schedule(*schedule)) return fail(VGICP_E_INVALID_ARG, "unsupported schedule");
  hipError_t e = hipDeviceSynchronize();
  if (e) return hip_fail(e, "hipDeviceSynchronize");
  return apply_schedule(batch, *schedule);
}

VGICP_API vgicp_status vgicp_batch_get_schedule(vgicp_batch batch, vgicp_schedule* schedule) {
  if (!batch || !schedule) return fail(VGICP_E_INVALID_ARG, "NULL argument");
  *schedule = batch->sched;
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_batch_linearize(vgicp_batch batch, const double* poses,
                                             vgicp_precision precision, double* H, double* b,
                                             double* err, int64_t* inliers,
                                             vgicp_stream stream) {
  vgicp_status st = check_batch_call(batch, poses, (int)precision);
  if (st != VGICP_OK) return st;
  if (batch->F > 0 && (!H || !b || !err || !inliers))
    return fail(VGICP_E_INVALID_ARG, "NULL output");
  hipStream_t s = stream_of(stream);
  if ((st = batch_begin(batch, s)) != VGICP_OK) return st;
  return batch_end(batch, s, run_batch(batch, poses, (int)precision, true, H, b, err, inliers, s));
}

VGICP_API vgicp_status vgicp_batch_evaluate(vgicp_batch batch, const double* poses,
                                            vgicp_precision precision, double* err,
                                            int64_t* inliers, vgicp_stream stream) {
  vgicp_status st = check_batch_call(batch, poses, (int)precision);
  if (st != VGICP_OK) return st;
  if (batch->F > 0 && (!err || !inliers)) return fail(VGICP_E_INVALID_ARG, "NULL output");
  hipStream_t s = stream_of(stream);
  if ((st = batch_begin(batch, s)) != VGICP_OK) return st;
  return batch_end(batch, s,
                   run_batch(batch, poses, (int)precision, false, nullptr, nullptr, err,
                             inliers, s));
}

VGICP_API vgicp_status vgicp_batch_overlap(vgicp_batch batch, const double* poses,
                                           double* rates, int64_t* inliers,
                                           vgicp_stream stream) {
  vgicp_status st = check_batch_call(batch, poses, VGICP_ACC_FP64);
  if (st != VGICP_OK) return st;
  if (batch->F > 0 && (!rates || !inliers)) return fail(VGICP_E_INVALID_ARG, "NULL output");
  hipStream_t s = stream_of(stream);
  if ((st = batch_begin(batch, s)) != VGICP_OK) return st;
  return batch_end(batch, s,
                   run_batch(batch, poses, kCountOnly, false, nullptr, nullptr, rates, inliers,
                             s));
}

extern "C++" {
namespace {

vgicp_status autotune(vgicp_batch batch, const double* poses, vgicp_precision precision,
                      const char* cache_path, vgicp_schedule* chosen, hipStream_t s);
vgicp_status lm_step(vgicp_batch batch, const double* poses, vgicp_precision precision,
                     double lambda, int32_t fixed_pose, double* poses_new, double* delta,
                     double* cost, hipStream_t s);
vgicp_status lm_iterate(vgicp_batch batch, double* poses, vgicp_precision precision,
                        double* lambda, int32_t fixed_pose, int32_t iterations, double* cost,
                        hipStream_t s);
vgicp_status grad_prepare(vgicp_batch b);
void free_lm(vgicp_batch b);

template <typename T>
hipError_t upload(T** d, const std::vector<T>& h) {
  hipError_t e = hipMalloc(d, std::max<size_t>(h.size(), 1) * sizeof(T));
  if (e == hipSuccess && !h.empty())
    e = hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

// Frees the LM step's buffers; the next LM call prepares them again.
void free_lm(vgicp_batch b) {
  for (void** p : {(void**)&b->d_lm_blocks, (void**)&b->d_lm_contrib, (void**)&b->d_lm_bptr,
                   (void**)&b->d_lm_bcontrib, (void**)&b->d_lm_H, (void**)&b->d_lm_b,
                   (void**)&b->d_lm_e0, (void**)&b->d_lm_e1, (void**)&b->d_lm_n0,
                   (void**)&b->d_lm_n1, (void**)&b->d_lm_A, (void**)&b->d_lm_diag,
                   (void**)&b->d_lm_x, (void**)&b->d_lm_dinv, (void**)&b->d_lm_Hc,
                   (void**)&b->d_lm_bc, (void**)&b->d_lm_cand, (void**)&b->d_lm_lambda,
                   (void**)&b->d_lm_pos, (void**)&b->d_lm_accept}) {
    (void)hipFree(*p);
    *p = nullptr;
  }
  b->lm_ready = false;
}

vgicp_status grad_prepare(vgicp_batch b) {
  if (b->grad_ready) return VGICP_OK;
  LmStructure L;
  build_lm_structure(b->hf, b->P, L);
  const int C = (int)b->clouds.size();
  std::vector<std::vector<int>> by_cloud((size_t)C);
  for (int f = 0; f < b->F; ++f) by_cloud[b->hf[f].source_cloud].push_back(f);
  std::vector<int> cptr((size_t)C + 1, 0), cfac;
  std::vector<long long> cn((size_t)C), coff((size_t)C);
  for (int c = 0; c < C; ++c) {
    cptr[c] = (int)cfac.size();
    cfac.insert(cfac.end(), by_cloud[c].begin(), by_cloud[c].end());
    cn[c] = b->clouds[c].n;
    coff[c] = b->cov6_offset[c];
    b->max_cloud_n = std::max<long long>(b->max_cloud_n, cn[c]);
  }
  cptr[C] = (int)cfac.size();
  hipError_t e;
  if ((e = hipMalloc(&b->d_gpts, (size_t)std::max<int64_t>(b->gpts_total, 1) * 3 * sizeof(float))) ||
      (e = hipMalloc(&b->d_gf, (size_t)std::max(b->F, 1) * 12 * sizeof(double))) ||
      (e = upload(&b->d_gbptr, L.bptr)) || (e = upload(&b->d_gbcontrib, L.bcontrib)) ||
      (e = upload(&b->d_cptr, cptr)) || (e = upload(&b->d_cfac, cfac)) ||
      (e = upload(&b->d_cloud_n, cn)) || (e = upload(&b->d_cloud_off, coff)) ||
      (e = hipMalloc(&b->d_gout, (size_t)std::max(C, 1) * sizeof(float*))) ||
      (e = hipHostMalloc(&b->h_gout, (size_t)std::max(C, 1) * sizeof(float*), 0)))
    return hip_fail(e, "hipMalloc (batch backward)");
  b->gout_last.assign((size_t)C, reinterpret_cast<float*>(1));  // forces the first upload
  b->grad_ready = true;
  return VGICP_OK;
}

vgicp_status lm_prepare(vgicp_batch b) {
  if (b->lm_ready) return VGICP_OK;
  build_lm_structure(b->hf, b->P, b->lm);
  if (b->lm_solver == 1 || (b->lm_solver == 2 && !b->lm.one_sweep)) b->lm.band = false;
  if (b->lm_solver != 0 || !b->lm.band) {
    b->lm.split = false;
    b->lm.m_top = b->lm.m_bot = 0;
  }
  const LmStructure& L = b->lm;
  const size_t F1 = (size_t)std::max(b->F, 1), P1 = (size_t)std::max(b->P, 1);
  const size_t n = (size_t)std::max(L.n, 64);
  // banded: the band rows of the permuted system, a spare block and 64 spare values (the
  // solver's scratch); split, after them the bottom end's and the separator's rows, each with
  // its spare block and values; dense: the whole matrix and the 64 x 64 block inverses
  const size_t W1 = (size_t)L.w + 1;
  const size_t top_vals = 6 * (P1 + 1) * W1 + 64;
  const size_t bot_vals = L.split ? (6 * (size_t)L.m_bot + W1 + 6) * W1 + 64 : 0;
  const size_t sep_vals = L.split ? (W1 + 6) * W1 + 64 : 0;
  const size_t mat = L.band ? top_vals + bot_vals + sep_vals : n * n;
  // right-hand sides / solutions: [n + 64], split: then [6 m_bot + w + 1 + 64] and [w + 1 + 64]
  const size_t xv = (n + 64) + (L.split ? (6 * (size_t)L.m_bot + W1 + 64) + (W1 + 64) : 0);
  const size_t inv = L.band ? 64 : n * 64;
  hipError_t e;
  if ((e = upload(&b->d_lm_blocks, L.blocks)) || (e = upload(&b->d_lm_contrib, L.contrib)) ||
      (e = upload(&b->d_lm_bptr, L.bptr)) || (e = upload(&b->d_lm_bcontrib, L.bcontrib)) ||
      (e = upload(&b->d_lm_pos, L.pos)) ||
      (e = hipMalloc(&b->d_lm_H, F1 * 144 * sizeof(double))) ||
      (e = hipMalloc(&b->d_lm_b, F1 * 12 * sizeof(double))) ||
      (e = hipMalloc(&b->d_lm_Hc, F1 * 144 * sizeof(double))) ||
      (e = hipMalloc(&b->d_lm_bc, F1 * 12 * sizeof(double))) ||
      (e = hipMalloc(&b->d_lm_e0, F1 * sizeof(double))) ||
      (e = hipMalloc(&b->d_lm_e1, F1 * sizeof(double))) ||
      (e = hipMalloc(&b->d_lm_n0, F1 * sizeof(int64_t))) ||
      (e = hipMalloc(&b->d_lm_n1, F1 * sizeof(int64_t))) ||
      (e = hipMalloc(&b->d_lm_cand, P1 * 12 * sizeof(double))) ||
      (e = hipMalloc(&b->d_lm_lambda, sizeof(double))) ||
      (e = hipMalloc(&b->d_lm_accept, sizeof(int))) ||
      (e = hipMalloc(&b->d_lm_A, mat * sizeof(double))) ||
      (e = hipMalloc(&b->d_lm_diag, n * sizeof(double))) ||
      (e = hipMalloc(&b->d_lm_x, xv * sizeof(double))) ||
      (e = hipMalloc(&b->d_lm_dinv, inv * sizeof(double))))
    return hip_fail(e, "hipMalloc (LM step)");
  b->lm_ready = true;
  return VGICP_OK;
}

}  // namespace
}  // extern "C++"

VGICP_API vgicp_status vgicp_batch_backward(vgicp_batch batch, const double* poses,
                                            vgicp_precision precision,
                                            const double* grad_err, double* grad_poses,
                                            double* grad_factors, float* const* grad_points,
                                            vgicp_stream stream) {
  vgicp_status st = check_batch_call(batch, poses, (int)precision);
  if (st != VGICP_OK) return st;
  if (precision != VGICP_ACC_FP64 && precision != VGICP_MATH_FP64)
    return fail(VGICP_E_INVALID_ARG, "backward supports VGICP_ACC_FP64 and VGICP_MATH_FP64");
  if ((batch->F > 0 && !grad_err) || (batch->P > 0 && !grad_poses))
    return fail(VGICP_E_INVALID_ARG, "NULL argument");
  if (batch->clouds.size() > 65535)
    return fail(VGICP_E_CAPACITY, "backward: more than 65,535 clouds in one batch");
  if ((st = grad_prepare(batch)) != VGICP_OK) return st;
  hipStream_t s = stream_of(stream);
  if ((st = batch_begin(batch, s)) != VGICP_OK) return st;
  hipError_t e;
  const int C = (int)batch->clouds.size();
  // the caller's point-gradient arrays: uploaded when they change (the pinned staging is
  // rewritten only after the batch's previous call, which read it, has completed)
  std::vector<float*> want((size_t)C, nullptr);
  if (grad_points)
    for (int c = 0; c < C; ++c) want[c] = grad_points[c];
  if (C > 0 && want != batch->gout_last) {
    if (batch->done_recorded && (e = hipEventSynchronize(batch->done)))
      return batch_end(batch, s, hip_fail(e, "hipEventSynchronize"));
    std::memcpy(batch->h_gout, want.data(), (size_t)C * sizeof(float*));
    if ((e = hipMemcpyAsync(batch->d_gout, batch->h_gout, (size_t)C * sizeof(float*),
                            hipMemcpyHostToDevice, s)))
      return batch_end(batch, s, hip_fail(e, "upload point-gradient pointers"));
    batch->gout_last = want;
  }
  if (batch->F == 0 && batch->P > 0 &&
      (e = hipMemsetAsync(grad_poses, 0, (size_t)batch->P * 6 * sizeof(double), s)))
    return batch_end(batch, s, hip_fail(e, "hipMemsetAsync"));
  if (batch->F > 0) {
    const BatchLaunch L = make_launch(batch, poses, (int)precision, false, nullptr, nullptr,
                                      nullptr, nullptr);
    BatchGrad G;
    G.grad_err = grad_err;
    G.gpts = batch->d_gpts;
    G.gf = grad_factors ? grad_factors : batch->d_gf;
    G.grad_poses = grad_poses;
    G.bptr = batch->d_gbptr;
    G.bcontrib = batch->d_gbcontrib;
    G.P = batch->P;
    G.cptr = batch->d_cptr;
    G.cfac = batch->d_cfac;
    G.cloud_n = batch->d_cloud_n;
    G.cloud_off = batch->d_cloud_off;
    G.perm = batch->d_perm;
    G.out = batch->d_gout;
    G.n_clouds = grad_points ? C : 0;
    G.max_n = batch->max_cloud_n;
    launch_batched_backward(L, G, s);
    if ((e = hipGetLastError())) return batch_end(batch, s, hip_fail(e, "backward launch"));
  }
  return batch_end(batch, s, VGICP_OK);
}


VGICP_API vgicp_status vgicp_batch_lm_step(vgicp_batch batch, const double* poses,
                                           vgicp_precision precision, double lambda,
                                           int32_t fixed_pose, double* poses_new, double* delta,
                                           double* cost, vgicp_stream stream) {
  vgicp_status st = check_batch_call(batch, poses, (int)precision);
  if (st != VGICP_OK) return st;
  if (!poses || !poses_new || !cost) return fail(VGICP_E_INVALID_ARG, "NULL argument");
  if (!(lambda >= 0.0) || !std::isfinite(lambda))
    return fail(VGICP_E_INVALID_ARG, "lambda must be finite and >= 0");
  if (fixed_pose < -1 || fixed_pose >= batch->P)
    return fail(VGICP_E_INVALID_ARG, "fixed_pose out of range");
  if ((st = lm_prepare(batch)) != VGICP_OK) return st;
  if (!batch->lm.band && 6LL * batch->P >= (1LL << 15))
    return fail(VGICP_E_CAPACITY, "LM step: more than 5,460 poses in a graph that is not banded");
  hipStream_t s = stream_of(stream);
  if ((st = batch_begin(batch, s)) != VGICP_OK) return st;
  return batch_end(batch, s, lm_step(batch, poses, precision, lambda, fixed_pose, poses_new,
                                     delta, cost, s));
}

VGICP_API vgicp_status vgicp_batch_lm_iterate(vgicp_batch batch, double* poses,
                                              vgicp_precision precision, double* lambda,
                                              int32_t fixed_pose, int32_t iterations,
                                              double* cost, vgicp_stream stream) {
  vgicp_status st = check_batch_call(batch, poses, (int)precision);
  if (st != VGICP_OK) return st;
  if (!poses || !lambda || !cost) return fail(VGICP_E_INVALID_ARG, "NULL argument");
  if (iterations < 0) return fail(VGICP_E_INVALID_ARG, "negative iteration count");
  if (fixed_pose < -1 || fixed_pose >= batch->P)
    return fail(VGICP_E_INVALID_ARG, "fixed_pose out of range");
  if ((st = lm_prepare(batch)) != VGICP_OK) return st;
  if (!batch->lm.band && 6LL * batch->P >= (1LL << 15))
    return fail(VGICP_E_CAPACITY, "LM step: more than 5,460 poses in a graph that is not banded");
  hipStream_t s = stream_of(stream);
  if ((st = batch_begin(batch, s)) != VGICP_OK) return st;
  return batch_end(batch, s, lm_iterate(batch, poses, precision, lambda, fixed_pose, iterations,
                                        cost, s));
}

VGICP_API vgicp_status vgicp_batch_lm_solver(vgicp_batch batch, int32_t solver) {
  if (!batch) return fail(VGICP_E_INVALID_ARG, "batch is NULL");
  if (solver < 0 || solver > 2) return fail(VGICP_E_INVALID_ARG, "solver must be 0, 1 or 2");
  if (batch->lm_solver == solver) return VGICP_OK;
  const hipError_t e = hipDeviceSynchronize();
  if (e) return hip_fail(e, "hipDeviceSynchronize");
  free_lm(batch);
  batch->lm_solver = solver;
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_batch_lm_info(vgicp_batch batch, int32_t* banded,
                                           int32_t* half_bandwidth) {
  if (!batch) return fail(VGICP_E_INVALID_ARG, "batch is NULL");
  vgicp_status st = lm_prepare(batch);
  if (st != VGICP_OK) return st;
  if (banded) *banded = batch->lm.band ? (batch->lm.split ? 2 : 1) : 0;
  if (half_bandwidth) *half_bandwidth = batch->lm.w;
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_pose_order(int32_t P, const int32_t* links, int32_t n_links,
                                        int32_t* pos, int32_t* bandwidth) {
  if (P < 0 || n_links < 0) return fail(VGICP_E_INVALID_ARG, "negative pose or link count");
  if ((n_links > 0 && !links) || (P > 0 && !pos))
    return fail(VGICP_E_INVALID_ARG, "links or pos is NULL");
  std::vector<std::set<int>> nb((size_t)P);
  for (int32_t k = 0; k < n_links; ++k) {
    const int32_t a = links[2 * (size_t)k], b = links[2 * (size_t)k + 1];
    if (a < 0 || a >= P || b < 0 || b >= P)
      return fail(VGICP_E_INVALID_ARG, "link with a pose index out of range");
    if (a == b) continue;
    nb[a].insert(b);
    nb[b].insert(a);
  }
  std::vector<std::vector<int>> adj((size_t)P);
  for (int p = 0; p < P; ++p) adj[p].assign(nb[p].begin(), nb[p].end());
  std::vector<int> order;
  int bw = 0;
  order_poses(adj, order, bw);
  for (int p = 0; p < P; ++p) pos[p] = order[p];
  if (bandwidth) *bandwidth = bw;
  return VGICP_OK;
}

}  // extern "C"

namespace {

LmDevice lm_device(vgicp_batch batch, const double* Hf, const double* bf) {
  LmDevice d;
  d.blocks = batch->d_lm_blocks;
  d.nblocks = (int)batch->lm.blocks.size();
  d.contrib = batch->d_lm_contrib;
  d.bptr = batch->d_lm_bptr;
  d.bcontrib = batch->d_lm_bcontrib;
  d.Hf = Hf;
  d.bf = bf;
  d.A = batch->d_lm_A;
  d.diag_raw = batch->d_lm_diag;
  d.x = batch->d_lm_x;
  d.Dinv = batch->d_lm_dinv;
  d.n = batch->lm.n;
  d.n_real = batch->lm.n_real;
  d.lambda = batch->d_lm_lambda;
  d.band = batch->lm.band ? 1 : 0;
  d.Ab = batch->d_lm_A;
  d.pos = batch->d_lm_pos;
  d.w = batch->lm.w;
  const LmStructure& L = batch->lm;
  d.split = L.split ? 1 : 0;
  d.m_top = L.m_top;
  d.m_bot = L.m_bot;
  d.Ab_bot = d.Ab_sep = d.x_bot = d.x_sep = nullptr;
  if (L.split) {
    const size_t W1 = (size_t)L.w + 1, P1 = (size_t)std::max(batch->P, 1);
    const size_t n = (size_t)std::max(L.n, 64);
    d.Ab_bot = batch->d_lm_A + 6 * (P1 + 1) * W1 + 64;
    d.Ab_sep = d.Ab_bot + (6 * (size_t)L.m_bot + W1 + 6) * W1 + 64;
    d.x_bot = batch->d_lm_x + n + 64;
    d.x_sep = d.x_bot + 6 * (size_t)L.m_bot + W1 + 64;
  }
  return d;
}

// One step from `poses`: linearize there, solve, retract into poses_new, linearize at poses_new
// (its cost is the step's second cost; its H and b stay in the candidate buffers).
vgicp_status lm_step(vgicp_batch batch, const double* poses, vgicp_precision precision,
                     double lambda, int32_t fixed_pose, double* poses_new, double* delta,
                     double* cost, hipStream_t s) {
  vgicp_status st = VGICP_OK;
  const int F = batch->F;
  if (F > 0 &&
      (st = run_batch(batch, poses, (int)precision, true, batch->d_lm_H, batch->d_lm_b,
                      batch->d_lm_e0, batch->d_lm_n0, s)) != VGICP_OK)
    return st;
  launch_lm_set(batch->d_lm_lambda, lambda, s);
  if (batch->P > 0)
    launch_lm_solve(lm_device(batch, batch->d_lm_H, batch->d_lm_b), batch->P, fixed_pose, poses,
                    poses_new, delta, device_flags(batch->device), s);
  if (F > 0 &&
      (st = run_batch(batch, poses_new, (int)precision, true, batch->d_lm_Hc, batch->d_lm_bc,
                      batch->d_lm_e1, batch->d_lm_n1, s)) != VGICP_OK)
    return st;
  launch_lm_cost(batch->d_lm_e0, batch->d_lm_e1, F, cost, s);
  hipError_t e = hipGetLastError();
  if (e) return hip_fail(e, "LM step launch");
  return VGICP_OK;
}

// `iterations` LM iterations, every decision on the device: the linearization at the current
// poses is kept between iterations, so each iteration linearizes once (at its candidate).
vgicp_status lm_iterate(vgicp_batch batch, double* poses, vgicp_precision precision,
                        double* lambda, int32_t fixed_pose, int32_t iterations, double* cost,
                        hipStream_t s) {
  vgicp_status st = VGICP_OK;
  const int F = batch->F, P = batch->P;
  if (F > 0 &&
      (st = run_batch(batch, poses, (int)precision, true, batch->d_lm_H, batch->d_lm_b,
                      batch->d_lm_e0, batch->d_lm_n0, s)) != VGICP_OK)
    return st;
  hipError_t e;
  if ((e = hipMemcpyAsync(batch->d_lm_lambda, lambda, sizeof(double), hipMemcpyDeviceToDevice,
                          s)))
    return hip_fail(e, "lambda");
  const LmDevice d = lm_device(batch, batch->d_lm_H, batch->d_lm_b);
  for (int it = 0; it < iterations; ++it) {
    if (P > 0)
      launch_lm_solve(d, P, fixed_pose, poses, batch->d_lm_cand, nullptr,
                      device_flags(batch->device), s);
    if (F > 0 &&
        (st = run_batch(batch, batch->d_lm_cand, (int)precision, true, batch->d_lm_Hc,
                        batch->d_lm_bc, batch->d_lm_e1, batch->d_lm_n1, s)) != VGICP_OK)
      return st;
    launch_lm_decide(batch->d_lm_e0, batch->d_lm_e1, F, batch->d_lm_lambda, batch->d_lm_accept,
                     it == 0 ? cost : nullptr, cost + it + 1, s);
    launch_lm_commit(batch->d_lm_accept, P, F, batch->d_lm_cand, poses, batch->d_lm_Hc,
                     batch->d_lm_bc, batch->d_lm_e1, batch->d_lm_H, batch->d_lm_b,
                     batch->d_lm_e0, s);
  }
  if ((e = hipMemcpyAsync(lambda, batch->d_lm_lambda, sizeof(double), hipMemcpyDeviceToDevice,
                          s)))
    return hip_fail(e, "lambda");
  if ((e = hipGetLastError())) return hip_fail(e, "LM iteration launch");
  return VGICP_OK;
}

}  // namespace

extern "C" {

VGICP_API vgicp_status vgicp_batch_autotune(vgicp_batch batch, const double* poses,
                                            vgicp_precision precision, const char* cache_path,
                                            vgicp_schedule* chosen, vgicp_stream stream) {
  vgicp_status st = check_batch_call(batch, poses, (int)precision);
  if (st != VGICP_OK) return st;
  hipStream_t s = stream_of(stream);
  if ((st = batch_begin(batch, s)) != VGICP_OK) return st;
  if ((st = batch_end(batch, s, autotune(batch, poses, precision, cache_path, chosen, s))) !=
      VGICP_OK)
    return st;
  const hipError_t e = hipStreamSynchronize(s);
  return e == hipSuccess ? VGICP_OK : hip_fail(e, "hipStreamSynchronize");
}

}  // extern "C"

namespace {

vgicp_status autotune(vgicp_batch batch, const double* poses, vgicp_precision precision,
                      const char* cache_path, vgicp_schedule* chosen, hipStream_t s) {
  vgicp_status st = VGICP_OK;
  const std::string key = tune_key(batch, (int)precision);
  if (cache_path) {
    auto m = read_cache(cache_path);
    auto it = m.find(key);
    if (it != m.end()) {
      vgicp_schedule sc{it->second[0], it->second[1], it->second[2], it->second[3]};
      if (valid_schedule(sc)) {
        if ((st = vgicp_batch_set_schedule(batch, &sc)) != VGICP_OK) return st;
        if (chosen) *chosen = sc;
        return VGICP_OK;
      }
    }
  }
  if (batch->F == 0) {
    if (chosen) *chosen = batch->sched;
    return VGICP_OK;
  }
  double *H = nullptr, *bb = nullptr, *err = nullptr;
  int64_t* nin = nullptr;
  hipError_t e;
  const size_t F = (size_t)batch->F;
  if ((e = hipMalloc(&H, F * 144 * 8)) || (e = hipMalloc(&bb, F * 12 * 8)) ||
      (e = hipMalloc(&err, F * 8)) || (e = hipMalloc(&nin, F * 8))) {
    (void)hipFree(H);
    (void)hipFree(bb);
    (void)hipFree(err);
    return hip_fail(e, "hipMalloc (autotune outputs)");
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  vgicp_schedule best = batch->sched;
  // optional trace of every candidate: stage block tile blocks_per_cu lookahead min median max
  const char* tlog_path = std::getenv("VGICP_AUTOTUNE_LOG");
  FILE* tlog = tlog_path ? std::fopen(tlog_path, "a") : nullptr;
  if (tlog) std::fprintf(tlog, "# %s\n", key.c_str());
  // median of `reps` timed launches (after one warm-up), or a negative value
  auto time_schedule = [&](const vgicp_schedule& sc, int reps, int stage) -> float {
    if (hipStreamSynchronize(s) != hipSuccess) return -1.0f;
    if (apply_schedule(batch, sc) != VGICP_OK) return -1.0f;
    const BatchLaunch L = make_launch(batch, poses, (int)precision, true, H, bb, err, nin);
    launch_batched(L, s);  // warm-up
    std::vector<float> times((size_t)reps);
    for (float& t : times) {
      (void)hipEventRecord(e0, s);
      launch_batched(L, s);
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      (void)hipEventElapsedTime(&t, e0, e1);
    }
    std::sort(times.begin(), times.end());
    if (tlog)
      std::fprintf(tlog, "%d %d %d %d %d %.4f %.4f %.4f\n", stage, sc.block, sc.tile,
                   sc.blocks_per_cu, sc.lookahead, times.front(), times[times.size() / 2],
                   times.back());
    return times[times.size() / 2];
  };
  // stage 1: every candidate, median of 3; stage 2: the six fastest again, median of 31
  const int blocks[] = {256, 512};
  const int per_lane[] = {8, 16, 32};
  const int bpcs[] = {1, 2, 3, 4, 8};
  const int looks[] = {2, 4, 8};
  std::vector<std::pair<float, vgicp_schedule>> ranked;
  for (int blk : blocks)
    for (int pl : per_lane)
      for (int bpc : bpcs)
        for (int la : looks) {
          vgicp_schedule sc{blk, blk * pl, bpc, la};
          if (!valid_schedule(sc)) continue;
          const float t = time_schedule(sc, 3, 1);
          if (t >= 0.0f) ranked.push_back({t, sc});
        }
  std::stable_sort(ranked.begin(), ranked.end(),
                   [](const std::pair<float, vgicp_schedule>& a,
                      const std::pair<float, vgicp_schedule>& c) { return a.first < c.first; });
  float best_ms = 1e30f;
  for (size_t i = 0; i < ranked.size() && i < 6; ++i) {
    const float t = time_schedule(ranked[i].second, 31, 2);
    if (t >= 0.0f && t < best_ms) {
      best_ms = t;
      best = ranked[i].second;
    }
  }
  if (tlog) std::fclose(tlog);
  (void)hipStreamSynchronize(s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(H);
  (void)hipFree(bb);
  (void)hipFree(err);
  (void)hipFree(nin);
  if ((e = hipGetLastError())) return hip_fail(e, "autotune launches");
  if ((st = apply_schedule(batch, best)) != VGICP_OK) return st;
  if (chosen) *chosen = best;
  if (cache_path) {
    auto m = read_cache(cache_path);
    m[key] = {best.block, best.tile, best.blocks_per_cu, best.lookahead};
    write_cache(cache_path, m);
  }
  return VGICP_OK;
}

}  // namespace

extern "C" {

VGICP_API vgicp_status vgicp_batch_destroy(vgicp_batch batch) {
  if (!batch) return VGICP_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != batch->device) (void)hipSetDevice(batch->device);
  (void)hipDeviceSynchronize();
  batch->drop_graphs();
  if (batch->capture_stream) (void)hipStreamDestroy(batch->capture_stream);
  if (batch->done) (void)hipEventDestroy(batch->done);
  (void)hipFree(batch->d_factors);
  (void)hipFree(batch->d_boxes);
  (void)hipFree(batch->d_rel);
  (void)hipFree(batch->d_items);
  (void)hipFree(batch->d_seg);
  (void)hipFree(batch->d_heads);
  (void)hipFree(batch->d_partials);
  (void)hipFree(batch->d_cov6);
  (void)hipFree(batch->d_xyz);
  (void)hipFree(batch->d_perm);
  for (void* p : {(void*)batch->d_gpts, (void*)batch->d_gf, (void*)batch->d_gbptr,
                  (void*)batch->d_gbcontrib, (void*)batch->d_cptr, (void*)batch->d_cfac,
                  (void*)batch->d_cloud_n, (void*)batch->d_cloud_off, (void*)batch->d_gout})
    (void)hipFree(p);
  if (batch->h_gout) (void)hipHostFree(batch->h_gout);
  free_lm(batch);
  if (cur != batch->device) (void)hipSetDevice(cur);
  delete batch;
  return VGICP_OK;
}

VGICP_API vgicp_status vgicp_linearize_batched(const vgicp_voxelmap* maps, int32_t n_maps,
                                               const vgicp_cloud* clouds, int32_t n_clouds,
                                               const double* poses, int32_t n_poses,
                                               const vgicp_factor* factors, int32_t n_factors,
                                               vgicp_precision precision, double* H, double* b,
                                               double* err, int64_t* inliers,
                                               vgicp_stream stream) {
  vgicp_batch bt = nullptr;
  vgicp_status st =
      vgicp_batch_create(maps, n_maps, clouds, n_clouds, factors, n_factors, n_poses, &bt);
  if (st != VGICP_OK) return st;
  st = vgicp_batch_linearize(bt, poses, precision, H, b, err, inliers, stream);
  hipError_t e = hipStreamSynchronize(stream_of(stream));
  vgicp_batch_destroy(bt);
  if (st != VGICP_OK) return st;
  if (e) return hip_fail(e, "hipStreamSynchronize");
  return VGICP_OK;
}

}  // extern "C"
