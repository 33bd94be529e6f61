// Types shared by the host runtime and the gfx950 kernels of the VGICP library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vgicp {

constexpr long long kKeyLimit = 1LL << 20;  // |voxel coordinate| < 2^20
constexpr long long kEmptyKey = -1;         // packed keys are non-negative
constexpr int kNumAcc = 28;                 // target-frame sums per factor (see PointSums)
constexpr int kPartialStride = 29;          // kNumAcc values + inlier count, per work item
constexpr int kNumXcd = 8;                  // XCDs of an MI355X; blocks are dealt round-robin

enum DevFlag : unsigned { kFlagNonFinite = 1u, kFlagKeyRange = 2u, kFlagInternal = 4u };

enum Precision : int { kAccFp64 = 0, kAccKahan = 1, kNaiveWorld = 2, kMathFp64 = 3 };

// One voxel of a map, stored in its open-addressing slot: a hit costs one 64-byte line.
struct alignas(64) VoxelRec {
  long long key;   // packed voxel key, kEmptyKey for a free slot
  double mean[3];  // FP64 mean of the member points
  float cov[6];    // mean of the member covariances (xx xy xz yy yz zz), rounded to FP32
  int id;          // canonical voxel id (rank of the key)
  int count;       // member points
};
static_assert(sizeof(VoxelRec) == 64, "VoxelRec must fill one 64-byte line");

// What a kernel needs to know about a voxel map.
struct MapView {
  const VoxelRec* table;  // [mask + 1]
  unsigned mask;          // capacity - 1 (capacity is a power of two, >= 2 V)
  int pow2;               // 1 when res is a power of two: v * inv_res == v / res exactly
  double res;
  double inv_res;
  const double* mean;     // canonical order [3][V]
  const float* cov;       // canonical order [6][V]
  long long V;
};

// Relative pose T_ts = T_t^-1 T_s of one factor, in the forms the kernels use.
struct RelPose {
  double R[9];   // row-major, FP64 (fixed evaluation order)
  double t[3];
  float Rf[9];   // rounded copies for FP32 per-point math
  float tf[3];
  // world-coordinate FP32 form (precision baseline): source-to-world and world-to-target
  float Rs[9], ts[3];   // T_s
  float Rti[9], tti[3]; // T_t^-1
};

// One factor of a batch as the persistent kernel sees it.
struct FactorView {
  MapView map;
  const float* xyz;     // [3][n]
  const float* cov;     // [6][n]
  long long n;
  int binary;
  int tile_base;        // index of the factor's first work item in canonical (factor) order
  int ntiles;
  int target_pose;
  int source_pose;
};

struct WorkItem {
  int factor;
  int tile;
};

}  // namespace vgicp
