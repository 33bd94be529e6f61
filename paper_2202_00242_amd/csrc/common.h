// Types shared by the host runtime and the gfx950 kernels of the VGICP library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vgicp {

constexpr long long kKeyLimit = 1LL << 20;  // |voxel coordinate| < 2^20
constexpr unsigned kEmpty32 = 0xffffffffu;  // free slot of a 32-bit-key table
constexpr long long kEmpty64 = -1;          // free slot of a 64-bit-key table
constexpr int kNumAcc = 28;                 // target-frame sums per factor (see device_math.h)
constexpr int kPartialStride = 29;          // kNumAcc values + inlier count, per work item
constexpr int kNumXcd = 8;                  // XCDs of an MI355X; blocks are dealt round-robin
constexpr int kNoAllocMaxTiles = 4096;      // tiles of the allocation-free single-factor call
constexpr int kMaxPointsPerLane = 32;       // tile <= 32 * block (bounds FP32 lane sums)
constexpr long long kMaxCloudPoints = 1LL << 30;  // per cloud: 32-bit byte offsets per plane
// Word 3 of a raw (untyped, stride 0) buffer descriptor on gfx9-family GPUs: 32-bit data
// format, so range checking is in bytes against num_records.
constexpr int kRawBufferFlags = 0x00020000;

// Lookup structure of a voxel map.
enum Layout : int { kLayoutGrid = 0, kLayoutHash32 = 1, kLayoutHash64 = 2 };

// Grid layout: the map's voxel bounding box is cut into bricks of 4 x 4 x 2 voxels, stored
// x-major. A brick is one 8-byte record: the occupancy mask (bit ((x&3)<<3)|((y&3)<<1)|(z&1)
// for the voxel at (x, y, z) relative to the box) and the position of its first occupied
// voxel in the brick-ordered voxel records; the voxel with mask bit j sits at
// base + popcount(mask & (2^j - 1)).
struct alignas(8) Brick {
  unsigned mask;
  int base;
};

enum DevFlag : unsigned { kFlagNonFinite = 1u, kFlagKeyRange = 2u, kFlagInternal = 4u };

// The four public precision forms, and an internal count-only mode (FP64 keys, no inlier
// arithmetic) for overlap rates.
enum Precision : int { kAccFp64 = 0, kAccKahan = 1, kNaiveWorld = 2, kMathFp64 = 3, kCountOnly = 4 };

// Gaussian of one voxel, in voxel-id (canonical) order. Both moments stay FP64: a plane-like
// voxel covariance has entries ~1e-2 m^2 and a smallest eigenvalue ~1e-5 m^2, which FP32
// rounding of the entries would perturb by ~1e-4 relative.
struct alignas(16) VoxelData {
  double mean[3];  // mean of the member points
  double cov[6];   // mean of the member covariances (xx xy xz yy yz zz)
  int count;
  int pad;
};
static_assert(sizeof(VoxelData) == 80, "VoxelData is five 16-byte words");

// What a kernel needs to know about a voxel map. Voxel coordinates k are first tested
// against the map's bounding box [lo, lo + ext). Inside it, one of three structures gives the
// voxel id:
//  * grid: occupancy bricks over the box (one 16-byte load per point); the lookup gives a
//      position in the brick-ordered records, rec_id maps it back to the voxel id;
//  * hash32: an open-addressing table of {rk, id} pairs (8 bytes) keyed by the relative key
//      rk = ((kx - lo0) << (by + bz)) | ((ky - lo1) << bz) | (kz - lo2)  (rk fits in 31 bits);
//  * hash64: the same with {packed absolute key, id} pairs (16 bytes).
struct MapView {
  const Brick* bricks;        // [gbx * gby * gbz] or nullptr
  unsigned brick_bytes;       // gbx * gby * gbz * sizeof(Brick) (< 2^28)
  const uint2* slots32;       // [mask + 1] or nullptr
  const longlong2* slots64;   // [mask + 1] or nullptr
  int gby, gbz;               // bricks along y and z
  unsigned mask;              // capacity - 1 (capacity is a power of two, >= 4 V)
  int pow2;                   // 1 when res is a power of two: v * inv_res == v / res exactly
  double res;
  double inv_res;
  int lo[3];
  int ext[3];
  int by, bz;
  const VoxelData* vox;       // [V] in voxel-id order
  const VoxelData* rec;       // [V] in the order lookups return: brick order (grid) or id order
  const int* rec_id;          // [V] voxel id of each record (grid), nullptr when rec == vox
  long long V;
};

// Relative pose T_ts = T_t^-1 T_s of one factor, in the forms the kernels use.
// Right Jacobians of the two pose tangents at which a backward pass is evaluated: the
// right-perturbation gradient g at T Exp(xi) becomes the tangent-coordinate gradient J^T g.
// use = 0: identity (xi = 0).
struct TangentMap {
  double Js[36];  // source, row-major 6x6
  double Jt[36];  // target
  int use;
};

struct RelPose {
  double R[9];   // row-major, FP64 (fixed evaluation order)
  double t[3];
  double Rk[9];  // R and t times 1/res of the target map: when res is a power of two the
  double tk[3];  // same transform order gives q / res exactly (scaling by 2^j is exact)
  float Rf[9];   // rounded copies for FP32 per-point math
  float tf[3];
  // world-coordinate FP32 form (precision baseline): source-to-world and world-to-target
  float Rs[9], ts[3];   // T_s
  float Rti[9], tti[3]; // T_t^-1
  int skip;             // the source's bounding box misses the map's voxels: no inlier possible
};

// One factor of a batch as the persistent kernel sees it.
struct FactorView {
  MapView map;
  const float* xyz;     // [3][n] (the batch's copy, in spatial order)
  const float* cov6;    // [n][6] (the batch's interleaved copy, same order)
  long long n;
  int binary;
  int tile_base;        // index of the factor's first work item in canonical (factor) order
  int ntiles;
  int target_pose;
  int source_pose;
  int source_cloud;     // index of the source's bounding box
  long long gbase;      // first point of the factor in the batch's point-gradient rows
};

struct WorkItem {
  int factor;
  int tile;
};

}  // namespace vgicp
