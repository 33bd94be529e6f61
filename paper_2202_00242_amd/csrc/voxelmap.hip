// Voxel map of a target cloud (Sec. III-A): every voxel holds the arithmetic mean of its
// member points' means and covariances. Deterministic GPU build:
//   1. FP64 voxel coordinates of every point, range and finiteness checks, coordinate bounds;
//   2. a dense sort key (the coordinates relative to their minimum, packed with just enough
//      bits per axis so that key order is lexicographic (x, y, z) order);
//   3. a stable LSD radix sort of (key, point index) - members of a voxel stay in increasing
//      point index;
//   4. segment heads and an exclusive scan: voxel id = rank of the key (canonical, independent
//      of point order and of the hash layout);
//   5. per voxel, FP64 sums in increasing point index -> mean and covariance;
//   6. the voxel Gaussians in id order (80-byte records) and a lookup structure: occupancy
//      bricks of 4 x 4 x 2 voxels over the map's voxel bounding box (with a copy of the records
//      in brick order) when the box is moderate, else an open-addressing table of {key, id} slots (capacity a power of two >= 4 V,
//      linear probing), the key relative to the bounding box and 32-bit whenever the box needs
//      at most 31 bits.
#include <algorithm>
#include <cmath>
#include <vector>

#include "device_math.h"
#include "internal.h"

namespace vgicp {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 8;
constexpr int kTile = kBlock * kItems;  // elements per block in scans and radix passes
constexpr long long kGridMaxBricks = 1LL << 24;   // 128 MiB of brick records (24-bit indexing)
constexpr long long kGridAutoBricks = 1LL << 23;  // 64 MiB of brick records

// ------------------------------------------------------------------ step 1: coordinates

__global__ __launch_bounds__(kBlock) void coords_kernel(const float* __restrict__ xyz,
                                                        const float* __restrict__ cov,
                                                        long long n, int pow2, double res,
                                                        double inv_res, int* __restrict__ kc,
                                                        int* __restrict__ bounds,
                                                        unsigned* __restrict__ flags) {
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
  unsigned fl = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    for (int a = 0; a < 6; ++a)
      if (!isfinite(cov[a * n + i])) fl |= kFlagNonFinite;
    for (int a = 0; a < 3; ++a) {
      int k = 0;
      const int st = pow2 ? voxel_coord<false>((double)xyz[a * n + i], res, inv_res, &k)
                          : voxel_coord<true>((double)xyz[a * n + i], res, inv_res, &k);
      if (st == 1) fl |= kFlagNonFinite;
      if (st == 2) fl |= kFlagKeyRange;
      kc[a * n + i] = k;
      lo[a] = min(lo[a], k);
      hi[a] = max(hi[a], k);
    }
  }
  for (int a = 0; a < 3; ++a) {
    for (int off = 32; off > 0; off >>= 1) {
      lo[a] = min(lo[a], __shfl_xor(lo[a], off, 64));
      hi[a] = max(hi[a], __shfl_xor(hi[a], off, 64));
    }
  }
  // one set of atomics per block: same-address atomics from every wave serialize in L2
  __shared__ int red[6][kBlock / 64];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 3; ++a) {
      red[a][w] = lo[a];
      red[3 + a][w] = hi[a];
    }
  if (fl) atomicOr(flags, fl);
  __syncthreads();
  if (threadIdx.x < 6) {
    int v = red[threadIdx.x][0];
    for (int ww = 1; ww < kBlock / 64; ++ww)
      v = threadIdx.x < 3 ? min(v, red[threadIdx.x][ww]) : max(v, red[threadIdx.x][ww]);
    if (threadIdx.x < 3)
      atomicMin(&bounds[threadIdx.x], v);
    else
      atomicMax(&bounds[threadIdx.x], v);
  }
}

__global__ void bounds_init_kernel(int* bounds, unsigned* flags) {
  if (threadIdx.x < 3) {
    bounds[threadIdx.x] = INT_MAX;
    bounds[3 + threadIdx.x] = INT_MIN;
  }
  if (threadIdx.x == 0) *flags = 0u;
}

// ------------------------------------------------------------------ step 2: sort keys

__global__ __launch_bounds__(kBlock) void sortkey_kernel(const int* __restrict__ kc, long long n,
                                                         int lx, int ly, int lz, int by, int bz,
                                                         unsigned long long* __restrict__ key,
                                                         int* __restrict__ val) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long x = (unsigned long long)(kc[i] - lx);
    const unsigned long long y = (unsigned long long)(kc[n + i] - ly);
    const unsigned long long z = (unsigned long long)(kc[2 * n + i] - lz);
    key[i] = (x << (by + bz)) | (y << bz) | z;
    val[i] = (int)i;
  }
}

// ------------------------------------------------------------------ exclusive scan (int)

// Block-wide exclusive scan of kTile ints (thread t owns elements t*kItems..t*kItems+7 of the
// tile); in and out may be the same array. Writes each block's total to block_sums when it is
// not null.
__global__ __launch_bounds__(kBlock) void scan_tile_kernel(const int* in, int* out, long long n,
                                                           int* __restrict__ block_sums) {
  __shared__ int wsum[kBlock / 64];
  const long long base = (long long)blockIdx.x * kTile + (long long)threadIdx.x * kItems;
  int v[kItems];
  int run = 0;
  for (int k = 0; k < kItems; ++k) {
    const long long i = base + k;
    v[k] = (i < n) ? in[i] : 0;
    run += v[k];
  }
  // inclusive scan of thread totals within the wave
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = run;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int before = 0;
  for (int k = 0; k < w; ++k) before += wsum[k];
  int excl = before + x - run;
  for (int k = 0; k < kItems; ++k) {
    const long long i = base + k;
    if (i < n) out[i] = excl;
    excl += v[k];
  }
  if (block_sums && threadIdx.x == kBlock - 1) block_sums[blockIdx.x] = before + x;
}

__global__ __launch_bounds__(kBlock) void scan_add_kernel(int* __restrict__ out, long long n,
                                                          const int* __restrict__ offs) {
  const long long base = (long long)blockIdx.x * kTile;
  const int o = offs[blockIdx.x];
  for (int k = threadIdx.x; k < kTile; k += kBlock) {
    const long long i = base + k;
    if (i < n) out[i] += o;
  }
}

// Exclusive scan of n ints (in -> out, may alias), recursive over block totals.
hipError_t exclusive_scan(const int* in, int* out, long long n, hipStream_t s, Scratch& sc) {
  if (n <= 0) return hipSuccess;
  const long long nb = (n + kTile - 1) / kTile;
  if (nb == 1) {
    scan_tile_kernel<<<1, kBlock, 0, s>>>(in, out, n, nullptr);
    return hipGetLastError();
  }
  int* sums = nullptr;
  hipError_t e = sc.alloc(&sums, (size_t)nb);
  if (e != hipSuccess) return e;
  scan_tile_kernel<<<(unsigned)nb, kBlock, 0, s>>>(in, out, n, sums);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = exclusive_scan(sums, sums, nb, s, sc)) != hipSuccess) return e;
  scan_add_kernel<<<(unsigned)nb, kBlock, 0, s>>>(out, n, sums);
  return hipGetLastError();
}

// ------------------------------------------------------------------ stable LSD radix sort

__global__ __launch_bounds__(kBlock) void radix_hist_kernel(
    const unsigned long long* __restrict__ key, long long n, int shift, int* __restrict__ hist,
    int ntiles) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kTile;
  for (int r = 0; r < kItems; ++r) {
    const long long i = base + r * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(int)((key[i] >> shift) & 255ull)], 1);
  }
  __syncthreads();
  hist[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Scatter of one 8-bit digit. The tile's items are visited in rounds r of kBlock consecutive
// elements; within a round, a lane's rank among equal digits comes from wave ballots and the
// per-wave counts of lower waves, so the output keeps input order among equal digits.
__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(
    const unsigned long long* __restrict__ kin, const int* __restrict__ vin,
    unsigned long long* __restrict__ kout, int* __restrict__ vout, long long n, int shift,
    const int* __restrict__ offsets, int ntiles, unsigned* __restrict__ flags) {
  __shared__ int running[256];
  __shared__ int wcount[kBlock / 64][256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  running[t] = offsets[t * ntiles + blockIdx.x];
  const long long base = (long long)blockIdx.x * kTile;
  const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  for (int r = 0; r < kItems; ++r) {
    for (int j = t; j < (kBlock / 64) * 256; j += kBlock) (&wcount[0][0])[j] = 0;
    __syncthreads();
    const long long i = base + r * kBlock + t;
    const bool valid = i < n;
    const unsigned long long k = valid ? kin[i] : 0ull;
    const int v = valid ? vin[i] : 0;
    const int dgt = (int)((k >> shift) & 255ull);
    unsigned long long peers = __ballot(valid);
    for (int bit = 0; bit < 8; ++bit) {
      const bool set = (dgt >> bit) & 1;
      const unsigned long long m = __ballot(set);
      peers &= set ? m : ~m;
    }
    const int rank = __popcll(peers & lt);
    if (valid && rank == 0) wcount[w][dgt] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int off = running[dgt] + rank;
      for (int ww = 0; ww < w; ++ww) off += wcount[ww][dgt];
      if (off >= 0 && off < n) {
        kout[off] = k;
        vout[off] = v;
      } else {
        atomicOr(flags, kFlagInternal);
      }
    }
    __syncthreads();
    int add = 0;
    for (int ww = 0; ww < kBlock / 64; ++ww) add += wcount[ww][t];
    running[t] += add;
    __syncthreads();
  }
}

// ------------------------------------------------------------------ steps 4-6

__global__ __launch_bounds__(kBlock) void heads_kernel(const unsigned long long* __restrict__ key,
                                                       long long n, int* __restrict__ head) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    head[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void seg_start_kernel(const int* __restrict__ head,
                                                           const int* __restrict__ vid,
                                                           long long n, int* __restrict__ start,
                                                           int V, unsigned* __restrict__ flags) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    if (head[i]) {
      const int v = vid[i];
      if (v >= 0 && v < V)
        start[v] = (int)i;
      else
        atomicOr(flags, kFlagInternal);
    }
  if (blockIdx.x == 0 && threadIdx.x == 0) start[V] = (int)n;
}

// One thread per voxel: FP64 sums over the members in increasing point index.
__global__ __launch_bounds__(kBlock) void stats_kernel(
    const float* __restrict__ xyz, const float* __restrict__ cov, long long n,
    const int* __restrict__ kc, const int* __restrict__ order,
    const unsigned long long* __restrict__ skey, const int* __restrict__ start, int V,
    long long* __restrict__ keys, unsigned* __restrict__ rkey, double* __restrict__ mean,
    double* __restrict__ vcov, int* __restrict__ count, VoxelData* __restrict__ vox,
    unsigned* __restrict__ flags) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int s = start[v], e = start[v + 1];
  if (!(s >= 0 && s < e && e <= n)) {
    atomicOr(flags, kFlagInternal);
    return;
  }
  double m0 = 0.0, m1 = 0.0, m2 = 0.0;
  double c[6] = {0, 0, 0, 0, 0, 0};
  for (int k = s; k < e; ++k) {
    const long long j = order[k];
    if (j < 0 || j >= n) {
      atomicOr(flags, kFlagInternal);
      return;
    }
    m0 += (double)xyz[j];
    m1 += (double)xyz[n + j];
    m2 += (double)xyz[2 * n + j];
    for (int a = 0; a < 6; ++a) c[a] += (double)cov[a * n + j];
  }
  const double cnt = (double)(e - s);
  const long long j0 = order[s];
  keys[v] = pack_key(kc[j0], kc[n + j0], kc[2 * n + j0]);
  rkey[v] = (unsigned)skey[s];
  VoxelData d;
  d.mean[0] = m0 / cnt;
  d.mean[1] = m1 / cnt;
  d.mean[2] = m2 / cnt;
  for (int a = 0; a < 6; ++a) d.cov[a] = c[a] / cnt;
  d.count = e - s;
  d.pad = 0;
  vox[v] = d;
  mean[v] = d.mean[0];
  mean[(long long)V + v] = d.mean[1];
  mean[2LL * V + v] = d.mean[2];
  for (int a = 0; a < 6; ++a) vcov[(long long)a * V + v] = d.cov[a];
  count[v] = e - s;
}

__global__ __launch_bounds__(kBlock) void slots32_init_kernel(uint2* __restrict__ t, long long cap) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cap;
       i += (long long)gridDim.x * blockDim.x)
    t[i] = make_uint2(kEmpty32, 0xffffffffu);
}

__global__ __launch_bounds__(kBlock) void slots64_init_kernel(longlong2* __restrict__ t,
                                                              long long cap) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cap;
       i += (long long)gridDim.x * blockDim.x) {
    longlong2 e;
    e.x = kEmpty64;
    e.y = -1;
    t[i] = e;
  }
}

// One thread per voxel; keys are distinct, so every insertion claims a fresh slot. The table
// keeps at least three quarters of its slots free, so the probe ends within capacity steps.
__global__ __launch_bounds__(kBlock) void insert32_kernel(const unsigned* __restrict__ rkey, int V,
                                                          uint2* __restrict__ t, unsigned mask) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const unsigned k = rkey[v];
  unsigned slot = hash32(k) & mask;
  for (unsigned p = 0; p <= mask; ++p) {
    if (atomicCAS(&t[slot].x, kEmpty32, k) == kEmpty32) {
      t[slot].y = (unsigned)v;
      return;
    }
    slot = (slot + 1) & mask;
  }
}

__global__ __launch_bounds__(kBlock) void insert64_kernel(const long long* __restrict__ keys, int V,
                                                          longlong2* __restrict__ t,
                                                          unsigned mask) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const long long k = keys[v];
  unsigned slot = hash64(k) & mask;
  for (unsigned p = 0; p <= mask; ++p) {
    unsigned long long* kp = reinterpret_cast<unsigned long long*>(&t[slot].x);
    if (atomicCAS(kp, (unsigned long long)kEmpty64, (unsigned long long)k) ==
        (unsigned long long)kEmpty64) {
      t[slot].y = v;
      return;
    }
    slot = (slot + 1) & mask;
  }
}

// Grid layout, step 1: one thread per voxel sets its bit in its brick's occupancy mask.
__device__ inline void voxel_box_coords(long long k, int lo0, int lo1, int lo2, unsigned& dx,
                                        unsigned& dy, unsigned& dz) {
  const int m21 = (1 << 21) - 1;
  dx = (unsigned)((int)((k >> 42) & m21) - (int)kKeyLimit - lo0);
  dy = (unsigned)((int)((k >> 21) & m21) - (int)kKeyLimit - lo1);
  dz = (unsigned)((int)(k & m21) - (int)kKeyLimit - lo2);
}

__global__ __launch_bounds__(kBlock) void brick_mark_kernel(const long long* __restrict__ keys,
                                                            int V, int lo0, int lo1, int lo2,
                                                            int gby, int gbz,
                                                            Brick* __restrict__ bricks) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  unsigned dx, dy, dz;
  voxel_box_coords(keys[v], lo0, lo1, lo2, dx, dy, dz);
  atomicOr(&bricks[brick_of(dx, dy, dz, (unsigned)gby, (unsigned)gbz)].mask,
           1u << bit_in_brick(dx, dy, dz));
}

// Step 2: occupied voxels per brick (then an exclusive scan gives each brick's base).
__global__ __launch_bounds__(kBlock) void brick_count_kernel(const Brick* __restrict__ bricks,
                                                             long long nb, int* __restrict__ cnt) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nb;
       i += (long long)gridDim.x * blockDim.x)
    cnt[i] = __popc(bricks[i].mask);
}

__global__ __launch_bounds__(kBlock) void brick_base_kernel(Brick* __restrict__ bricks,
                                                            long long nb,
                                                            const int* __restrict__ base) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nb;
       i += (long long)gridDim.x * blockDim.x)
    bricks[i].base = base[i];
}

// Step 3: one thread per voxel copies its record to its brick-ordered position.
__global__ __launch_bounds__(kBlock) void brick_place_kernel(
    const long long* __restrict__ keys, int V, int lo0, int lo1, int lo2, int gby, int gbz,
    const Brick* __restrict__ bricks, const VoxelData* __restrict__ vox,
    VoxelData* __restrict__ voxb, int* __restrict__ rec_id) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  unsigned dx, dy, dz;
  voxel_box_coords(keys[v], lo0, lo1, lo2, dx, dy, dz);
  const Brick br = bricks[brick_of(dx, dy, dz, (unsigned)gby, (unsigned)gbz)];
  const unsigned bit = bit_in_brick(dx, dy, dz);
  const int pos = br.base + __popc(br.mask & ((1u << bit) - 1u));
  voxb[pos] = vox[v];
  rec_id[pos] = v;
}

// ------------------------------------------------------------------ spatial order of a cloud

// Morton code of the point's cell (floor(v / cell) per axis, offset by 2^20 and clamped to 21
// bits; bits interleaved x, y, z from the lowest) and the point index.
__global__ __launch_bounds__(kBlock) void morton_kernel(const float* __restrict__ xyz, long long n,
                                                       double inv_cell,
                                                       unsigned long long* __restrict__ code,
                                                       int* __restrict__ idx) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    unsigned long long c = 0;
    for (int a = 0; a < 3; ++a) {
      double f = floor((double)xyz[a * n + i] * inv_cell) + (double)kKeyLimit;
      f = fmin(fmax(f, 0.0), (double)(2 * kKeyLimit - 1));  // NaN -> 0
      const unsigned long long k = (unsigned long long)f;
      for (int b = 0; b < 21; ++b) c |= ((k >> b) & 1ull) << (3 * b + a);
    }
    code[i] = c;
    idx[i] = (int)i;
  }
}

// Per block: min and max of every axis of a cloud, and whether a coordinate is not finite.
__global__ __launch_bounds__(kBlock) void cloud_bounds_kernel(const float* __restrict__ xyz,
                                                              long long n,
                                                              float* __restrict__ part,
                                                              unsigned* __restrict__ flags) {
  __shared__ float red[6][kBlock / 64];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  unsigned fl = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    for (int a = 0; a < 3; ++a) {
      const float v = xyz[a * n + i];
      if (!isfinite(v)) fl |= kFlagNonFinite;
      lo[a] = fminf(lo[a], v);
      hi[a] = fmaxf(hi[a], v);
    }
  for (int a = 0; a < 3; ++a)
    for (int off = 32; off > 0; off >>= 1) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], off, 64));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off, 64));
    }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 3; ++a) {
      red[a][w] = lo[a];
      red[3 + a][w] = hi[a];
    }
  if (fl) atomicOr(flags, fl);
  __syncthreads();
  if (threadIdx.x < 6) {
    float v = red[threadIdx.x][0];
    for (int ww = 1; ww < kBlock / 64; ++ww)
      v = threadIdx.x < 3 ? fminf(v, red[threadIdx.x][ww]) : fmaxf(v, red[threadIdx.x][ww]);
    part[blockIdx.x * 6 + threadIdx.x] = v;
  }
}

// Positions [3][n] and interleaved covariances [n][6] in the order perm.
__global__ __launch_bounds__(kBlock) void gather_cloud_kernel(
    const float* __restrict__ xyz, const float* __restrict__ cov, long long n,
    const int* __restrict__ perm, float* __restrict__ xyz_out, float* __restrict__ cov6_out,
    unsigned* __restrict__ flags) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long j = perm[i];
    if (j < 0 || j >= n) {
      atomicOr(flags, kFlagInternal);
      continue;
    }
    for (int a = 0; a < 3; ++a) xyz_out[a * n + i] = xyz[a * n + j];
    float2* o = reinterpret_cast<float2*>(cov6_out) + 3 * i;
    o[0] = make_float2(cov[j], cov[n + j]);
    o[1] = make_float2(cov[2 * n + j], cov[3 * n + j]);
    o[2] = make_float2(cov[4 * n + j], cov[5 * n + j]);
  }
}

int grid_for(long long n) {
  return (int)std::max<long long>(1, std::min<long long>((n + kBlock - 1) / kBlock, 65536));
}

int bits_for(long long span) {  // bits to hold values 0..span
  int b = 0;
  while ((1LL << b) <= span) ++b;
  return b;
}

}  // namespace

hipError_t scan_exclusive(const int* in, int* out, long long n, hipStream_t s, Scratch& sc) {
  return exclusive_scan(in, out, n, s, sc);
}

hipError_t radix_sort_pairs(unsigned long long** k, int** v, unsigned long long** kt, int** vt,
                            long long n, int bits, unsigned* flags, hipStream_t s, Scratch& sc) {
  if (n <= 0) return hipSuccess;
  const long long ntiles = (n + kTile - 1) / kTile;
  int* hist = nullptr;
  hipError_t e = sc.alloc(&hist, (size_t)(256 * ntiles));
  if (e != hipSuccess) return e;
  for (int shift = 0; shift < bits; shift += 8) {
    radix_hist_kernel<<<(unsigned)ntiles, kBlock, 0, s>>>(*k, n, shift, hist, (int)ntiles);
    if ((e = exclusive_scan(hist, hist, 256 * ntiles, s, sc)) != hipSuccess) return e;
    radix_scatter_kernel<<<(unsigned)ntiles, kBlock, 0, s>>>(*k, *v, *kt, *vt, n, shift, hist,
                                                             (int)ntiles, flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    std::swap(*k, *kt);
    std::swap(*v, *vt);
  }
  return hipSuccess;
}

vgicp_status spatial_copy(const float* xyz, const float* cov, int64_t n, double cell,
                          float* xyz_out, float* cov6_out, float* box, int* perm_out,
                          hipStream_t s) {
  for (int a = 0; a < 3; ++a) {
    box[a] = INFINITY;
    box[3 + a] = -INFINITY;
  }
  if (n <= 0) return VGICP_OK;
  Scratch sc;
  unsigned long long *kA = nullptr, *kB = nullptr;
  int *vA = nullptr, *vB = nullptr, *hist = nullptr;
  unsigned* flags = nullptr;
  const long long ntiles = (n + kTile - 1) / kTile;
  hipError_t e;
  if ((e = sc.alloc(&kA, (size_t)n)) || (e = sc.alloc(&kB, (size_t)n)) ||
      (e = sc.alloc(&vA, (size_t)n)) || (e = sc.alloc(&vB, (size_t)n)) ||
      (e = sc.alloc(&hist, (size_t)(256 * ntiles))) || (e = sc.alloc(&flags, 1)))
    return hip_fail(e, "hipMalloc (cloud order)");
  if ((e = hipMemsetAsync(flags, 0, sizeof(unsigned), s))) return hip_fail(e, "hipMemsetAsync");
  morton_kernel<<<grid_for(n), kBlock, 0, s>>>(xyz, n, 1.0 / cell, kA, vA);
  for (int shift = 0; shift < 63; shift += 8) {
    radix_hist_kernel<<<(unsigned)ntiles, kBlock, 0, s>>>(kA, n, shift, hist, (int)ntiles);
    if ((e = exclusive_scan(hist, hist, 256 * ntiles, s, sc)) != hipSuccess)
      return hip_fail(e, "radix scan (cloud order)");
    radix_scatter_kernel<<<(unsigned)ntiles, kBlock, 0, s>>>(kA, vA, kB, vB, n, shift, hist,
                                                             (int)ntiles, flags);
    std::swap(kA, kB);
    std::swap(vA, vB);
  }
  gather_cloud_kernel<<<grid_for(n), kBlock, 0, s>>>(xyz, cov, n, vA, xyz_out, cov6_out, flags);
  if (perm_out &&
      (e = hipMemcpyAsync(perm_out, vA, (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, s)))
    return hip_fail(e, "copy of the cloud order");
  const int nb = std::min(grid_for(n), 64);
  float* part = nullptr;
  unsigned* bflags = nullptr;
  if ((e = sc.alloc(&part, (size_t)nb * 6)) || (e = sc.alloc(&bflags, 1)) ||
      (e = hipMemsetAsync(bflags, 0, sizeof(unsigned), s)))
    return hip_fail(e, "cloud bounds scratch");
  cloud_bounds_kernel<<<nb, kBlock, 0, s>>>(xyz, n, part, bflags);
  std::vector<float> hp((size_t)nb * 6);
  unsigned hf = 0, hb = 0;
  if ((e = hipGetLastError()) ||
      (e = hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s)) ||
      (e = hipMemcpyAsync(&hb, bflags, sizeof(hb), hipMemcpyDeviceToHost, s)) ||
      (e = hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(float), hipMemcpyDeviceToHost, s)) ||
      (e = hipStreamSynchronize(s)))
    return hip_fail(e, "cloud order");
  if (hf) return fail(VGICP_E_HIP, "internal error in the cloud order");
  for (int b = 0; b < nb; ++b)
    for (int a = 0; a < 3; ++a) {
      box[a] = std::min(box[a], hp[6 * b + a]);
      box[3 + a] = std::max(box[3 + a], hp[6 * b + 3 + a]);
    }
  if (hb)  // a non-finite coordinate: never skipped, so the kernels report it
    for (int a = 0; a < 3; ++a) {
      box[a] = -INFINITY;
      box[3 + a] = INFINITY;
    }
  return VGICP_OK;
}

vgicp_status build_voxelmap(const float* xyz, const float* cov, int64_t n, double res,
                            int layout, hipStream_t s, vgicp_voxelmap* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  auto* m = new vgicp_voxelmap_s;
  m->device = dev;
  m->res = res;
  m->inv_res = 1.0 / res;
  int ex = 0;
  m->pow2 = (std::frexp(res, &ex) == 0.5) ? 1 : 0;
  Scratch sc;
  auto cleanup = [&](vgicp_status st) {
    destroy_voxelmap(m);
    return st;
  };
  int* kc = nullptr;
  int* bounds = nullptr;
  unsigned* flags = nullptr;  // the map build's own error word (the sticky one is not touched)
  if ((e = sc.alloc(&kc, 3 * (size_t)n)) != hipSuccess ||
      (e = sc.alloc(&bounds, 6)) != hipSuccess || (e = sc.alloc(&flags, 1)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMalloc (voxel map scratch)"));
  bounds_init_kernel<<<1, 64, 0, s>>>(bounds, flags);
  if (n > 0)
    coords_kernel<<<std::min(grid_for(n), 128), kBlock, 0, s>>>(xyz, cov, n, m->pow2, res, m->inv_res, kc,
                                                 bounds, flags);
  int hb[6];
  unsigned hf = 0;
  if ((e = hipGetLastError()) != hipSuccess ||
      (e = hipMemcpyAsync(hb, bounds, sizeof(hb), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return cleanup(hip_fail(e, "voxel coordinates"));
  if (hf) {
    if (hf & kFlagNonFinite) return cleanup(fail(VGICP_E_NONFINITE, "non-finite map point"));
    return cleanup(fail(VGICP_E_KEY_RANGE, "map point outside the voxel key range |k| < 2^20"));
  }

  long long V = 0;
  int* order = nullptr;  // point index in key order
  unsigned long long* keyA = nullptr;
  unsigned* rkey = nullptr;
  int bits = 0;
  if (n > 0) {
    const int bx = bits_for((long long)hb[3] - hb[0]);
    const int by = bits_for((long long)hb[4] - hb[1]);
    const int bz = bits_for((long long)hb[5] - hb[2]);
    bits = bx + by + bz;  // <= 63
    for (int a = 0; a < 3; ++a) {
      m->lo[a] = hb[a];
      m->ext[a] = hb[3 + a] - hb[a] + 1;
    }
    m->by = by;
    m->bz = bz;
    m->key32 = bits <= 31;
    unsigned long long* keyB = nullptr;
    int *valA = nullptr, *valB = nullptr;
    if ((e = sc.alloc(&keyA, (size_t)n)) != hipSuccess ||
        (e = sc.alloc(&keyB, (size_t)n)) != hipSuccess ||
        (e = sc.alloc(&valA, (size_t)n)) != hipSuccess ||
        (e = sc.alloc(&valB, (size_t)n)) != hipSuccess)
      return cleanup(hip_fail(e, "hipMalloc (sort buffers)"));
    sortkey_kernel<<<grid_for(n), kBlock, 0, s>>>(kc, n, hb[0], hb[1], hb[2], by, bz, keyA,
                                                  valA);
    const long long ntiles = (n + kTile - 1) / kTile;
    if (ntiles * 256 >= (1LL << 31))
      return cleanup(fail(VGICP_E_CAPACITY, "map too large for the 32-bit sort offsets"));
    int* hist = nullptr;
    if ((e = sc.alloc(&hist, (size_t)(256 * ntiles))) != hipSuccess)
      return cleanup(hip_fail(e, "hipMalloc (histograms)"));
    for (int shift = 0; shift < bits; shift += 8) {
      radix_hist_kernel<<<(unsigned)ntiles, kBlock, 0, s>>>(keyA, n, shift, hist, (int)ntiles);
      if ((e = exclusive_scan(hist, hist, 256 * ntiles, s, sc)) != hipSuccess)
        return cleanup(hip_fail(e, "radix scan"));
      radix_scatter_kernel<<<(unsigned)ntiles, kBlock, 0, s>>>(keyA, valA, keyB, valB, n,
                                                               shift, hist, (int)ntiles, flags);
      std::swap(keyA, keyB);
      std::swap(valA, valB);
    }
    order = valA;
    int *head = nullptr, *vid = nullptr;
    if ((e = sc.alloc(&head, (size_t)n)) != hipSuccess ||
        (e = sc.alloc(&vid, (size_t)n)) != hipSuccess)
      return cleanup(hip_fail(e, "hipMalloc (segments)"));
    heads_kernel<<<grid_for(n), kBlock, 0, s>>>(keyA, n, head);
    if ((e = exclusive_scan(head, vid, n, s, sc)) != hipSuccess)
      return cleanup(hip_fail(e, "segment scan"));
    int last[2] = {0, 0};
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(&last[0], vid + (n - 1), sizeof(int), hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(&last[1], head + (n - 1), sizeof(int), hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return cleanup(hip_fail(e, "voxel count"));
    V = (long long)last[0] + last[1];
    if (V <= 0 || V > n) return cleanup(fail(VGICP_E_HIP, "internal error: voxel count"));
    int* start = nullptr;
    if ((e = sc.alloc(&start, (size_t)V + 1)) != hipSuccess ||
        (e = sc.alloc(&rkey, (size_t)V)) != hipSuccess)
      return cleanup(hip_fail(e, "hipMalloc (segment starts)"));
    seg_start_kernel<<<grid_for(n), kBlock, 0, s>>>(head, vid, n, start, (int)V, flags);
    m->V = V;
    if ((e = hipMalloc(&m->keys, std::max<size_t>(V, 1) * sizeof(int64_t))) != hipSuccess ||
        (e = hipMalloc(&m->mean, std::max<size_t>(3 * V, 1) * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&m->cov, std::max<size_t>(6 * V, 1) * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&m->count, std::max<size_t>(V, 1) * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&m->vox, std::max<size_t>(V, 1) * sizeof(VoxelData))) != hipSuccess)
      return cleanup(fail(VGICP_E_OOM, "hipMalloc (voxel arrays)"));
    stats_kernel<<<(unsigned)((V + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        xyz, cov, n, kc, order, keyA, start, (int)V, reinterpret_cast<long long*>(m->keys), rkey,
        m->mean, m->cov, m->count, m->vox, flags);
  } else {
    if ((e = hipMalloc(&m->keys, sizeof(int64_t))) != hipSuccess ||
        (e = hipMalloc(&m->mean, sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&m->cov, sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&m->count, sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&m->vox, sizeof(VoxelData))) != hipSuccess)
      return cleanup(fail(VGICP_E_OOM, "hipMalloc (voxel arrays)"));
  }
  // Grid layout: occupancy bricks of 4 x 4 x 2 voxels over the bounding box. The automatic
  // choice takes it while it needs at most kGridAutoBricks bricks or 32 per voxel; else the
  // hash table.
  const long long gbx = ((long long)m->ext[0] + 3) / 4, gby = ((long long)m->ext[1] + 3) / 4,
                  gbz = ((long long)m->ext[2] + 1) / 2;
  const long long nb = (n > 0) ? gbx * gby * gbz : 0;
  bool use_grid = false;
  if (layout == VGICP_LAYOUT_GRID) {
    if (nb > kGridMaxBricks)
      return cleanup(fail(VGICP_E_CAPACITY, "voxel grid above 2^24 bricks; use the hash layout"));
    use_grid = true;
  } else if (layout == VGICP_LAYOUT_AUTO) {
    use_grid = nb <= kGridMaxBricks && (nb <= kGridAutoBricks || nb <= 32 * V);
  }
  if (use_grid) {
    m->layout = kLayoutGrid;
    m->gby = (int)gby;
    m->gbz = (int)gbz;
    m->nbricks = std::max<long long>(nb, 1);
    int* cnt = nullptr;
    if ((e = hipMalloc(&m->bricks, (size_t)m->nbricks * sizeof(Brick))) != hipSuccess ||
        (e = hipMalloc(&m->voxb, std::max<size_t>(V, 1) * sizeof(VoxelData))) != hipSuccess ||
        (e = hipMalloc(&m->rec_id, std::max<size_t>(V, 1) * sizeof(int))) != hipSuccess)
      return cleanup(fail(VGICP_E_OOM, "hipMalloc (voxel grid)"));
    if ((e = sc.alloc(&cnt, (size_t)m->nbricks)) != hipSuccess ||
        (e = hipMemsetAsync(m->bricks, 0, (size_t)m->nbricks * sizeof(Brick), s)) != hipSuccess)
      return cleanup(hip_fail(e, "voxel grid scratch"));
    if (V > 0) {
      const unsigned vb = (unsigned)((V + kBlock - 1) / kBlock);
      const long long* keys = reinterpret_cast<const long long*>(m->keys);
      brick_mark_kernel<<<vb, kBlock, 0, s>>>(keys, (int)V, m->lo[0], m->lo[1], m->lo[2],
                                               (int)gby, (int)gbz, m->bricks);
      brick_count_kernel<<<grid_for(nb), kBlock, 0, s>>>(m->bricks, nb, cnt);
      if ((e = exclusive_scan(cnt, cnt, nb, s, sc)) != hipSuccess)
        return cleanup(hip_fail(e, "brick scan"));
      brick_base_kernel<<<grid_for(nb), kBlock, 0, s>>>(m->bricks, nb, cnt);
      brick_place_kernel<<<vb, kBlock, 0, s>>>(keys, (int)V, m->lo[0], m->lo[1], m->lo[2],
                                                (int)gby, (int)gbz, m->bricks, m->vox, m->voxb,
                                                m->rec_id);
    }
  } else {
    m->layout = m->key32 ? kLayoutHash32 : kLayoutHash64;
  }
  long long cap = 16;
  while (cap < 4 * V) cap <<= 1;
  if (cap > (1LL << 31)) return cleanup(fail(VGICP_E_CAPACITY, "voxel table above 2^31 slots"));
  m->cap = use_grid ? 0 : cap;
  if (use_grid) {
    // no table: the grid resolves every key
  } else if (m->key32) {
    if ((e = hipMalloc(&m->slots32, (size_t)cap * sizeof(uint2))) != hipSuccess)
      return cleanup(fail(VGICP_E_OOM, "hipMalloc (voxel table)"));
    slots32_init_kernel<<<grid_for(cap), kBlock, 0, s>>>(m->slots32, cap);
    if (V > 0)
      insert32_kernel<<<(unsigned)((V + kBlock - 1) / kBlock), kBlock, 0, s>>>(
          rkey, (int)V, m->slots32, (unsigned)(cap - 1));
  } else {
    if ((e = hipMalloc(&m->slots64, (size_t)cap * sizeof(longlong2))) != hipSuccess)
      return cleanup(fail(VGICP_E_OOM, "hipMalloc (voxel table)"));
    slots64_init_kernel<<<grid_for(cap), kBlock, 0, s>>>(m->slots64, cap);
    if (V > 0)
      insert64_kernel<<<(unsigned)((V + kBlock - 1) / kBlock), kBlock, 0, s>>>(
          reinterpret_cast<const long long*>(m->keys), (int)V, m->slots64, (unsigned)(cap - 1));
  }
  if ((e = hipGetLastError()) != hipSuccess ||
      (e = hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return cleanup(hip_fail(e, "voxel table"));
  if (hf & kFlagInternal) return cleanup(fail(VGICP_E_HIP, "internal error in the voxel map build"));
  *out = m;
  return VGICP_OK;
}

void destroy_voxelmap(vgicp_voxelmap m) {
  if (!m) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != m->device) (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(m->bricks);
  (void)hipFree(m->voxb);
  (void)hipFree(m->rec_id);
  (void)hipFree(m->slots32);
  (void)hipFree(m->slots64);
  (void)hipFree(m->vox);
  (void)hipFree(m->keys);
  (void)hipFree(m->mean);
  (void)hipFree(m->cov);
  (void)hipFree(m->count);
  if (cur != m->device) (void)hipSetDevice(cur);
  delete m;
}

}  // namespace vgicp
