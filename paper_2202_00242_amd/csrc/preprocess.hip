// Preprocessing of Sec. III-C on the GPU:
//   * voxel-grid filter: one output point per voxel, the FP64 mean of its members' positions
//     (and timestamps); with timestamps, a cell's points are taken in time order and a point
//     whose timestamp leaves the running mean timestamp of the cell's current voxel by more than
//     a tenth of the scan duration starts a new voxel of that cell, so that the first and last
//     points of a sweep do not fuse;
//   * the k nearest neighbours of every point (exact, ties by the lower index): uniform grid of
//     power-of-two cells over the Morton-sorted cloud, a hash of the occupied cells, and per
//     point a search over growing cubic shells of cells that stops once the k-th distance is
//     below the distance to the unsearched space;
//   * the point covariances C_k of Sec. III-A from those neighbours, plane-regularized as in
//     GICP (the eigenvalues of the neighbours' scatter replaced by scale * (1, 1, eps)).
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "device_math.h"
#include "internal.h"

namespace vgicp {
namespace {

constexpr int kBlock = 256;
constexpr unsigned long long kEmptyCell = ~0ull;

int grid_for(long long n) {
  return (int)std::max<long long>(1, std::min<long long>((n + kBlock - 1) / kBlock, 65536));
}

int bits_for(long long span) {  // bits to hold values 0..span
  int b = 0;
  while ((1LL << b) <= span) ++b;
  return b;
}

__global__ void bounds_reset_kernel(int* bounds, unsigned* flags) {
  if (threadIdx.x < 3) {
    bounds[threadIdx.x] = INT_MAX;
    bounds[3 + threadIdx.x] = INT_MIN;
  }
  if (threadIdx.x == 0) *flags = 0u;
}

// ------------------------------------------------------------------ voxel-grid filter

// Cells floor(p / res) per axis in FP64 (a multiply for a power-of-two res, where it is exact),
// their bounds, and the finiteness / range checks of positions and timestamps.
__global__ __launch_bounds__(kBlock) void ds_cells_kernel(const float* __restrict__ xyz,
                                                          const float* __restrict__ t,
                                                          long long n, int pow2, double res,
                                                          double inv_res, int* __restrict__ kc,
                                                          int* __restrict__ bounds,
                                                          unsigned* __restrict__ flags) {
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
  unsigned fl = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    if (t && !isfinite(t[i])) fl |= kFlagNonFinite;
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
  for (int a = 0; a < 3; ++a)
    for (int off = 32; off > 0; off >>= 1) {
      lo[a] = min(lo[a], __shfl_xor(lo[a], off, 64));
      hi[a] = max(hi[a], __shfl_xor(hi[a], off, 64));
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

// Sort key of a timestamp: its FP32 bits made monotone as unsigned (-0 counted as +0).
__global__ __launch_bounds__(kBlock) void ds_time_key_kernel(const float* __restrict__ t,
                                                             long long n,
                                                             unsigned long long* __restrict__ key,
                                                             int* __restrict__ idx) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    unsigned b = __float_as_uint(t[i] + 0.0f);
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    key[i] = b;
    idx[i] = (int)i;
  }
}

// Cell key of the point at each position of `order` (identity if null): coordinates relative to
// the bounds, packed x-major so that key order is (x, y, z) lexicographic order.
__global__ __launch_bounds__(kBlock) void ds_cell_key_kernel(const int* __restrict__ kc,
                                                             long long n,
                                                             const int* __restrict__ order,
                                                             int lx, int ly, int lz, int sy,
                                                             int sz,
                                                             unsigned long long* __restrict__ key,
                                                             int* __restrict__ val) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long j = order ? order[i] : i;
    key[i] = ((unsigned long long)(kc[j] - lx) << sy) |
             ((unsigned long long)(kc[n + j] - ly) << sz) |
             (unsigned long long)(kc[2 * n + j] - lz);
    val[i] = (int)j;
  }
}

// One thread per cell (its first sorted position) walks the cell's points in (time, index)
// order: the count pass stores the number of voxels at the cell's first position, the emit
// pass writes every voxel's means at the offsets of the scanned counts.
template <bool EMIT>
__global__ __launch_bounds__(kBlock) void ds_walk_kernel(
    const unsigned long long* __restrict__ key, const int* __restrict__ val, long long n,
    const float* __restrict__ xyz, const float* __restrict__ t, double thr,
    int* __restrict__ vcount, const int* __restrict__ voff, long long m, float* __restrict__ out,
    float* __restrict__ tout) {
#pragma clang fp contract(off)
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long k0 = key[i];
    if (i > 0 && key[i - 1] == k0) {
      if (!EMIT) vcount[i] = 0;
      continue;
    }
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, st = 0.0;
    int cnt = 0, nv = 0;
    const long long o = EMIT ? voff[i] : 0;
    for (long long j = i; j < n && key[j] == k0; ++j) {
      const long long p = val[j];
      const double tj = t ? (double)t[p] : 0.0;
      if (t && cnt > 0 && fabs(tj - st / (double)cnt) > thr) {
        if (EMIT && o + nv < m) {
          out[o + nv] = (float)(s0 / (double)cnt);
          out[m + o + nv] = (float)(s1 / (double)cnt);
          out[2 * m + o + nv] = (float)(s2 / (double)cnt);
          if (tout) tout[o + nv] = (float)(st / (double)cnt);
        }
        ++nv;
        s0 = s1 = s2 = st = 0.0;
        cnt = 0;
      }
      s0 = s0 + (double)xyz[p];
      s1 = s1 + (double)xyz[n + p];
      s2 = s2 + (double)xyz[2 * n + p];
      st = st + tj;
      ++cnt;
    }
    if (EMIT && o + nv < m) {
      out[o + nv] = (float)(s0 / (double)cnt);
      out[m + o + nv] = (float)(s1 / (double)cnt);
      out[2 * m + o + nv] = (float)(s2 / (double)cnt);
      if (tout) tout[o + nv] = (float)(st / (double)cnt);
    }
    ++nv;
    if (!EMIT) vcount[i] = nv;
  }
}

// ------------------------------------------------------------------ k nearest neighbours

struct CellSlot {
  unsigned long long key;  // Morton code of the cell, kEmptyCell if free
  int start, count;        // the cell's points in the sorted cloud
};

// The bits of x (21 at most) spread to every third bit.
__host__ __device__ inline unsigned long long spread3(unsigned long long x) {
  x &= 0x1fffffull;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

__device__ inline unsigned long long morton3(int x, int y, int z) {
  return spread3((unsigned)x) | (spread3((unsigned)y) << 1) | (spread3((unsigned)z) << 2);
}

__device__ inline unsigned cell_hash(unsigned long long k) {  // SplitMix64 finalizer
  k ^= k >> 30;
  k *= 0xbf58476d1ce4e5b9ull;
  k ^= k >> 27;
  k *= 0x94d049bb133111ebull;
  k ^= k >> 31;
  return (unsigned)k;
}

// Per block: min and max of every axis, and the finiteness check.
__global__ __launch_bounds__(kBlock) void knn_bounds_kernel(const float* __restrict__ xyz,
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

// Cell size estimate: for S sampled points (one block each), the binary exponent e of the
// squared distance at which the count of points reaches k; the k-th neighbour then lies within
// 2^((e + 1) / 2). est = INT_MAX if the cloud has fewer than k points, INT_MIN for duplicates.
constexpr int kExpBins = 128;
__global__ __launch_bounds__(kBlock) void knn_sample_kernel(const float* __restrict__ xyz,
                                                            long long n, int S, int k,
                                                            int* __restrict__ est) {
#pragma clang fp contract(off)
  __shared__ int hist[kExpBins];
  for (int b = threadIdx.x; b < kExpBins; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  const long long q = (long long)blockIdx.x * n / S;
  const double q0 = xyz[q], q1 = xyz[n + q], q2 = xyz[2 * n + q];
  for (long long j = threadIdx.x; j < n; j += blockDim.x) {
    const double dx = (double)xyz[j] - q0, dy = (double)xyz[n + j] - q1,
                 dz = (double)xyz[2 * n + j] - q2;
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    const int b = d2 > 0.0 ? min(max(ilogb(d2), -62), 62) + 64 : 0;
    atomicAdd(&hist[b], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int cum = 0, e = INT_MAX;
    for (int b = 0; b < kExpBins; ++b) {
      cum += hist[b];
      if (cum >= k) {
        e = b == 0 ? INT_MIN : b - 64;
        break;
      }
    }
    est[blockIdx.x] = e;
  }
}

// Morton code of every point's cell (coordinates relative to the cloud's lowest cell).
__global__ __launch_bounds__(kBlock) void knn_code_kernel(const float* __restrict__ xyz,
                                                          long long n, double inv_h, int lx,
                                                          int ly, int lz,
                                                          unsigned long long* __restrict__ code,
                                                          int* __restrict__ idx) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int cx = (int)floor((double)xyz[i] * inv_h) - lx;
    const int cy = (int)floor((double)xyz[n + i] * inv_h) - ly;
    const int cz = (int)floor((double)xyz[2 * n + i] * inv_h) - lz;
    code[i] = morton3(cx, cy, cz);
    idx[i] = (int)i;
  }
}

// Sorted copy of the positions.
__global__ __launch_bounds__(kBlock) void knn_gather_kernel(const float* __restrict__ xyz,
                                                            long long n,
                                                            const int* __restrict__ perm,
                                                            float* __restrict__ xs) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long p = perm[i];
    for (int a = 0; a < 3; ++a) xs[a * n + i] = xyz[a * n + p];
  }
}

// Grid level L has cells 8^L times the finest along each axis; its cell of a point is the
// finest cell's relative coordinates shifted right by 3L, so its Morton code is the finest code
// shifted right by 9L and every level's cells are contiguous runs of the one sorted order.
// Two passes per level: a cell's first position claims a hash slot and stores its start, then
// its last position finds the slot and stores the count.
__global__ __launch_bounds__(kBlock) void knn_level_head_kernel(
    long long n, const unsigned long long* __restrict__ code, int shift,
    CellSlot* __restrict__ slots, unsigned mask, unsigned* __restrict__ flags) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long c = code[i] >> shift;
    if (i > 0 && (code[i - 1] >> shift) == c) continue;
    unsigned s = cell_hash(c) & mask;
    bool placed = false;
    for (unsigned probe = 0; probe <= mask; ++probe) {
      const unsigned long long prev = atomicCAS(&slots[s].key, kEmptyCell, c);
      if (prev == kEmptyCell) {
        slots[s].start = (int)i;
        placed = true;
        break;
      }
      s = (s + 1) & mask;
    }
    if (!placed) atomicOr(flags, kFlagInternal);
  }
}

__global__ __launch_bounds__(kBlock) void knn_level_tail_kernel(
    long long n, const unsigned long long* __restrict__ code, int shift,
    CellSlot* __restrict__ slots, unsigned mask, unsigned* __restrict__ flags) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long c = code[i] >> shift;
    if (i + 1 < n && (code[i + 1] >> shift) == c) continue;
    unsigned s = cell_hash(c) & mask;
    bool found = false;
    for (unsigned probe = 0; probe <= mask; ++probe) {
      if (slots[s].key == c) {
        slots[s].count = (int)(i + 1 - slots[s].start);
        found = true;
        break;
      }
      s = (s + 1) & mask;
    }
    if (!found) atomicOr(flags, kFlagInternal);
  }
}

constexpr int kMaxLevels = 8;  // 3 more bits per level: 8 levels cover 2^21 finest cells

struct KnnGrid {
  const float* xs;         // [3][n] sorted positions
  const int* perm;         // [n] original index of each sorted position
  const CellSlot* slots[kMaxLevels];
  unsigned mask[kMaxLevels];
  int levels;
  double h, inv_h;         // finest cell edge (a power of two) and its inverse
  int lo[3];               // lowest finest cell per axis
  int ext[3];              // highest relative finest cell per axis
  long long n;
};

__device__ inline const CellSlot* find_cell(const CellSlot* slots, unsigned mask,
                                            unsigned long long c) {
  unsigned s = cell_hash(c) & mask;
  for (unsigned probe = 0; probe <= mask; ++probe) {
    const unsigned long long k = slots[s].key;
    if (k == c) return &slots[s];
    if (k == kEmptyCell) return nullptr;
    s = (s + 1) & mask;
  }
  return nullptr;
}

// Offers candidate (d, id) to the k best pairs kept sorted in bd/bi (K >= k slots): a better
// candidate bubbles down with selects; kth/kthi track slot k - 1.
template <int K>
__device__ inline void offer(double d, int id, double (&bd)[K], int (&bi)[K], double& kth,
                             int& kthi, int k) {
  if (!(d < kth || (d == kth && id < kthi))) return;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const bool lt = d < bd[s] || (d == bd[s] && id < bi[s]);
    const double td = bd[s];
    const int ti = bi[s];
    bd[s] = lt ? d : td;
    bi[s] = lt ? id : ti;
    d = lt ? td : d;
    id = lt ? ti : id;
  }
  kth = bd[0];
  kthi = bi[0];
#pragma unroll
  for (int s = 1; s < K; ++s)
    if (s == k - 1) {
      kth = bd[s];
      kthi = bi[s];
    }
}

// Shells searched on one level before the search moves to the next, coarser one.
constexpr int kMaxShell = 3;
// Lanes that share one query.
constexpr int kGroup = 16;

__device__ inline double shfl_xor_d(double v, int m) {
  const int lo = __shfl_xor(__double2loint(v), m, kGroup);
  const int hi = __shfl_xor(__double2hiint(v), m, kGroup);
  return __hiloint2double(hi, lo);
}

// The group's `rounds` best pairs in order: every lane offers the head of its own sorted list,
// a butterfly over the group's lanes picks the least (distance, index), its owner advances.
// Returns the pair of the last round (the group's k-th); `out`, if given, receives round s at
// out[s * n] from lane s mod kGroup.
template <int K>
__device__ inline void group_select(const double (&bd)[K], const int (&bi)[K], int rounds,
                                    int lane, double& kd, int& ki, int* out, long long n) {
  int head = 0;
  for (int s = 0; s < rounds; ++s) {
    double hd = INFINITY;
    int hi = INT_MAX;
#pragma unroll
    for (int t = 0; t < K; ++t)
      if (t == head) {
        hd = bd[t];
        hi = bi[t];
      }
    double md = hd;
    int mi = hi;
#pragma unroll
    for (int m = 1; m < kGroup; m <<= 1) {
      const double od = shfl_xor_d(md, m);
      const int oi = __shfl_xor(mi, m, kGroup);
      if (od < md || (od == md && oi < mi)) {
        md = od;
        mi = oi;
      }
    }
    if (mi != INT_MAX && mi == hi) ++head;  // indices are unique: exactly one owner
    if (out && (s % kGroup) == lane) out[(long long)s * n] = mi == INT_MAX ? -1 : mi;
    kd = md;
    ki = mi;
  }
}

// kGroup lanes per query, queries in sorted order (neighbouring groups query neighbouring
// points). On level L the search grows cubes of level-L cells around the query's cell: first
// the 3 x 3 x 3 cube, then the shells at Chebyshev distance 2, 3, ...; the lanes look up the
// cells of a step kGroup at a time, one each, and then share out the points of those cells
// (every lane takes every kGroup-th point, so the few large cells of an isolated query's coarse
// levels are split too); each lane keeps the best pairs it has seen sorted in registers
// (K >= k slots; a better candidate bubbles down with selects). After
// every step the group's k-th pair is merged from the lanes' lists. Every unvisited point lies
// outside the searched cube, at least `bound` away, so the search ends once the k-th distance is
// below bound^2 (with a relative margin far above the rounding of either side). A query still open
// after shell kMaxShell moves one level up: there the first 3 x 3 x 3 cube covers the previous
// level's cube (kMaxShell < 8), whose points were visited already and are skipped. The top level
// is one cell, so every query ends.
template <int K>
__global__ __launch_bounds__(kBlock) void knn_query_kernel(KnnGrid g, int k,
                                                           int* __restrict__ nbr) {
#pragma clang fp contract(off)
  const long long n = g.n;
  const int lane = threadIdx.x & (kGroup - 1);
  const long long stride = (long long)gridDim.x * blockDim.x / kGroup;
  for (long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kGroup; i < n;
       i += stride) {
    const double q0 = g.xs[i], q1 = g.xs[n + i], q2 = g.xs[2 * n + i];
    const int f0 = (int)floor(q0 * g.inv_h) - g.lo[0];
    const int f1 = (int)floor(q1 * g.inv_h) - g.lo[1];
    const int f2 = (int)floor(q2 * g.inv_h) - g.lo[2];
    double bd[K];
    int bi[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
      bd[s] = INFINITY;
      bi[s] = INT_MAX;
    }
    double kth = INFINITY;  // this lane's k-th
    int kthi = INT_MAX;
    double gk = INFINITY;   // the group's k-th (equal in all its lanes)
    int gki = INT_MAX;
    const double o0 = (double)g.lo[0] * g.h, o1 = (double)g.lo[1] * g.h,
                 o2 = (double)g.lo[2] * g.h;
    bool done = false;
    for (int L = 0; L < g.levels && !done; ++L) {
      const int sh = 3 * L;
      const double hl = g.h * (double)(1 << sh);
      const int c0 = f0 >> sh, c1 = f1 >> sh, c2 = f2 >> sh;
      const int x1 = g.ext[0] >> sh, y1 = g.ext[1] >> sh, z1 = g.ext[2] >> sh;
      const int psh = sh - 3;  // previous level's cells (L > 0)
      const int p0 = L > 0 ? f0 >> psh : 0, p1 = L > 0 ? f1 >> psh : 0,
                p2 = L > 0 ? f2 >> psh : 0;
      const CellSlot* slots = g.slots[L];
      const unsigned mask = g.mask[L];
      for (int r = 1; r <= kMaxShell; ++r) {
        const bool first = r == 1;  // the whole 3 x 3 x 3 cube
        const bool skip_seen = L > 0 && first;
        // the step's cells, indexed over the cube of side 2r + 1 (the interior of a shell is
        // skipped): each lane looks up one cell per round, then the group walks the points of
        // the round's cells together, every lane taking every kGroup-th point
        const int side = 2 * r + 1, ncube = side * side * side;
        for (int base = 0; base < ncube; base += kGroup) {
          int start = 0, count = 0;
          const int t = base + lane;
          if (t < ncube) {
            const int dx = t % side - r, dy = (t / side) % side - r, dz = t / (side * side) - r;
            const int x = c0 + dx, y = c1 + dy, z = c2 + dz;
            const bool in_step = first || abs(dx) == r || abs(dy) == r || abs(dz) == r;
            bool want = in_step && x >= 0 && x <= x1 && y >= 0 && y <= y1 && z >= 0 && z <= z1;
            if (want && gk < INFINITY) {  // skip cells that cannot hold a better point
              const double b0 = o0 + (double)x * hl, b1 = o1 + (double)y * hl,
                           b2 = o2 + (double)z * hl;
              const double e0 = q0 < b0 ? b0 - q0 : (q0 > b0 + hl ? q0 - (b0 + hl) : 0.0);
              const double e1 = q1 < b1 ? b1 - q1 : (q1 > b1 + hl ? q1 - (b1 + hl) : 0.0);
              const double e2 = q2 < b2 ? b2 - q2 : (q2 > b2 + hl ? q2 - (b2 + hl) : 0.0);
              want = ((e0 * e0 + e1 * e1) + e2 * e2) * (1.0 - 1e-12) <= gk;
            }
            if (want) {
              const CellSlot* cs = find_cell(slots, mask, morton3(x, y, z));
              if (cs) {
                start = cs->start;
                count = cs->count;
              }
            }
          }
#pragma unroll 1
          for (int src = 0; src < kGroup; ++src) {
            const int st = __shfl(start, src, kGroup), ct = __shfl(count, src, kGroup);
            for (int j = st + lane; j < st + ct; j += kGroup) {
              const double x0 = g.xs[j], x1_ = g.xs[n + j], x2 = g.xs[2 * n + j];
              if (skip_seen) {
                const int d0 = (((int)floor(x0 * g.inv_h) - g.lo[0]) >> psh) - p0;
                const int d1 = (((int)floor(x1_ * g.inv_h) - g.lo[1]) >> psh) - p1;
                const int d2 = (((int)floor(x2 * g.inv_h) - g.lo[2]) >> psh) - p2;
                if (abs(d0) <= kMaxShell && abs(d1) <= kMaxShell && abs(d2) <= kMaxShell)
                  continue;  // visited on the previous level
              }
              const double dx_ = x0 - q0, dy_ = x1_ - q1, dz_ = x2 - q2;
              const double d = (dx_ * dx_ + dy_ * dy_) + dz_ * dz_;
              const int id = g.perm[j];
              if (d > gk || (d == gk && id > gki)) continue;  // cannot reach the group's k
              offer<K>(d, id, bd, bi, kth, kthi, k);
            }
          }
        }
        group_select<K>(bd, bi, k, lane, gk, gki, nullptr, n);
        if (c0 - r <= 0 && c1 - r <= 0 && c2 - r <= 0 && c0 + r >= x1 && c1 + r >= y1 &&
            c2 + r >= z1) {
          done = true;  // every cell visited
          break;
        }
        const double g0 = fmin(q0 - (o0 + (double)(c0 - r) * hl), o0 + (double)(c0 + r + 1) * hl - q0);
        const double g1 = fmin(q1 - (o1 + (double)(c1 - r) * hl), o1 + (double)(c1 + r + 1) * hl - q1);
        const double g2 = fmin(q2 - (o2 + (double)(c2 - r) * hl), o2 + (double)(c2 + r + 1) * hl - q2);
        const double bound = fmax(fmin(fmin(g0, g1), g2), 0.0);
        if (gk < bound * bound * (1.0 - 1e-12)) {
          done = true;
          break;
        }
      }
    }
    group_select<K>(bd, bi, k, lane, gk, gki, nbr + g.perm[i], n);
  }
}

// ------------------------------------------------------------------ point covariances

// Cyclic Jacobi iteration on a symmetric 3x3 A (Golub & Van Loan, symmetric Schur rotations):
// A -> V^T A V diagonal, V orthogonal.
__device__ inline void rotate(double (&A)[3][3], double (&V)[3][3], int p, int q) {
  if (A[p][q] == 0.0) return;
  const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
  const double at = fabs(theta);
  const double t = at > 1e150 ? 0.5 / theta
                              : (theta >= 0.0 ? 1.0 : -1.0) / (at + sqrt(at * at + 1.0));
  const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double arp = A[r][p], arq = A[r][q];
    A[r][p] = c * arp - s * arq;
    A[r][q] = s * arp + c * arq;
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double apr = A[p][r], aqr = A[q][r];
    A[p][r] = c * apr - s * aqr;
    A[q][r] = s * apr + c * aqr;
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double vrp = V[r][p], vrq = V[r][q];
    V[r][p] = c * vrp - s * vrq;
    V[r][q] = s * vrp + c * vrq;
  }
}

__global__ __launch_bounds__(kBlock) void cov_kernel(const float* __restrict__ xyz, long long n,
                                                     const int* __restrict__ nbr, int k,
                                                     double scale, double eps,
                                                     float* __restrict__ cov,
                                                     unsigned* __restrict__ flags) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    int m = 0;
    bool bad = false;
    for (int s = 0; s < k; ++s) {
      const int j = nbr[s * n + i];
      if (j < 0) continue;
      if (j >= n) {
        bad = true;
        continue;
      }
      m0 += (double)xyz[j];
      m1 += (double)xyz[n + j];
      m2 += (double)xyz[2 * n + j];
      ++m;
    }
    if (bad) atomicOr(flags, kFlagBadIndex);
    const double inv_m = m > 0 ? 1.0 / (double)m : 0.0;
    m0 *= inv_m;
    m1 *= inv_m;
    m2 *= inv_m;
    double A[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int s = 0; s < k; ++s) {
      const int j = nbr[s * n + i];
      if (j < 0 || j >= n) continue;
      const double v[3] = {(double)xyz[j] - m0, (double)xyz[n + j] - m1,
                           (double)xyz[2 * n + j] - m2};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) A[a][b] += v[a] * v[b];
    }
    A[1][0] = A[0][1];
    A[2][0] = A[0][2];
    A[2][1] = A[1][2];
    double c6[6];
    if (scale > 0.0) {
      double V[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
      for (int sweep = 0; sweep < 12; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-36 * dia) break;
        rotate(A, V, 0, 1);
        rotate(A, V, 0, 2);
        rotate(A, V, 1, 2);
      }
      int c = 0;
      if (A[1][1] < A[c][c]) c = 1;
      if (A[2][2] < A[c][c]) c = 2;
      const double u[3] = {c == 0 ? V[0][0] : (c == 1 ? V[0][1] : V[0][2]),
                           c == 0 ? V[1][0] : (c == 1 ? V[1][1] : V[1][2]),
                           c == 0 ? V[2][0] : (c == 1 ? V[2][1] : V[2][2])};
      const double g = 1.0 - eps;
      c6[0] = scale * (1.0 - g * u[0] * u[0]);
      c6[1] = scale * (-g * u[0] * u[1]);
      c6[2] = scale * (-g * u[0] * u[2]);
      c6[3] = scale * (1.0 - g * u[1] * u[1]);
      c6[4] = scale * (-g * u[1] * u[2]);
      c6[5] = scale * (1.0 - g * u[2] * u[2]);
    } else {
      c6[0] = A[0][0] * inv_m;
      c6[1] = A[0][1] * inv_m;
      c6[2] = A[0][2] * inv_m;
      c6[3] = A[1][1] * inv_m;
      c6[4] = A[1][2] * inv_m;
      c6[5] = A[2][2] * inv_m;
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) cov[a * n + i] = (float)c6[a];
  }
}

bool pow2_res(double res) {
  int e = 0;
  return std::frexp(res, &e) == 0.5;
}

}  // namespace

vgicp_status downsample(const float* xyz, const float* t, int64_t n, double res, double d_scan,
                        float* xyz_out, float* t_out, int64_t capacity, int64_t* n_out,
                        hipStream_t s) {
  *n_out = 0;
  if (n == 0) return VGICP_OK;
  Scratch sc;
  int *kc = nullptr, *bounds = nullptr, *vA = nullptr, *vB = nullptr, *vcnt = nullptr,
      *voff = nullptr;
  unsigned long long *kA = nullptr, *kB = nullptr;
  unsigned* flags = nullptr;
  hipError_t e;
  if ((e = sc.alloc(&kc, 3 * (size_t)n)) || (e = sc.alloc(&bounds, 6)) ||
      (e = sc.alloc(&flags, 1)) || (e = sc.alloc(&kA, (size_t)n)) ||
      (e = sc.alloc(&kB, (size_t)n)) || (e = sc.alloc(&vA, (size_t)n)) ||
      (e = sc.alloc(&vB, (size_t)n)) || (e = sc.alloc(&vcnt, (size_t)n)) ||
      (e = sc.alloc(&voff, (size_t)n)))
    return hip_fail(e, "hipMalloc (downsample)");
  const bool p2 = pow2_res(res);
  bounds_reset_kernel<<<1, 64, 0, s>>>(bounds, flags);
  ds_cells_kernel<<<std::min(grid_for(n), 128), kBlock, 0, s>>>(xyz, t, n, p2 ? 1 : 0, res, 1.0 / res, kc,
                                                 bounds, flags);
  int hb[6];
  unsigned hf = 0;
  if ((e = hipGetLastError()) || (e = hipMemcpyAsync(hb, bounds, sizeof(hb), hipMemcpyDeviceToHost, s)) ||
      (e = hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s)) ||
      (e = hipStreamSynchronize(s)))
    return hip_fail(e, "downsample cells");
  if (hf & kFlagNonFinite) return fail(VGICP_E_NONFINITE, "non-finite point or timestamp");
  if (hf & kFlagKeyRange) return fail(VGICP_E_KEY_RANGE, "cell coordinate out of range");
  const int bx = bits_for((long long)hb[3] - hb[0]), by = bits_for((long long)hb[4] - hb[1]),
            bz = bits_for((long long)hb[5] - hb[2]);
  const int* order = nullptr;
  if (t) {  // (time, index) order first; the stable cell sort below keeps it within a cell
    ds_time_key_kernel<<<grid_for(n), kBlock, 0, s>>>(t, n, kA, vA);
    if ((e = hipGetLastError()) || (e = radix_sort_pairs(&kA, &vA, &kB, &vB, n, 32, flags, s, sc)))
      return hip_fail(e, "downsample time sort");
    order = vA;
  }
  ds_cell_key_kernel<<<grid_for(n), kBlock, 0, s>>>(kc, n, order, hb[0], hb[1], hb[2], by + bz,
                                                    bz, kB, vB);
  std::swap(kA, kB);
  std::swap(vA, vB);
  if ((e = hipGetLastError()) ||
      (e = radix_sort_pairs(&kA, &vA, &kB, &vB, n, bx + by + bz, flags, s, sc)))
    return hip_fail(e, "downsample cell sort");
  const double thr = d_scan / 10.0;
  ds_walk_kernel<false><<<grid_for(n), kBlock, 0, s>>>(kA, vA, n, xyz, t, thr, vcnt, nullptr, 0,
                                                       nullptr, nullptr);
  if ((e = hipGetLastError()) || (e = scan_exclusive(vcnt, voff, n, s, sc)))
    return hip_fail(e, "downsample count");
  int last[2] = {0, 0};
  if ((e = hipMemcpyAsync(&last[0], voff + n - 1, sizeof(int), hipMemcpyDeviceToHost, s)) ||
      (e = hipMemcpyAsync(&last[1], vcnt + n - 1, sizeof(int), hipMemcpyDeviceToHost, s)) ||
      (e = hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s)) ||
      (e = hipStreamSynchronize(s)))
    return hip_fail(e, "downsample count");
  if (hf & kFlagInternal) return fail(VGICP_E_HIP, "internal error in the downsample sort");
  const int64_t m = (int64_t)last[0] + last[1];
  *n_out = m;
  if (m > capacity) return fail(VGICP_E_CAPACITY, "downsampled cloud exceeds the output capacity");
  ds_walk_kernel<true><<<grid_for(n), kBlock, 0, s>>>(kA, vA, n, xyz, t, thr, nullptr, voff, m,
                                                      xyz_out, t ? t_out : nullptr);
  if ((e = hipGetLastError()) || (e = hipStreamSynchronize(s)))
    return hip_fail(e, "downsample emit");
  return VGICP_OK;
}

vgicp_status knn(const float* xyz, int64_t n, int k, double cell, int32_t* nbr, hipStream_t s) {
  if (n == 0) return VGICP_OK;
  Scratch sc;
  hipError_t e;
  const int nb = std::min<int>(grid_for(n), 1024);
  float* part = nullptr;
  unsigned* flags = nullptr;
  if ((e = sc.alloc(&part, (size_t)nb * 6)) || (e = sc.alloc(&flags, 1)))
    return hip_fail(e, "hipMalloc (knn)");
  if ((e = hipMemsetAsync(flags, 0, sizeof(unsigned), s))) return hip_fail(e, "hipMemsetAsync");
  knn_bounds_kernel<<<nb, kBlock, 0, s>>>(xyz, n, part, flags);
  // the cell estimate runs beside the bounds (a non-finite cloud is rejected after it)
  const int S = cell > 0.0 ? 0 : (int)std::min<int64_t>(n, 64);
  int* est = nullptr;
  if (S > 0) {
    if ((e = sc.alloc(&est, (size_t)S))) return hip_fail(e, "hipMalloc (knn)");
    knn_sample_kernel<<<S, kBlock, 0, s>>>(xyz, n, S, k, est);
  }
  std::vector<float> hp((size_t)nb * 6);
  std::vector<int> he(S);
  unsigned hf = 0;
  if ((e = hipGetLastError()) ||
      (e = hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(float), hipMemcpyDeviceToHost, s)) ||
      (S > 0 && (e = hipMemcpyAsync(he.data(), est, S * sizeof(int), hipMemcpyDeviceToHost, s))) ||
      (e = hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s)) ||
      (e = hipStreamSynchronize(s)))
    return hip_fail(e, "knn bounds");
  if (hf & kFlagNonFinite) return fail(VGICP_E_NONFINITE, "non-finite point");
  double lo[3], hi[3], maxabs = 0.0;
  for (int a = 0; a < 3; ++a) {
    lo[a] = hp[a];
    hi[a] = hp[3 + a];
    for (int b = 1; b < nb; ++b) {
      lo[a] = std::min<double>(lo[a], hp[b * 6 + a]);
      hi[a] = std::max<double>(hi[a], hp[b * 6 + 3 + a]);
    }
    maxabs = std::max(maxabs, std::max(std::fabs(lo[a]), std::fabs(hi[a])));
  }
  int eh = 0;  // cell edge 2^eh
  if (cell > 0.0) {
    eh = (int)std::ceil(std::log2(cell));
  } else {
    std::vector<int> r;
    for (int v : he)
      if (v != INT_MIN) r.push_back(v == INT_MAX ? 62 : (v + 2) / 2);  // 2^r >= k-th distance
    if (!r.empty()) {
      std::nth_element(r.begin(), r.begin() + r.size() / 2, r.end());
      eh = r[r.size() / 2];
    }
  }
  // every cell coordinate stays below 2^19 in magnitude
  eh = std::max(eh, (int)std::ceil(std::log2(std::max(maxabs, 1e-300))) - 19);
  eh = std::min(std::max(eh, -60), 150);
  const double h = std::ldexp(1.0, eh), inv_h = std::ldexp(1.0, -eh);
  KnnGrid g;
  int ext_max = 0;
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = (int)std::floor(lo[a] * inv_h);
    g.ext[a] = (int)std::floor(hi[a] * inv_h) - g.lo[a];
    ext_max = std::max(ext_max, g.ext[a]);
  }
  const int bits = 3 * bits_for(ext_max);
  int levels = 1;
  while (levels < kMaxLevels && (ext_max >> (3 * (levels - 1))) > 0) ++levels;
  unsigned long long *kA = nullptr, *kB = nullptr;
  int *vA = nullptr, *vB = nullptr;
  float* xs = nullptr;
  if ((e = sc.alloc(&kA, (size_t)n)) || (e = sc.alloc(&kB, (size_t)n)) ||
      (e = sc.alloc(&vA, (size_t)n)) || (e = sc.alloc(&vB, (size_t)n)) ||
      (e = sc.alloc(&xs, 3 * (size_t)n)))
    return hip_fail(e, "hipMalloc (knn)");
  knn_code_kernel<<<grid_for(n), kBlock, 0, s>>>(xyz, n, inv_h, g.lo[0], g.lo[1], g.lo[2], kA, vA);
  if ((e = hipGetLastError()) || (e = radix_sort_pairs(&kA, &vA, &kB, &vB, n, bits, flags, s, sc)))
    return hip_fail(e, "knn sort");
  knn_gather_kernel<<<grid_for(n), kBlock, 0, s>>>(xyz, n, vA, xs);
  for (int L = 0; L < levels; ++L) {
    // cells on level L: at most n, and at most the product of the level's extents
    long long cells = 1;
    for (int a = 0; a < 3; ++a) cells = std::min<long long>(cells * ((g.ext[a] >> (3 * L)) + 1), n);
    unsigned cap = 1;
    while ((long long)cap < 2 * cells) cap <<= 1;
    CellSlot* slots = nullptr;
    if ((e = sc.alloc(&slots, (size_t)cap))) return hip_fail(e, "hipMalloc (knn)");
    if ((e = hipMemsetAsync(slots, 0xff, (size_t)cap * sizeof(CellSlot), s)))
      return hip_fail(e, "hipMemsetAsync");
    knn_level_head_kernel<<<grid_for(n), kBlock, 0, s>>>(n, kA, 9 * L, slots, cap - 1, flags);
    knn_level_tail_kernel<<<grid_for(n), kBlock, 0, s>>>(n, kA, 9 * L, slots, cap - 1, flags);
    g.slots[L] = slots;
    g.mask[L] = cap - 1;
  }
  g.levels = levels;
  g.xs = xs;
  g.perm = vA;
  g.h = h;
  g.inv_h = inv_h;
  g.n = n;
  const int qgrid = grid_for(n * kGroup);
  if (k <= 8)
    knn_query_kernel<8><<<qgrid, kBlock, 0, s>>>(g, k, nbr);
  else if (k <= 16)
    knn_query_kernel<16><<<qgrid, kBlock, 0, s>>>(g, k, nbr);
  else
    knn_query_kernel<32><<<qgrid, kBlock, 0, s>>>(g, k, nbr);
  if ((e = hipGetLastError()) ||
      (e = hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s)) ||
      (e = hipStreamSynchronize(s)))
    return hip_fail(e, "knn query");
  if (hf & kFlagInternal) return fail(VGICP_E_HIP, "internal error in the neighbour search");
  return VGICP_OK;
}

void launch_point_covariances(const float* xyz, int64_t n, const int32_t* nbr, int k,
                              double scale, double eps, float* cov, unsigned* flags,
                              hipStream_t s) {
  if (n == 0) return;
  cov_kernel<<<grid_for(n), kBlock, 0, s>>>(xyz, n, nbr, k, scale, eps, cov, flags);
}

}  // namespace vgicp
