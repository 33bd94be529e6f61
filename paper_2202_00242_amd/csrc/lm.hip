// One Levenberg-Marquardt step of the pose graph formed by a batch's matching-cost factors
// (Sec. III-F: the global mapping graph over submap poses, optimized with LM; Eq. (2) supplies
// every factor's cost and its Gauss-Newton blocks).
//
//   1. linearize every factor at the current poses (the batched kernel);
//   2. assemble the 6P x 6P system: each 6x6 block and each 6-vector is the sum of its factors'
//      contributions in factor order (one thread per entry, so the result is deterministic);
//   3. damp it as H + lambda diag(H) (Marquardt); a pose that no factor reaches, and an optional
//      fixed pose, get an identity row (their step is zero);
//   4. solve (H + lambda diag H) delta = -b in FP64: with the poses in a bandwidth-reducing order
//      (chosen once per batch) the system is banded and one workgroup factors it with a sliding
//      window of the band in LDS; a graph too wide for that uses a dense right-looking blocked
//      Cholesky factorization (64 x 64 blocks) instead;
//   5. retract every pose, T_i <- T_i Exp(delta_i), and linearize there (the cost at the new poses,
//      and the next iteration's system when the step is taken).
// The iteration form decides on the device: the step is taken when the cost decreases (lambda
// divided by 10), otherwise lambda is multiplied by 10 and the poses stay.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <set>
#include <type_traits>
#include <vector>

#include "device_math.h"
#include "internal.h"

namespace vgicp {
namespace {

constexpr int kNB = 64;  // Cholesky block size

// Orders a wave's LDS writes before its lanes read them.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// ------------------------------------------------------------------ assembly

__global__ __launch_bounds__(256) void lm_clear_kernel(double* __restrict__ A, long long nn,
                                                       int n, int n_real,
                                                       double* __restrict__ diag_raw) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nn;
       i += (long long)gridDim.x * blockDim.x) {
    const long long r = i / n, c = i % n;
    A[i] = (r == c && r >= n_real) ? 1.0 : 0.0;  // padding rows: identity
    if (c == 0) diag_raw[r] = 0.0;
  }
}

// One thread per entry of every nonzero 6x6 block; contributions are (factor << 2) | (a << 1)
// | b, the 6x6 sub-block (a, b) of the factor's 12x12 [source | target] matrix.
__global__ __launch_bounds__(256) void lm_assemble_kernel(
    const LmBlock* __restrict__ blocks, int nblocks, const int* __restrict__ contrib,
    const double* __restrict__ Hf, const double* __restrict__ lambda, int fixed, int n,
    double* __restrict__ A,
    double* __restrict__ diag_raw) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nblocks * 36) return;
  const LmBlock bk = blocks[t / 36];
  const int e = t % 36, r = e / 6, c = e % 6;
  if (bk.row == fixed || bk.col == fixed) return;
  double s = 0.0;
#pragma unroll 8  // loads issued together, the sum in its order
  for (int q = 0; q < bk.count; ++q) {
    const int w = contrib[bk.first + q];
    const int f = w >> 2, a = (w >> 1) & 1, b = w & 1;
    s += Hf[144LL * f + (6 * a + r) * 12 + 6 * b + c];
  }
  const long long i = 6LL * bk.row + r, j = 6LL * bk.col + c;
  if (i == j) {
    diag_raw[i] = s;
    s = s > 0.0 ? s * (1.0 + *lambda) : 1.0;
  }
  A[i * n + j] = s;
}

// Right-hand side -b (contributions (factor << 1) | half), and identity rows for poses without
// a factor, for zero diagonal entries and for the fixed pose.
__global__ __launch_bounds__(256) void lm_rhs_kernel(const int* __restrict__ bptr,
                                                     const int* __restrict__ bcontrib,
                                                     const double* __restrict__ bf, int P,
                                                     int fixed, int n, double* __restrict__ A,
                                                     const double* __restrict__ diag_raw,
                                                     double* __restrict__ g) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  if (t >= 6 * P) {  // padding
    g[t] = 0.0;
    return;
  }
  const int p = t / 6, r = t % 6;
  double s = 0.0;
#pragma unroll 8  // loads issued together, the sum in its order
  for (int q = bptr[p]; q < bptr[p + 1]; ++q) {
    const int w = bcontrib[q];
    s += bf[12LL * (w >> 1) + 6 * (w & 1) + r];
  }
  if (p == fixed || !(diag_raw[t] > 0.0)) {
    A[(long long)t * n + t] = 1.0;
    s = 0.0;
  }
  g[t] = -s;
}

// ------------------------------------------------------------------ Cholesky (lower, in place)

// Broadcast of lane l's double (l uniform) through two scalar reads.
__device__ inline double readlane_d(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Diagonal block k on 256 threads, the block and its inverse in LDS, in 16 x 16 tiles. Per
// diagonal tile kk: one wave factors the tile, a lane per row in registers (the pivot row's
// entries reach the other lanes by scalar broadcasts), and inverts it (lane r solves
// x L^T = e_r by substitution); then all threads form the panel below it, L_ik = A_ik L_kk^-T,
// as a product with that inverse, and update the trailing lower triangle. The inverse of the
// whole factor follows block row by block row, X_ij = -X_ii sum_{j <= m < i} L_im X_mj. Only
// the 16 x 16 tile factorizations are a serial chain. The factor overwrites the block (zeros
// above the diagonal) and its inverse goes to Dinv (row-major): the panel and the triangular
// solves then multiply by it instead of substituting. A non-positive pivot sets the non-finite
// flag (the damped system must be positive definite) and continues with 1.
constexpr int kTile = 16;
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ A, int n, int k,
                                                         double* __restrict__ Dinv,
                                                         unsigned* __restrict__ flags) {
  __shared__ double S[kNB][kNB + 1];
  __shared__ double X[kNB][kNB + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const long long o = (long long)k * kNB;
  for (int e = t; e < kNB * kNB; e += 256) {
    const int r = e / kNB, c = e % kNB;
    S[r][c] = A[(o + r) * n + o + c];
    X[r][c] = 0.0;
  }
  __syncthreads();
  for (int kk = 0; kk < kNB / kTile; ++kk) {
    const int b = kk * kTile;
    if (w == 0) {
      const int r = lane & (kTile - 1);  // lanes 16..63 repeat rows 0..15 and store nothing
      double a[kTile];
#pragma unroll
      for (int p = 0; p < kTile; ++p) a[p] = S[b + r][b + p];
#pragma unroll
      for (int j = 0; j < kTile; ++j) {
        double d = readlane_d(a[j], j);
        if (!(d > 0.0)) {
          if (lane == 0) atomicOr(flags, kFlagNonFinite);
          d = 1.0;
        }
        d = sqrt(d);
        const double lij = (r > j) ? a[j] / d : (r == j ? d : a[j]);
        a[j] = lij;
#pragma unroll
        for (int l = j + 1; l < kTile; ++l) {
          const double llj = readlane_d(lij, l);
          a[l] = (r >= l) ? a[l] - lij * llj : a[l];
        }
      }
      if (lane < kTile)
#pragma unroll
        for (int p = 0; p < kTile; ++p) S[b + r][b + p] = (p <= r) ? a[p] : 0.0;
      wave_lds_sync();
      double x[kTile];
#pragma unroll
      for (int c = 0; c < kTile; ++c) {
        double v = (c == r) ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < c; ++q) v -= x[q] * S[b + c][b + q];
        x[c] = v / S[b + c][b + c];
      }
      if (lane < kTile)
#pragma unroll
        for (int c = 0; c < kTile; ++c) X[b + c][b + r] = x[c];  // (L_kk^-1)_{c, r}
    }
    __syncthreads();
    // panel below the tile: L[r][b + c] = sum_q A[r][b + q] (L_kk^-1)[c][q]
    const int rows = kNB - b - kTile;
    double tmp[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int e = t + 256 * u;
      tmp[u] = 0.0;
      if (e < rows * kTile) {
        const int r = b + kTile + e / kTile, c = e % kTile;
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < kTile; ++q) v += S[r][b + q] * X[b + c][b + q];
        tmp[u] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int e = t + 256 * u;
      if (e < rows * kTile) S[b + kTile + e / kTile][b + e % kTile] = tmp[u];
    }
    __syncthreads();
    // trailing lower triangle: A[r][c] -= sum_q L[r][b + q] L[c][b + q]
    for (int e = t; e < rows * rows; e += 256) {
      const int rr = e / rows, cc = e % rows;
      if (cc > rr) continue;
      const int r = b + kTile + rr, c = b + kTile + cc;
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < kTile; ++q) v += S[r][b + q] * S[c][b + q];
      S[r][c] -= v;
    }
    __syncthreads();
  }
  // the inverse below its diagonal tiles, block row bi: Y = sum_{j <= m < bi} L_{bi,m} X_{m,j},
  // then X_{bi,j} = -X_{bi,bi} Y (Y parked in X_{bi,j} between the two products)
  for (int bi = 1; bi < kNB / kTile; ++bi) {
    double tmp[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int e = t + 256 * u;
      tmp[u] = 0.0;
      if (e < bi * kTile * kTile) {
        const int j = e / (kTile * kTile), rr = (e / kTile) % kTile, cc = e % kTile;
        const int r = kTile * bi + rr, c = kTile * j + cc;
        double v = 0.0;
        for (int m = j; m < bi; ++m)
#pragma unroll
          for (int q = 0; q < kTile; ++q) v += S[r][kTile * m + q] * X[kTile * m + q][c];
        tmp[u] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int e = t + 256 * u;
      if (e < bi * kTile * kTile)
        X[kTile * bi + (e / kTile) % kTile][kTile * (e / (kTile * kTile)) + e % kTile] = tmp[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int e = t + 256 * u;
      tmp[u] = 0.0;
      if (e < bi * kTile * kTile) {
        const int j = e / (kTile * kTile), rr = (e / kTile) % kTile, cc = e % kTile;
        const int c = kTile * j + cc;
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < kTile; ++q)
          v += X[kTile * bi + rr][kTile * bi + q] * X[kTile * bi + q][c];
        tmp[u] = -v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int e = t + 256 * u;
      if (e < bi * kTile * kTile)
        X[kTile * bi + (e / kTile) % kTile][kTile * (e / (kTile * kTile)) + e % kTile] = tmp[u];
    }
    __syncthreads();
  }
  for (int e = t; e < kNB * kNB; e += 256) {
    const int r = e / kNB, c = e % kNB;
    A[(o + r) * n + o + c] = c <= r ? S[r][c] : 0.0;
    Dinv[(o + r) * kNB + c] = c <= r ? X[r][c] : 0.0;  // (L^-1)_{r, c}
  }
}

// Panel: block rows below k, X = A_ik L_kk^-T (X L_kk^T = A_ik), as a 64 x 64 x 64 product:
// 256 threads, 4 x 4 entries each, the inner dimension staged through LDS in halves.
__global__ __launch_bounds__(256) void trsm_kernel(double* __restrict__ A, int n, int k,
                                                   const double* __restrict__ Dinv) {
  __shared__ double Xs[kNB][33];
  __shared__ double Is[kNB][33];
  const long long o = (long long)k * kNB, bi = (long long)(k + 1 + blockIdx.x) * kNB;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  for (int h = 0; h < 2; ++h) {
    for (int e = threadIdx.x; e < kNB * 32; e += blockDim.x) {
      const int rr = e / 32, pp = e % 32;
      Xs[rr][pp] = A[(bi + rr) * n + o + 32 * h + pp];
      Is[rr][pp] = Dinv[(o + rr) * kNB + 32 * h + pp];
    }
    __syncthreads();
    for (int p = 0; p < 32; ++p) {
      double a[4], b[4];
      for (int q = 0; q < 4; ++q) {
        a[q] = Xs[4 * ty + q][p];
        b[q] = Is[4 * tx + q][p];
      }
      for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) A[(bi + 4 * ty + u) * n + o + 4 * tx + v] = acc[u][v];
}

// Trailing update of the lower-triangle block (i, j), k < j <= i: A_ij -= L_ik L_jk^T. 256
// threads, 4 x 4 entries each; the 64-wide inner dimension is staged through LDS in halves.
__global__ __launch_bounds__(256) void update_kernel(double* __restrict__ A, int n, int k,
                                                     int nblk) {
  __shared__ double Li[kNB][33];
  __shared__ double Lj[kNB][33];
  const int t = blockIdx.x;
  int ip = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);  // t -> (ip, jp), jp <= ip
  while ((ip + 1) * (ip + 2) / 2 <= t) ++ip;
  while (ip * (ip + 1) / 2 > t) --ip;
  const int jp = t - ip * (ip + 1) / 2;
  const long long bi = (long long)(k + 1 + ip) * kNB, bj = (long long)(k + 1 + jp) * kNB;
  const long long ok = (long long)k * kNB;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  for (int h = 0; h < 2; ++h) {
    for (int e = threadIdx.x; e < kNB * 32; e += blockDim.x) {
      const int rr = e / 32, pp = e % 32;
      Li[rr][pp] = A[(bi + rr) * n + ok + 32 * h + pp];
      Lj[rr][pp] = A[(bj + rr) * n + ok + 32 * h + pp];
    }
    __syncthreads();
    for (int p = 0; p < 32; ++p) {
      double a[4], b[4];
      for (int q = 0; q < 4; ++q) {
        a[q] = Li[4 * ty + q][p];
        b[q] = Lj[4 * tx + q][p];
      }
      for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) A[(bi + 4 * ty + u) * n + bj + 4 * tx + v] -= acc[u][v];
  (void)nblk;
}

// Triangular solves L y = g, then L^T x = y, block by block: the diagonal block by its inverse,
// then the other rows are updated by a grid (forward: a wave per row reads its 64 contiguous
// entries; backward: a thread per row reads a column, contiguous across the threads).
// Diagonal block k: x_k <- L_kk^-1 x_k (forward) or L_kk^-T x_k (backward), a lane per row,
// the inverse staged through LDS by coalesced rows.
template <bool FWD>
__global__ __launch_bounds__(64) void trsv_diag_kernel(const double* __restrict__ Dinv, int k,
                                                       double* __restrict__ x) {
  __shared__ double xb[kNB];
  __shared__ double Ds[kNB][kNB + 1];
  const int lane = threadIdx.x, o = k * kNB;
  xb[lane] = x[o + lane];
  const double* D = Dinv + (long long)o * kNB;
#pragma unroll 8
  for (int r = 0; r < kNB; ++r) Ds[r][lane] = D[r * kNB + lane];  // coalesced rows
  wave_lds_sync();
  double s = 0.0;
  if (FWD)
    for (int p = 0; p <= lane; ++p) s += Ds[lane][p] * xb[p];
  else
    for (int p = lane; p < kNB; ++p) s += Ds[p][lane] * xb[p];
  x[o + lane] = s;
}

// forward: rows below block k, a wave per row
__global__ __launch_bounds__(256) void trsv_fwd_update_kernel(const double* __restrict__ A,
                                                              int n, int k,
                                                              double* __restrict__ x) {
  const int o = k * kNB, lane = threadIdx.x & 63;
  const int i = o + kNB + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double s = A[(long long)i * n + o + lane] * x[o + lane];
  for (int w = 32; w > 0; w >>= 1) s += __shfl_xor(s, w);
  if (lane == 0) x[i] -= s;
}

// backward: rows above block k, a thread per row
__global__ __launch_bounds__(256) void trsv_bwd_update_kernel(const double* __restrict__ A,
                                                              int n, int k,
                                                              double* __restrict__ x) {
  __shared__ double xb[kNB];
  const int o = k * kNB, i = blockIdx.x * blockDim.x + threadIdx.x;
  if (threadIdx.x < kNB) xb[threadIdx.x] = x[o + threadIdx.x];
  __syncthreads();
  if (i >= o) return;
  double s = 0.0;
  for (int c = 0; c < kNB; ++c) s += A[(long long)(o + c) * n + i] * xb[c];
  x[i] -= s;
}

// ------------------------------------------------------------------ retraction and costs

__global__ __launch_bounds__(256) void lm_retract_kernel(const double* __restrict__ poses,
                                                         const double* __restrict__ x, int P,
                                                         double* __restrict__ poses_new,
                                                         double* __restrict__ delta) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double xi[6], o[12];
  for (int a = 0; a < 6; ++a) xi[a] = x[6 * p + a];
  se3_retract(poses + 12LL * p, xi, o);
  for (int a = 0; a < 12; ++a) poses_new[12LL * p + a] = o[a];
  if (delta)
    for (int a = 0; a < 6; ++a) delta[6LL * p + a] = xi[a];
}

// The sums of e0 and of e1 over F factors by one 256-thread block, each in a fixed order
// (strided partial sums, then a tree over the threads); the result is in thread 0. The loads of
// eight strides are issued together (the sums keep their order).
__device__ inline void block_cost_sums(const double* __restrict__ e0,
                                       const double* __restrict__ e1, int F, double& c0,
                                       double& c1) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, b = 0.0;
#pragma unroll 8
  for (int f = threadIdx.x; f < F; f += 256) {
    a += e0[f];
    b += e1[f];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  c0 = s0[0];
  c1 = s1[0];
}

// cost[0] = sum of e0, cost[1] = sum of e1 (block_cost_sums).
__global__ __launch_bounds__(256) void lm_cost_kernel(const double* __restrict__ e0,
                                                      const double* __restrict__ e1, int F,
                                                      double* __restrict__ cost) {
  double c0, c1;
  block_cost_sums(e0, e1, F, c0, c1);
  if (threadIdx.x == 0) {
    cost[0] = c0;
    cost[1] = c1;
  }
}

unsigned grid1(long long n, int block) {
  return (unsigned)std::max<long long>(1, std::min<long long>((n + block - 1) / block, 65536));
}

// ------------------------------------------------------------------ banded solve

// The pose graph of a mapping run is banded once its poses are put in a suitable order (each
// submap is linked to the submaps near it; along a loop a spectral order interleaves the two
// sides). The damped system is then factored by one workgroup that keeps a sliding window of
// the band in LDS: block step s (the 6 unknowns of one pose position, columns j0 = 6 s ..)
// factors the 6 x 6 diagonal block, forms the panel below it, applies the rank-6 update to the
// window, and the block's rows leave the window (to global memory) while the next rows come in.
// The forward substitution rides along; the backward substitution walks the blocks in reverse.
// Every sum has a fixed order (deterministic). A long band is solved from both ends: no entry
// couples the unknowns before a run of w + 1 consecutive unknowns (the separator) with those
// after it, so two workgroups eliminate the two sides at once (the far side stored in reverse
// order, so that the same forward sweep eliminates its last block first), the separator's system
// is the sum of the Schur complements the two sides leave on it, and the two backward sweeps
// then run side by side.
//
// Eight compute waves never touch global memory inside the sweeps: two producer waves move the
// rows in and out, beside each step's trailing update. They load a step's incoming rows two
// steps ahead, into registers, with branch-free loads and stores (clamped addresses), so that
// waiting for the oldest loads does not also wait for the newest ones or for the stores of the
// rows leaving the window.
constexpr int kBandMaxW = 131;            // half-bandwidth w = 6 * pose bandwidth + 5
constexpr int kBandMaxW1 = kBandMaxW + 1;
constexpr int kBandMaxR = kBandMaxW + 6;  // window rows
constexpr int kBandWaves = 8;             // compute waves
constexpr int kBandProd = 2;              // producer waves
constexpr int kBandThreads = 64 * (kBandWaves + kBandProd);
constexpr int kBandLD = kBandMaxW1 + 1;   // LDS row stride of the window (odd: no bank conflicts
                                           // when lanes walk a column)
constexpr int kBandMaxN = kBandMaxR * kBandLD;  // LDS doubles of the window
constexpr int kBandPer = (6 * kBandMaxW1 + 64 * kBandProd - 1) / (64 * kBandProd);  // band values
                                                                             // of one block per
                                                                             // producer lane
constexpr int kBandSplitMin = 8;  // blocks per end below which one sweep solves the system
constexpr int kBandPcLD = 144;  // panel stride: the four lane groups of an MFMA operand read fall
                                // in disjoint LDS banks (144 = 16 mod 32 doubles)
static_assert(kBandPcLD >= kBandMaxR, "panel stride");
typedef double dbl4 __attribute__((ext_vector_type(4)));

// 1 / sqrt(d) for d > 0: the hardware's reciprocal square root refined by two Newton steps
// (r <- r (3 - d r^2) / 2; each squares the relative error), a short dependent chain where the
// library's square root and division are long ones. Accurate to a few units in the last place.
__device__ inline double rsqrt_refined(double d) {
  double r = __builtin_amdgcn_rsq(d);
  r = r * (1.5 - 0.5 * d * r * r);
  r = r * (1.5 - 0.5 * d * r * r);
  return r;
}

// The 6 x 6 diagonal block of block step s (its rows in the window, slots (j0 + a) mod R):
// M = L L^T (Cholesky), X = L^-1 and the block of the forward substitution z = L^-1 y. The
// window's rows get L with the reciprocals of its diagonal on the diagonal (what the backward
// substitution uses); X (row-major, lower triangle) goes to Xs for the panel, z to zs and the
// window's right-hand side. Called by a whole wave; lane 0 does the arithmetic in registers (the
// chain of the 6 pivots, then X column by column and z), so the block costs one round of LDS
// reads and one of writes.
__device__ inline void band_diag_block(int s, int R, double* Wn, double* yw, double* Xs,
                                       double* zs, int* bad_flag, int lane) {
  const int j0 = 6 * s;
  if (lane == 0) {
    double L[6][6], inv[6], yv[6];
    int sl[6];
    const int s0 = j0 % R;
#pragma unroll
    for (int a = 0; a < 6; ++a) sl[a] = s0 + a < R ? s0 + a : s0 + a - R;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      yv[a] = yw[sl[a]];
#pragma unroll
      for (int b = 0; b <= a; ++b) L[a][b] = Wn[sl[a] * kBandLD + (a - b)];
    }
    bool bad = false;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      double dd = L[c][c];
#pragma unroll
      for (int k = 0; k < c; ++k) dd -= L[c][k] * L[c][k];
      if (!(dd > 0.0) || !isfinite(dd)) {
        bad = true;
        dd = 1.0;
      }
      const double r = rsqrt_refined(dd);
      inv[c] = r;
#pragma unroll
      for (int q = c + 1; q < 6; ++q) {
        double v = L[q][c];
#pragma unroll
        for (int k = 0; k < c; ++k) v -= L[q][k] * L[c][k];
        L[q][c] = v * r;
      }
    }
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) Wn[sl[a] * kBandLD + (a - b)] = b < a ? L[a][b] : inv[a];
    // X = L^-1 by columns: X_cc = inv_c, X_rc = -inv_r sum_{c <= k < r} L_rk X_kc; then
    // z_a = sum_{c <= a} X_ac y_c
    double X[6][6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      X[c][c] = inv[c];
#pragma unroll
      for (int r = c + 1; r < 6; ++r) {
        double v = 0.0;
#pragma unroll
        for (int k = c; k < r; ++k) v += L[r][k] * X[k][c];
        X[r][c] = -v * inv[r];
      }
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      double z = 0.0;
#pragma unroll
      for (int c = 0; c <= a; ++c) {
        Xs[6 * a + c] = X[a][c];
        z += X[a][c] * yv[c];
      }
      zs[a] = z;
      yw[sl[a]] = z;
    }
    if (bad) *bad_flag = 1;
  }
  wave_lds_sync();
}

// One banded system of a band_solve_kernel launch (workgroup b takes system b).
// Ab: [n + 6][w + 1] band rows of the damped system, Ab[i][d] = A[i][i - d] (d <= min(i, w)),
// then 6 spare rows (at least 64 values: scratch); overwritten by the rows of L (reciprocal
// diagonal). y: [n + 64] right-hand side, overwritten by the solution (64 spare values). n is a
// multiple of 6, and n + 18 (w + 1) <= kBandMaxN (the backward sweep keeps y and three blocks of
// rows of L in LDS).
// Partial sweeps (the two ends of a split system): nf is the number of 6-unknown blocks that
// are eliminated; the rows from 6 nf on are the separator. xs holds the separator's solution
// for the backward sweep, separator unknown r at row 6 nf + r, or at row n - 1 - r when the
// system is stored in reverse order (xs_rev).
struct BandSystem {
  double* Ab;
  double* y;
  int n, nf;
  const double* xs;
  int xs_rev;
};
struct BandSystems {
  BandSystem a, b;
};
constexpr int kBandFull = 0;  // factor, forward and backward substitution
constexpr int kBandFwd = 1;   // eliminate blocks 0 .. nf - 1 (factor rows and forward
                              // substitution); the separator's rows, reduced by the eliminated
                              // blocks (their Schur complement and right-hand side), are written
                              // back to Ab and y
constexpr int kBandBwd = 2;   // backward substitution of blocks nf - 1 .. 0, the separator's
                              // unknowns read from xs; y gets the whole solution
// Layout: the window's rows at an odd stride, the panel column-major (Pc[b][slot]). The rank-6
// update runs on FP64 matrix cores, 16 x 16 tiles read from and written back to the window.
// Lookahead: wave 0 updates the tile that holds the next diagonal block first and then factors
// that block while the other waves finish the update, so the serial 6 x 6 factorizations
// overlap the bulk of the work.
template <int MODE>
__global__ __launch_bounds__(kBandThreads) void band_solve_kernel(BandSystems sys, int w,
                                                                  unsigned* __restrict__ flags) {
  // the workgroup's system (uniform selects: no indexing of the argument block)
  const bool second = blockIdx.x != 0;
  double* __restrict__ Ab = second ? sys.b.Ab : sys.a.Ab;
  double* __restrict__ y = second ? sys.b.y : sys.a.y;
  const int n = second ? sys.b.n : sys.a.n;
  const double* __restrict__ xs = second ? sys.b.xs : sys.a.xs;
  const int xs_rev = second ? sys.b.xs_rev : sys.a.xs_rev;
  __shared__ double lds[kBandMaxN + 80];
  double* Wn = lds;                // the window (forward), y and the ring (backward)
  double* dump = lds + kBandMaxN;  // words for writes that must land nowhere (one per lane, and
                                   // 12 more for the update's rows that do not exist)
  __shared__ double Pc[6][kBandPcLD];
  __shared__ double yw[kBandMaxR];
  __shared__ double Xs[36];
  __shared__ double zs[6];
  __shared__ double zsb[2][6];
  __shared__ int s_bad;
  const int t = threadIdx.x, lane = t & 63;
  // whole waves take the producer's or the compute branch (a wave-uniform condition), and the
  // two branches pass the same barriers in the same order
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int W1 = w + 1, R = w + 6;
  const int nb = n / 6;
  const int nf = MODE == kBandFull ? nb : (second ? sys.b.nf : sys.a.nf);  // blocks eliminated
  const int rv = 6 * W1;  // band values of one block's rows
  double* ys = Wn;        // backward sweep: the right-hand side
  double* ring = Wn + n;  // backward sweep: the rows of L of three blocks
  // the backward sweep's right-hand side: z of the forward sweep, the separator's solution where
  // it is given
  auto band_rhs_in = [&](int i) {
    if (MODE == kBandBwd && i >= 6 * nf) return xs[xs_rev ? n - 1 - i : i - 6 * nf];
    return y[i];
  };
  if (t == 0) s_bad = 0;
  if (MODE != kBandBwd) {
    for (int e = t; e < R * W1; e += kBandThreads) {
      const int i = e / W1, d = e % W1;
      Wn[i * kBandLD + d] = (i < n && d <= i) ? Ab[(long long)i * W1 + d] : 0.0;
    }
    for (int i = t; i < R; i += kBandThreads) yw[i] = i < n ? y[i] : 0.0;
    __syncthreads();
    if (t < 64 && nf > 0) band_diag_block(0, R, Wn, yw, Xs, zs, &s_bad, t);
  }
  __syncthreads();
  if (wv >= kBandWaves) {
    // ---- producers (element e of a block's rows goes to producer lane e mod 128)
    const int pl = 64 * (wv - kBandWaves) + lane;
    // value u of a lane is element e = lane + 64 u of a block's rows (row e / W1, band column
    // e mod W1); lanes past the end load from and store to the spare block after the matrix, so
    // every load and store is issued on every step
    const float inv_w1 = 1.0f / (float)W1;
    auto row_of = [&](int e) { return (int)(((float)e + 0.5f) * inv_w1); };  // exact: e < 2^10
    // global accesses: a block-uniform base and a 32-bit byte offset per lane
    auto ld = [](const double* base, unsigned off) {
      return *(const double*)((const char*)base + off);
    };
    auto st = [](double* base, unsigned off, double v) { *(double*)((char*)base + off) = v; };
    // rows entering the window after step s: 6 s + R + a (raw values; masked where they are
    // used); past the matrix the block is read from the spare rows
    // (the lane index passes through an empty asm statement on every step, so that the per-lane
    // offsets are recomputed rather than hoisted out of the loop and spilled)
    auto fresh_lane = [&]() {
      int l = pl;
      asm volatile("" : "+v"(l));
      return l;
    };
    auto load_in = [&](int s, double(&buf)[kBandPer], double& by) {
      const long long o = min(6LL * s + R, (long long)n) * W1;
      const double* base = Ab + o;
      const int ln = fresh_lane();
#pragma unroll
      for (int u = 0; u < kBandPer; ++u) {
        const int e = ln + 64 * kBandProd * u;
        buf[u] = ld(base, 8u * (unsigned)(e < rv ? e : rv - 1));
      }
      const long long iy = min(6LL * s + R, (long long)n);
      by = ld(y + iy, 8u * (unsigned)lane);
    };
    // step s: the rows of block s leave (rows of L and z to global memory), the rows loaded for
    // step s take their slots
    auto swap_rows = [&](int s, const double(&buf)[kBandPer], double by) {
      const int j0 = 6 * s, b0 = j0 % R;
      const long long r0 = (long long)j0 + R;
      double* base = Ab + (long long)j0 * W1;
      const int ln = fresh_lane();
      const unsigned spare = 8u * (unsigned)((n - j0) * W1 + lane);  // in the spare rows
      int loc[kBandPer];
      double old[kBandPer];
#pragma unroll
      for (int u = 0; u < kBandPer; ++u) {
        const int e = ln + 64 * kBandProd * u;
        const int a = row_of(e), d = e - a * W1;
        const int sr = b0 + a < R ? b0 + a : b0 + a - R;
        loc[u] = e < rv ? sr * kBandLD + d : -1;
        old[u] = Wn[loc[u] >= 0 ? loc[u] : 0];
      }
      const bool ly = ln < 6;
      const int sy = ly ? (b0 + ln < R ? b0 + ln : b0 + ln - R) : 0;
      const double oy = yw[sy];
#pragma unroll
      for (int u = 0; u < kBandPer; ++u)
        st(base, loc[u] >= 0 ? 8u * (unsigned)(ln + 64 * kBandProd * u) : spare, old[u]);
      st(y + j0, 8u * (unsigned)(ly ? ln : n - j0 + lane), oy);
#pragma unroll
      for (int u = 0; u < kBandPer; ++u) {
        const int e = ln + 64 * kBandProd * u;
        const int a = row_of(e), d = e - a * W1;
        *(loc[u] >= 0 ? &Wn[loc[u]] : &dump[lane]) = (r0 + a < n && d <= r0 + a) ? buf[u] : 0.0;
      }
      *(ly ? &yw[sy] : &dump[lane]) = r0 + ln < n ? by : 0.0;
    };
    double bufA[kBandPer], bufB[kBandPer], byA = 0.0, byB = 0.0;
    if (MODE != kBandBwd) {
      if (nf > 0) {
        load_in(0, bufA, byA);
        load_in(1, bufB, byB);
      }
      // two steps per iteration, so that each buffer keeps its registers (straight-line code:
      // the waits before a buffer is used count the loads and stores issued after it). The
      // swap of step s runs beside the step's trailing update, after the panel's barrier: the
      // rows of block s are final and no longer read, and the slots they free are read from
      // step s + 1 on.
      int s = 0;
      for (; s + 1 < nf; s += 2) {
        __syncthreads();
        swap_rows(s, bufA, byA);
        load_in(s + 2, bufA, byA);
        __syncthreads();
        __syncthreads();
        swap_rows(s + 1, bufB, byB);
        load_in(s + 3, bufB, byB);
        __syncthreads();
      }
      if (s < nf) {
        __syncthreads();
        swap_rows(s, bufA, byA);
        __syncthreads();
      }
    }
    if constexpr (MODE != kBandFwd) {
      // the rows of L and z are in global memory for the backward sweep
      __threadfence();
      __syncthreads();
      for (int i = t; i < n; i += kBandThreads) ys[i] = band_rhs_in(i);
      // block sb's rows of L, all of them (rows 6 sb .. 6 sb + 5 are contiguous)
      auto load_blk = [&](int sb, double(&buf)[kBandPer]) {
        const double* base = Ab + 6LL * (sb > 0 ? sb : 0) * W1;
        const int ln = fresh_lane();
#pragma unroll
        for (int u = 0; u < kBandPer; ++u) {
          const int e = ln + 64 * kBandProd * u;
          buf[u] = ld(base, 8u * (unsigned)(e < rv ? e : rv - 1));
        }
      };
      auto put_blk = [&](int sb, const double(&buf)[kBandPer]) {
        double* r = ring + (sb % 3) * rv;
        const int ln = fresh_lane();
#pragma unroll
        for (int u = 0; u < kBandPer; ++u) {
          const int e = ln + 64 * kBandProd * u;
          *(e < rv ? &r[e] : &dump[lane]) = buf[u];
        }
      };
      // the ring holds three blocks: step s reads block s (updates) and block s - 1 (the
      // lookahead solve) while the producer writes block s - 2; bufA holds the block that goes
      // into the ring next, bufB the one after it
      if (nb > 0) {
        load_blk(nb - 1, bufA);
        load_blk(nb - 2, bufB);
        put_blk(nb - 1, bufA);
        if (nb > 1) put_blk(nb - 2, bufB);
        load_blk(nb - 3, bufA);
        load_blk(nb - 4, bufB);
      }
      __syncthreads();
      __syncthreads();
      // two steps per iteration as above
      int sb = nb - 1;
      for (; sb >= 3; sb -= 2) {
        put_blk(sb - 2, bufA);
        load_blk(sb - 4, bufA);
        __syncthreads();
        put_blk(sb - 3, bufB);
        load_blk(sb - 5, bufB);
        __syncthreads();
      }
      for (; sb >= 0; --sb) {
        if (sb == 2) put_blk(0, bufA);
        __syncthreads();
      }
    }
  } else {
    // ---- compute waves
    // rank-6 update in 16 x 16 tiles of the trailing window (rows and columns tt, tk below the
    // block, tk <= tt): tile (0, 0) belongs to wave 0, which then factors the next diagonal
    // block (lookahead); the others are dealt to waves 1 .. 7 and the rest to wave 0
    const int nT = (w + 15) / 16;
    const int ntile = nT * (nT + 1) / 2;
    const int tiles_per_wave = (ntile - 1 + kBandWaves - 1) / kBandWaves;
    // tile row of tile q in the row-major order of the lower triangle of tiles
    auto tile_row_of = [](int q) {
      int TI = (int)((sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
      while ((TI + 1) * (TI + 2) / 2 <= q) ++TI;
      while (TI * (TI + 1) / 2 > q) --TI;
      return TI;
    };
    const int g = lane >> 4, c16 = lane & 15;
    const int dump_word = kBandMaxN + lane;  // a lane's dump word, as an index of Wn
    for (int s = 0; s < (MODE == kBandBwd ? 0 : nf); ++s) {
      const int j0 = 6 * s;
      const int base = (j0 + 6) % R;  // slot of the window row j0 + 6 (tt = 0)
      auto slot = [&](int tt) { return base + tt < R ? base + tt : base + tt - R; };
      // (2) panel: L_i = A_i L_D^-T = A_i X^T for the window rows below the block, and the
      // forward substitution's update of their right-hand side
      for (int tt = t; tt < w; tt += 64 * kBandWaves) {
        const int i = j0 + 6 + tt;
        const int si = slot(tt);
        double p[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (i < n) {
          double a[6];
#pragma unroll
          for (int b = 0; b < 6; ++b) {
            const int d = 6 + tt - b;
            a[b] = d <= w ? Wn[si * kBandLD + d] : 0.0;
          }
#pragma unroll
          for (int b = 0; b < 6; ++b) {
            double v = 0.0;
#pragma unroll
            for (int c = 0; c <= b; ++c) v += Xs[6 * b + c] * a[c];
            p[b] = v;
          }
#pragma unroll
          for (int b = 0; b < 6; ++b) {
            const int d = 6 + tt - b;
            if (d <= w) Wn[si * kBandLD + d] = p[b];
          }
          double yy = yw[si];
#pragma unroll
          for (int b = 0; b < 6; ++b) yy -= p[b] * zs[b];
          yw[si] = yy;
        }
#pragma unroll
        for (int b = 0; b < 6; ++b) Pc[b][si] = p[b];
      }
      __syncthreads();
      // (3) C -= P_I P_K^T on the 16 x 16 tiles (TI, TK), TK <= TI, of the trailing window: two
      // FP64 MFMAs per tile (16 x 16 x 4, the panel's 6 columns padded to 8), on the transposed
      // tile D = C^T: D -= P_K P_I^T. Lane layout: A[p][k] and B[k][q] in lane (p or q) + 16 k,
      // D[p][q] in lane q + 16 (p mod 4), element p / 4. So lane (q, g) holds window row
      // i0 + q, columns k0 + g + 4 v: one row address per lane and four constant offsets (and
      // the lanes of a 16-lane group walk rows, whose stride of kBandLD + 1 doubles spreads them
      // over the LDS banks). Branch-free: operands are read at clamped addresses and zeroed where
      // they do not exist; a lane whose row does not exist, or whose entry of a diagonal tile
      // lies above the diagonal, reads and writes its dump words. The tiles of one tile row
      // share the row side (the row address and mask, the B operand).
      int rrow = 0;       // window index of (row i0 + c16, column g) plus k0: rrow - k0 - 4 v
      bool rok = false;   // the lane's row exists
      double a0 = 0.0, a1 = 0.0;
      auto row_setup = [&](int TI) {
        const int tt = 16 * TI + c16;
        rok = tt < w && j0 + 6 + tt < n;
        const int st = tt < w ? slot(tt) : 0;
        rrow = st * kBandLD + tt - g;
        const double x0 = Pc[g][st], x1 = Pc[4 + (g & 1)][st];
        a0 = tt < w ? -x0 : 0.0;
        a1 = (tt < w && g < 2) ? -x1 : 0.0;
      };
      // NT tiles (TI, TK0 .. TK0 + NT - 1) of one tile row: every load first, then the MFMA
      // chains side by side, then the stores (their entries are disjoint)
      auto tiles = [&](auto nt_tag, int TI, int TK0) {
        constexpr int NT = decltype(nt_tag)::value;
        double b0[NT], b1[NT];
        int addr[NT][4];
        dbl4 c[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const int TK = TK0 + j, k0 = 16 * TK;
          const int rb = k0 + c16;
          const int sb = rb < w ? slot(rb) : 0;
          const double y0 = Pc[g][sb], y1 = Pc[4 + (g & 1)][sb];
          b0[j] = rb < w ? y0 : 0.0;
          b1[j] = (rb < w && g < 2) ? y1 : 0.0;
          if (TK != TI) {
            // below the diagonal: every entry of an existing row exists (band offset <= w)
            const int base = rok ? rrow - k0 - 12 : dump_word;
#pragma unroll
            for (int v = 0; v < 4; ++v) addr[j][v] = base + 12 - 4 * v;
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v)
              addr[j][v] = rok && g + 4 * v <= c16 ? rrow - k0 - 4 * v : dump_word;
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) c[j][v] = Wn[addr[j][v]];
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) c[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0[j], a0, c[j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < NT; ++j) c[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1[j], a1, c[j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) Wn[addr[j][v]] = c[j][v];
      };
      using one = std::integral_constant<int, 1>;
      using two = std::integral_constant<int, 2>;
      if (wv == 0) {
        // tile (0, 0) holds the next diagonal block
        row_setup(0);
        tiles(one{}, 0, 0);
        wave_lds_sync();
        if (s + 1 < nf) band_diag_block(s + 1, R, Wn, yw, Xs, zs, &s_bad, lane);
      }
      if (j0 + 6 + 16 < n) {
        // the other tiles in row-major order, (1, 0), (1, 1), (2, 0), ...: contiguous shares of
        // ceil(tiles / 8) for waves 1 .. 7, what is left for wave 0 after its diagonal block
        // (tiles whose rows are all past the matrix are skipped)
        const int q0 = 1 + (wv == 0 ? kBandWaves - 1 : wv - 1) * tiles_per_wave;
        const int q1 = wv == 0 ? ntile : min(ntile, q0 + tiles_per_wave);
        if (q0 < q1) {
          int TI = tile_row_of(q0), TK = q0 - TI * (TI + 1) / 2;
          row_setup(TI);
          for (int q = q0; q < q1;) {
            if (j0 + 6 + 16 * TI >= n) break;
            if (q + 1 < q1 && TK + 1 <= TI) {
              tiles(two{}, TI, TK);
              q += 2;
              TK += 2;
            } else {
              tiles(one{}, TI, TK);
              q += 1;
              TK += 1;
            }
            if (TK > TI) {
              ++TI;
              TK = 0;
              if (q < q1) row_setup(TI);
            }
          }
        }
      }
      __syncthreads();
    }
    if constexpr (MODE != kBandFwd) {
      __syncthreads();
      __threadfence();  // no stale cached copy of y: the producer has stored z there
      for (int i = t; i < n; i += kBandThreads) ys[i] = band_rhs_in(i);
      __syncthreads();
      // backward substitution L^T x = z: x of block s is known at step s; the w unknowns before
      // the block subtract its contribution, and wave 0, which holds the 6 of them that form block
      // s - 1, then solves that block by substitution with its L_D (lookahead)
      auto solve_blk = [&](int sb) {
        const double* rs = ring + (sb % 3) * rv;
        const int j0 = 6 * sb;
        if (MODE == kBandBwd && sb >= nf) {  // a separator block: its unknowns are given
#pragma unroll
          for (int b = 0; b < 6; ++b) zsb[sb & 1][b] = ys[j0 + b];
          return;
        }
        double x[6];
#pragma unroll
        for (int b = 5; b >= 0; --b) {
          double v = ys[j0 + b];
#pragma unroll
          for (int c = b + 1; c < 6; ++c) v -= rs[c * W1 + (c - b)] * x[c];
          x[b] = v * rs[b * W1];
        }
#pragma unroll
        for (int b = 0; b < 6; ++b) {
          ys[j0 + b] = x[b];
          zsb[sb & 1][b] = x[b];
        }
      };
      if (t == 0 && nb > 0) solve_blk(nb - 1);
      __syncthreads();
      for (int s = nb - 1; s >= 0; --s) {
        const int j0 = 6 * s;
        const double* rs = ring + (s % 3) * rv;
        const double* zc = zsb[s & 1];
        // (a separator block's contribution goes to the eliminated unknowns only)
        if (t < w && j0 - 1 - t >= 0 && (MODE != kBandBwd || j0 - 1 - t < 6 * nf)) {
          const int k = j0 - 1 - t;
          double v = ys[k];
#pragma unroll
          for (int b = 0; b < 6; ++b) {
            const int d = b + 1 + t;
            if (d <= w) v -= rs[b * W1 + d] * zc[b];
          }
          ys[k] = v;
        }
        if (wv == 0) {
          wave_lds_sync();
          if (t == 0 && s > 0) solve_blk(s - 1);
        }
        __syncthreads();
      }
    }
  }
  __syncthreads();
  if (MODE == kBandFwd) {
    // the separator's rows: the rows of L towards the eliminated blocks, the Schur complement,
    // and the right-hand side after the forward substitution
    const int r0 = 6 * nf;
    for (int e = t; e < (n - r0) * W1; e += kBandThreads) {
      const int i = r0 + e / W1, d = e % W1;
      Ab[(long long)i * W1 + d] = Wn[(i % R) * kBandLD + d];
    }
    for (int i = r0 + t; i < n; i += kBandThreads) y[i] = yw[i % R];
  } else {
    for (int i = t; i < n; i += kBandThreads) y[i] = ys[i];
  }
  if (t == 0 && s_bad) atomicOr(flags, kFlagNonFinite);
}

// ------------------------------------------------------------------ banded assembly

// Zeroes the band rows (Ab: total values; a split system's bottom end: total2 values of Ab2 and
// its right-hand side y2, whose separator rows no pose writes) and diag_raw.
__global__ __launch_bounds__(256) void band_clear_kernel(double* __restrict__ Ab, long long total,
                                                         double* __restrict__ Ab2,
                                                         long long total2,
                                                         double* __restrict__ y2, int n2,
                                                         double* __restrict__ diag_raw, int n) {
  const long long m = max(total, total2);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (long long)gridDim.x * blockDim.x) {
    if (i < total) Ab[i] = 0.0;
    if (i < total2) Ab2[i] = 0.0;
    if (i < n2) y2[i] = 0.0;
    if (i < n) diag_raw[i] = 0.0;
  }
}

// As lm_assemble_kernel, into the band rows of the permuted system: pose p moves to position
// pos[p]; only the lower triangle is stored (entry (I, J), I >= J, at Ab[I][I - J]). A split
// system keeps rows I < n_top in Ab and the rows below in Ab_bot, in reverse order: entry
// (I, J) is entry (n - 1 - J, n - 1 - I) of the reversed matrix, at Ab_bot[n - 1 - J][I - J].
__global__ __launch_bounds__(256) void band_assemble_kernel(
    const LmBlock* __restrict__ blocks, int nblocks, const int* __restrict__ contrib,
    const double* __restrict__ Hf, const double* __restrict__ lambda, int fixed,
    const int* __restrict__ pos, int w, double* __restrict__ Ab, double* __restrict__ diag_raw,
    int n_top, int n, double* __restrict__ Ab_bot) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nblocks * 36) return;
  const LmBlock bk = blocks[t / 36];
  const int e = t % 36, r = e / 6, c = e % 6;
  if (bk.row == fixed || bk.col == fixed) return;
  const long long I = 6LL * pos[bk.row] + r, J = 6LL * pos[bk.col] + c;
  if (J > I) return;  // the upper triangle is implied
  double s = 0.0;
#pragma unroll 8  // loads issued together, the sum in its order
  for (int q = 0; q < bk.count; ++q) {
    const int wq = contrib[bk.first + q];
    const int f = wq >> 2, a = (wq >> 1) & 1, b = wq & 1;
    s += Hf[144LL * f + (6 * a + r) * 12 + 6 * b + c];
  }
  if (I == J) {
    diag_raw[6LL * bk.row + r] = s;
    s = s > 0.0 ? s * (1.0 + *lambda) : 1.0;
  }
  if (I < n_top)
    Ab[I * (w + 1) + (I - J)] = s;
  else
    Ab_bot[(n - 1 - J) * (w + 1) + (I - J)] = s;
}

// Right-hand side -b in the permuted order, and unit diagonals for poses without a factor,
// for zero diagonal entries and for the fixed pose.
__global__ __launch_bounds__(256) void band_rhs_kernel(const int* __restrict__ bptr,
                                                       const int* __restrict__ bcontrib,
                                                       const double* __restrict__ bf, int P,
                                                       int fixed, const int* __restrict__ pos,
                                                       int w, double* __restrict__ Ab,
                                                       const double* __restrict__ diag_raw,
                                                       double* __restrict__ g, int n_top, int n,
                                                       double* __restrict__ Ab_bot,
                                                       double* __restrict__ g_bot) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 6 * P) return;
  const int p = t / 6, r = t % 6;
  double s = 0.0;
#pragma unroll 8  // loads issued together, the sum in its order
  for (int q = bptr[p]; q < bptr[p + 1]; ++q) {
    const int wq = bcontrib[q];
    s += bf[12LL * (wq >> 1) + 6 * (wq & 1) + r];
  }
  const long long I = 6LL * pos[p] + r;
  const bool top = I < n_top;  // else a row of a split system's bottom end (reverse order)
  const long long Ir = top ? I : n - 1 - I;
  if (p == fixed || !(diag_raw[t] > 0.0)) {
    (top ? Ab : Ab_bot)[Ir * (w + 1)] = 1.0;
    s = 0.0;
  }
  (top ? g : g_bot)[Ir] = -s;
}

// The separator's system of a split solve: the Schur complements and right-hand sides that the
// two ends leave on it, summed (top + bottom, a fixed order). Separator row r is row r0 + r of
// the top end and row n_bot - 1 - r of the bottom end (reverse order). w + 1 rows.
__global__ __launch_bounds__(256) void band_sep_kernel(const double* __restrict__ Ab_top,
                                                       const double* __restrict__ y_top, int r0,
                                                       const double* __restrict__ Ab_bot,
                                                       const double* __restrict__ y_bot,
                                                       int n_bot, int w,
                                                       double* __restrict__ Ab_sep,
                                                       double* __restrict__ y_sep) {
  const int W1 = w + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < W1 * W1) {
    const int r = e / W1, d = e % W1;
    double v = 0.0;
    if (d <= r)
      v = Ab_top[(long long)(r0 + r) * W1 + d] + Ab_bot[(long long)(n_bot - 1 - (r - d)) * W1 + d];
    Ab_sep[e] = v;
  }
  if (e < W1) y_sep[e] = y_top[r0 + e] + y_bot[n_bot - 1 - e];
}

// poses_new[p] = poses[p] Exp(x[6 pos[p] ..]), delta[p] = that step.
__global__ __launch_bounds__(256) void band_retract_kernel(const double* __restrict__ poses,
                                                           const double* __restrict__ x,
                                                           const int* __restrict__ pos, int P,
                                                           double* __restrict__ poses_new,
                                                           double* __restrict__ delta,
                                                           const double* __restrict__ x_bot,
                                                           int n_top, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double xi[6], o[12];
  for (int a = 0; a < 6; ++a) {
    const long long I = 6LL * pos[p] + a;
    xi[a] = I < n_top ? x[I] : x_bot[n - 1 - I];  // a split system's bottom end: reverse order
  }
  se3_retract(poses + 12LL * p, xi, o);
  for (int a = 0; a < 12; ++a) poses_new[12LL * p + a] = o[a];
  if (delta)
    for (int a = 0; a < 6; ++a) delta[6LL * p + a] = xi[a];
}

// ------------------------------------------------------------------ iteration on the device

__global__ void lm_set_kernel(double* __restrict__ p, double v) { *p = v; }

// Sum of F costs in a fixed order (strided partial sums over 256 threads, then a tree).
// The step is taken when the candidate's cost is finite and below the current one: lambda / 10,
// else lambda * 10 (kept within [1e-12, 1e12]). cost_out: the cost after the iteration.
__global__ __launch_bounds__(256) void lm_decide_kernel(const double* __restrict__ e_cur,
                                                        const double* __restrict__ e_cand, int F,
                                                        double* __restrict__ lambda,
                                                        int* __restrict__ accept,
                                                        double* __restrict__ cost_first,
                                                        double* __restrict__ cost_out) {
  double c0, c1;
  block_cost_sums(e_cur, e_cand, F, c0, c1);  // the same order as lm_cost_kernel's
  if (threadIdx.x == 0) {
    const bool take = isfinite(c1) && c1 < c0;
    *accept = take ? 1 : 0;
    const double l = take ? *lambda * 0.1 : *lambda * 10.0;
    *lambda = fmin(fmax(l, 1e-12), 1e12);
    if (cost_first) *cost_first = c0;
    *cost_out = take ? c1 : c0;
  }
}

// On a taken step the candidate becomes the current state: poses and the linearization.
__global__ __launch_bounds__(256) void lm_commit_kernel(const int* __restrict__ accept, int P,
                                                        int F, const double* __restrict__ cand,
                                                        double* __restrict__ poses,
                                                        const double* __restrict__ Hc,
                                                        const double* __restrict__ bc,
                                                        const double* __restrict__ ec,
                                                        double* __restrict__ H,
                                                        double* __restrict__ b,
                                                        double* __restrict__ e) {
  if (!*accept) return;
  const long long nH = 144LL * F, nb = 12LL * F, nP = 12LL * P;
  const long long total = nH + nb + F + nP;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    if (i < nH)
      H[i] = Hc[i];
    else if (i < nH + nb)
      b[i - nH] = bc[i - nH];
    else if (i < nH + nb + F)
      e[i - nH - nb] = ec[i - nH - nb];
    else
      poses[i - nH - nb - F] = cand[i - nH - nb - F];
  }
}

}  // namespace

// ------------------------------------------------------------------ pose order

namespace {

// Largest distance, in positions, between two poses linked by a factor.
int pose_bandwidth(const std::vector<std::vector<int>>& adj, const std::vector<int>& pos) {
  int bw = 0;
  for (int p = 0; p < (int)adj.size(); ++p)
    for (int q : adj[p]) bw = std::max(bw, std::abs(pos[p] - pos[q]));
  return bw;
}

// Breadth-first levels from `start` (distances; -1 unreached).
std::vector<int> bfs_dist(const std::vector<std::vector<int>>& adj, int start) {
  std::vector<int> d(adj.size(), -1), q;
  q.push_back(start);
  d[start] = 0;
  for (size_t h = 0; h < q.size(); ++h)
    for (int v : adj[q[h]])
      if (d[v] < 0) {
        d[v] = d[q[h]] + 1;
        q.push_back(v);
      }
  return d;
}

// Reverse Cuthill-McKee order (Cuthill and McKee 1969; reversed as George 1971): breadth-first
// from `start`, neighbours by increasing degree, every further component from its lowest-degree
// pose, then the whole order reversed. Returns the position of every pose.
std::vector<int> rcm_positions(const std::vector<std::vector<int>>& adj, int start) {
  const int P = (int)adj.size();
  std::vector<int> order, seen(P, 0);
  order.reserve(P);
  auto deg = [&](int v) { return (int)adj[v].size(); };
  int next = start;
  while ((int)order.size() < P) {
    if (next < 0) {
      for (int v = 0; v < P; ++v)
        if (!seen[v] && (next < 0 || deg(v) < deg(next))) next = v;
    }
    size_t h = order.size();
    order.push_back(next);
    seen[next] = 1;
    for (; h < order.size(); ++h) {
      std::vector<int> nb;
      for (int v : adj[order[h]])
        if (!seen[v]) {
          seen[v] = 1;
          nb.push_back(v);
        }
      std::stable_sort(nb.begin(), nb.end(), [&](int a, int b) { return deg(a) < deg(b); });
      order.insert(order.end(), nb.begin(), nb.end());
    }
    next = -1;
  }
  std::vector<int> pos(P);
  for (int i = 0; i < P; ++i) pos[order[P - 1 - i]] = i;
  return pos;
}

// Spectral order (the poses sorted by their entry of the graph Laplacian's second eigenvector):
// power iteration on c I - L (c above L's largest eigenvalue) with the constant vector removed,
// from a ramp, for a fixed budget of iterations. Deterministic; ties by pose index.
std::vector<int> spectral_positions(const std::vector<std::vector<int>>& adj) {
  const int P = (int)adj.size();
  long long nnz = 0;
  int maxdeg = 0;
  for (auto& a : adj) {
    nnz += (long long)a.size();
    maxdeg = std::max(maxdeg, (int)a.size());
  }
  const double c = 2.0 * maxdeg + 1.0;
  std::vector<double> v(P), u(P);
  for (int i = 0; i < P; ++i) v[i] = (double)i - 0.5 * (P - 1);
  const long long iters = std::max<long long>(
      50, std::min<long long>(4000, 50000000LL / std::max<long long>(1, nnz + P)));
  for (long long it = 0; it < iters; ++it) {
    for (int i = 0; i < P; ++i) {
      double s = (c - (double)adj[i].size()) * v[i];
      for (int q : adj[i]) s += v[q];
      u[i] = s;
    }
    double mean = 0.0;
    for (double x : u) mean += x;
    mean /= P;
    double nrm = 0.0;
    for (int i = 0; i < P; ++i) {
      u[i] -= mean;
      nrm += u[i] * u[i];
    }
    nrm = std::sqrt(nrm);
    if (!(nrm > 0.0)) break;
    for (int i = 0; i < P; ++i) v[i] = u[i] / nrm;
  }
  std::vector<int> order(P);
  for (int i = 0; i < P; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return v[a] < v[b]; });
  std::vector<int> pos(P);
  for (int i = 0; i < P; ++i) pos[order[i]] = i;
  return pos;
}

}  // namespace

// A bandwidth-reducing order of the poses: the identity, reverse Cuthill-McKee from a
// pseudo-peripheral pose (George and Liu's repeated breadth-first search) and from the lowest-
// degree poses, and the spectral order; the one with the smallest bandwidth is kept.
void order_poses(const std::vector<std::vector<int>>& adj, std::vector<int>& pos, int& bw) {
  const int P = (int)adj.size();
  pos.resize(P);
  for (int i = 0; i < P; ++i) pos[i] = i;
  bw = pose_bandwidth(adj, pos);
  if (P < 3) return;
  auto consider = [&](std::vector<int> cand) {
    const int b = pose_bandwidth(adj, cand);
    if (b < bw) {
      bw = b;
      pos = std::move(cand);
    }
  };
  // pseudo-peripheral pose of the first component
  int s = 0;
  for (int round = 0; round < 8; ++round) {
    const std::vector<int> d = bfs_dist(adj, s);
    int far = s;
    for (int v = 0; v < P; ++v)
      if (d[v] > d[far] || (d[v] == d[far] && d[v] >= 0 && adj[v].size() < adj[far].size()))
        far = v;
    if (far == s) break;
    s = far;
  }
  consider(rcm_positions(adj, s));
  std::vector<int> bydeg(P);
  for (int i = 0; i < P; ++i) bydeg[i] = i;
  std::stable_sort(bydeg.begin(), bydeg.end(),
                   [&](int a, int b) { return adj[a].size() < adj[b].size(); });
  for (int k = 0; k < std::min(P, 4); ++k) consider(rcm_positions(adj, bydeg[k]));
  consider(spectral_positions(adj));
}

void build_lm_structure(const std::vector<FactorView>& hf, int P, LmStructure& s) {
  std::map<std::pair<int, int>, std::vector<int>> blocks;
  std::vector<std::vector<int>> rhs((size_t)P);
  for (int f = 0; f < (int)hf.size(); ++f) {
    const int sp = hf[f].source_pose, tp = hf[f].target_pose;
    blocks[{sp, sp}].push_back(f << 2);
    rhs[sp].push_back(f << 1);
    if (hf[f].binary) {
      blocks[{sp, tp}].push_back((f << 2) | 1);
      blocks[{tp, sp}].push_back((f << 2) | 2);
      blocks[{tp, tp}].push_back((f << 2) | 3);
      rhs[tp].push_back((f << 1) | 1);
    }
  }
  s.blocks.clear();
  s.contrib.clear();
  for (auto& kv : blocks) {
    LmBlock b;
    b.row = kv.first.first;
    b.col = kv.first.second;
    b.first = (int)s.contrib.size();
    b.count = (int)kv.second.size();
    s.contrib.insert(s.contrib.end(), kv.second.begin(), kv.second.end());
    s.blocks.push_back(b);
  }
  s.bptr.assign((size_t)P + 1, 0);
  s.bcontrib.clear();
  for (int p = 0; p < P; ++p) {
    s.bptr[p] = (int)s.bcontrib.size();
    s.bcontrib.insert(s.bcontrib.end(), rhs[p].begin(), rhs[p].end());
  }
  s.bptr[P] = (int)s.bcontrib.size();
  s.n_real = 6 * P;
  s.n = ((6 * P + kNB - 1) / kNB) * kNB;
  // the pose order of the banded solve
  std::vector<std::set<int>> nb((size_t)P);
  for (const LmBlock& b : s.blocks)
    if (b.row != b.col) nb[b.row].insert(b.col);
  std::vector<std::vector<int>> adj((size_t)P);
  for (int p = 0; p < P; ++p) adj[p].assign(nb[p].begin(), nb[p].end());
  order_poses(adj, s.pos, s.pose_bw);
  s.w = 6 * s.pose_bw + 5;
  // one sweep keeps the right-hand side and three blocks of rows in LDS for the backward
  // sweep; from both ends each end does, so a long graph fits when its longer end fits
  const int ns = s.pose_bw + 1;  // separator blocks
  const bool narrow = P > 0 && s.w <= kBandMaxW;
  const bool split = narrow && P - ns >= 2 * kBandSplitMin;  // each end >= kBandSplitMin blocks
  const int m_top = split ? (P - ns) / 2 : 0, m_bot = split ? P - ns - m_top : 0;
  s.one_sweep = narrow && 6LL * P + 18LL * (s.w + 1) <= kBandMaxN;
  const bool ends_fit = split && 6LL * (m_bot + ns) + 18LL * (s.w + 1) <= kBandMaxN;
  s.band = s.one_sweep || ends_fit;
  s.split = s.band && split;
  s.m_top = s.split ? m_top : 0;
  s.m_bot = s.split ? m_bot : 0;
}

void launch_lm_solve(const LmDevice& d, int P, int fixed, const double* poses,
                     double* poses_new, double* delta, unsigned* flags, hipStream_t s) {
  if (d.band) {
    const int W1 = d.w + 1, n = 6 * P;
    // split: the top end holds rows 0 .. n_top - 1 (its blocks and the separator), the bottom
    // end the separator and the rows below it, reversed
    const int n_top = d.split ? 6 * d.m_top + W1 : n;
    const int n_bot = d.split ? 6 * d.m_bot + W1 : 0;
    const long long t1 = (long long)n_top * W1, t2 = (long long)n_bot * W1;
    band_clear_kernel<<<grid1(std::max(t1, t2), 256), 256, 0, s>>>(d.Ab, t1, d.Ab_bot, t2,
                                                                   d.x_bot, n_bot, d.diag_raw, n);
    if (d.nblocks > 0)
      band_assemble_kernel<<<grid1(36LL * d.nblocks, 256), 256, 0, s>>>(
          d.blocks, d.nblocks, d.contrib, d.Hf, d.lambda, fixed, d.pos, d.w, d.Ab, d.diag_raw,
          n_top, n, d.Ab_bot);
    band_rhs_kernel<<<grid1(n, 256), 256, 0, s>>>(d.bptr, d.bcontrib, d.bf, P, fixed, d.pos, d.w,
                                                  d.Ab, d.diag_raw, d.x, n_top, n, d.Ab_bot,
                                                  d.x_bot);
    if (!d.split) {
      BandSystems one{};
      one.a = {d.Ab, d.x, n, n / 6, nullptr, 0};
      one.b = one.a;
      band_solve_kernel<kBandFull><<<1, kBandThreads, 0, s>>>(one, d.w, flags);
    } else {
      // the two ends side by side (one workgroup each), the separator, then the two backward
      // sweeps side by side
      BandSystems ends{};
      ends.a = {d.Ab, d.x, n_top, d.m_top, d.x_sep, 0};
      ends.b = {d.Ab_bot, d.x_bot, n_bot, d.m_bot, d.x_sep, 1};
      band_solve_kernel<kBandFwd><<<2, kBandThreads, 0, s>>>(ends, d.w, flags);
      band_sep_kernel<<<grid1((long long)W1 * W1, 256), 256, 0, s>>>(
          d.Ab, d.x, 6 * d.m_top, d.Ab_bot, d.x_bot, n_bot, d.w, d.Ab_sep, d.x_sep);
      BandSystems sep{};
      sep.a = {d.Ab_sep, d.x_sep, W1, W1 / 6, nullptr, 0};
      sep.b = sep.a;
      band_solve_kernel<kBandFull><<<1, kBandThreads, 0, s>>>(sep, d.w, flags);
      band_solve_kernel<kBandBwd><<<2, kBandThreads, 0, s>>>(ends, d.w, flags);
    }
    band_retract_kernel<<<grid1(P, 256), 256, 0, s>>>(poses, d.x, d.pos, P, poses_new, delta,
                                                      d.x_bot, n_top, n);
    return;
  }
  const int n = d.n;
  const long long nn = (long long)n * n;
  lm_clear_kernel<<<grid1(nn, 256), 256, 0, s>>>(d.A, nn, n, d.n_real, d.diag_raw);
  if (d.nblocks > 0)
    lm_assemble_kernel<<<grid1(36LL * d.nblocks, 256), 256, 0, s>>>(
        d.blocks, d.nblocks, d.contrib, d.Hf, d.lambda, fixed, n, d.A, d.diag_raw);
  lm_rhs_kernel<<<grid1(n, 256), 256, 0, s>>>(d.bptr, d.bcontrib, d.bf, P, fixed, n, d.A,
                                               d.diag_raw, d.x);
  const int nblk = n / kNB;
  for (int k = 0; k < nblk; ++k) {
    potrf_diag_kernel<<<1, 256, 0, s>>>(d.A, n, k, d.Dinv, flags);
    const int below = nblk - k - 1;
    if (below > 0) {
      trsm_kernel<<<below, 256, 0, s>>>(d.A, n, k, d.Dinv);
      update_kernel<<<below * (below + 1) / 2, 256, 0, s>>>(d.A, n, k, nblk);
    }
  }
  for (int k = 0; k < nblk; ++k) {
    trsv_diag_kernel<true><<<1, 64, 0, s>>>(d.Dinv, k, d.x);
    const int rows = n - (k + 1) * kNB;
    if (rows > 0) trsv_fwd_update_kernel<<<(rows + 3) / 4, 256, 0, s>>>(d.A, n, k, d.x);
  }
  for (int k = nblk - 1; k >= 0; --k) {
    trsv_diag_kernel<false><<<1, 64, 0, s>>>(d.Dinv, k, d.x);
    if (k > 0) trsv_bwd_update_kernel<<<(k * kNB + 255) / 256, 256, 0, s>>>(d.A, n, k, d.x);
  }
  lm_retract_kernel<<<grid1(P, 256), 256, 0, s>>>(poses, d.x, P, poses_new, delta);
}

void launch_lm_set(double* p, double v, hipStream_t s) { lm_set_kernel<<<1, 1, 0, s>>>(p, v); }

void launch_lm_decide(const double* e_cur, const double* e_cand, int F, double* lambda,
                      int* accept, double* cost_first, double* cost_out, hipStream_t s) {
  lm_decide_kernel<<<1, 256, 0, s>>>(e_cur, e_cand, F, lambda, accept, cost_first, cost_out);
}

void launch_lm_commit(const int* accept, int P, int F, const double* cand, double* poses,
                      const double* Hc, const double* bc, const double* ec, double* H, double* b,
                      double* e, hipStream_t s) {
  const long long total = 157LL * F + 12LL * P;
  lm_commit_kernel<<<grid1(total, 256), 256, 0, s>>>(accept, P, F, cand, poses, Hc, bc, ec, H, b,
                                                     e);
}

void launch_lm_cost(const double* e0, const double* e1, int F, double* cost, hipStream_t s) {
  lm_cost_kernel<<<1, 256, 0, s>>>(e0, e1, F, cost);
}

}  // namespace vgicp
