// One Levenberg-Marquardt step of the pose graph formed by a batch's matching-cost factors
// (Sec. III-F: the global mapping graph over submap poses, optimized with LM; Eq. (2) supplies
// every factor's cost and its Gauss-Newton blocks).
//
//   1. linearize every factor at the current poses (the batched kernel);
//   2. assemble the 6P x 6P system: each 6x6 block and each 6-vector is the sum of its factors'
//      contributions in factor order (one thread per entry, so the result is deterministic);
//   3. damp it as H + lambda diag(H) (Marquardt); a pose that no factor reaches, and an optional
//      fixed pose, get an identity row (their step is zero);
//   4. solve (H + lambda diag H) delta = -b by a dense right-looking blocked Cholesky
//      factorization in FP64 (64 x 64 blocks: diagonal factorization and inverse, panel
//      product, trailing update) and two blocked triangular solves;
//   5. retract every pose, T_i <- T_i Exp(delta_i), and evaluate the cost there.
#include <algorithm>
#include <map>
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
    const double* __restrict__ Hf, double lambda, int fixed, int n, double* __restrict__ A,
    double* __restrict__ diag_raw) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nblocks * 36) return;
  const LmBlock bk = blocks[t / 36];
  const int e = t % 36, r = e / 6, c = e % 6;
  if (bk.row == fixed || bk.col == fixed) return;
  double s = 0.0;
  for (int q = 0; q < bk.count; ++q) {
    const int w = contrib[bk.first + q];
    const int f = w >> 2, a = (w >> 1) & 1, b = w & 1;
    s += Hf[144LL * f + (6 * a + r) * 12 + 6 * b + c];
  }
  const long long i = 6LL * bk.row + r, j = 6LL * bk.col + c;
  if (i == j) {
    diag_raw[i] = s;
    s = s > 0.0 ? s * (1.0 + lambda) : 1.0;
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

// cost[0] = sum of e0, cost[1] = sum of e1, each in a fixed order (strided partial sums, then a
// tree over the 256 threads).
__global__ __launch_bounds__(256) void lm_cost_kernel(const double* __restrict__ e0,
                                                      const double* __restrict__ e1, int F,
                                                      double* __restrict__ cost) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, b = 0.0;
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
  if (threadIdx.x == 0) {
    cost[0] = s0[0];
    cost[1] = s1[0];
  }
}

unsigned grid1(long long n, int block) {
  return (unsigned)std::max<long long>(1, std::min<long long>((n + block - 1) / block, 65536));
}

}  // namespace

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
}

void launch_lm_solve(const LmDevice& d, int P, double lambda, int fixed, const double* poses,
                     double* poses_new, double* delta, unsigned* flags, hipStream_t s) {
  const int n = d.n;
  const long long nn = (long long)n * n;
  lm_clear_kernel<<<grid1(nn, 256), 256, 0, s>>>(d.A, nn, n, d.n_real, d.diag_raw);
  if (d.nblocks > 0)
    lm_assemble_kernel<<<grid1(36LL * d.nblocks, 256), 256, 0, s>>>(
        d.blocks, d.nblocks, d.contrib, d.Hf, lambda, fixed, n, d.A, d.diag_raw);
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

void launch_lm_cost(const double* e0, const double* e1, int F, double* cost, hipStream_t s) {
  lm_cost_kernel<<<1, 256, 0, s>>>(e0, e1, F, cost);
}

}  // namespace vgicp
