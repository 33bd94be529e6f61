// Per-point arithmetic of the VGICP factor for gfx950 (wave64).
//
// Sec. III-A, Eqs. (2)-(3): for a source point (mu, C) and the relative pose T_ts = [R | t]:
//   q = R mu + t, voxel v = floor(q / res), d = mu'_v - q,
//   Omega = (C'_v + R C R^T)^-1, e = d^T Omega d.
// The Gauss-Newton terms are accumulated in the TARGET frame with J_t = [-[q]x, I]:
//   H_t = J_t^T Omega J_t, b_t = J_t^T Omega d (21 + 6 values, plus e), and the source and
// binary blocks are recovered once per factor from J_s = -J_t Ad(T_ts):
//   unary  H_s = Ad^T H_t Ad,  b_s = -Ad^T b_t
//   binary H = B^T H_t B, b = B^T b_t with B = [-Ad | I]  (order [source | target]).
#pragma once

#include "common.h"

namespace vgicp {

// ------------------------------------------------------------------ address spaces

// Pointers fetched from structures in device memory are generic (flat) to the compiler; these
// casts state that the data is in global memory, so that accesses become global loads with a
// scalar base and a 32-bit lane offset instead of flat loads with 64-bit lane addresses.
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <class T>
using gptr = T*;  // the host pass only type-checks device code
#endif

template <class T>
__device__ __forceinline__ gptr<const T> gbl(const T* p) {
  return (gptr<const T>)p;
}

template <class T>
__device__ __forceinline__ gptr<T> gblw(T* p) {
  return (gptr<T>)p;
}

// ------------------------------------------------------------------ voxel keys and hashing

__host__ __device__ inline long long pack_key(int kx, int ky, int kz) {
  return ((long long)(kx + kKeyLimit) << 42) | ((long long)(ky + kKeyLimit) << 21) |
         (long long)(kz + kKeyLimit);
}

// Right perturbation out = T Exp(xi), xi = [omega; rho], T and out row-major [R|t] (12 doubles):
// R = I + A K + B K^2, V = I + B K + C K^2 with K = [omega]x (Rodrigues; series below 1e-6 rad).
__host__ __device__ inline void se3_retract(const double* T, const double* xi, double* o) {
  const double w[3] = {xi[0], xi[1], xi[2]}, rho[3] = {xi[3], xi[4], xi[5]};
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double th = sqrt(th2);
  double A, B, C;
  if (th < 1e-6) {
    A = 1.0 - th2 / 6.0;
    B = 0.5 - th2 / 24.0;
    C = 1.0 / 6.0 - th2 / 120.0;
  } else {
    A = sin(th) / th;
    B = (1.0 - cos(th)) / th2;
    C = (th - sin(th)) / (th2 * th);
  }
  const double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
  double K2[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += K[3 * r + k] * K[3 * k + c];
      K2[3 * r + c] = s;
    }
  double R[9], V[9];
  for (int i = 0; i < 9; ++i) {
    const double I = (i % 4 == 0) ? 1.0 : 0.0;
    R[i] = I + A * K[i] + B * K2[i];
    V[i] = I + B * K[i] + C * K2[i];
  }
  double te[3];
  for (int r = 0; r < 3; ++r)
    te[r] = V[3 * r] * rho[0] + V[3 * r + 1] * rho[1] + V[3 * r + 2] * rho[2];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c)
      o[4 * r + c] = T[4 * r] * R[c] + T[4 * r + 1] * R[3 + c] + T[4 * r + 2] * R[6 + c];
    o[4 * r + 3] = T[4 * r] * te[0] + T[4 * r + 1] * te[1] + T[4 * r + 2] * te[2] + T[4 * r + 3];
  }
}

// Brick of the voxel (dx, dy, dz) (relative to the bounding box; gby x gbz bricks per x-slab)
// and its bit in the brick's occupancy mask.
__host__ __device__ inline unsigned brick_of(unsigned dx, unsigned dy, unsigned dz, unsigned gby,
                                             unsigned gbz) {
  return ((dx >> 2) * gby + (dy >> 2)) * gbz + (dz >> 1);
}
__host__ __device__ inline unsigned bit_in_brick(unsigned dx, unsigned dy, unsigned dz) {
  return ((dx & 3u) << 3) | ((dy & 3u) << 1) | (dz & 1u);
}

// 32-bit finaliser of MurmurHash3 (Appleby): spreads the dense relative keys of surface voxels
// over the table.
__host__ __device__ inline unsigned hash32(unsigned h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

__host__ __device__ inline unsigned hash64(long long k) {
  return hash32((unsigned)k ^ ((unsigned)((unsigned long long)k >> 32) * 0x9e3779b9u));
}

// q = R mu + t in FP64 with one fixed evaluation order and no fused multiply-add, so that the
// voxel a point falls in is decided exactly as the definition writes it.
__device__ inline void transform_exact(const double* R, const double* t, float x, float y,
                                       float z, double q[3]) {
#pragma clang fp contract(off)
  const double X = x, Y = y, Z = z;
  q[0] = ((R[0] * X + R[1] * Y) + R[2] * Z) + t[0];
  q[1] = ((R[3] * X + R[4] * Y) + R[5] * Z) + t[1];
  q[2] = ((R[6] * X + R[7] * Y) + R[8] * Z) + t[2];
}

// Voxel coordinate of one axis: floor(v / res) toward -inf. DIV = false multiplies by 1/res,
// which rounds identically when res is a power of two; callers pick DIV from the map (a uniform
// branch around the whole tile, so the division is only paid where it is needed). Returns 0 and
// sets k, 1 for non-finite v, 2 when |k| >= 2^20.
template <bool DIV>
__device__ inline int voxel_coord(double v, double res, double inv_res, int* k) {
  const double s = DIV ? v / res : v * inv_res;
  const double f = floor(s);
  if (!isfinite(f)) return 1;
  if (!(fabs(f) < (double)kKeyLimit)) return 2;
  *k = (int)f;
  return 0;
}

// Branch-free voxel coordinate from s = v / res: floor(s) as an int32, saturated by the
// hardware conversion (NaN gives 0; the caller rejects non-finite points). Every map voxel has
// |k| < 2^20, so an out-of-range coordinate always fails the map's bounding-box test (computed
// in unsigned arithmetic): out-of-range points become misses without control flow.
__device__ inline int floor_sat_i32(double s) {
  int k;
  asm("v_cvt_i32_f64 %0, %1" : "=v"(k) : "v"(floor(s)));
  return k;
}

__device__ inline int floor_sat_i32_f32(float s) {
  int k;
  asm("v_cvt_i32_f32 %0, %1" : "=v"(k) : "v"(floorf(s)));
  return k;
}

// ------------------------------------------------------------------ fused covariance inverse

// Omega = (Cv + R C R^T)^-1, formed in FP64 whatever the precision of the rest of the point's
// arithmetic: with plane-like covariances the fused covariance has a smallest eigenvalue ~1e-3
// of its entries, and forming or inverting it in FP32 would lose about that factor of accuracy
// in the surface-normal direction (FP64 vector arithmetic runs at the FP32 rate on this GPU).
// Adjugate inverse with Sylvester's criterion; o = (xx, xy, xz, yy, yz, zz). False when the
// fused covariance is not positive definite or not finite.
template <typename T>
__device__ inline bool fused_inverse(const double* R, const double* cv, const float* c, T o[6]) {
  const double c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3], c4 = c[4], c5 = c[5];
  // rows of R C
  const double a0 = R[0] * c0 + R[1] * c1 + R[2] * c2;
  const double a1 = R[0] * c1 + R[1] * c3 + R[2] * c4;
  const double a2 = R[0] * c2 + R[1] * c4 + R[2] * c5;
  const double b0 = R[3] * c0 + R[4] * c1 + R[5] * c2;
  const double b1 = R[3] * c1 + R[4] * c3 + R[5] * c4;
  const double b2 = R[3] * c2 + R[4] * c4 + R[5] * c5;
  const double g0 = R[6] * c0 + R[7] * c1 + R[8] * c2;
  const double g1 = R[6] * c1 + R[7] * c3 + R[8] * c4;
  const double g2 = R[6] * c2 + R[7] * c4 + R[8] * c5;
  const double s00 = cv[0] + (a0 * R[0] + a1 * R[1] + a2 * R[2]);
  const double s01 = cv[1] + (a0 * R[3] + a1 * R[4] + a2 * R[5]);
  const double s02 = cv[2] + (a0 * R[6] + a1 * R[7] + a2 * R[8]);
  const double s11 = cv[3] + (b0 * R[3] + b1 * R[4] + b2 * R[5]);
  const double s12 = cv[4] + (b0 * R[6] + b1 * R[7] + b2 * R[8]);
  const double s22 = cv[5] + (g0 * R[6] + g1 * R[7] + g2 * R[8]);
  const double A00 = s11 * s22 - s12 * s12;
  const double A01 = s02 * s12 - s01 * s22;
  const double A02 = s01 * s12 - s02 * s11;
  const double A11 = s00 * s22 - s02 * s02;
  const double A12 = s01 * s02 - s00 * s12;
  const double A22 = s00 * s11 - s01 * s01;
  const double det = s00 * A00 + s01 * A01 + s02 * A02;
  // Sylvester's criterion: leading principal minors s00, A22 and det all positive
  if (!(s00 > 0.0) || !(A22 > 0.0) || !(det > 0.0) || !isfinite(det)) return false;
  const double inv = 1.0 / det;
  o[0] = (T)(A00 * inv);
  o[1] = (T)(A01 * inv);
  o[2] = (T)(A02 * inv);
  o[3] = (T)(A11 * inv);
  o[4] = (T)(A12 * inv);
  o[5] = (T)(A22 * inv);
  return true;
}

// ------------------------------------------------------------------ accumulators

// FP64 running sums (FP64 per-point math).
struct AccF64 {
  double v[kNumAcc];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < kNumAcc; ++i) v[i] = 0.0;
  }
  __device__ void add(int i, float x) { v[i] += (double)x; }
  __device__ void add(int i, double x) { v[i] += x; }
  __device__ double get(int i) const { return v[i]; }
};

// FP32 partial sums of one lane over one work item (at most kMaxPointsPerLane points), taken
// to FP64 for every sum above the lane. A partial of m FP32 terms carries a relative rounding
// error below m * 2^-24 of the sum of magnitudes (2e-6 for m = 32), the same order as the
// rounding of the FP32 per-point terms themselves; half the registers of FP64 sums.
struct AccF32 {
  float v[kNumAcc];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < kNumAcc; ++i) v[i] = 0.0f;
  }
  __device__ void add(int i, float x) { v[i] += x; }
  __device__ void add(int i, double x) { v[i] += (float)x; }
  __device__ double get(int i) const { return (double)v[i]; }
};

// Kahan-compensated FP32 running sums (Kahan 1965): c carries the low-order part lost by the
// last addition; the value is s - c, taken to FP64 for every reduction above the thread.
struct AccKahan {
  float s[kNumAcc], c[kNumAcc];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < kNumAcc; ++i) s[i] = c[i] = 0.0f;
  }
  __device__ void add(int i, float x) {
    const float y = x - c[i];
    const float t = s[i] + y;
    c[i] = (t - s[i]) - y;
    s[i] = t;
  }
  __device__ void add(int i, double x) { add(i, (float)x); }
  __device__ double get(int i) const { return (double)s[i] - (double)c[i]; }
};

// Order of the kNumAcc sums:
//   0..5   H_rr (xx xy xz yy yz zz)      rotation-rotation block of H_t
//   6..14  H_rt row-major (3x3)          rotation-translation block
//   15..20 H_tt = sum Omega (xx..zz)
//   21..23 b_r = sum q x (Omega d)
//   24..26 b_t = sum Omega d
//   27     e   = sum d^T Omega d
enum : int { kHrr = 0, kHrt = 6, kHtt = 15, kBr = 21, kBt = 24, kE = 27 };

// Adds one inlier's contribution (q, d in the target frame, Omega = o).
template <bool LIN, typename T, class Acc>
__device__ inline void add_point_terms(const T q[3], const T d[3], const T o[6], Acc& acc) {
  const T u0 = o[0] * d[0] + o[1] * d[1] + o[2] * d[2];
  const T u1 = o[1] * d[0] + o[3] * d[1] + o[4] * d[2];
  const T u2 = o[2] * d[0] + o[4] * d[1] + o[5] * d[2];
  acc.add(kE, d[0] * u0 + d[1] * u1 + d[2] * u2);
  if constexpr (LIN) {
    const T q0 = q[0], q1 = q[1], q2 = q[2];
    // M = [q]x Omega (= H_rt), column j = q x Omega[:, j]
    const T m00 = q1 * o[2] - q2 * o[1], m10 = q2 * o[0] - q0 * o[2], m20 = q0 * o[1] - q1 * o[0];
    const T m01 = q1 * o[4] - q2 * o[3], m11 = q2 * o[1] - q0 * o[4], m21 = q0 * o[3] - q1 * o[1];
    const T m02 = q1 * o[5] - q2 * o[4], m12 = q2 * o[2] - q0 * o[5], m22 = q0 * o[4] - q1 * o[2];
    // H_rr = [q]x^T Omega [q]x = -M [q]x
    acc.add(kHrr + 0, m02 * q1 - m01 * q2);
    acc.add(kHrr + 1, m00 * q2 - m02 * q0);
    acc.add(kHrr + 2, m01 * q0 - m00 * q1);
    acc.add(kHrr + 3, m10 * q2 - m12 * q0);
    acc.add(kHrr + 4, m11 * q0 - m10 * q1);
    acc.add(kHrr + 5, m21 * q0 - m20 * q1);
    acc.add(kHrt + 0, m00);
    acc.add(kHrt + 1, m01);
    acc.add(kHrt + 2, m02);
    acc.add(kHrt + 3, m10);
    acc.add(kHrt + 4, m11);
    acc.add(kHrt + 5, m12);
    acc.add(kHrt + 6, m20);
    acc.add(kHrt + 7, m21);
    acc.add(kHrt + 8, m22);
#pragma unroll
    for (int i = 0; i < 6; ++i) acc.add(kHtt + i, o[i]);
    acc.add(kBr + 0, q1 * u2 - q2 * u1);
    acc.add(kBr + 1, q2 * u0 - q0 * u2);
    acc.add(kBr + 2, q0 * u1 - q1 * u0);
    acc.add(kBt + 0, u0);
    acc.add(kBt + 1, u1);
    acc.add(kBt + 2, u2);
  }
}

// ------------------------------------------------------------------ block reduction

// Sums NV doubles over the block (fixed order: butterfly within each wave, then waves in
// index order) and writes them to out[0..NV) from the first NV threads. Deterministic. For
// small NV (one shuffle pass per value).
template <int BLOCK, int NV>
__device__ inline void block_sum_store(double (&v)[NV], double* __restrict__ out) {
  constexpr int W = BLOCK / 64;
  __shared__ double sh[W][NV];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double x = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[i] = x;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[w][i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = sh[0][threadIdx.x];
#pragma unroll
    for (int k = 1; k < W; ++k) s += sh[k][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Same result shape for up to 32 values with a reduce-scatter butterfly: at the step with
// lane mask m (32, 16, 8, 4, 2) a lane keeps half of its values (the upper half if its m-bit
// is set) and adds the partner's copy of that half, so the values left to exchange halve at
// every step (32 double shuffles in all instead of 6 per value). Lanes 2k and 2k+1 end with
// the wave total of value k.
template <int BLOCK, int NV>
__device__ inline void block_sum_store_rs(double (&v)[32], double* __restrict__ out) {
  static_assert(NV <= 32, "at most 32 values");
  constexpr int W = BLOCK / 64;
  __shared__ double sh[W][32];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int step = 0; step < 5; ++step) {
    const int m = 32 >> step;
    const int half = 16 >> step;
    const bool upper = (lane & m) != 0;
    // blend on the bit patterns, so that the choice stays a register operation (a select of
    // array elements would become a select of addresses into private memory)
    const long long up = upper ? -1LL : 0LL;
#pragma unroll
    for (int j = 0; j < half; ++j) {
      const long long lo_bits = __double_as_longlong(v[j]);
      const long long hi_bits = __double_as_longlong(v[j + half]);
      const double send = __longlong_as_double((lo_bits & up) | (hi_bits & ~up));
      const double keep = __longlong_as_double((hi_bits & up) | (lo_bits & ~up));
      v[j] = keep + __shfl_xor(send, m, 64);
    }
  }
  v[0] += __shfl_xor(v[0], 1, 64);
  if ((lane & 1) == 0) sh[w][lane >> 1] = v[0];
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = sh[0][threadIdx.x];
#pragma unroll
    for (int k = 1; k < W; ++k) s += sh[k][threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ per-factor expansion

// Ad(T) = [[R, 0], [[t]x R, R]] for xi = [omega; rho].
__device__ inline void adjoint(const double* R, const double* t, double A[36]) {
  for (int i = 0; i < 36; ++i) A[i] = 0.0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      A[6 * r + c] = R[3 * r + c];
      A[6 * (r + 3) + (c + 3)] = R[3 * r + c];
    }
  const double tx[9] = {0.0, -t[2], t[1], t[2], 0.0, -t[0], -t[1], t[0], 0.0};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += tx[3 * r + k] * R[3 * k + c];
      A[6 * (r + 3) + c] = s;
    }
}

}  // namespace vgicp
