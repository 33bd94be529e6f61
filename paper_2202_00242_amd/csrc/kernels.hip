// Linearize / evaluate / backward kernels of the VGICP matching-cost factor on gfx950.
//
// Work unit: a tile of one factor's source points, in two phases per wave.
//   A. Lookup: every lane takes U points (the schedule's lookahead; structure-of-arrays loads,
//      coalesced across the wave),
//      transforms them in FP64, tests the voxel against the map's bounding box and probes the
//      {key, id} table for all of them at once. Hits are compacted into a per-wave LDS queue.
//   B. Inliers: whenever 64 are queued, all lanes run the full per-point work on one each
//      (covariance load, voxel Gaussian load, fused covariance inverse, residual, 28
//      target-frame sums in registers). Misses thus cost only phase A.
// The block reduces its sums in a fixed order and writes one partial per tile; a second kernel
// adds the partials of each factor in tile order and expands them to the factor's H and b.
// Results are therefore bitwise reproducible whatever the scheduling.
#include <algorithm>
#include <type_traits>

#include "device_math.h"
#include "internal.h"

namespace vgicp {

// ------------------------------------------------------------------ relative pose

// T_ts = T_t^-1 T_s in the fixed FP64 order of the definition (no fused multiply-add), and
// the rounded forms used by the FP32 variants. Runs on the host (single calls) and on the
// device (batches, from the pose buffer at graph replay).
__host__ __device__ inline void compute_rel_pose(const double* Tt, const double* Ts,
                                                 double inv_res, RelPose& o) {
#pragma clang fp contract(off)
  o.skip = 0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      o.R[3 * r + c] = (Tt[r] * Ts[c] + Tt[4 + r] * Ts[4 + c]) + Tt[8 + r] * Ts[8 + c];
  const double dt[3] = {Ts[3] - Tt[3], Ts[7] - Tt[7], Ts[11] - Tt[11]};
  for (int r = 0; r < 3; ++r)
    o.t[r] = (Tt[r] * dt[0] + Tt[4 + r] * dt[1]) + Tt[8 + r] * dt[2];
  for (int i = 0; i < 9; ++i) o.Rk[i] = o.R[i] * inv_res;
  for (int i = 0; i < 3; ++i) o.tk[i] = o.t[i] * inv_res;
  for (int i = 0; i < 9; ++i) o.Rf[i] = (float)o.R[i];
  for (int i = 0; i < 3; ++i) o.tf[i] = (float)o.t[i];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) {
      o.Rs[3 * r + c] = (float)Ts[4 * r + c];
      o.Rti[3 * r + c] = (float)Tt[4 * c + r];
    }
    o.ts[r] = (float)Ts[4 * r + 3];
    o.tti[r] = (float)(-(Tt[r] * Tt[3] + Tt[4 + r] * Tt[7] + Tt[8 + r] * Tt[11]));
  }
}

void relative_pose(const double* Tt, const double* Ts, double* Tts) {
  RelPose o;
  compute_rel_pose(Tt, Ts, 1.0, o);
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) Tts[4 * r + c] = o.R[3 * r + c];
    Tts[4 * r + 3] = o.t[r];
  }
}

RelPose make_rel_pose(const double* Tt, const double* Ts, double inv_res) {
  RelPose o;
  compute_rel_pose(Tt, Ts, inv_res, o);
  return o;
}

namespace {

// ------------------------------------------------------------------ phase A: voxel lookup

// Voxel coordinates of one source point in the target frame, branch-free (saturated, see
// floor_sat_i32), and the transformed point: q, or q / res when res is a power of two (the
// caller scales it back). Returns false when the transformed point is not finite.
template <int PREC, bool DIV>
__device__ inline bool point_key(const MapView& m, const RelPose& T, float x, float y, float z,
                                 int k[3], double q[3]) {
  if constexpr (PREC == kNaiveWorld) {
    // world point in FP32, then into the target frame in FP32
    const float w0 = T.Rs[0] * x + T.Rs[1] * y + T.Rs[2] * z + T.ts[0];
    const float w1 = T.Rs[3] * x + T.Rs[4] * y + T.Rs[5] * z + T.ts[1];
    const float w2 = T.Rs[6] * x + T.Rs[7] * y + T.Rs[8] * z + T.ts[2];
    const float q0 = T.Rti[0] * w0 + T.Rti[1] * w1 + T.Rti[2] * w2 + T.tti[0];
    const float q1 = T.Rti[3] * w0 + T.Rti[4] * w1 + T.Rti[5] * w2 + T.tti[1];
    const float q2 = T.Rti[6] * w0 + T.Rti[7] * w1 + T.Rti[8] * w2 + T.tti[2];
    const float ir = (float)m.inv_res;
    k[0] = floor_sat_i32_f32(q0 * ir);
    k[1] = floor_sat_i32_f32(q1 * ir);
    k[2] = floor_sat_i32_f32(q2 * ir);
    q[0] = q0;
    q[1] = q1;
    q[2] = q2;
    return isfinite(q0 + q1 + q2);
  } else {
    if constexpr (DIV) {
      transform_exact(T.R, T.t, x, y, z, q);
      for (int a = 0; a < 3; ++a) k[a] = floor_sat_i32(q[a] / m.res);
      return isfinite(q[0] + q[1] + q[2]);
    } else {
      // q / res exactly (power-of-two res); returned scaled, the inlier phase multiplies by
      // res (exact again)
      transform_exact(T.Rk, T.tk, x, y, z, q);
      for (int a = 0; a < 3; ++a) k[a] = floor_sat_i32(q[a]);
      return isfinite(q[0] + q[1] + q[2]);
    }
  }
}

// Orders a wave's LDS writes before other lanes of the same wave read them.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inliers a wave may hold between batches: fewer than 64 left over plus 64 * U new ones.
template <int U>
constexpr int queue_cap() {
  return 64 * (U + 1);
}

// Buffer descriptors over the three position planes of a source cloud (n < 2^30): loads take
// a 32-bit VGPR offset against an SGPR descriptor (no per-lane 64-bit address arithmetic), and
// offsets past a plane read 0 instead of touching memory.
struct Planes {
  __amdgpu_buffer_rsrc_t x, y, z;
};

__device__ inline __amdgpu_buffer_rsrc_t raw_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           kRawBufferFlags);
}

__device__ inline Planes make_planes(const float* xyz, int n) {
  const unsigned bytes = (unsigned)n * 4u;
  return {raw_rsrc(xyz, bytes), raw_rsrc(xyz + n, bytes), raw_rsrc(xyz + 2 * (size_t)n, bytes)};
}

// Positions of the points base + u*64 + lane, u < U. Lanes past the tile read neighbouring
// points or zeros (past the cloud), without a branch; the caller ignores them.
template <int U>
struct Chunk {
  float x[U], y[U], z[U];

  __device__ inline void load(const Planes& P, int base, int lane) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned off = (unsigned)(base + u * 64 + lane) * 4u;
      x[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(P.x, off, 0, 0));
      y[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(P.y, off, 0, 0));
      z[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(P.z, off, 0, 0));
    }
  }
};

// One queued inlier: its transformed point (FP64, target frame), voxel record, point index.
struct alignas(16) QueueEntry {
  double q0, q1, q2;
  int rec;
  int point;
};

// Phase A of a wave-chunk: lane l resolves the points base + u*64 + l, u < U (positions in
// c), with all their lookups in flight together. Hits are appended (in (u, lane) order) to the
// wave's queue: transformed point, voxel record index (MapView::rec) and point index; cnt
// stays wave-uniform. corr receives voxel ids.
// The next chunk's positions (nxt, at next_base) are loaded here, after this chunk's lookups
// are issued: vector-memory counters retire in issue order, so loads issued earlier would have
// to complete before the lookups could be consumed.
template <int PREC, bool DIV, int LAYOUT, int U, bool GRAD = false>
__device__ inline void resolve(const MapView& m, const RelPose& T, const Chunk<U>& c,
                               Chunk<U>& nxt, const Planes& P, int next_base, int base, int end,
                               int lane, QueueEntry* qe, int& cnt, int* __restrict__ corr,
                               unsigned& fl, float* __restrict__ gz = nullptr) {
  const float* x = c.x;
  const float* y = c.y;
  const float* z = c.z;
  bool valid[U];
#pragma unroll
  for (int u = 0; u < U; ++u) valid[u] = base + u * 64 + lane < end;
  unsigned slot[U], klo[U], khi[U];
  int st[U], id[U];  // st: 0 probing, 1 hit, 2 miss
  double q[U][3];    // transformed point (target frame)
#pragma unroll
  for (int u = 0; u < U; ++u) {
    id[u] = -1;
    int k[3];
    const bool finite = point_key<PREC, DIV>(m, T, x[u], y[u], z[u], k, q[u]);
    if (valid[u] && !finite) fl |= kFlagNonFinite;
    const unsigned dx = (unsigned)k[0] - (unsigned)m.lo[0];
    const unsigned dy = (unsigned)k[1] - (unsigned)m.lo[1];
    const unsigned dz = (unsigned)k[2] - (unsigned)m.lo[2];
    // outside the map's voxel bounding box (or out of range, or not finite): a miss
    const bool inbox = valid[u] && finite && dx < (unsigned)m.ext[0] &&
                       dy < (unsigned)m.ext[1] && dz < (unsigned)m.ext[2];
    if constexpr (LAYOUT == kLayoutGrid) {
      // 24-bit multiplies: a grid has fewer than 2^24 bricks
      slot[u] = __umul24(__umul24(dx >> 2, (unsigned)m.gby) + (dy >> 2), (unsigned)m.gbz) +
                (dz >> 1);
      klo[u] = bit_in_brick(dx, dy, dz);
      khi[u] = 0;
    } else if constexpr (LAYOUT == kLayoutHash32) {
      klo[u] = (dx << (m.by + m.bz)) | (dy << m.bz) | dz;
      khi[u] = 0;
      slot[u] = hash32(klo[u]) & m.mask;
    } else {
      const long long pk = pack_key(k[0], k[1], k[2]);
      klo[u] = (unsigned)pk;
      khi[u] = (unsigned)((unsigned long long)pk >> 32);
      slot[u] = hash64(pk) & m.mask;
    }
    st[u] = inbox ? 0 : 2;
  }
  if constexpr (LAYOUT == kLayoutGrid) {
    // one 8-byte brick load per point, all lookahead points at once; the record position is
    // the brick's base plus the occupied voxels below the point's bit. Points outside the box
    // load past the end of the bricks, which reads an empty brick (no branch around the loads).
    const __amdgpu_buffer_rsrc_t rb = raw_rsrc(m.bricks, m.brick_bytes);
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    u32x2 br[U];  // {mask, base}, one 8-byte load each
#pragma unroll
    for (int u = 0; u < U; ++u)
      br[u] = __builtin_amdgcn_raw_buffer_load_b64(rb, st[u] == 0 ? slot[u] * 8u : 0x80000000u,
                                                   0, 0);
    nxt.load(P, next_base, lane);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned hit = (br[u].x >> klo[u]) & 1u;
      const int pos = (int)br[u].y + __popc(br[u].x & ((1u << klo[u]) - 1u));
      id[u] = hit ? pos : -1;
      st[u] = 2 - (int)hit;
    }
  } else {
    nxt.load(P, next_base, lane);
    // Linear probing, all lookahead points at once; at least three quarters of the slots are
    // free, so every probe sequence ends within capacity steps.
    for (unsigned p = 0; p <= m.mask; ++p) {
      bool pending = false;
#pragma unroll
      for (int u = 0; u < U; ++u) pending |= st[u] == 0;
      if (__ballot(pending) == 0ull) break;
      // branch-free update of every lookahead point (selects, no divergent control flow)
      if constexpr (LAYOUT == kLayoutHash32) {
        uint2 sv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) sv[u] = gbl(m.slots32)[slot[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool pend = st[u] == 0;
          const bool hit = pend && sv[u].x == klo[u];
          const bool empty = pend && sv[u].x == kEmpty32;
          id[u] = hit ? (int)sv[u].y : id[u];
          st[u] = hit ? 1 : (empty ? 2 : st[u]);
          slot[u] = (pend && !hit && !empty) ? ((slot[u] + 1) & m.mask) : slot[u];
        }
      } else {
        longlong2 sv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) sv[u] = gbl(m.slots64)[slot[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const long long key = (long long)(((unsigned long long)khi[u] << 32) | klo[u]);
          const bool pend = st[u] == 0;
          const bool hit = pend && sv[u].x == key;
          const bool empty = pend && sv[u].x == kEmpty64;
          id[u] = hit ? (int)sv[u].y : id[u];
          st[u] = hit ? 1 : (empty ? 2 : st[u]);
          slot[u] = (pend && !hit && !empty) ? ((slot[u] + 1) & m.mask) : slot[u];
        }
      }
    }
  }
  if (corr) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (valid[u]) {
        int v = -1;
        if (st[u] == 1) v = (LAYOUT == kLayoutGrid) ? gbl(m.rec_id)[id[u]] : id[u];
        gblw(corr)[base + u * 64 + lane] = v;
      }
  }
  if constexpr (GRAD) {  // a point without a voxel has no gradient
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (valid[u] && st[u] != 1) {
        const gptr<float> g = gblw(gz) + 3 * (size_t)(unsigned)(base + u * 64 + lane);
        g[0] = 0.0f;
        g[1] = 0.0f;
        g[2] = 0.0f;
      }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const bool h = st[u] == 1;
    const unsigned long long mk = __ballot(h);
    if (h) {
      const int pos = cnt + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mk >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((unsigned)mk, 0u));
      if constexpr (PREC != kCountOnly)
        qe[pos] = QueueEntry{q[u][0], q[u][1], q[u][2], id[u], base + u * 64 + lane};
    }
    cnt += __popcll(mk);
  }
}

// ------------------------------------------------------------------ phase B: inlier terms

template <int PREC>
using RealOf = typename std::conditional<PREC == kMathFp64, double, float>::type;

// Full per-point work of one inlier (its voxel is known): fused covariance, inverse,
// residual and target-frame Gauss-Newton terms.
template <int PREC, bool LIN, bool AOS, class Acc>
__device__ inline void inlier_terms(const MapView& m, const RelPose& T,
                                    const float* __restrict__ cov, int n, QueueEntry e,
                                    double qscale, Acc& acc, int& nin, unsigned& fl) {
  using Real = RealOf<PREC>;
  float c[6];
  if constexpr (AOS) {  // interleaved [n][6] (24 bytes): three 8-byte loads
    const float2* c2 = gbl(reinterpret_cast<const float2*>(cov)) + 3 * (size_t)(unsigned)e.point;
    const float2 c01 = c2[0], c23 = c2[1], c45 = c2[2];
    c[0] = c01.x, c[1] = c01.y, c[2] = c23.x, c[3] = c23.y, c[4] = c45.x, c[5] = c45.y;
  } else {  // the caller's planes [6][n]
#pragma unroll
    for (int a = 0; a < 6; ++a) c[a] = gbl(cov + (size_t)a * n)[(unsigned)e.point];
  }
  const VoxelData vd = gbl(m.rec)[(unsigned)e.rec];
  // queued as q / res when res is a power of two (qscale = res, exact) else q (qscale = 1)
  const double q[3] = {e.q0 * qscale, e.q1 * qscale, e.q2 * qscale};
  Real qq[3], d[3];
  if constexpr (PREC == kNaiveWorld) {  // q holds the FP32 world-path point
    for (int a = 0; a < 3; ++a) {
      qq[a] = (float)q[a];
      d[a] = (float)vd.mean[a] - qq[a];
    }
  } else {
    for (int a = 0; a < 3; ++a) {
      qq[a] = (Real)q[a];
      d[a] = (Real)(vd.mean[a] - q[a]);
    }
  }
  Real o[6];
  const bool ok = fused_inverse<Real>(T.R, vd.cov, c, o);
  if (!ok) {
    fl |= kFlagNonFinite;
    return;
  }
  add_point_terms<LIN>(qq, d, o, acc);
  ++nin;
}

// Gradient terms of one inlier (the backward of Eq. (2) with its correspondence held):
// w = R^T Omega d (source frame); the source pose's right-perturbation gradient gains
// 2 w x (mu + C w) (rotation) and -2 w (translation), and the point's gradient is -2 w
// (scaled by the factor's upstream gradient later). Omega is formed in FP64 as everywhere.
struct GradAcc {
  double v[6];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = 0.0;
  }
};

template <int PREC>
__device__ inline void inlier_grad(const MapView& m, const RelPose& T,
                                   const float* __restrict__ xyz, const float* __restrict__ cov,
                                   int n, QueueEntry e, double qscale, GradAcc& acc, int& nin,
                                   unsigned& fl, float* __restrict__ gz) {
  using Real = RealOf<PREC>;
  float c[6];
  const float2* c2 = gbl(reinterpret_cast<const float2*>(cov)) + 3 * (size_t)(unsigned)e.point;
  const float2 c01 = c2[0], c23 = c2[1], c45 = c2[2];
  c[0] = c01.x, c[1] = c01.y, c[2] = c23.x, c[3] = c23.y, c[4] = c45.x, c[5] = c45.y;
  const float mx = gbl(xyz)[(unsigned)e.point];
  const float my = gbl(xyz + (size_t)n)[(unsigned)e.point];
  const float mz = gbl(xyz + 2 * (size_t)n)[(unsigned)e.point];
  const VoxelData vd = gbl(m.rec)[(unsigned)e.rec];
  const double q[3] = {e.q0 * qscale, e.q1 * qscale, e.q2 * qscale};
  Real d[3];
  for (int a = 0; a < 3; ++a) d[a] = (Real)(vd.mean[a] - q[a]);
  const gptr<float> g = gblw(gz) + 3 * (size_t)(unsigned)e.point;
  Real o[6];
  if (!fused_inverse<Real>(T.R, vd.cov, c, o)) {
    fl |= kFlagNonFinite;
    g[0] = 0.0f;
    g[1] = 0.0f;
    g[2] = 0.0f;
    return;
  }
  Real R[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = (Real)T.R[i];
  const Real u0 = o[0] * d[0] + o[1] * d[1] + o[2] * d[2];
  const Real u1 = o[1] * d[0] + o[3] * d[1] + o[4] * d[2];
  const Real u2 = o[2] * d[0] + o[4] * d[1] + o[5] * d[2];
  const Real w0 = R[0] * u0 + R[3] * u1 + R[6] * u2;
  const Real w1 = R[1] * u0 + R[4] * u1 + R[7] * u2;
  const Real w2 = R[2] * u0 + R[5] * u1 + R[8] * u2;
  const Real a0 = (Real)mx + (c[0] * w0 + c[1] * w1 + c[2] * w2);
  const Real a1 = (Real)my + (c[1] * w0 + c[3] * w1 + c[4] * w2);
  const Real a2 = (Real)mz + (c[2] * w0 + c[4] * w1 + c[5] * w2);
  acc.v[0] += 2.0 * (double)(w1 * a2 - w2 * a1);
  acc.v[1] += 2.0 * (double)(w2 * a0 - w0 * a2);
  acc.v[2] += 2.0 * (double)(w0 * a1 - w1 * a0);
  acc.v[3] -= 2.0 * (double)w0;
  acc.v[4] -= 2.0 * (double)w1;
  acc.v[5] -= 2.0 * (double)w2;
  g[0] = (float)(-2.0 * (double)w0);
  g[1] = (float)(-2.0 * (double)w1);
  g[2] = (float)(-2.0 * (double)w2);
  ++nin;
}

// Phase B of one queued inlier: linearization / evaluation terms, or gradient terms.
template <int PREC, bool LIN, bool AOS, bool GRAD, class Acc>
__device__ inline void phase_b(const MapView& m, const RelPose& T, const float* __restrict__ xyz,
                               const float* __restrict__ cov, int n, QueueEntry e,
                               double qscale, Acc& acc, int& nin, unsigned& fl,
                               float* __restrict__ gz) {
  if constexpr (GRAD)
    inlier_grad<PREC>(m, T, xyz, cov, n, e, qscale, acc, nin, fl, gz);
  else
    inlier_terms<PREC, LIN, AOS>(m, T, cov, n, e, qscale, acc, nin, fl);
}

// ------------------------------------------------------------------ one tile

template <int PREC>
struct AccOf {
  using type = AccF32;
};
template <>
struct AccOf<kAccKahan> {
  using type = AccKahan;
};
template <>
struct AccOf<kMathFp64> {
  using type = AccF64;
};

// Each wave takes chunks of 64 * U points of the tile (chunk c of wave w starts at
// start + (c * BLOCK/64 + w) * 64 * U), resolves them (phase A) and, whenever at
// least 64 inliers are queued, runs them with all 64 lanes busy (phase B). The queue tail is
// flushed at the end of the tile.
template <int PREC, bool LIN, int BLOCK, int U, bool DIV, int LAYOUT, bool AOS, bool GRAD,
          class Acc>
__device__ inline void tile_body(const MapView& m, const RelPose& T,
                                 const float* __restrict__ xyz, const float* __restrict__ cov,
                                 int n, int start, int end, int* __restrict__ corr, Acc& acc,
                                 int& nin, unsigned& fl, QueueEntry* qe,
                                 float* __restrict__ gz) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const Planes P = make_planes(xyz, n);
  const double qscale = (DIV || PREC == kNaiveWorld) ? 1.0 : m.res;
  int cnt = 0;
  // positions double-buffered: chunk c + 1 is loaded while chunk c is resolved
  Chunk<U> cur;
  cur.load(P, start + w * 64 * U, lane);
  for (int base = start + w * 64 * U; base < end; base += BLOCK * U) {
    Chunk<U> nxt;
    resolve<PREC, DIV, LAYOUT, U, GRAD>(m, T, cur, nxt, P, base + BLOCK * U, base, end, lane,
                                        qe, cnt, corr, fl, gz);
    cur = nxt;
    if constexpr (PREC == kCountOnly) {  // overlap: count the hits, no inlier phase
      if (lane == 0) nin += cnt;
      cnt = 0;
      continue;
    }
    if (cnt >= 64) {
      wave_sync();
      int head = 0;
      for (; cnt - head >= 64; head += 64)
        phase_b<PREC, LIN, AOS, GRAD>(m, T, xyz, cov, n, qe[head + lane], qscale, acc, nin, fl,
                                      gz);
      const int rem = cnt - head;
      // move the tail to the front (through registers: every lane reads before any writes)
      const int src = min(head + lane, cnt - 1);
      const double e0 = qe[src].q0, e1 = qe[src].q1, e2 = qe[src].q2;
      const int er = qe[src].rec, ep = qe[src].point;
      wave_sync();
      if (lane < rem) {
        qe[lane].q0 = e0;
        qe[lane].q1 = e1;
        qe[lane].q2 = e2;
        qe[lane].rec = er;
        qe[lane].point = ep;
      }
      cnt = rem;
      wave_sync();
    }
  }
  wave_sync();
  if constexpr (PREC != kCountOnly)
    if (lane < cnt)
      phase_b<PREC, LIN, AOS, GRAD>(m, T, xyz, cov, n, qe[lane], qscale, acc, nin, fl, gz);
  wave_sync();
}

// One tile [start, end) of a factor's source; writes the tile's partial sums (kPartialStride
// doubles: the 28 sums then the inlier count; evaluate writes only e and the count).
template <int PREC, bool LIN, int BLOCK, int U, bool AOS, bool GRAD = false>
__device__ inline void process_tile(const MapView& m, const RelPose& T,
                                    const float* __restrict__ xyz,
                                    const float* __restrict__ cov, int n, int start, int end,
                                    int* __restrict__ corr, double* __restrict__ partial,
                                    unsigned* flags, float* __restrict__ gz = nullptr) {
  __shared__ QueueEntry s_qe[BLOCK / 64][queue_cap<U>()];
  const int w = threadIdx.x >> 6;
  typename std::conditional<GRAD, GradAcc, typename AccOf<PREC>::type>::type acc;
  acc.zero();
  int nin = 0;
  unsigned fl = 0;
  QueueEntry* qe = s_qe[w];
  // uniform per tile: lookup structure and key arithmetic (multiply when res is a power of 2)
#define VGICP_TILE(DIV, LAYOUT)                                                         \
  tile_body<PREC, LIN, BLOCK, U, DIV, LAYOUT, AOS, GRAD>(m, T, xyz, cov, n, start, end, corr, \
                                                         acc, nin, fl, qe, gz)
  if (m.bricks) {
    if (m.pow2) VGICP_TILE(false, kLayoutGrid); else VGICP_TILE(true, kLayoutGrid);
  } else if (m.slots32) {
    if (m.pow2) VGICP_TILE(false, kLayoutHash32); else VGICP_TILE(true, kLayoutHash32);
  } else {
    if (m.pow2) VGICP_TILE(false, kLayoutHash64); else VGICP_TILE(true, kLayoutHash64);
  }
#undef VGICP_TILE
  if constexpr (GRAD) {
    double v[7];
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = acc.v[i];
    v[6] = (double)nin;
    block_sum_store<BLOCK, 7>(v, partial);
  } else if constexpr (LIN) {
    double v[32];
#pragma unroll
    for (int i = 0; i < kNumAcc; ++i) v[i] = acc.get(i);
    v[kNumAcc] = (double)nin;
#pragma unroll
    for (int i = kPartialStride; i < 32; ++i) v[i] = 0.0;
    block_sum_store_rs<BLOCK, kPartialStride>(v, partial);
  } else {
    double v[2] = {acc.get(kE), (double)nin};
    block_sum_store<BLOCK, 2>(v, partial + kE);
  }
  if (fl) atomicOr(flags, fl);
}

// Adjoint expansion of a factor's 28 target-frame sums (s, in LDS) shared out over the first 64
// threads of the block, an entry per thread: the target-frame blocks H_t, b_t, A = Ad(T_ts),
// G = H_t A; source block A^T G, source gradient -A^T b_t, and for a binary factor the cross
// blocks -G^T, -G and the target block H_t. H is written with row stride ld (12: the batch's
// [F][144] rows, zero blocks for a unary factor; 6 or 12: a single factor's own dimension).
// Every thread of the block must call it (it synchronises).
// Work space of expand_shared in the caller kernel's LDS (kernel-scope arrays: a __shared__
// array inside a device function that several kernels call is laid out once for all of them,
// which sized every such kernel's LDS to the largest).
struct ExpandLds {
  double Ht[36], A[36], G[36], bt[6];
};

__device__ inline void expand_shared(const double* s, const RelPose& T, int binary, double* Hf,
                                     int ld, double* bf, int i, ExpandLds& w) {
  double* Ht = w.Ht;
  double* A = w.A;
  double* G = w.G;
  double* bt = w.bt;
  if (i < 36) {
    const int r = i / 6, c = i % 6;
    const int rr = r % 3, cc = c % 3;
    const int lo = min(rr, cc), hi = max(rr, cc);
    const int sym = lo == 0 ? hi : (lo == 1 ? hi + 2 : 5);
    Ht[i] = r < 3 ? (c < 3 ? s[kHrr + sym] : s[kHrt + 3 * rr + cc])
                  : (c < 3 ? s[kHrt + 3 * cc + rr] : s[kHtt + sym]);
    double a = 0.0;
    if ((r < 3) == (c < 3)) {
      a = T.R[3 * rr + cc];
    } else if (r >= 3) {  // [t]x R: row rr of t x (column cc of R); no local array (an indexed
                          // private array would be moved to LDS, one copy per thread)
      const double c0 = T.R[cc], c1 = T.R[3 + cc], c2 = T.R[6 + cc];
      a = rr == 0 ? T.t[1] * c2 - T.t[2] * c1
                  : (rr == 1 ? T.t[2] * c0 - T.t[0] * c2 : T.t[0] * c1 - T.t[1] * c0);
    }
    A[i] = a;
  }
  if (i < 6) bt[i] = i < 3 ? s[kBr + i] : s[kBt + i - 3];
  __syncthreads();
  if (i < 36) {
    const int r = i / 6, c = i % 6;
    double x = 0.0;
    for (int k = 0; k < 6; ++k) x += Ht[6 * r + k] * A[6 * k + c];
    G[i] = x;
  }
  __syncthreads();
  const int dim = ld == 12 ? 12 : (binary ? 12 : 6);
  for (int e = i; e < dim * dim && i < 64; e += 64) {
    const int R = e / dim, C = e % dim;
    double v = 0.0;
    if (R < 6 && C < 6) {
      for (int k = 0; k < 6; ++k) v += A[6 * k + R] * G[6 * k + C];
    } else if (binary) {
      v = R < 6 ? -G[6 * (C - 6) + R] : (C < 6 ? -G[6 * (R - 6) + C] : Ht[6 * (R - 6) + C - 6]);
    }
    Hf[e] = v;
  }
  if (i < dim) {
    double y = 0.0;
    if (i < 6) {
      for (int k = 0; k < 6; ++k) y += A[6 * k + i] * bt[k];
      y = -y;
    } else if (binary) {
      y = bt[i - 6];
    }
    bf[i] = y;
  }
}

// ------------------------------------------------------------------ single factor

template <int PREC, bool LIN, int BLOCK>
__global__ __launch_bounds__(BLOCK) void plain_tile_kernel(MapView m, RelPose T,
                                                           const float* __restrict__ xyz,
                                                           const float* __restrict__ cov,
                                                           long long n, int tile,
                                                           int* __restrict__ corr,
                                                           double* __restrict__ partials,
                                                           unsigned* flags) {
  const int start = blockIdx.x * tile;
  const int end = (int)min((long long)start + tile, n);
  process_tile<PREC, LIN, BLOCK, 4, false>(m, T, xyz, cov, (int)n, start, end, corr,
                                    partials + (size_t)blockIdx.x * kPartialStride, flags);
}

// Sums the tile partials (each of the 29 values by 8 threads over every 8th tile, the 8 in
// order: a fixed order) and expands them to H and b (dimension 6 or 12, row stride =
// dimension); writes the cost and inlier count. 256 threads.
constexpr int kFinParts = 8;
template <bool LIN>
__global__ __launch_bounds__(256) void plain_finalize_kernel(const double* __restrict__ partials,
                                                             int ntiles, RelPose T, int binary,
                                                             double* __restrict__ H,
                                                             double* __restrict__ b,
                                                             double* __restrict__ err,
                                                             long long* __restrict__ inliers) {
  __shared__ double part[kPartialStride][kFinParts];
  __shared__ double s[kPartialStride];
  __shared__ ExpandLds ew;
  const int i = threadIdx.x;
  if (i < kPartialStride * kFinParts) {
    const int v = i / kFinParts, q = i % kFinParts;
    double a = 0.0;
    if (LIN || v >= kE)
      for (int t = q; t < ntiles; t += kFinParts) a += partials[(long long)t * kPartialStride + v];
    part[v][q] = a;
  }
  __syncthreads();
  if (i < kPartialStride) {
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < kFinParts; ++q) a += part[i][q];
    s[i] = a;
  }
  __syncthreads();
  if (i == 0) {
    *err = s[kE];
    *inliers = (long long)s[kNumAcc];
  }
  if constexpr (LIN) expand_shared(s, T, binary, H, binary ? 12 : 6, b, i, ew);
}

// ------------------------------------------------------------------ backward

// Per point with a correspondence: w = R^T Omega d; de/domega_s += 2 w x (mu + C w),
// de/drho_s += -2 w, de/dmu = -2 w (times the upstream gradient g).
template <int PREC, int BLOCK>
__global__ __launch_bounds__(BLOCK) void backward_tile_kernel(
    MapView m, RelPose T, const float* __restrict__ xyz, const float* __restrict__ cov,
    long long n, int tile, const int* __restrict__ corr, const double* __restrict__ grad_err,
    double* __restrict__ partials, float* __restrict__ grad_xyz) {
  using Real = RealOf<PREC>;
  const long long start = (long long)blockIdx.x * tile;
  const long long end = min(start + (long long)tile, n);
  const double g = *grad_err;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const Real* R;
  if constexpr (PREC == kMathFp64)
    R = T.R;
  else
    R = T.Rf;
  for (long long i = start + threadIdx.x; i < end; i += BLOCK) {
    const int v = corr[i];
    if (v < 0 || v >= m.V) {
      if (grad_xyz) {
        grad_xyz[i] = 0.0f;
        grad_xyz[n + i] = 0.0f;
        grad_xyz[2 * n + i] = 0.0f;
      }
      continue;
    }
    const float x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
    float c[6];
    for (int a = 0; a < 6; ++a) c[a] = cov[a * n + i];
    double q[3];
    transform_exact(T.R, T.t, x, y, z, q);
    const VoxelData vd = gbl(m.vox)[v];
    const Real d0 = (Real)(vd.mean[0] - q[0]);
    const Real d1 = (Real)(vd.mean[1] - q[1]);
    const Real d2 = (Real)(vd.mean[2] - q[2]);
    Real o[6];
    if (!fused_inverse<Real>(T.R, vd.cov, c, o)) {
      if (grad_xyz) {
        grad_xyz[i] = 0.0f;
        grad_xyz[n + i] = 0.0f;
        grad_xyz[2 * n + i] = 0.0f;
      }
      continue;
    }
    const Real u0 = o[0] * d0 + o[1] * d1 + o[2] * d2;
    const Real u1 = o[1] * d0 + o[3] * d1 + o[4] * d2;
    const Real u2 = o[2] * d0 + o[4] * d1 + o[5] * d2;
    const Real w0 = R[0] * u0 + R[3] * u1 + R[6] * u2;
    const Real w1 = R[1] * u0 + R[4] * u1 + R[7] * u2;
    const Real w2 = R[2] * u0 + R[5] * u1 + R[8] * u2;
    const Real a0 = (Real)x + (c[0] * w0 + c[1] * w1 + c[2] * w2);
    const Real a1 = (Real)y + (c[1] * w0 + c[3] * w1 + c[4] * w2);
    const Real a2 = (Real)z + (c[2] * w0 + c[4] * w1 + c[5] * w2);
    acc[0] += 2.0 * (double)(w1 * a2 - w2 * a1);
    acc[1] += 2.0 * (double)(w2 * a0 - w0 * a2);
    acc[2] += 2.0 * (double)(w0 * a1 - w1 * a0);
    acc[3] -= 2.0 * (double)w0;
    acc[4] -= 2.0 * (double)w1;
    acc[5] -= 2.0 * (double)w2;
    if (grad_xyz) {
      grad_xyz[i] = (float)(-2.0 * g * (double)w0);
      grad_xyz[n + i] = (float)(-2.0 * g * (double)w1);
      grad_xyz[2 * n + i] = (float)(-2.0 * g * (double)w2);
    }
  }
  block_sum_store<BLOCK, 6>(acc, partials + (long long)blockIdx.x * 6);
}

// g_s = g * sum; binary: g_t = -Ad(T_st)^T g_s with T_st = [R^T | -R^T t].
// Sums the tiles' source gradients, scales by the upstream gradient, forms the target's
// (de/dxi_t = -Ad(T_st)^T de/dxi_s) and maps both to tangent coordinates (J^T g).
__global__ void backward_finalize_kernel(const double* __restrict__ partials, int ntiles,
                                         RelPose T, int binary, TangentMap J,
                                         const double* __restrict__ grad_err,
                                         double* __restrict__ grad_xi) {
  __shared__ double s[6];
  const int i = threadIdx.x;
  if (i < 6) {
    double a = 0.0;
    for (int t = 0; t < ntiles; ++t) a += partials[(long long)t * 6 + i];
    s[i] = a * (*grad_err);
  }
  __syncthreads();
  if (i == 0) {
    double g[12];
    for (int k = 0; k < 6; ++k) g[k] = s[k];
    if (binary) {
      double Rt[9], st[3], A[36];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Rt[3 * r + c] = T.R[3 * c + r];
      for (int r = 0; r < 3; ++r)
        st[r] = -(Rt[3 * r] * T.t[0] + Rt[3 * r + 1] * T.t[1] + Rt[3 * r + 2] * T.t[2]);
      adjoint(Rt, st, A);
      for (int c = 0; c < 6; ++c) {
        double x = 0.0;
        for (int r = 0; r < 6; ++r) x += A[6 * r + c] * s[r];
        g[6 + c] = -x;
      }
    }
    for (int h = 0; h < (binary ? 2 : 1); ++h) {
      const double* Jh = h == 0 ? J.Js : J.Jt;
      for (int c = 0; c < 6; ++c) {
        double x = g[6 * h + c];
        if (J.use) {
          x = 0.0;
          for (int r = 0; r < 6; ++r) x += Jh[6 * r + c] * g[6 * h + r];
        }
        grad_xi[6 * h + c] = x;
      }
    }
  }
}

// ------------------------------------------------------------------ batches

// Per factor: the relative pose, and whether the source's bounding box (its local frame, the
// eight corners moved by T_ts in FP64 and widened by a margin far above the rounding of any
// point's transform) misses the voxel box of the map: then no point can fall in a voxel and the
// factor's work items are skipped (its sums are zero). Boxes are [lo, hi] per cloud; a cloud
// with a non-finite point has an infinite box and is never skipped, so its error still shows.
__global__ void batch_prep_kernel(const FactorView* __restrict__ F, int nF,
                                  const double* __restrict__ poses,
                                  const float* __restrict__ boxes, int allow_skip,
                                  RelPose* __restrict__ rel, unsigned long long* __restrict__ heads) {
#pragma clang fp contract(off)
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < kNumXcd) heads[f] = 0ull;
  if (f >= nF) return;
  RelPose& o = rel[f];
  compute_rel_pose(poses + 12LL * F[f].target_pose, poses + 12LL * F[f].source_pose,
                   F[f].map.inv_res, o);
  if (allow_skip && boxes) {
    const float* bx = boxes + 6LL * F[f].source_cloud;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool finite = true;
    for (int c = 0; c < 8; ++c) {
      const double p[3] = {(double)bx[(c & 1) ? 3 : 0], (double)bx[(c & 2) ? 4 : 1],
                           (double)bx[(c & 4) ? 5 : 2]};
      for (int r = 0; r < 3; ++r) {
        const double q = ((o.R[3 * r] * p[0] + o.R[3 * r + 1] * p[1]) + o.R[3 * r + 2] * p[2]) + o.t[r];
        finite = finite && isfinite(q);
        lo[r] = fmin(lo[r], q);
        hi[r] = fmax(hi[r], q);
      }
    }
    const MapView& m = F[f].map;
    bool miss = finite;
    if (finite) {
      miss = false;
      for (int r = 0; r < 3; ++r) {
        const double mg = 1e-6 * (1.0 + fabs(lo[r]) + fabs(hi[r]));
        const double klo = floor((lo[r] - mg) * m.inv_res), khi = floor((hi[r] + mg) * m.inv_res);
        // the map's voxel coordinates are lo .. lo + ext - 1 (none when the map is empty)
        if (khi < (double)m.lo[r] || klo > (double)m.lo[r] + (double)m.ext[r] - 1.0) miss = true;
      }
    }
    o.skip = miss ? 1 : 0;
  }
}

// Persistent kernel: block b serves the queue of XCD (b mod 8) first (blocks are dealt to the
// XCDs round-robin, and each queue holds the work of whole target groups, so an XCD's L2 sees
// few voxel tables at a time), then helps the other queues. The owner's blocks take a queue's
// items from its head and helpers from its tail, so a helper works on the queue's last target
// groups, which the owner has not reached, rather than pulling the owner's current target into
// a second L2. One 64-bit counter per queue holds both counts: an atomic add returns how many
// items were taken before it from either end, so every item is taken exactly once and every
// block leaves once all queues are drained.
// Occupancy target per lookahead (waves per SIMD): the register budget of 512 / waves.
template <int U>
constexpr int waves_for_lookahead() {
  return U <= 2 ? 4 : (U <= 4 ? 3 : 2);
}

template <int PREC, bool LIN, int BLOCK, int U, bool GRAD = false>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(waves_for_lookahead<U>()))) void batch_kernel(const FactorView* __restrict__ F,
                                                      const RelPose* __restrict__ rel,
                                                      const WorkItem* __restrict__ items,
                                                      const int* __restrict__ seg,
                                                      unsigned long long* __restrict__ heads,
                                                      int tile,
                                                      double* __restrict__ partials,
                                                      unsigned* flags,
                                                      float* __restrict__ gpts = nullptr) {
  __shared__ int s_item;
  const int xcd = blockIdx.x & (kNumXcd - 1);
  for (int qi = 0; qi < kNumXcd; ++qi) {
    const int x = (xcd + qi) & (kNumXcd - 1);
    const int base = seg[x];
    const int count = seg[x + 1] - base;
    const unsigned long long inc = qi == 0 ? 1ull : (1ull << 32);
    for (;;) {
      if (threadIdx.x == 0) {
        const unsigned long long old = atomicAdd(&heads[x], inc);
        const long long from_head = (long long)(old & 0xffffffffull), from_tail = (long long)(old >> 32);
        s_item = from_head + from_tail < count ? (qi == 0 ? (int)from_head : count - 1 - (int)from_tail)
                                               : -1;
      }
      __syncthreads();
      // the item index is the same for the whole block: keep it (and what it selects) scalar
      const int it = __builtin_amdgcn_readfirstlane(s_item);
      __syncthreads();
      if (it < 0) break;
      const int wf = __builtin_amdgcn_readfirstlane(items[base + it].factor);
      const int wt = __builtin_amdgcn_readfirstlane(items[base + it].tile);
      if (__builtin_amdgcn_readfirstlane(rel[wf].skip)) continue;  // the finalize writes zeros
      const FactorView& f = F[wf];
      const int start = wt * tile;
      const int end = (int)min((long long)start + tile, f.n);
      process_tile<PREC, LIN, BLOCK, U, true, GRAD>(
          f.map, rel[wf], f.xyz, f.cov6, (int)f.n, start, end, nullptr,
          partials + (size_t)(f.tile_base + wt) * kPartialStride, flags,
          GRAD ? gpts + 3 * (size_t)f.gbase : nullptr);
    }
  }
}

// RATE (count-only mode): err receives the overlap rate inliers / n instead of the cost.
template <bool LIN, bool RATE>
__global__ __launch_bounds__(64) void batch_finalize_kernel(const FactorView* __restrict__ F,
                                      const RelPose* __restrict__ rel,
                                      const double* __restrict__ partials,
                                      double* __restrict__ H, double* __restrict__ b,
                                      double* __restrict__ err, long long* __restrict__ inliers) {
  __shared__ double s[kPartialStride];
  __shared__ ExpandLds ew;
  const int f = blockIdx.x;
  const int i = threadIdx.x;
  const int base = F[f].tile_base, nt = rel[f].skip ? 0 : F[f].ntiles;
  if (i < kPartialStride && (LIN || i >= kE)) {
    double a = 0.0;
    for (int t = 0; t < nt; ++t) a += partials[(long long)(base + t) * kPartialStride + i];
    s[i] = a;
  }
  __syncthreads();
  if (i == 0) {
    if constexpr (RATE)
      err[f] = F[f].n > 0 ? s[kNumAcc] / (double)F[f].n : 0.0;
    else
      err[f] = s[kE];
    inliers[f] = (long long)s[kNumAcc];
  }
  if constexpr (LIN) expand_shared(s, rel[f], F[f].binary, H + 144LL * f, 12, b + 12LL * f, i, ew);
}

// ------------------------------------------------------------------ batched backward

// Per factor: the source pose's gradient summed over the tiles in order, scaled by the
// factor's upstream gradient; a binary factor's target gradient is -Ad(T_st)^T of it.
// gf[f] = [source | target] (the target half is zero for a unary factor).
__global__ void batch_grad_finalize_kernel(const FactorView* __restrict__ F,
                                           const RelPose* __restrict__ rel,
                                           const double* __restrict__ partials,
                                           const double* __restrict__ grad_err,
                                           double* __restrict__ gf) {
  __shared__ double s[6];
  const int f = blockIdx.x;
  const int i = threadIdx.x;
  const int base = F[f].tile_base, nt = rel[f].skip ? 0 : F[f].ntiles;
  if (i < 6) {
    double a = 0.0;
    for (int t = 0; t < nt; ++t) a += partials[(long long)(base + t) * kPartialStride + i];
    s[i] = a * grad_err[f];
  }
  __syncthreads();
  if (i < 12) {
    double v = 0.0;
    if (i < 6) {
      v = s[i];
    } else if (F[f].binary) {
      // A = Ad(T_st), T_st = T_ts^-1 = [R^T | -R^T t]; entry (r, c) of A^T is A[c][r]
      const RelPose& T = rel[f];
      const int c = i - 6;
      double st[3];
      for (int r = 0; r < 3; ++r)
        st[r] = -(T.R[r] * T.t[0] + T.R[3 + r] * T.t[1] + T.R[6 + r] * T.t[2]);
      double A[36];
      double Rt[9];
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) Rt[3 * r + k] = T.R[3 * k + r];
      adjoint(Rt, st, A);
      for (int r = 0; r < 6; ++r) v += A[6 * r + c] * s[r];
      v = -v;
    }
    gf[12LL * f + i] = v;
  }
}

// Per pose and tangent entry: the factors' gradients summed in factor order (deterministic).
__global__ void batch_grad_pose_kernel(const int* __restrict__ bptr,
                                       const int* __restrict__ bcontrib,
                                       const double* __restrict__ gf, int P,
                                       double* __restrict__ grad_poses) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 6 * P) return;
  const int p = t / 6, r = t % 6;
  double s = 0.0;
  for (int q = bptr[p]; q < bptr[p + 1]; ++q) {
    const int w = bcontrib[q];
    s += gf[12LL * (w >> 1) + 6 * (w & 1) + r];
  }
  grad_poses[t] = s;
}

// Per source cloud (blockIdx.y) and point of its spatial order: the gradients of the factors
// that read it, summed in factor order and scaled by their upstream gradients, written to the
// caller's [3][n] array at the point's original index. A skipped factor has no inlier.
__global__ __launch_bounds__(256) void batch_grad_points_kernel(
    const FactorView* __restrict__ F, const RelPose* __restrict__ rel,
    const int* __restrict__ cptr, const int* __restrict__ cfac,
    const long long* __restrict__ cloud_n, const long long* __restrict__ cloud_off,
    const int* __restrict__ perm, float* const* __restrict__ out,
    const double* __restrict__ grad_err, const float* __restrict__ gpts) {
  const int c = blockIdx.y;
  const long long n = cloud_n[c];
  float* o = out[c];
  if (!o) return;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int j = cptr[c]; j < cptr[c + 1]; ++j) {
      const int f = cfac[j];
      if (rel[f].skip) continue;
      const double g = grad_err[f];
      const float* v = gpts + 3 * (size_t)(F[f].gbase + k);
      s0 += g * (double)v[0];
      s1 += g * (double)v[1];
      s2 += g * (double)v[2];
    }
    // a cloud no factor reads was never put in spatial order: its points keep their index
    const long long i = cptr[c] == cptr[c + 1] ? k : perm[cloud_off[c] + k];
    o[i] = (float)s0;
    o[n + i] = (float)s1;
    o[2 * n + i] = (float)s2;
  }
}

// ------------------------------------------------------------------ dispatch

template <int PREC, bool LIN>
void launch_plain_t(const MapView& m, const RelPose& T, const float* xyz, const float* cov,
                    int64_t n, int binary, double* partials, int ntiles, int tile,
                    int32_t* corr, unsigned* flags, double* H, double* b, double* err,
                    int64_t* inliers, hipStream_t s) {
  if (ntiles > 0)
    plain_tile_kernel<PREC, LIN, 256><<<ntiles, 256, 0, s>>>(m, T, xyz, cov, n, tile, corr,
                                                             partials, flags);
  plain_finalize_kernel<LIN><<<1, 256, 0, s>>>(partials, ntiles, T, binary, H, b, err,
                                             reinterpret_cast<long long*>(inliers));
}

template <int PREC, bool LIN, int BLOCK, int U>
void launch_batch_t(const BatchLaunch& L, hipStream_t s) {
  batch_prep_kernel<<<(L.F + 255) / 256, 256, 0, s>>>(L.factors, L.F, L.poses, L.boxes,
                                                      PREC != kNaiveWorld, L.rel, L.heads);
  batch_kernel<PREC, LIN, BLOCK, U><<<L.grid, BLOCK, 0, s>>>(L.factors, L.rel, L.items, L.seg,
                                                            L.heads, L.tile, L.partials, L.flags);
  batch_finalize_kernel<LIN, PREC == kCountOnly><<<L.F, 64, 0, s>>>(
      L.factors, L.rel, L.partials, L.H, L.b, L.err, reinterpret_cast<long long*>(L.inliers));
}

template <int PREC, bool LIN, int BLOCK>
void launch_batch_u(const BatchLaunch& L, hipStream_t s) {
  if (L.lookahead == 8)
    launch_batch_t<PREC, LIN, BLOCK, 8>(L, s);
  else if (L.lookahead == 2)
    launch_batch_t<PREC, LIN, BLOCK, 2>(L, s);
  else
    launch_batch_t<PREC, LIN, BLOCK, 4>(L, s);
}

template <int PREC, bool LIN>
void launch_batch_b(const BatchLaunch& L, hipStream_t s) {
  if (L.block == 512)
    launch_batch_u<PREC, LIN, 512>(L, s);
  else
    launch_batch_u<PREC, LIN, 256>(L, s);
}

}  // namespace

void launch_plain(const MapView& m, const RelPose& T, const float* xyz, const float* cov,
                  int64_t n, int binary, int precision, bool linearize, double* partials,
                  int ntiles, int tile, int32_t* corr, unsigned* flags, double* H, double* b,
                  double* err, int64_t* inliers, hipStream_t s) {
#define VGICP_PLAIN(P)                                                                        \
  (linearize ? launch_plain_t<P, true>(m, T, xyz, cov, n, binary, partials, ntiles, tile, corr, \
                                       flags, H, b, err, inliers, s)                          \
             : launch_plain_t<P, false>(m, T, xyz, cov, n, binary, partials, ntiles, tile,    \
                                        corr, flags, H, b, err, inliers, s))
  switch (precision) {
    case kAccKahan: VGICP_PLAIN(kAccKahan); break;
    case kNaiveWorld: VGICP_PLAIN(kNaiveWorld); break;
    case kMathFp64: VGICP_PLAIN(kMathFp64); break;
    default: VGICP_PLAIN(kAccFp64); break;
  }
#undef VGICP_PLAIN
}

void launch_backward(const MapView& m, const RelPose& T, const TangentMap& J, const float* xyz,
                     const float* cov, int64_t n, int binary, int precision,
                     const int32_t* corr, const double* grad_err, double* partials, int ntiles,
                     int tile, double* grad_xi, float* grad_xyz, hipStream_t s) {
  if (ntiles > 0) {
    if (precision == kMathFp64)
      backward_tile_kernel<kMathFp64, 256><<<ntiles, 256, 0, s>>>(
          m, T, xyz, cov, n, tile, corr, grad_err, partials, grad_xyz);
    else
      backward_tile_kernel<kAccFp64, 256><<<ntiles, 256, 0, s>>>(
          m, T, xyz, cov, n, tile, corr, grad_err, partials, grad_xyz);
  }
  backward_finalize_kernel<<<1, 64, 0, s>>>(partials, ntiles, T, binary, J, grad_err, grad_xi);
}

namespace {
template <int PREC, int BLOCK, int U>
void launch_batch_grad_t(const BatchLaunch& L, const BatchGrad& G, hipStream_t s) {
  batch_prep_kernel<<<(L.F + 255) / 256, 256, 0, s>>>(L.factors, L.F, L.poses, L.boxes, 1,
                                                      L.rel, L.heads);
  batch_kernel<PREC, false, BLOCK, U, true><<<L.grid, BLOCK, 0, s>>>(
      L.factors, L.rel, L.items, L.seg, L.heads, L.tile, L.partials, L.flags, G.gpts);
  batch_grad_finalize_kernel<<<L.F, 64, 0, s>>>(L.factors, L.rel, L.partials, G.grad_err,
                                                G.gf);
  if (G.P > 0)
    batch_grad_pose_kernel<<<(6 * G.P + 255) / 256, 256, 0, s>>>(G.bptr, G.bcontrib, G.gf, G.P,
                                                               G.grad_poses);
  if (G.n_clouds > 0 && G.max_n > 0) {
    const long long gx = std::min<long long>((G.max_n + 255) / 256, 4096);
    batch_grad_points_kernel<<<dim3((unsigned)gx, (unsigned)G.n_clouds), 256, 0, s>>>(
        L.factors, L.rel, G.cptr, G.cfac, G.cloud_n, G.cloud_off, G.perm, G.out, G.grad_err,
        G.gpts);
  }
}

template <int PREC, int BLOCK>
void launch_batch_grad_u(const BatchLaunch& L, const BatchGrad& G, hipStream_t s) {
  if (L.lookahead == 8)
    launch_batch_grad_t<PREC, BLOCK, 8>(L, G, s);
  else if (L.lookahead == 2)
    launch_batch_grad_t<PREC, BLOCK, 2>(L, G, s);
  else
    launch_batch_grad_t<PREC, BLOCK, 4>(L, G, s);
}

template <int PREC>
void launch_batch_grad_b(const BatchLaunch& L, const BatchGrad& G, hipStream_t s) {
  if (L.block == 512)
    launch_batch_grad_u<PREC, 512>(L, G, s);
  else
    launch_batch_grad_u<PREC, 256>(L, G, s);
}
}  // namespace

void launch_batched_backward(const BatchLaunch& L, const BatchGrad& G, hipStream_t s) {
  if (L.precision == kMathFp64)
    launch_batch_grad_b<kMathFp64>(L, G, s);
  else
    launch_batch_grad_b<kAccFp64>(L, G, s);
}

void launch_batched(const BatchLaunch& L, hipStream_t s) {
#define VGICP_BATCH(P) \
  (L.linearize ? launch_batch_b<P, true>(L, s) : launch_batch_b<P, false>(L, s))
  switch (L.precision) {
    case kAccKahan: VGICP_BATCH(kAccKahan); break;
    case kNaiveWorld: VGICP_BATCH(kNaiveWorld); break;
    case kMathFp64: VGICP_BATCH(kMathFp64); break;
    case kCountOnly: launch_batch_b<kCountOnly, false>(L, s); break;
    default: VGICP_BATCH(kAccFp64); break;
  }
#undef VGICP_BATCH
}

}  // namespace vgicp
