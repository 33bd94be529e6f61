// IMU preintegration factor of Sec. III-B (Eqs. (4)-(9)), batched over factors, FP64.
//   * preintegration: per factor, its samples in order (Eqs. (4)-(6) from the body frame at
//     time i, no gravity): dR <- dR Exp((w - b_w) dt), dv <- dv + dR (a - b_a) dt,
//     dp <- dp + dv dt + dR (a - b_a) dt^2 / 2, with the covariance of the preintegration noise
//     (dphi, dv, dp) propagated to first order, S <- A S A^T + B Q B^T (the on-manifold
//     preintegration the section cites);
//   * linearization: residual r = [Log(dR^T R_i^T R_j); R_i^T (v_j - v_i - g dt) - dv;
//     R_i^T (t_j - t_i - v_i dt - g dt^2 / 2) - dp] (Eqs. (7)-(9)), its Jacobian over
//     [xi_i, v_i, xi_j, v_j] (right perturbation of the poses, additive velocities), whitened by
//     the Cholesky factor of S: H = J^T S^-1 J, b = J^T S^-1 r, e = r^T S^-1 r.
//   * with bias states: the preintegration's derivatives with respect to the biases, the
//     first-order bias correction and the bias random walk (15 residuals, 30 unknowns).
// A factor holds tens to hundreds of samples and a graph a few thousand factors: one thread per
// factor, everything in registers, for the preintegration and the 18-unknown factor; one block
// of 64 threads per factor for the 30-unknown one (its 900-entry Hessian is formed in parallel).
#include <cmath>

#include "internal.h"

namespace vgicp {
namespace {

constexpr int kImuBlock = 64;

__device__ inline void hat3(const double w[3], double K[3][3]) {
  K[0][0] = 0.0;
  K[0][1] = -w[2];
  K[0][2] = w[1];
  K[1][0] = w[2];
  K[1][1] = 0.0;
  K[1][2] = -w[0];
  K[2][0] = -w[1];
  K[2][1] = w[0];
  K[2][2] = 0.0;
}

// Exp(w) (Rodrigues), and with J non-null the right Jacobian J_r(w) (series near zero).
__device__ inline void so3_exp_jr(const double w[3], double E[3][3], double (*J)[3]) {
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double th = sqrt(th2);
  double K[3][3], K2[3][3];
  hat3(w, K);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) K2[r][c] = K[r][0] * K[0][c] + K[r][1] * K[1][c] + K[r][2] * K[2][c];
  double a, b, ja, jb;  // E = I + a K + b K^2, J_r = I - ja K + jb K^2
  if (th < 1e-8) {
    a = 1.0;
    b = 0.5;
    ja = 0.5;
    jb = 1.0 / 6.0;
  } else {
    const double s = sin(th), c = cos(th);
    a = s / th;
    b = (1.0 - c) / th2;
    ja = b;
    jb = (th - s) / (th2 * th);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double id = r == c ? 1.0 : 0.0;
      E[r][c] = id + a * K[r][c] + b * K2[r][c];
      if (J) J[r][c] = id - ja * K[r][c] + jb * K2[r][c];
    }
}

// Log(R) as a rotation vector (angle below pi), and J_r^-1 of that vector.
__device__ inline void so3_log_jrinv(const double R[3][3], double w[3], double Ji[3][3]) {
  const double c = fmin(fmax((R[0][0] + R[1][1] + R[2][2] - 1.0) * 0.5, -1.0), 1.0);
  const double th = acos(c);
  const double v[3] = {R[2][1] - R[1][2], R[0][2] - R[2][0], R[1][0] - R[0][1]};
  const double f = th < 1e-8 ? 0.5 : th / (2.0 * sin(th));
#pragma unroll
  for (int i = 0; i < 3; ++i) w[i] = f * v[i];
  double K[3][3], K2[3][3];
  hat3(w, K);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
      K2[r][cc] = K[r][0] * K[0][cc] + K[r][1] * K[1][cc] + K[r][2] * K[2][cc];
  const double g = th < 1e-8 ? 1.0 / 12.0
                             : 1.0 / (th * th) - (1.0 + cos(th)) / (2.0 * th * sin(th));
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) Ji[r][cc] = (r == cc ? 1.0 : 0.0) + 0.5 * K[r][cc] + g * K2[r][cc];
}

// COV: the mean and the noise covariance (pre, cov). JAC: the mean's derivatives with respect to
// the biases instead (jac [F][9][6], rows (dphi, dv, dp), columns (b_a, b_w)): perturbing b_w by
// d moves dR_{k+1} = dR_k E_k by dR_{k+1} Exp((E_k^T J_R + ... ) d), see the recursions below;
// they use the values before the sample, as the covariance does.
template <bool COV, bool JAC>
__global__ __launch_bounds__(kImuBlock) void imu_preintegrate_kernel(
    const double* __restrict__ imu, long long m, const long long* __restrict__ seg, int F,
    const double* __restrict__ bias, double sg2, double sa2, double* __restrict__ pre,
    double* __restrict__ cov, double* __restrict__ jac, unsigned* __restrict__ flags) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  const long long k0 = seg[f], k1 = seg[f + 1];
  if (k0 < 0 || k1 < k0 || k1 > m) {
    atomicOr(flags, kFlagBadIndex);
    return;
  }
  const double ba[3] = {bias[6 * f], bias[6 * f + 1], bias[6 * f + 2]};
  const double bw[3] = {bias[6 * f + 3], bias[6 * f + 4], bias[6 * f + 5]};
  double dR[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  double dv[3] = {0.0, 0.0, 0.0}, dp[3] = {0.0, 0.0, 0.0}, T = 0.0;
  double S[COV ? 9 : 1][COV ? 9 : 1];
  if constexpr (COV) {
#pragma unroll
    for (int r = 0; r < 9; ++r)
#pragma unroll
      for (int c = 0; c < 9; ++c) S[r][c] = 0.0;
  }
  // bias derivatives: JR = d(dphi)/d(b_w), Jva / Jvw, Jpa / Jpw
  double JR[JAC ? 3 : 1][3], Jva[JAC ? 3 : 1][3], Jvw[JAC ? 3 : 1][3], Jpa[JAC ? 3 : 1][3],
      Jpw[JAC ? 3 : 1][3];
  if constexpr (JAC) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) JR[r][c] = Jva[r][c] = Jvw[r][c] = Jpa[r][c] = Jpw[r][c] = 0.0;
  }
  bool bad = false;
  for (long long k = k0; k < k1; ++k) {
    const double* row = imu + 7 * k;
    const double dt = row[6];
    if (!(dt > 0.0) || !isfinite(dt)) bad = true;
    const double wt[3] = {(row[0] - bw[0]) * dt, (row[1] - bw[1]) * dt, (row[2] - bw[2]) * dt};
    const double at[3] = {row[3] - ba[0], row[4] - ba[1], row[5] - ba[2]};
    double E[3][3], Jr[3][3];
    so3_exp_jr(wt, E, Jr);
    // M1 = -dR [a]x dt; the position row of A is M1 dt / 2 and dt I
    double Ka[3][3], M1[3][3];
    hat3(at, Ka);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        M1[r][c] = -(dR[r][0] * Ka[0][c] + dR[r][1] * Ka[1][c] + dR[r][2] * Ka[2][c]) * dt;
    if constexpr (JAC) {
      // with D = -dR [a]x JR (the rotation's bias derivative seen by the acceleration):
      //   Jp += Jv dt + (-dR dt^2/2 | D dt^2/2), Jv += (-dR dt | D dt), JR <- E^T JR - J_r dt
      double KJ[3][3], D[3][3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          KJ[r][c] = Ka[r][0] * JR[0][c] + Ka[r][1] * JR[1][c] + Ka[r][2] * JR[2][c];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          D[r][c] = -(dR[r][0] * KJ[0][c] + dR[r][1] * KJ[1][c] + dR[r][2] * KJ[2][c]);
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          Jpa[r][c] += Jva[r][c] * dt - 0.5 * dR[r][c] * dt * dt;
          Jpw[r][c] += Jvw[r][c] * dt + 0.5 * D[r][c] * dt * dt;
          Jva[r][c] -= dR[r][c] * dt;
          Jvw[r][c] += D[r][c] * dt;
        }
      double nJ[3][3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          nJ[r][c] = E[0][r] * JR[0][c] + E[1][r] * JR[1][c] + E[2][r] * JR[2][c] - Jr[r][c] * dt;
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) JR[r][c] = nJ[r][c];
    }
    if constexpr (COV) {
    // X = A S (row blocks: E^T S0, M1 S0 + S1, M1 dt/2 S0 + dt S1 + S2)
    double X[9][9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double s0 = E[0][r] * S[0][c] + E[1][r] * S[1][c] + E[2][r] * S[2][c];
        const double m = M1[r][0] * S[0][c] + M1[r][1] * S[1][c] + M1[r][2] * S[2][c];
        X[r][c] = s0;
        X[3 + r][c] = m + S[3 + r][c];
        X[6 + r][c] = 0.5 * dt * m + dt * S[3 + r][c] + S[6 + r][c];
      }
    }
    // S = X A^T (column blocks: X0 E, X0 M1^T + X1, X0 M1^T dt/2 + dt X1 + X2)
#pragma unroll
    for (int r = 0; r < 9; ++r) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double e0 = X[r][0] * E[0][c] + X[r][1] * E[1][c] + X[r][2] * E[2][c];
        const double m = X[r][0] * M1[c][0] + X[r][1] * M1[c][1] + X[r][2] * M1[c][2];
        S[r][c] = e0;
        S[r][3 + c] = m + X[r][3 + c];
        S[r][6 + c] = 0.5 * dt * m + dt * X[r][3 + c] + X[r][6 + c];
      }
    }
    // + B Q B^T: gyro noise through J_r dt into dphi; accelerometer noise through dR dt into dv
    // and dR dt^2 / 2 into dp
    const double qg = sg2 / dt * dt * dt, qa = sa2 / dt * dt * dt;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double jj = Jr[r][0] * Jr[c][0] + Jr[r][1] * Jr[c][1] + Jr[r][2] * Jr[c][2];
        const double rr = dR[r][0] * dR[c][0] + dR[r][1] * dR[c][1] + dR[r][2] * dR[c][2];
        S[r][c] += qg * jj;
        S[3 + r][3 + c] += qa * rr;
        S[3 + r][6 + c] += 0.5 * dt * qa * rr;
        S[6 + r][3 + c] += 0.5 * dt * qa * rr;
        S[6 + r][6 + c] += 0.25 * dt * dt * qa * rr;
      }
    }
    // the mean
    double ra[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) ra[r] = dR[r][0] * at[0] + dR[r][1] * at[1] + dR[r][2] * at[2];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      dp[r] += dv[r] * dt + 0.5 * ra[r] * dt * dt;
      dv[r] += ra[r] * dt;
    }
    double nR[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        nR[r][c] = dR[r][0] * E[0][c] + dR[r][1] * E[1][c] + dR[r][2] * E[2][c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) dR[r][c] = nR[r][c];
    T += dt;
  }
  if (bad) atomicOr(flags, kFlagNonFinite);
  if constexpr (COV) {
    double* o = pre + 16 * (long long)f;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) o[3 * r + c] = dR[r][c];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      o[9 + r] = dv[r];
      o[12 + r] = dp[r];
    }
    o[15] = T;
    if (cov) {
      double* oc = cov + 81 * (long long)f;
#pragma unroll
      for (int r = 0; r < 9; ++r)
#pragma unroll
        for (int c = 0; c < 9; ++c) oc[9 * r + c] = 0.5 * (S[r][c] + S[c][r]);
    }
  }
  if constexpr (JAC) {
    double* o = jac + 54 * (long long)f;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        o[6 * r + c] = 0.0;
        o[6 * r + 3 + c] = JR[r][c];
        o[6 * (3 + r) + c] = Jva[r][c];
        o[6 * (3 + r) + 3 + c] = Jvw[r][c];
        o[6 * (6 + r) + c] = Jpa[r][c];
        o[6 * (6 + r) + 3 + c] = Jpw[r][c];
      }
  }
}

__global__ __launch_bounds__(kImuBlock) void imu_linearize_kernel(
    const double* __restrict__ pre, const double* __restrict__ cov, const int* __restrict__ idx,
    int F, const double* __restrict__ poses, const double* __restrict__ vel, int P, double g0,
    double g1, double g2, double* __restrict__ H, double* __restrict__ bout,
    double* __restrict__ err, unsigned* __restrict__ flags) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  const int i = idx[2 * f], j = idx[2 * f + 1];
  if (i < 0 || i >= P || j < 0 || j >= P) {
    atomicOr(flags, kFlagBadIndex);
    return;
  }
  const double* p = pre + 16 * (long long)f;
  const double* Ti = poses + 12 * (long long)i;
  const double* Tj = poses + 12 * (long long)j;
  double Ri[3][3], Rj[3][3], ti[3], tj[3], vi[3], vj[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Ri[r][c] = Ti[4 * r + c];
      Rj[r][c] = Tj[4 * r + c];
    }
    ti[r] = Ti[4 * r + 3];
    tj[r] = Tj[4 * r + 3];
    vi[r] = vel[3 * i + r];
    vj[r] = vel[3 * j + r];
  }
  const double dt = p[15];
  const double g[3] = {g0, g1, g2};
  // rotation residual: Log(dR^T Ri^T Rj)
  double M[3][3], Rij[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Rij[r][c] = Ri[0][r] * Rj[0][c] + Ri[1][r] * Rj[1][c] + Ri[2][r] * Rj[2][c];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      M[r][c] = p[r] * Rij[0][c] + p[3 + r] * Rij[1][c] + p[6 + r] * Rij[2][c];
  double res[9], Ji[3][3];
  so3_log_jrinv(M, res, Ji);
  double uv[3], up[3];  // Ri^T (vj - vi - g dt), Ri^T (tj - ti - vi dt - g dt^2 / 2)
  {
    double a[3], b[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      a[r] = vj[r] - vi[r] - g[r] * dt;
      b[r] = tj[r] - ti[r] - vi[r] * dt - 0.5 * g[r] * dt * dt;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      uv[r] = Ri[0][r] * a[0] + Ri[1][r] * a[1] + Ri[2][r] * a[2];
      up[r] = Ri[0][r] * b[0] + Ri[1][r] * b[1] + Ri[2][r] * b[2];
      res[3 + r] = uv[r] - p[9 + r];
      res[6 + r] = up[r] - p[12 + r];
    }
  }
  // Jacobian 9 x 18 over [xi_i (omega, rho), v_i, xi_j (omega, rho), v_j]
  double J[9][18];
#pragma unroll
  for (int r = 0; r < 9; ++r)
#pragma unroll
    for (int c = 0; c < 18; ++c) J[r][c] = 0.0;
  double Kv[3][3], Kp[3][3];
  hat3(uv, Kv);
  hat3(up, Kp);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // -Jr^-1 Rj^T Ri = -Jr^-1 Rij^T
      J[r][c] = -(Ji[r][0] * Rij[c][0] + Ji[r][1] * Rij[c][1] + Ji[r][2] * Rij[c][2]);
      J[r][9 + c] = Ji[r][c];
      J[3 + r][c] = Kv[r][c];
      J[3 + r][6 + c] = -Ri[c][r];
      J[3 + r][15 + c] = Ri[c][r];
      J[6 + r][c] = Kp[r][c];
      J[6 + r][3 + c] = r == c ? -1.0 : 0.0;
      J[6 + r][6 + c] = -Ri[c][r] * dt;
      J[6 + r][12 + c] = Rij[r][c];
    }
  // whiten with the Cholesky factor L of the covariance (S = L L^T): solve L Y = [J | r]
  double L[9][9];
  const double* S = cov + 81 * (long long)f;
  bool pd = true;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    double d = S[9 * c + c];
#pragma unroll
    for (int q = 0; q < c; ++q) d -= L[c][q] * L[c][q];
    if (!(d > 1e-13 * S[9 * c + c])) {  // not positive definite to working precision
      pd = false;
      d = 1.0;
    }
    const double lc = sqrt(d);
    L[c][c] = lc;
#pragma unroll
    for (int r = c + 1; r < 9; ++r) {
      double v = S[9 * r + c];
#pragma unroll
      for (int q = 0; q < c; ++q) v -= L[r][q] * L[c][q];
      L[r][c] = v / lc;
    }
  }
  if (!pd) atomicOr(flags, kFlagNonFinite);
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const double inv = 1.0 / L[r][r];
#pragma unroll
    for (int c = 0; c < 18; ++c) {
      double v = J[r][c];
#pragma unroll
      for (int q = 0; q < r; ++q) v -= L[r][q] * J[q][c];
      J[r][c] = v * inv;
    }
    double v = res[r];
#pragma unroll
    for (int q = 0; q < r; ++q) v -= L[r][q] * res[q];
    res[r] = v * inv;
  }
  double* Ho = H + 324 * (long long)f;
#pragma unroll
  for (int a = 0; a < 18; ++a)
#pragma unroll
    for (int c = 0; c < 18; ++c) {
      double v = 0.0;
#pragma unroll
      for (int r = 0; r < 9; ++r) v += J[r][a] * J[r][c];
      Ho[18 * a + c] = v;
    }
#pragma unroll
  for (int a = 0; a < 18; ++a) {
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < 9; ++r) v += J[r][a] * res[r];
    bout[18 * (long long)f + a] = v;
  }
  double e = 0.0;
#pragma unroll
  for (int r = 0; r < 9; ++r) e += res[r] * res[r];
  err[f] = e;
}

// Factor with bias states (the state of Eq. (1) holds the biases): the preintegrated values
// corrected to first order for the bias of state i (db = b_i - b0, b0 the preintegration's),
//   dR Exp(J_R,w db_w), dv + J_v db, dp + J_p db,
// the residual above with them, and the bias random walk b_j - b_i (covariance
// diag(sigma_ba^2, sigma_bw^2) dt): 15 residuals over 30 unknowns [xi_i, v_i, b_i, xi_j, v_j, b_j].
// One block of 64 threads per factor: thread 0 forms the residual and the Jacobian's nonzero
// blocks in LDS and the Cholesky factor of the preintegration covariance; the threads whiten the
// 31 columns of [J | r] (one each) and form H = J~^T J~ (an entry each), b = J~^T r~, e = |r~|^2.
constexpr int kImuBiasThreads = 64;
__global__ __launch_bounds__(kImuBiasThreads) void imu_linearize_bias_kernel(
    const double* __restrict__ pre, const double* __restrict__ cov,
    const double* __restrict__ jac, const double* __restrict__ bias0,
    const int* __restrict__ idx, int F, const double* __restrict__ poses,
    const double* __restrict__ vel, const double* __restrict__ biases, int P, double g0,
    double g1, double g2, double qa, double qw, double* __restrict__ H,
    double* __restrict__ bout, double* __restrict__ err, unsigned* __restrict__ flags) {
  __shared__ double J[15][31];  // column 30: the residual
  __shared__ double L[9][9];
  __shared__ double wb[6];
  __shared__ int ok;
  const int f = blockIdx.x, t = threadIdx.x;
  for (int e = t; e < 15 * 31; e += kImuBiasThreads) J[e / 31][e % 31] = 0.0;
  __syncthreads();
  if (t == 0) {
    ok = 1;
    const int i = idx[2 * f], j = idx[2 * f + 1];
    if (i < 0 || i >= P || j < 0 || j >= P) {
      atomicOr(flags, kFlagBadIndex);
      ok = 0;
    } else {
      const double* p = pre + 16 * (long long)f;
      const double* Jb = jac + 54 * (long long)f;  // [9][6]
      const double* Ti = poses + 12 * (long long)i;
      const double* Tj = poses + 12 * (long long)j;
      double Ri[3][3], Rj[3][3], ti[3], tj[3], vi[3], vj[3], db[6];
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) {
          Ri[r][c] = Ti[4 * r + c];
          Rj[r][c] = Tj[4 * r + c];
        }
        ti[r] = Ti[4 * r + 3];
        tj[r] = Tj[4 * r + 3];
        vi[r] = vel[3 * i + r];
        vj[r] = vel[3 * j + r];
      }
      for (int k = 0; k < 6; ++k) db[k] = biases[6 * i + k] - bias0[6 * (long long)f + k];
      const double dt = p[15];
      const double g[3] = {g0, g1, g2};
      // the corrected preintegration
      double phi[3], Ephi[3][3], Jphi[3][3], dRc[3][3], dvc[3], dpc[3];
      for (int r = 0; r < 3; ++r)
        phi[r] = Jb[6 * r + 3] * db[3] + Jb[6 * r + 4] * db[4] + Jb[6 * r + 5] * db[5];
      so3_exp_jr(phi, Ephi, Jphi);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          dRc[r][c] = p[3 * r] * Ephi[0][c] + p[3 * r + 1] * Ephi[1][c] + p[3 * r + 2] * Ephi[2][c];
      for (int r = 0; r < 3; ++r) {
        double sv = p[9 + r], sp = p[12 + r];
        for (int k = 0; k < 6; ++k) {
          sv += Jb[6 * (3 + r) + k] * db[k];
          sp += Jb[6 * (6 + r) + k] * db[k];
        }
        dvc[r] = sv;
        dpc[r] = sp;
      }
      // rotation residual Log(dRc^T Ri^T Rj) and its right Jacobian's inverse
      double Rij[3][3], M[3][3], rR[3], Ji[3][3];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          Rij[r][c] = Ri[0][r] * Rj[0][c] + Ri[1][r] * Rj[1][c] + Ri[2][r] * Rj[2][c];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          M[r][c] = dRc[0][r] * Rij[0][c] + dRc[1][r] * Rij[1][c] + dRc[2][r] * Rij[2][c];
      so3_log_jrinv(M, rR, Ji);
      double uv[3], up[3];
      {
        double a[3], b[3];
        for (int r = 0; r < 3; ++r) {
          a[r] = vj[r] - vi[r] - g[r] * dt;
          b[r] = tj[r] - ti[r] - vi[r] * dt - 0.5 * g[r] * dt * dt;
        }
        for (int r = 0; r < 3; ++r) {
          uv[r] = Ri[0][r] * a[0] + Ri[1][r] * a[1] + Ri[2][r] * a[2];
          up[r] = Ri[0][r] * b[0] + Ri[1][r] * b[1] + Ri[2][r] * b[2];
        }
      }
      for (int r = 0; r < 3; ++r) {
        J[r][30] = rR[r];
        J[3 + r][30] = uv[r] - dvc[r];
        J[6 + r][30] = up[r] - dpc[r];
      }
      for (int k = 0; k < 6; ++k) J[9 + k][30] = biases[6 * j + k] - biases[6 * i + k];
      // the gyro-bias column of the rotation: -J_r^-1(rR) Exp(rR)^T J_r(phi) J_R,w, Exp(rR) = M
      double G[3][3], Q[3][3];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          G[r][c] = Jphi[r][0] * Jb[3 + c] + Jphi[r][1] * Jb[6 + 3 + c] +
                    Jphi[r][2] * Jb[12 + 3 + c];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          Q[r][c] = M[0][r] * G[0][c] + M[1][r] * G[1][c] + M[2][r] * G[2][c];
      double Kv[3][3], Kp[3][3];
      hat3(uv, Kv);
      hat3(up, Kp);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          J[r][c] = -(Ji[r][0] * Rij[c][0] + Ji[r][1] * Rij[c][1] + Ji[r][2] * Rij[c][2]);
          J[r][15 + c] = Ji[r][c];
          J[r][12 + c] = -(Ji[r][0] * Q[0][c] + Ji[r][1] * Q[1][c] + Ji[r][2] * Q[2][c]);
          J[3 + r][c] = Kv[r][c];
          J[3 + r][6 + c] = -Ri[c][r];
          J[3 + r][21 + c] = Ri[c][r];
          J[6 + r][c] = Kp[r][c];
          J[6 + r][3 + c] = r == c ? -1.0 : 0.0;
          J[6 + r][6 + c] = -Ri[c][r] * dt;
          J[6 + r][18 + c] = Rij[r][c];
        }
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 6; ++k) {
          J[3 + r][9 + k] = -Jb[6 * (3 + r) + k];
          J[6 + r][9 + k] = -Jb[6 * (6 + r) + k];
        }
      for (int k = 0; k < 6; ++k) {
        J[9 + k][9 + k] = -1.0;
        J[9 + k][24 + k] = 1.0;
        const double q = (k < 3 ? qa : qw) * dt;
        wb[k] = 1.0 / sqrt(q);
        if (!(q > 0.0) || !isfinite(q)) ok = 0;
      }
      // Cholesky factor of the preintegration covariance
      const double* S = cov + 81 * (long long)f;
      bool pd = true;
      for (int c = 0; c < 9; ++c) {
        double d = S[9 * c + c];
        for (int q = 0; q < c; ++q) d -= L[c][q] * L[c][q];
        if (!(d > 1e-13 * S[9 * c + c])) {
          pd = false;
          d = 1.0;
        }
        const double lc = sqrt(d);
        L[c][c] = lc;
        const double inv = 1.0 / lc;
        for (int r = c + 1; r < 9; ++r) {
          double v = S[9 * r + c];
          for (int q = 0; q < c; ++q) v -= L[r][q] * L[c][q];
          L[r][c] = v * inv;
        }
        for (int r = 0; r < c; ++r) L[r][c] = 0.0;
      }
      if (!pd || !ok) {
        atomicOr(flags, kFlagNonFinite);
        ok = pd && ok;
      }
    }
  }
  __syncthreads();
  if (!ok) return;
  // whiten the columns of [J | r]: L^-1 for the preintegration rows, 1 / sqrt(q dt) for the walk
  if (t < 31) {
    for (int r = 0; r < 9; ++r) {
      double v = J[r][t];
      for (int q = 0; q < r; ++q) v -= L[r][q] * J[q][t];
      J[r][t] = v / L[r][r];
    }
    for (int r = 9; r < 15; ++r) J[r][t] *= wb[r - 9];
  }
  __syncthreads();
  double* Ho = H + 900 * (long long)f;
  for (int e = t; e < 900; e += kImuBiasThreads) {
    const int a = e / 30, c = e % 30;
    double v = 0.0;
    for (int r = 0; r < 15; ++r) v += J[r][a] * J[r][c];
    Ho[e] = v;
  }
  if (t < 30) {
    double v = 0.0;
    for (int r = 0; r < 15; ++r) v += J[r][t] * J[r][30];
    bout[30 * (long long)f + t] = v;
  }
  if (t == 0) {
    double e = 0.0;
    for (int r = 0; r < 15; ++r) e += J[r][30] * J[r][30];
    err[f] = e;
  }
}

}  // namespace

void launch_imu_preintegrate(const double* imu, int64_t m, const int64_t* seg, int F,
                             const double* bias,
                             double sigma_g, double sigma_a, double* pre, double* cov,
                             double* jac, unsigned* flags, hipStream_t s) {
  if (F <= 0) return;
  const unsigned grid = (unsigned)((F + kImuBlock - 1) / kImuBlock);
  imu_preintegrate_kernel<true, false><<<grid, kImuBlock, 0, s>>>(
      imu, (long long)m, reinterpret_cast<const long long*>(seg), F, bias, sigma_g * sigma_g,
      sigma_a * sigma_a, pre, cov, nullptr, flags);
  if (jac)
    imu_preintegrate_kernel<false, true><<<grid, kImuBlock, 0, s>>>(
        imu, (long long)m, reinterpret_cast<const long long*>(seg), F, bias, 0.0, 0.0, nullptr,
        nullptr, jac, flags);
}

void launch_imu_linearize_bias(const double* pre, const double* cov, const double* jac,
                               const double* bias0, const int32_t* idx, int F,
                               const double* poses, const double* vel, const double* biases,
                               int P, const double g[3], double sigma_ba, double sigma_bw,
                               double* H, double* b, double* err, unsigned* flags,
                               hipStream_t s) {
  if (F <= 0) return;
  imu_linearize_bias_kernel<<<F, kImuBiasThreads, 0, s>>>(
      pre, cov, jac, bias0, idx, F, poses, vel, biases, P, g[0], g[1], g[2],
      sigma_ba * sigma_ba, sigma_bw * sigma_bw, H, b, err, flags);
}

void launch_imu_linearize(const double* pre, const double* cov, const int32_t* idx, int F,
                          const double* poses, const double* vel, int P, const double g[3],
                          double* H, double* b, double* err, unsigned* flags, hipStream_t s) {
  if (F <= 0) return;
  imu_linearize_kernel<<<(F + kImuBlock - 1) / kImuBlock, kImuBlock, 0, s>>>(
      pre, cov, idx, F, poses, vel, P, g[0], g[1], g[2], H, b, err, flags);
}

}  // namespace vgicp
