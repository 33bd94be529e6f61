// VGICP matching-cost oracle: plain, slow, FP64 CPU reference.
//
// TEST INFRASTRUCTURE ONLY. This file is loaded by the test-suite, by the smoke check and by
// the CPU-baseline leg of the benchmark. The product library never includes, links or calls
// it, and it includes nothing from the product library.
//
// What it computes (Koide et al., "Globally Consistent and Tightly Coupled 3D LiDAR Inertial
// Mapping", ICRA 2022):
//   * Sec. III-A: every point p_k is a Gaussian (mu_k, C_k); the target cloud P_j is cut into
//     voxels, and each voxel holds a Gaussian aggregated from the means and covariances of the
//     points inside it.
//   * Eq. (2): the matching cost e^M is the sum of e^D2D over the source points p_k of P_i.
//   * Eq. (3): e^D2D = d_k^T (C'_k + R C_k R^T)^-1 d_k with d_k = mu'_k - T mu_k, where
//     (mu'_k, C'_k) is the voxel that the transformed point falls in (a single voxel lookup).
//   * Sec. III-A, last paragraph: a Hessian factor (H, b, e) is formed from the derivatives of
//     Eq. (2) at the current linearization point.
//
// Readings taken where the paper is silent (each one is listed with its reason in the design
// notes of the repository):
//   * frame: T_ts = T_t^-1 T_s maps source-local points into the target's local frame (the
//     voxel map is built in the target's own frame);
//   * the 4x4 transform around C_k in Eq. (3) acts through its rotation only: R C_k R^T;
//   * voxel Gaussian = arithmetic mean of member means and of member covariances, n >= 1;
//   * a point whose voxel is absent is skipped (it is not an inlier);
//   * voxel coordinate = floor(v / res) in FP64, |k| < 2^20; voxel ids = rank of the key among
//     the distinct keys in ascending order;
//   * Gauss-Newton with the inverse covariance frozen at the linearization point:
//     e(xi) ~= e + 2 b^T xi + xi^T H xi, H = sum J^T Omega J, b = sum J^T Omega d;
//   * tangent xi = [omega; rho], right perturbation T Exp(xi); binary blocks ordered
//     [source | target].
//
// Floating point: compiled with -ffp-contract=off and without fast-math, so every product and
// sum below rounds exactly as written. The relative pose and the transformed point are written
// with one fixed evaluation order, because the voxel a point falls in is decided by them.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <unordered_map>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// Status codes; the numeric values mirror the product's documented error contract.
constexpr int kOk = 0;
constexpr int kInvalidArg = 1;
constexpr int kNonFinite = 2;
constexpr int kKeyRange = 3;

constexpr int64_t kKeyLimit = int64_t(1) << 20;  // |voxel coordinate| must stay below this

// Neumaier's compensated sum (Neumaier 1974): keeps the oracle's own summation error far below
// the tolerances it is used to check.
struct CompSum {
  double s = 0.0, c = 0.0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

// Voxel coordinate of one axis: floor toward -inf of v / res, in FP64.
int voxel_coord(double v, double res, int64_t* k) {
  double f = std::floor(v / res);
  if (!std::isfinite(f)) return kNonFinite;
  if (!(std::fabs(f) < double(kKeyLimit))) return kKeyRange;
  *k = int64_t(f);
  return kOk;
}

// Packs three voxel coordinates into 63 bits. Ascending packed order is lexicographic (x, y, z).
int64_t pack_key(int64_t kx, int64_t ky, int64_t kz) {
  return ((kx + kKeyLimit) << 42) | ((ky + kKeyLimit) << 21) | (kz + kKeyLimit);
}

struct Map {
  double res = 1.0;
  std::vector<int64_t> keys;     // ascending; position = voxel id
  std::vector<double> mean;      // [V][3]
  std::vector<double> cov;       // [V][6]: xx xy xz yy yz zz
  std::vector<int32_t> count;    // [V]
  std::unordered_map<int64_t, int32_t> id_of;
};

// Pose as a row-major 3x4 [R | t].
struct Pose {
  double R[3][3];
  double t[3];
};

Pose load_pose(const double* T) {
  Pose p;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) p.R[r][c] = T[4 * r + c];
    p.t[r] = T[4 * r + 3];
  }
  return p;
}

// T_ts = T_t^-1 T_s in one fixed evaluation order.
Pose relative_pose(const Pose& Tt, const Pose& Ts) {
  Pose o;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      o.R[r][c] = (Tt.R[0][r] * Ts.R[0][c] + Tt.R[1][r] * Ts.R[1][c]) + Tt.R[2][r] * Ts.R[2][c];
  double dt[3] = {Ts.t[0] - Tt.t[0], Ts.t[1] - Tt.t[1], Ts.t[2] - Tt.t[2]};
  for (int r = 0; r < 3; ++r)
    o.t[r] = (Tt.R[0][r] * dt[0] + Tt.R[1][r] * dt[1]) + Tt.R[2][r] * dt[2];
  return o;
}

// q = R mu + t in one fixed evaluation order.
void transform_point(const Pose& T, const double mu[3], double q[3]) {
  for (int r = 0; r < 3; ++r)
    q[r] = ((T.R[r][0] * mu[0] + T.R[r][1] * mu[1]) + T.R[r][2] * mu[2]) + T.t[r];
}

void sym_from6(const double* c6, double S[3][3]) {
  S[0][0] = c6[0]; S[0][1] = c6[1]; S[0][2] = c6[2];
  S[1][0] = c6[1]; S[1][1] = c6[3]; S[1][2] = c6[4];
  S[2][0] = c6[2]; S[2][1] = c6[4]; S[2][2] = c6[5];
}

// Lower Cholesky factor of a 3x3 symmetric matrix; false when it is not positive definite or
// not finite.
bool cholesky3(const double A[3][3], double L[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) L[i][j] = 0.0;
  for (int j = 0; j < 3; ++j) {
    double d = A[j][j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    L[j][j] = std::sqrt(d);
    for (int i = j + 1; i < 3; ++i) {
      double s = A[i][j];
      for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
      L[i][j] = s / L[j][j];
    }
  }
  return true;
}

// Solves L y = v (forward substitution).
void forward_sub(const double L[3][3], const double v[3], double y[3]) {
  for (int i = 0; i < 3; ++i) {
    double s = v[i];
    for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
    y[i] = s / L[i][i];
  }
}

// Solves L^T x = y (back substitution).
void back_sub(const double L[3][3], const double y[3], double x[3]) {
  for (int i = 2; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < 3; ++k) s -= L[k][i] * x[k];
    x[i] = s / L[i][i];
  }
}

// Fused covariance of Eq. (3): Sigma = C'_v + R C_k R^T.
void fused_covariance(const Pose& T, const double* cvox6, const double Ck[3][3], double S[3][3]) {
  double RC[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += T.R[r][k] * Ck[k][c];
      RC[r][c] = s;
    }
  double V[3][3];
  sym_from6(cvox6, V);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += RC[r][k] * T.R[c][k];
      S[r][c] = V[r][c] + s;
    }
}

// [v]x, the cross-product matrix.
void skew(const double v[3], double S[3][3]) {
  S[0][0] = 0.0;   S[0][1] = -v[2]; S[0][2] = v[1];
  S[1][0] = v[2];  S[1][1] = 0.0;   S[1][2] = -v[0];
  S[2][0] = -v[1]; S[2][1] = v[0];  S[2][2] = 0.0;
}

// Source-pose Jacobian of d:  J_s = [ R [mu]x , -R ]  (3x6).
void jacobian_source(const Pose& T, const double mu[3], double J[3][6]) {
  double M[3][3];
  skew(mu, M);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += T.R[r][k] * M[k][c];
      J[r][c] = s;
      J[r][3 + c] = -T.R[r][c];
    }
}

// Target-pose Jacobian of d:  J_t = [ -[q]x , I ]  (3x6).
void jacobian_target(const double q[3], double J[3][6]) {
  double Q[3][3];
  skew(q, Q);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      J[r][c] = -Q[r][c];
      J[r][3 + c] = (r == c) ? 1.0 : 0.0;
    }
}

struct Cloud {
  const double* xyz;  // [3][n]
  const double* cov;  // [6][n]
  int64_t n;
  void point(int64_t k, double mu[3], double C[3][3]) const {
    for (int a = 0; a < 3; ++a) mu[a] = xyz[a * n + k];
    double c6[6];
    for (int a = 0; a < 6; ++a) c6[a] = cov[a * n + k];
    sym_from6(c6, C);
  }
};

// Voxel id of a point already in the target frame, or -1. Status is kNonFinite for a
// non-finite point; an out-of-range coordinate cannot hold a voxel and is a plain miss.
int lookup(const Map& m, const double q[3], int32_t* id) {
  int64_t k[3];
  for (int a = 0; a < 3; ++a) {
    int st = voxel_coord(q[a], m.res, &k[a]);
    if (st == kNonFinite) return kNonFinite;
    if (st == kKeyRange) { *id = -1; return kOk; }
  }
  auto it = m.id_of.find(pack_key(k[0], k[1], k[2]));
  *id = (it == m.id_of.end()) ? -1 : it->second;
  return kOk;
}

// One Gauss-Newton factor, written straight from the definition: per inlier,
// Omega = (C'_v + R C_k R^T)^-1 by Cholesky, e += d^T Omega d, H += J^T Omega J, b += J^T Omega d
// with J = J_s (unary) or [J_s | J_t] (binary).
int linearize_one(const Map& m, const Cloud& src, const Pose& Tt, const Pose& Ts, int binary,
                  bool want_hb, double* H, double* b, double* e, int64_t* inliers,
                  int32_t* corr) {
  const Pose T = relative_pose(Tt, Ts);
  const int dim = binary ? 12 : 6;
  std::vector<CompSum> Hs(dim * dim), bs(dim);
  CompSum es;
  int64_t nin = 0;
  for (int64_t k = 0; k < src.n; ++k) {
    double mu[3], Ck[3][3], q[3];
    src.point(k, mu, Ck);
    transform_point(T, mu, q);
    int32_t v;
    if (lookup(m, q, &v) != kOk) return kNonFinite;
    if (corr) corr[k] = v;
    if (v < 0) continue;
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = m.mean[3 * v + a] - q[a];
    double S[3][3], L[3][3];
    fused_covariance(T, &m.cov[6 * v], Ck, S);
    if (!cholesky3(S, L)) return kNonFinite;
    // With Sigma = L L^T:  d^T Sigma^-1 d = |L^-1 d|^2 and J^T Sigma^-1 J = (L^-1 J)^T (L^-1 J).
    double z[3];
    forward_sub(L, d, z);
    es.add(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
    ++nin;
    if (!want_hb) continue;
    double J[3][12];
    double Js[3][6];
    jacobian_source(T, mu, Js);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 6; ++c) J[r][c] = Js[r][c];
    if (binary) {
      double Jt[3][6];
      jacobian_target(q, Jt);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 6; ++c) J[r][6 + c] = Jt[r][c];
    }
    double Y[3][12];
    for (int c = 0; c < dim; ++c) {
      double col[3] = {J[0][c], J[1][c], J[2][c]}, y[3];
      forward_sub(L, col, y);
      for (int r = 0; r < 3; ++r) Y[r][c] = y[r];
    }
    for (int i = 0; i < dim; ++i) {
      bs[i].add(Y[0][i] * z[0] + Y[1][i] * z[1] + Y[2][i] * z[2]);
      for (int j = 0; j < dim; ++j)
        Hs[i * dim + j].add(Y[0][i] * Y[0][j] + Y[1][i] * Y[1][j] + Y[2][i] * Y[2][j]);
    }
  }
  *e = es.value();
  *inliers = nin;
  if (want_hb) {
    for (int i = 0; i < dim * dim; ++i) H[i] = Hs[i].value();
    for (int i = 0; i < dim; ++i) b[i] = bs[i].value();
  }
  return kOk;
}

bool finite_array(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

extern "C" {

int oracle_voxel_coord(double v, double res, int64_t* k) {
  if (!(res > 0.0) || !std::isfinite(res)) return kInvalidArg;
  return voxel_coord(v, res, k);
}

int64_t oracle_pack_key(int64_t kx, int64_t ky, int64_t kz) { return pack_key(kx, ky, kz); }

void oracle_unpack_key(int64_t key, int64_t* kx, int64_t* ky, int64_t* kz) {
  const int64_t m = (int64_t(1) << 21) - 1;
  *kx = ((key >> 42) & m) - kKeyLimit;
  *ky = ((key >> 21) & m) - kKeyLimit;
  *kz = (key & m) - kKeyLimit;
}

// Builds the voxel map of one target cloud (Sec. III-A): group by voxel, average member means
// and member covariances in FP64 summing in increasing point index, number voxels by ascending
// key. xyz is [3][n], cov is [6][n] (xx xy xz yy yz zz), both FP64.
int oracle_map_build(const double* xyz, const double* cov, int64_t n, double res, void** out) {
  if (!out || n < 0 || (n > 0 && (!xyz || !cov))) return kInvalidArg;
  if (!(res > 0.0) || !std::isfinite(res)) return kInvalidArg;
  if (!finite_array(xyz, 3 * n) || !finite_array(cov, 6 * n)) return kNonFinite;
  Map* m = new Map;
  m->res = res;
  std::vector<int64_t> key(n);
  for (int64_t j = 0; j < n; ++j) {
    int64_t k[3];
    for (int a = 0; a < 3; ++a) {
      int st = voxel_coord(xyz[a * n + j], res, &k[a]);
      if (st != kOk) { delete m; return st; }
    }
    key[j] = pack_key(k[0], k[1], k[2]);
  }
  std::vector<int64_t> order(n);
  std::iota(order.begin(), order.end(), int64_t(0));
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return key[a] < key[b]; });
  for (int64_t s = 0; s < n;) {
    int64_t e = s;
    while (e < n && key[order[e]] == key[order[s]]) ++e;
    double sm[3] = {0, 0, 0}, sc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = s; i < e; ++i) {  // members in increasing point index (stable sort)
      const int64_t j = order[i];
      for (int a = 0; a < 3; ++a) sm[a] += xyz[a * n + j];
      for (int a = 0; a < 6; ++a) sc[a] += cov[a * n + j];
    }
    const double cnt = double(e - s);
    const int32_t id = int32_t(m->keys.size());
    m->keys.push_back(key[order[s]]);
    for (int a = 0; a < 3; ++a) m->mean.push_back(sm[a] / cnt);
    for (int a = 0; a < 6; ++a) m->cov.push_back(sc[a] / cnt);
    m->count.push_back(int32_t(e - s));
    m->id_of.emplace(key[order[s]], id);
    s = e;
  }
  *out = m;
  return kOk;
}

int64_t oracle_map_size(const void* m) { return int64_t(static_cast<const Map*>(m)->keys.size()); }

void oracle_map_export(const void* mp, int64_t* keys, double* mean, double* cov, int32_t* count) {
  const Map* m = static_cast<const Map*>(mp);
  const size_t V = m->keys.size();
  if (keys) std::memcpy(keys, m->keys.data(), V * sizeof(int64_t));
  if (mean) std::memcpy(mean, m->mean.data(), 3 * V * sizeof(double));
  if (cov) std::memcpy(cov, m->cov.data(), 6 * V * sizeof(double));
  if (count) std::memcpy(count, m->count.data(), V * sizeof(int32_t));
}

void oracle_map_free(void* m) { delete static_cast<Map*>(m); }

void oracle_relative_pose(const double* Tt, const double* Ts, double* Tts) {
  Pose o = relative_pose(load_pose(Tt), load_pose(Ts));
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) Tts[4 * r + c] = o.R[r][c];
    Tts[4 * r + 3] = o.t[r];
  }
}

// Linearizes one factor. H is row-major [dim*dim] and b is [dim], dim = 6 (unary: free source
// pose, fixed target pose) or 12 (binary, [source | target]). corr is nullable, [n].
int oracle_linearize(const void* m, const double* xyz, const double* cov, int64_t n,
                     const double* Tt, const double* Ts, int binary, double* H, double* b,
                     double* e, int64_t* inliers, int32_t* corr) {
  if (!m || !Tt || !Ts || !H || !b || !e || !inliers || n < 0) return kInvalidArg;
  if (!finite_array(Tt, 12) || !finite_array(Ts, 12)) return kNonFinite;
  Cloud c{xyz, cov, n};
  return linearize_one(*static_cast<const Map*>(m), c, load_pose(Tt), load_pose(Ts), binary,
                       true, H, b, e, inliers, corr);
}

// Eq. (2) only: the cost and the inlier count (the overlap numerator of Sec. III-D).
int oracle_evaluate(const void* m, const double* xyz, const double* cov, int64_t n,
                    const double* Tt, const double* Ts, double* e, int64_t* inliers,
                    int32_t* corr) {
  if (!m || !Tt || !Ts || !e || !inliers || n < 0) return kInvalidArg;
  if (!finite_array(Tt, 12) || !finite_array(Ts, 12)) return kNonFinite;
  Cloud c{xyz, cov, n};
  return linearize_one(*static_cast<const Map*>(m), c, load_pose(Tt), load_pose(Ts), 0, false,
                       nullptr, nullptr, e, inliers, corr);
}

// Cost of Eq. (2) with the correspondences given (corr[k] = voxel id or -1) and, optionally,
// every point's inverse fused covariance given as omega[k][9] instead of recomputed. Used to
// take finite differences of the cost with frozen correspondences / frozen Omega.
int oracle_cost_fixed(const void* mp, const double* xyz, const double* cov, int64_t n,
                      const double* Tt, const double* Ts, const int32_t* corr,
                      const double* omega, double* e) {
  if (!mp || !corr || !e) return kInvalidArg;
  const Map& m = *static_cast<const Map*>(mp);
  const Pose T = relative_pose(load_pose(Tt), load_pose(Ts));
  Cloud c{xyz, cov, n};
  CompSum es;
  for (int64_t k = 0; k < n; ++k) {
    const int32_t v = corr[k];
    if (v < 0) continue;
    double mu[3], Ck[3][3], q[3], d[3];
    c.point(k, mu, Ck);
    transform_point(T, mu, q);
    for (int a = 0; a < 3; ++a) d[a] = m.mean[3 * v + a] - q[a];
    if (omega) {
      const double* W = omega + 9 * k;
      double s = 0.0;
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) s += d[r] * W[3 * r + cc] * d[cc];
      es.add(s);
    } else {
      double S[3][3], L[3][3], z[3];
      fused_covariance(T, &m.cov[6 * v], Ck, S);
      if (!cholesky3(S, L)) return kNonFinite;
      forward_sub(L, d, z);
      es.add(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
    }
  }
  *e = es.value();
  return kOk;
}

// Inverse fused covariance of every point with a correspondence (omega[k][9], row-major);
// zeros for points without one.
int oracle_point_omega(const void* mp, const double* xyz, const double* cov, int64_t n,
                       const double* Tt, const double* Ts, const int32_t* corr, double* omega) {
  if (!mp || !corr || !omega) return kInvalidArg;
  const Map& m = *static_cast<const Map*>(mp);
  const Pose T = relative_pose(load_pose(Tt), load_pose(Ts));
  Cloud c{xyz, cov, n};
  for (int64_t k = 0; k < n; ++k) {
    double* W = omega + 9 * k;
    for (int a = 0; a < 9; ++a) W[a] = 0.0;
    const int32_t v = corr[k];
    if (v < 0) continue;
    double mu[3], Ck[3][3], S[3][3], L[3][3];
    c.point(k, mu, Ck);
    fused_covariance(T, &m.cov[6 * v], Ck, S);
    if (!cholesky3(S, L)) return kNonFinite;
    for (int col = 0; col < 3; ++col) {
      double u[3] = {0, 0, 0}, y[3], x[3];
      u[col] = 1.0;
      forward_sub(L, u, y);
      back_sub(L, y, x);
      for (int r = 0; r < 3; ++r) W[3 * r + col] = x[r];
    }
  }
  return kOk;
}

// Exact gradient of Eq. (2) with the correspondences frozen (corr given) and the inverse fused
// covariance NOT frozen. With w_k = R^T Omega_k d_k (R = rotation of T_ts):
//   de/d omega_s = sum 2 w_k x (mu_k + C_k w_k),  de/d rho_s = sum -2 w_k,  de/d mu_k = -2 w_k,
//   de/d xi_t   = -Ad(T_st)^T de/d xi_s,  Ad(R, t) = [[R, 0], [[t]x R, R]],  T_st = T_ts^-1.
// g_xi is [6] (unary) or [12] ([source | target]); g_pts is [3][n] or null.
int oracle_gradient(const void* mp, const double* xyz, const double* cov, int64_t n,
                    const double* Tt, const double* Ts, int binary, const int32_t* corr,
                    double* g_xi, double* g_pts, double* e) {
  if (!mp || !corr || !g_xi) return kInvalidArg;
  const Map& m = *static_cast<const Map*>(mp);
  const Pose T = relative_pose(load_pose(Tt), load_pose(Ts));
  Cloud c{xyz, cov, n};
  CompSum gs[6], es;
  for (int64_t k = 0; k < n; ++k) {
    const int32_t v = corr[k];
    if (v < 0) {
      if (g_pts)
        for (int a = 0; a < 3; ++a) g_pts[a * n + k] = 0.0;
      continue;
    }
    double mu[3], Ck[3][3], q[3], d[3], S[3][3], L[3][3], z[3], od[3];
    c.point(k, mu, Ck);
    transform_point(T, mu, q);
    for (int a = 0; a < 3; ++a) d[a] = m.mean[3 * v + a] - q[a];
    fused_covariance(T, &m.cov[6 * v], Ck, S);
    if (!cholesky3(S, L)) return kNonFinite;
    forward_sub(L, d, z);
    back_sub(L, z, od);  // od = Omega d
    es.add(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
    double w[3];
    for (int a = 0; a < 3; ++a) w[a] = T.R[0][a] * od[0] + T.R[1][a] * od[1] + T.R[2][a] * od[2];
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = mu[a] + (Ck[a][0] * w[0] + Ck[a][1] * w[1] + Ck[a][2] * w[2]);
    const double wxu[3] = {w[1] * u[2] - w[2] * u[1], w[2] * u[0] - w[0] * u[2],
                           w[0] * u[1] - w[1] * u[0]};
    for (int a = 0; a < 3; ++a) {
      gs[a].add(2.0 * wxu[a]);
      gs[3 + a].add(-2.0 * w[a]);
    }
    if (g_pts)
      for (int a = 0; a < 3; ++a) g_pts[a * n + k] = -2.0 * w[a];
  }
  double g[6];
  for (int a = 0; a < 6; ++a) g[a] = gs[a].value();
  for (int a = 0; a < 6; ++a) g_xi[a] = g[a];
  if (binary) {
    // T_st = [R^T | -R^T t];  Ad(T_st) = [[A, 0], [[s]x A, A]] with A = R^T, s = -R^T t.
    double A[3][3], s[3];
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) A[r][cc] = T.R[cc][r];
    for (int r = 0; r < 3; ++r) s[r] = -(A[r][0] * T.t[0] + A[r][1] * T.t[1] + A[r][2] * T.t[2]);
    double Sx[3][3], SA[3][3];
    skew(s, Sx);
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc)
        SA[r][cc] = Sx[r][0] * A[0][cc] + Sx[r][1] * A[1][cc] + Sx[r][2] * A[2][cc];
    double Ad[6][6];
    for (int r = 0; r < 6; ++r)
      for (int cc = 0; cc < 6; ++cc) Ad[r][cc] = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) {
        Ad[r][cc] = A[r][cc];
        Ad[3 + r][3 + cc] = A[r][cc];
        Ad[3 + r][cc] = SA[r][cc];
      }
    for (int cc = 0; cc < 6; ++cc) {
      double s2 = 0.0;
      for (int r = 0; r < 6; ++r) s2 += Ad[r][cc] * g[r];
      g_xi[6 + cc] = -s2;
    }
  }
  if (e) *e = es.value();
  return kOk;
}

// Many factors at once, OpenMP over factors (each factor is computed exactly as by
// oracle_linearize). factors is [F][5]: target map, source cloud, target pose, source pose,
// binary. Outputs: H [F][144] (unary factors fill the leading 6x6 block, row stride 12, rest 0),
// b [F][12], e [F], inliers [F].
int oracle_linearize_factors(const void* const* maps, int32_t n_maps, const double* const* xyz,
                             const double* const* cov, const int64_t* npts, int32_t n_clouds,
                             const double* poses, int32_t n_poses, const int32_t* factors,
                             int32_t F, int nthreads, double* H, double* b, double* e,
                             int64_t* inliers) {
  if (F < 0 || !factors) return kInvalidArg;
  for (int32_t f = 0; f < F; ++f) {
    const int32_t* fd = factors + 5 * f;
    if (fd[0] < 0 || fd[0] >= n_maps || fd[1] < 0 || fd[1] >= n_clouds || fd[2] < 0 ||
        fd[2] >= n_poses || fd[3] < 0 || fd[3] >= n_poses)
      return kInvalidArg;
  }
  int status = kOk;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int32_t f = 0; f < F; ++f) {
    const int32_t* fd = factors + 5 * f;
    const int binary = fd[4] ? 1 : 0;
    double h[144], bb[12];
    int st = oracle_linearize(maps[fd[0]], xyz[fd[1]], cov[fd[1]], npts[fd[1]],
                              poses + 12 * fd[2], poses + 12 * fd[3], binary, h, bb, e + f,
                              inliers + f, nullptr);
    double* Hf = H + 144 * f;
    double* bf = b + 12 * f;
    for (int i = 0; i < 144; ++i) Hf[i] = 0.0;
    for (int i = 0; i < 12; ++i) bf[i] = 0.0;
    const int dim = binary ? 12 : 6;
    for (int i = 0; i < dim; ++i) {
      bf[i] = bb[i];
      for (int j = 0; j < dim; ++j) Hf[12 * i + j] = h[dim * i + j];
    }
    if (st != kOk) {
#ifdef _OPENMP
#pragma omp critical
#endif
      status = st;
    }
  }
  return status;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
