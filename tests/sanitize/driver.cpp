// Host driver for the address / undefined-behaviour sanitizer runs of the oracle and of the
// input generator's native helpers: every exported function on small inputs, edge cases and
// error paths, with a hand-computed value checked so that the run is not vacuous.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

extern "C" {
int oracle_voxel_coord(double v, double res, int64_t* k);
int64_t oracle_pack_key(int64_t kx, int64_t ky, int64_t kz);
void oracle_unpack_key(int64_t key, int64_t* kx, int64_t* ky, int64_t* kz);
int oracle_map_build(const double* xyz, const double* cov, int64_t n, double res, void** out);
int64_t oracle_map_size(const void* m);
void oracle_map_export(const void* m, int64_t* keys, double* mean, double* cov, int32_t* count);
void oracle_map_free(void* m);
void oracle_relative_pose(const double* Tt, const double* Ts, double* Tts);
int oracle_linearize(const void* m, const double* xyz, const double* cov, int64_t n,
                     const double* Tt, const double* Ts, int binary, double* H, double* b,
                     double* e, int64_t* inliers, int32_t* corr);
int oracle_evaluate(const void* m, const double* xyz, const double* cov, int64_t n,
                    const double* Tt, const double* Ts, double* e, int64_t* inliers,
                    int32_t* corr);
int oracle_cost_fixed(const void* m, const double* xyz, const double* cov, int64_t n,
                      const double* Tt, const double* Ts, const int32_t* corr,
                      const double* omega, double* e);
int oracle_point_omega(const void* m, const double* xyz, const double* cov, int64_t n,
                       const double* Tt, const double* Ts, const int32_t* corr, double* omega);
int oracle_gradient(const void* m, const double* xyz, const double* cov, int64_t n,
                    const double* Tt, const double* Ts, int binary, const int32_t* corr,
                    double* g_xi, double* g_points, double* e);
int oracle_linearize_factors(const void* const* maps, int32_t n_maps, const double* const* xyz,
                             const double* const* cov, const int64_t* npts, int32_t n_clouds,
                             const double* poses, int32_t n_poses, const int32_t* factors,
                             int32_t F, int nthreads, double* H, double* b, double* e,
                             int64_t* inliers);
void synth_raycast(const double* boxes, int nb, const double* cyls, int nc, const double* sensors,
                   int ns, const double* elev, int nbeams, int naz, double max_range,
                   const double* noise, double* out, unsigned char* valid, int nthreads);
int64_t synth_downsample(const double* pts, int64_t n, double res, double* out);
void synth_plane_cov(const double* pts, int64_t n, const int64_t* nbr, int k, double scale,
                     double flat, float* out6, int nthreads);
}

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

int main() {
  const double I12[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
  // the single-point case with exact values: e = 0.125, b = (-1/8, 1/4, -1/8, 1/4, 0, -1/4)
  {
    const double txyz[3] = {0.25, 0.5, 0.75}, tcov[6] = {0.5, 0, 0, 0.5, 0, 0.5};
    const double sxyz[3] = {0.5, 0.5, 0.5}, scov[6] = {0.5, 0, 0, 0.5, 0, 0.5};
    void* m = nullptr;
    CHECK(oracle_map_build(txyz, tcov, 1, 1.0, &m) == 0);
    double H[144], b[12], e = 0;
    int64_t nin = 0;
    int32_t corr[1];
    CHECK(oracle_linearize(m, sxyz, scov, 1, I12, I12, 0, H, b, &e, &nin, corr) == 0);
    CHECK(e == 0.125 && nin == 1 && corr[0] == 0);
    const double bref[6] = {-0.125, 0.25, -0.125, 0.25, 0.0, -0.25};
    for (int i = 0; i < 6; ++i) CHECK(b[i] == bref[i]);
    CHECK(oracle_linearize(m, sxyz, scov, 1, I12, I12, 1, H, b, &e, &nin, nullptr) == 0);
    oracle_map_free(m);
  }
  // keys
  int64_t k = 0;
  CHECK(oracle_voxel_coord(1.0, 0.5, &k) == 0 && k == 2);
  CHECK(oracle_voxel_coord(-1e-30, 0.5, &k) == 0 && k == -1);
  CHECK(oracle_voxel_coord(-0.0, 0.5, &k) == 0 && k == 0);
  CHECK(oracle_voxel_coord(NAN, 0.5, &k) != 0);
  CHECK(oracle_voxel_coord(1e300, 0.5, &k) != 0);
  int64_t a, bb, c;
  oracle_unpack_key(oracle_pack_key(-5, 7, -1048575), &a, &bb, &c);
  CHECK(a == -5 && bb == 7 && c == -1048575);
  // random clouds through every entry point
  std::mt19937_64 rng(7);
  std::normal_distribution<double> N(0.0, 1.0);
  const int64_t n = 3000;
  std::vector<double> xyz(3 * n), cov(6 * n), sx(3 * n), sc(6 * n);
  for (int64_t i = 0; i < n; ++i) {
    for (int a2 = 0; a2 < 3; ++a2) {
      xyz[a2 * n + i] = 2.0 * N(rng);
      sx[a2 * n + i] = xyz[a2 * n + i] + 0.05 * N(rng);
    }
    const double d[6] = {0.01, 0, 0, 0.01, 0, 0.01};
    for (int a2 = 0; a2 < 6; ++a2) cov[a2 * n + i] = sc[a2 * n + i] = d[a2];
  }
  void* m = nullptr;
  CHECK(oracle_map_build(xyz.data(), cov.data(), n, 0.3, &m) == 0);
  const int64_t V = oracle_map_size(m);
  std::vector<int64_t> keys(V);
  std::vector<double> mean(3 * V), vcov(6 * V);
  std::vector<int32_t> count(V);
  oracle_map_export(m, keys.data(), mean.data(), vcov.data(), count.data());
  int64_t tot = 0;
  for (int32_t x : count) tot += x;
  CHECK(tot == n);
  double Ts[12] = {1, 0, 0, 0.01, 0, 1, 0, -0.02, 0, 0, 1, 0.03}, Tts[12];
  oracle_relative_pose(I12, Ts, Tts);
  std::vector<int32_t> corr(n);
  double H[144], b[12], e = 0, e2 = 0;
  int64_t nin = 0;
  CHECK(oracle_linearize(m, sx.data(), sc.data(), n, I12, Ts, 1, H, b, &e, &nin, corr.data()) == 0);
  CHECK(nin > 0);
  CHECK(oracle_evaluate(m, sx.data(), sc.data(), n, I12, Ts, &e2, &nin, corr.data()) == 0);
  CHECK(std::fabs(e - e2) <= 1e-9 * e);
  std::vector<double> om(9 * n), gp(3 * n);
  CHECK(oracle_point_omega(m, sx.data(), sc.data(), n, I12, Ts, corr.data(), om.data()) == 0);
  CHECK(oracle_cost_fixed(m, sx.data(), sc.data(), n, I12, Ts, corr.data(), om.data(), &e2) == 0);
  CHECK(oracle_cost_fixed(m, sx.data(), sc.data(), n, I12, Ts, corr.data(), nullptr, &e2) == 0);
  double g[12];
  CHECK(oracle_gradient(m, sx.data(), sc.data(), n, I12, Ts, 1, corr.data(), g, gp.data(), &e2) == 0);
  // a batch of factors, unary and binary, one empty cloud
  const void* maps[1] = {m};
  const double* xs[2] = {sx.data(), sx.data()};
  const double* cs[2] = {sc.data(), sc.data()};
  const int64_t np[2] = {n, 0};
  double poses[24];
  for (int i = 0; i < 12; ++i) {
    poses[i] = I12[i];
    poses[12 + i] = Ts[i];
  }
  const int32_t fac[15] = {0, 0, 0, 1, 1, 0, 0, 0, 1, 0, 0, 1, 0, 1, 1};
  double FH[3 * 144], Fb[36], Fe[3];
  int64_t Fn[3];
  CHECK(oracle_linearize_factors(maps, 1, xs, cs, np, 2, poses, 2, fac, 3, 2, FH, Fb, Fe, Fn) == 0);
  CHECK(Fn[2] == 0 && Fe[2] == 0.0);
  // error paths
  std::vector<double> bad = sx;
  bad[5] = NAN;
  void* m2 = nullptr;
  CHECK(oracle_map_build(bad.data(), cov.data(), n, 0.3, &m2) != 0 && m2 == nullptr);
  CHECK(oracle_map_build(xyz.data(), cov.data(), -1, 0.3, &m2) != 0);
  CHECK(oracle_linearize(m, bad.data(), sc.data(), n, I12, Ts, 1, H, b, &e, &nin, nullptr) != 0);
  void* m0 = nullptr;
  CHECK(oracle_map_build(nullptr, nullptr, 0, 0.5, &m0) == 0 && oracle_map_size(m0) == 0);
  CHECK(oracle_linearize(m0, sx.data(), sc.data(), n, I12, Ts, 0, H, b, &e, &nin, nullptr) == 0 &&
        nin == 0 && e == 0.0);
  oracle_map_free(m0);
  oracle_map_free(m);
  // generator helpers: a ray cast, a voxel filter, plane covariances from neighbour lists
  const double boxes[12] = {5, -2, -1, 8, 2, 3, -10, -10, -2, 10, 10, -1.9};
  const double cyls[5] = {0, 6, 0.2, -2, 3};
  const double sensors[4] = {0, 0, 0, 0.1};
  const int nbeams = 4, naz = 90;
  const double elev[4] = {-0.3, -0.1, 0.1, 0.3};
  std::vector<double> noise(nbeams * naz), hits(3 * nbeams * naz);
  for (double& x : noise) x = 0.01 * N(rng);
  std::vector<unsigned char> valid(nbeams * naz);
  synth_raycast(boxes, 2, cyls, 1, sensors, 1, elev, nbeams, naz, 50.0, noise.data(),
                hits.data(), valid.data(), 2);
  std::vector<double> pts;
  for (int i = 0; i < nbeams * naz; ++i)
    if (valid[i])
      for (int a2 = 0; a2 < 3; ++a2) pts.push_back(hits[3 * i + a2]);
  const int64_t np2 = (int64_t)pts.size() / 3;
  CHECK(np2 > 20);
  std::vector<double> ds(pts.size());
  const int64_t nd = synth_downsample(pts.data(), np2, 0.25, ds.data());
  CHECK(nd > 0 && nd <= np2);
  const int kk = 5;
  std::vector<int64_t> nbr(nd * kk);
  for (int64_t i = 0; i < nd; ++i)  // brute-force neighbours (the point itself included)
    for (int q = 0; q < kk; ++q) nbr[i * kk + q] = (i + q) % nd;
  std::vector<float> out6(6 * nd);
  synth_plane_cov(ds.data(), nd, nbr.data(), kk, 0.01, 1e-3, out6.data(), 2);
  for (float x : out6) CHECK(std::isfinite(x));
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("sanitized run ok: %lld voxels, %lld inliers, %lld hits, %lld filtered\n",
              (long long)V, (long long)Fn[0], (long long)np2, (long long)nd);
  return 0;
}
