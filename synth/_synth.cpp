// Native helpers of the synthetic LiDAR-scene generator: ray casting against a scene of
// ground plane, axis-aligned boxes and vertical cylinders; centroid voxel-grid downsampling;
// plane-regularised point covariances from given neighbour lists.
//
// Input generation only: nothing here evaluates the registration cost.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

struct Box { double x0, y0, z0, x1, y1, z1; };
struct Cyl { double cx, cy, r, z0, z1; };

// Ray p + t d against an axis-aligned box (slab method); returns the entry distance or +inf.
double hit_box(const double p[3], const double d[3], const Box& b) {
  double lo[3] = {b.x0, b.y0, b.z0}, hi[3] = {b.x1, b.y1, b.z1};
  double tmin = 0.0, tmax = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (std::fabs(d[a]) < 1e-15) {
      if (p[a] < lo[a] || p[a] > hi[a]) return INFINITY;
      continue;
    }
    double t0 = (lo[a] - p[a]) / d[a], t1 = (hi[a] - p[a]) / d[a];
    if (t0 > t1) std::swap(t0, t1);
    tmin = std::max(tmin, t0);
    tmax = std::min(tmax, t1);
    if (tmin > tmax) return INFINITY;
  }
  return tmin > 0.0 ? tmin : INFINITY;
}

// Ray against the side of a vertical finite cylinder.
double hit_cyl(const double p[3], const double d[3], const Cyl& c) {
  const double ox = p[0] - c.cx, oy = p[1] - c.cy;
  const double A = d[0] * d[0] + d[1] * d[1];
  if (A < 1e-15) return INFINITY;
  const double B = 2.0 * (ox * d[0] + oy * d[1]);
  const double C = ox * ox + oy * oy - c.r * c.r;
  const double disc = B * B - 4.0 * A * C;
  if (disc < 0.0) return INFINITY;
  const double t = (-B - std::sqrt(disc)) / (2.0 * A);
  if (t <= 0.0) return INFINITY;
  const double z = p[2] + t * d[2];
  return (z >= c.z0 && z <= c.z1) ? t : INFINITY;
}

}  // namespace

extern "C" {

// Casts nbeams x naz rays from each sensor. sensors: [ns][4] = (x, y, z, yaw). Ray (i, j) has
// elevation elev[i] and sensor-frame azimuth 2 pi j / naz. out: [ns][nbeams*naz][3] sensor-frame
// hit points with range noise noise[s][i*naz + j] added along the ray; valid marks hits within
// max_range (after noise).
void synth_raycast(const double* boxes, int nb, const double* cyls, int nc, const double* sensors,
                   int ns, const double* elev, int nbeams, int naz, double max_range,
                   const double* noise, double* out, unsigned char* valid, int nthreads) {
  const Box* B = reinterpret_cast<const Box*>(boxes);
  const Cyl* C = reinterpret_cast<const Cyl*>(cyls);
  const double two_pi = 2.0 * M_PI;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  for (int s = 0; s < ns; ++s) {
    const double* S = sensors + 4 * s;
    const double p[3] = {S[0], S[1], S[2]};
    const double yaw = S[3];
    // Per azimuth column, the objects whose bounding circle the column can meet.
    std::vector<std::vector<int>> col(naz);  // object id: box i -> i, cylinder i -> nb + i
    auto add_span = [&](int id, double cx, double cy, double rb) {
      const double dx = cx - p[0], dy = cy - p[1];
      const double rho = std::sqrt(dx * dx + dy * dy);
      if (rho - rb > max_range) return;
      if (rho <= rb * 1.0001) {
        for (int j = 0; j < naz; ++j) col[j].push_back(id);
        return;
      }
      const double centre = std::atan2(dy, dx) - yaw;
      const double hw = std::asin(std::min(1.0, rb / rho)) + two_pi / naz;
      int j0 = int(std::floor((centre - hw) / two_pi * naz));
      int j1 = int(std::ceil((centre + hw) / two_pi * naz));
      for (int j = j0; j <= j1; ++j) col[((j % naz) + naz) % naz].push_back(id);
    };
    for (int i = 0; i < nb; ++i) {
      const double hx = 0.5 * (B[i].x1 - B[i].x0), hy = 0.5 * (B[i].y1 - B[i].y0);
      add_span(i, B[i].x0 + hx, B[i].y0 + hy, std::sqrt(hx * hx + hy * hy));
    }
    for (int i = 0; i < nc; ++i) add_span(nb + i, C[i].cx, C[i].cy, C[i].r);
    for (auto& v : col) {
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    const int nr = nbeams * naz;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int r = 0; r < nr; ++r) {
      const int i = r / naz, j = r % naz;
      const double az = two_pi * j / naz;
      const double ce = std::cos(elev[i]), se = std::sin(elev[i]);
      const double ds[3] = {ce * std::cos(az), ce * std::sin(az), se};  // sensor frame
      const double cy = std::cos(yaw), sy = std::sin(yaw);
      const double dw[3] = {cy * ds[0] - sy * ds[1], sy * ds[0] + cy * ds[1], ds[2]};
      double t = INFINITY;
      if (dw[2] < -1e-12) t = -p[2] / dw[2];  // ground z = 0
      for (int id : col[j]) {
        const double th = id < nb ? hit_box(p, dw, B[id]) : hit_cyl(p, dw, C[id - nb]);
        if (th < t) t = th;
      }
      const size_t o = size_t(s) * nr + r;
      double tn = t + noise[o];
      if (std::isfinite(t) && t <= max_range && tn > 0.0 && tn <= max_range) {
        out[3 * o + 0] = tn * ds[0];
        out[3 * o + 1] = tn * ds[1];
        out[3 * o + 2] = tn * ds[2];
        valid[o] = 1;
      } else {
        out[3 * o + 0] = out[3 * o + 1] = out[3 * o + 2] = 0.0;
        valid[o] = 0;
      }
    }
  }
}

// Centroid voxel-grid filter: one output point per occupied cell (the mean of its points),
// cells in ascending (x, y, z) order. pts and out are [n][3]; returns the output count.
int64_t synth_downsample(const double* pts, int64_t n, double res, double* out) {
  std::vector<int64_t> kx(n), ky(n), kz(n);
  for (int64_t i = 0; i < n; ++i) {
    kx[i] = int64_t(std::floor(pts[3 * i] / res));
    ky[i] = int64_t(std::floor(pts[3 * i + 1] / res));
    kz[i] = int64_t(std::floor(pts[3 * i + 2] / res));
  }
  std::vector<int64_t> ord(n);
  std::iota(ord.begin(), ord.end(), int64_t(0));
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    if (kx[a] != kx[b]) return kx[a] < kx[b];
    if (ky[a] != ky[b]) return ky[a] < ky[b];
    if (kz[a] != kz[b]) return kz[a] < kz[b];
    return a < b;
  });
  int64_t m = 0;
  for (int64_t s = 0; s < n;) {
    int64_t e = s;
    double acc[3] = {0, 0, 0};
    while (e < n && kx[ord[e]] == kx[ord[s]] && ky[ord[e]] == ky[ord[s]] &&
           kz[ord[e]] == kz[ord[s]]) {
      for (int a = 0; a < 3; ++a) acc[a] += pts[3 * ord[e] + a];
      ++e;
    }
    for (int a = 0; a < 3; ++a) out[3 * m + a] = acc[a] / double(e - s);
    ++m;
    s = e;
  }
  return m;
}

// Point covariances from neighbour lists: the unit eigenvector n of the smallest eigenvalue of
// the neighbours' sample covariance is taken as the surface normal, and the covariance is set to
// scale * (I - (1 - flat) n n^T), i.e. eigenvalues (1, 1, flat) * scale around the surface.
// pts [n][3]; nbr [n][k] (int64 indices); out6 [6][n] FP32 (xx xy xz yy yz zz).
void synth_plane_cov(const double* pts, int64_t n, const int64_t* nbr, int k, double scale,
                     double flat, float* out6, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t i = 0; i < n; ++i) {
    double mu[3] = {0, 0, 0};
    for (int j = 0; j < k; ++j)
      for (int a = 0; a < 3; ++a) mu[a] += pts[3 * nbr[i * k + j] + a];
    for (int a = 0; a < 3; ++a) mu[a] /= k;
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int j = 0; j < k; ++j) {
      double v[3];
      for (int a = 0; a < 3; ++a) v[a] = pts[3 * nbr[i * k + j] + a] - mu[a];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A[a][b] += v[a] * v[b];
    }
    // Cyclic Jacobi eigenvalue iteration on the symmetric 3x3 matrix.
    double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 30; ++sweep) {
      const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
      const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
      if (off <= 1e-30 * dia + 1e-300) break;
      for (int p = 0; p < 2; ++p)
        for (int q = p + 1; q < 3; ++q) {
          if (std::fabs(A[p][q]) < 1e-300) continue;
          const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
          const double t = (theta >= 0 ? 1.0 : -1.0) /
                           (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
          const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
          for (int r = 0; r < 3; ++r) {
            const double arp = A[r][p], arq = A[r][q];
            A[r][p] = c * arp - s * arq;
            A[r][q] = s * arp + c * arq;
          }
          for (int r = 0; r < 3; ++r) {
            const double apr = A[p][r], aqr = A[q][r];
            A[p][r] = c * apr - s * aqr;
            A[q][r] = s * apr + c * aqr;
          }
          for (int r = 0; r < 3; ++r) {
            const double vrp = V[r][p], vrq = V[r][q];
            V[r][p] = c * vrp - s * vrq;
            V[r][q] = s * vrp + c * vrq;
          }
        }
    }
    int m = 0;
    for (int a = 1; a < 3; ++a)
      if (A[a][a] < A[m][m]) m = a;
    double nv[3] = {V[0][m], V[1][m], V[2][m]};
    const double nn = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    for (int a = 0; a < 3; ++a) nv[a] /= nn;
    const double g = 1.0 - flat;
    const double c6[6] = {scale * (1.0 - g * nv[0] * nv[0]), -scale * g * nv[0] * nv[1],
                          -scale * g * nv[0] * nv[2], scale * (1.0 - g * nv[1] * nv[1]),
                          -scale * g * nv[1] * nv[2], scale * (1.0 - g * nv[2] * nv[2])};
    for (int a = 0; a < 6; ++a) out6[a * n + i] = float(c6[a]);
  }
}

}  // extern "C"
