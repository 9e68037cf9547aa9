// TEST INFRASTRUCTURE ONLY -- the checking implementation ("oracle") of the
// track refit through a space-charge-distortion correction map, and of its
// gradient with respect to the map's coefficients.
//
// The paper names space-charge-distortion correction maps as a main source of
// track-quality problems (Abstract; Section 2) and describes the track fit as
// a Kalman filter over the attached clusters (Section 2).  The map form, the
// fit's seed and direction are readings recorded with the documentation:
//
//   map   three components (delta r, delta r*phi, delta z) [cm], each a
//         tensor-product uniform cubic B-spline over 36 phi nodes (every 10 deg,
//         periodic), 17 r nodes (85 + 10 j cm) and 20 z nodes (-250 + k 500/19
//         cm); nodes outside the r and z ranges are absent.
//   apply a measured cluster (x, y, z) in its sector frame, at radius r and
//         global azimuth phi, moves by delta r along (x, y)/r, by delta r*phi
//         along (-y, x)/r and by delta z along z.
//   refit outward from the innermost cluster of the track: y, z from that
//         cluster, sin(phi), dz/ds, q/pT from the tracking result (constants),
//         covariance diag(sy^2, sz^2, 1e-2, 1e-2, 1); then propagate to every
//         further cluster's own corrected x and update; no rejection.
//   loss  f(theta) = sum over tracks of dL_dchi2[track] * chi2[track].
//
// The gradient is computed here by forward-mode differentiation with dual
// numbers: one pass of the FP64 refit per cluster coordinate, then the chain
// rule through the (linear) map.  That is the exact derivative of the FP64
// arithmetic, by a method independent of any reverse sweep.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

#include "kalman.h"

namespace {

using namespace orc;

constexpr int kNPhi = 36, kNR = 17, kNZ = 20, kComp = 3;
constexpr int kNCoef = kComp * kNPhi * kNR * kNZ;
constexpr double kPi = 3.14159265358979323846;
constexpr double kDPhi = 2.0 * kPi / kNPhi;
constexpr double kR0 = 85.0, kDR = 10.0;
constexpr double kZ0 = -250.0, kDZ = 500.0 / 19.0;

// Uniform cubic B-spline centred at 0 with knots at the integers.
double bspline(double t) {
  const double a = std::fabs(t);
  if (a < 1.0) return (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0;
  if (a < 2.0) {
    const double b = 2.0 - a;
    return b * b * b / 6.0;
  }
  return 0.0;
}

int coef_index(int comp, int i, int j, int k) { return ((comp * kNPhi + i) * kNR + j) * kNZ + k; }

// The (up to) 4 x 4 x 4 nodes whose basis functions are non-zero at (r, phi,
// z), with their tensor-product weights.  Returns the number of terms.
int basis_terms(double r, double phi, double z, int* idx3, double* w) {
  double ph = std::fmod(phi, 2.0 * kPi);
  if (ph < 0) ph += 2.0 * kPi;
  const int i0 = int(std::floor(ph / kDPhi));
  const int j0 = int(std::floor((r - kR0) / kDR));
  const int k0 = int(std::floor((z - kZ0) / kDZ));
  int n = 0;
  for (int a = -1; a <= 2; ++a) {
    const int i = i0 + a;
    const double bi = bspline(ph / kDPhi - double(i));
    const int ii = ((i % kNPhi) + kNPhi) % kNPhi;
    for (int b = -1; b <= 2; ++b) {
      const int j = j0 + b;
      if (j < 0 || j >= kNR) continue;
      const double bj = bspline((r - (kR0 + kDR * j)) / kDR);
      for (int c = -1; c <= 2; ++c) {
        const int k = k0 + c;
        if (k < 0 || k >= kNZ) continue;
        const double bk = bspline((z - (kZ0 + kDZ * k)) / kDZ);
        const double ww = bi * bj * bk;
        if (ww == 0.0) continue;
        idx3[3 * n] = ii;
        idx3[3 * n + 1] = j;
        idx3[3 * n + 2] = k;
        w[n] = ww;
        ++n;
      }
    }
  }
  return n;
}

void map_eval(const double* theta, double r, double phi, double z, double* d3) {
  d3[0] = d3[1] = d3[2] = 0.0;
  if (!theta) return;
  int idx[3 * 64];
  double w[64];
  const int n = basis_terms(r, phi, z, idx, w);
  for (int c = 0; c < kComp; ++c)
    for (int t = 0; t < n; ++t) d3[c] += theta[coef_index(c, idx[3 * t], idx[3 * t + 1], idx[3 * t + 2])] * w[t];
}

struct Hit {
  double xm, ym, zm, r, phi;  // measured, sector frame; radius; global azimuth
  double xc, yc, zc;          // corrected
};

// z_map: the z at which the map is evaluated (the measured z, or a fixed z
// for time-frame input, whose drift coordinate is not z)
void correct(const double* theta, Hit& h, double z_map) {
  double d[3];
  map_eval(theta, h.r, h.phi, z_map, d);
  h.xc = h.xm + (d[0] * h.xm - d[1] * h.ym) / h.r;
  h.yc = h.ym + (d[0] * h.ym + d[1] * h.xm) / h.r;
  h.zc = h.zm + d[2];
}

// Outward refit over the corrected clusters; false if a propagation fails.
template <class T>
bool refit(const T* xc, const T* yc, const T* zc, int n, double s0, double t0, double w0,
           const Consts<T>& c, T* chi2_out) {
  State<T> st;
  st.x = xc[0];
  st.y = yc[0];
  st.z = zc[0];
  st.s = T(s0);
  st.t = T(t0);
  st.w = T(w0);
  diagonal_covariance(st, c.sy2, c.sz2, T(1e-2), T(1e-2), T(1));
  T chi2 = T(0);
  for (int i = 1; i < n; ++i) {
    if (!propagate(st, xc[i], c)) return false;
    chi2 = chi2 + update(st, yc[i], zc[i], c);
  }
  *chi2_out = chi2;
  return true;
}

struct RefitInput {
  const float* row_x;
  const OrcParams* p;
  int64_t n_tracks;
  const int64_t* hit_begin;
  const int32_t* hit_id;
  const uint8_t* hit_row;
  const int32_t* unit;
  const float* unit_alpha;
  const float* seed;  // [n][5] y, z, sin(phi), dz/ds, q/pT of the tracking result
  const float* y;
  const float* z;
  int z_fixed = 0;     // 1: the map is evaluated at z_map for every cluster
  double z_map = 0.0;
};

std::vector<Hit> track_hits(const RefitInput& in, int64_t t, const double* theta) {
  const bool fixed = in.z_fixed != 0;
  std::vector<Hit> hs;
  const double alpha = in.unit_alpha[in.unit[t]];
  for (int64_t q = in.hit_begin[t]; q < in.hit_begin[t + 1]; ++q) {
    Hit h;
    h.xm = double(in.row_x[in.hit_row[q]]);
    h.ym = double(in.y[in.hit_id[q]]);
    h.zm = double(in.z[in.hit_id[q]]);
    h.r = std::sqrt(h.xm * h.xm + h.ym * h.ym);
    h.phi = alpha + std::atan2(h.ym, h.xm);
    correct(theta, h, fixed ? in.z_map : h.zm);
    hs.push_back(h);
  }
  return hs;
}

}  // namespace

extern "C" {

int orc_map_ncoef() { return kNCoef; }

void orc_map_eval(const double* theta, double r, double phi, double z, double* out3) {
  map_eval(theta, r, phi, z, out3);
}

// Corrected position of a cluster measured at (x, y, z) in the frame of a
// sector whose centre line lies at azimuth alpha (the refit's correction):
// out3 = (x_c, y_c, z_c).
void orc_map_correct(const double* theta, double x, double y, double z, double alpha, double* out3) {
  Hit h;
  h.xm = x;
  h.ym = y;
  h.zm = z;
  h.r = std::sqrt(x * x + y * y);
  h.phi = alpha + std::atan2(y, x);
  correct(theta, h, h.zm);
  out3[0] = h.xc;
  out3[1] = h.yc;
  out3[2] = h.zc;
}

// Basis terms at a point: node indices (phi, r, z) and weights; returns count.
int orc_map_basis(double r, double phi, double z, int32_t* idx3, double* w) {
  return basis_terms(r, phi, z, idx3, w);
}

// FP64 refit chi2 per track (ok[t] = 0 when a propagation failed; chi2 = 0).
// z_fixed = 1: the map is evaluated at z = z_map for every cluster.
void orc_refit(const float* row_x, const OrcParams* p, int64_t n_tracks, const int64_t* hit_begin,
               const int32_t* hit_id, const uint8_t* hit_row, const int32_t* unit,
               const float* unit_alpha, const float* seed, const float* y, const float* z,
               const double* theta, int32_t z_fixed, double z_map, double* chi2, int32_t* ok) {
  RefitInput in{row_x, p, n_tracks, hit_begin, hit_id, hit_row, unit, unit_alpha, seed, y, z,
                z_fixed, z_map};
  const Consts<double> c = make_consts<double>(*p);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t t = 0; t < n_tracks; ++t) {
    std::vector<Hit> hs = track_hits(in, t, theta);
    const int n = int(hs.size());
    std::vector<double> xc(n), yc(n), zc(n);
    for (int i = 0; i < n; ++i) {
      xc[i] = hs[i].xc;
      yc[i] = hs[i].yc;
      zc[i] = hs[i].zc;
    }
    double ch = 0.0;
    const float* sd = seed + 5 * t;
    const bool good = n >= 2 && refit<double>(xc.data(), yc.data(), zc.data(), n, double(sd[2]),
                                              double(sd[3]), double(sd[4]), c, &ch);
    ok[t] = good ? 1 : 0;
    chi2[t] = good ? ch : 0.0;
  }
}

// Gradient of f = sum_t dL_dchi2[t] * chi2[t] with respect to theta (written
// to grad[kNCoef]) and, if hit_grad is not null, with respect to every corrected
// cluster coordinate (hit_grad[3 * hit] = df/d(xc, yc, zc)).
void orc_refit_grad(const float* row_x, const OrcParams* p, int64_t n_tracks,
                    const int64_t* hit_begin, const int32_t* hit_id, const uint8_t* hit_row,
                    const int32_t* unit, const float* unit_alpha, const float* seed, const float* y,
                    const float* z, const double* theta, const double* dL_dchi2, double* grad,
                    double* hit_grad) {
  RefitInput in{row_x, p, n_tracks, hit_begin, hit_id, hit_row, unit, unit_alpha, seed, y, z};
  const Consts<Dual> c = make_consts<Dual>(*p);
  const int64_t n_hits = hit_begin[n_tracks];
  std::vector<double> hg(3 * size_t(n_hits), 0.0);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4)
#endif
  for (int64_t t = 0; t < n_tracks; ++t) {
    std::vector<Hit> hs = track_hits(in, t, theta);
    const int n = int(hs.size());
    if (n < 2 || dL_dchi2[t] == 0.0) continue;
    const float* sd = seed + 5 * t;
    std::vector<Dual> xc(n), yc(n), zc(n);
    for (int q = 0; q < n; ++q) {
      for (int comp = 0; comp < 3; ++comp) {
        for (int i = 0; i < n; ++i) {
          xc[i] = Dual(hs[i].xc, (i == q && comp == 0) ? 1.0 : 0.0);
          yc[i] = Dual(hs[i].yc, (i == q && comp == 1) ? 1.0 : 0.0);
          zc[i] = Dual(hs[i].zc, (i == q && comp == 2) ? 1.0 : 0.0);
        }
        Dual ch;
        if (!refit<Dual>(xc.data(), yc.data(), zc.data(), n, double(sd[2]), double(sd[3]),
                         double(sd[4]), c, &ch))
          break;
        hg[3 * size_t(hit_begin[t] + q) + comp] = dL_dchi2[t] * ch.d;
      }
    }
  }
  // chain rule through the map, in a fixed order
  std::memset(grad, 0, sizeof(double) * kNCoef);
  for (int64_t t = 0; t < n_tracks; ++t) {
    std::vector<Hit> hs = track_hits(in, t, theta);
    for (size_t q = 0; q < hs.size(); ++q) {
      const Hit& h = hs[q];
      const double* g = &hg[3 * size_t(hit_begin[t] + int64_t(q))];
      // d(xc, yc)/d(delta r) = (x, y)/r; d(xc, yc)/d(delta r*phi) = (-y, x)/r
      const double gr = (g[0] * h.xm + g[1] * h.ym) / h.r;
      const double gp = (-g[0] * h.ym + g[1] * h.xm) / h.r;
      const double gz = g[2];
      int idx[3 * 64];
      double w[64];
      const int nt = basis_terms(h.r, h.phi, h.zm, idx, w);
      for (int k = 0; k < nt; ++k) {
        grad[coef_index(0, idx[3 * k], idx[3 * k + 1], idx[3 * k + 2])] += gr * w[k];
        grad[coef_index(1, idx[3 * k], idx[3 * k + 1], idx[3 * k + 2])] += gp * w[k];
        grad[coef_index(2, idx[3 * k], idx[3 * k + 1], idx[3 * k + 2])] += gz * w[k];
      }
    }
  }
  if (hit_grad) std::memcpy(hit_grad, hg.data(), sizeof(double) * hg.size());
}

}  // extern "C"
