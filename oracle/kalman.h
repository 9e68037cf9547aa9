// TEST INFRASTRUCTURE ONLY -- part of the checking implementation ("oracle").
//
// Track model and Kalman filter steps shared by the tracking oracle and the
// refit oracle, as templates over the number type: float (the decisions'
// precision), double (FP64 reference) and Dual (forward-mode derivatives of
// the FP64 arithmetic).  Formulas: the readings of the paper's Kalman filter
// (Section 2) recorded with the documentation -- exact circle propagation in
// the bending plane, block-diagonal covariance, 2-D measurement update.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>

extern "C" {
struct OrcParams {
  float win_y, win_z;      // neighbour-finder windows per row step [cm]
  float d2_max;            // neighbour-finder cut on the chord deviation [cm^2]
  float chi2_max;          // attachment cut (2 degrees of freedom)
  float sinphi_max;        // propagation guard on |sin(phi)|
  float u_max;             // propagation guard on |C| * chord / 2
  float sigma_y, sigma_z;  // cluster errors [cm]
  float cww0;              // seed variance of q/pT [(GeV/c)^-2]
  float bz;                // field [T]
  int32_t min_hits;        // tracklets with fewer hits are dropped
  int32_t max_misses;      // consecutive rows without attachment that stop following
  int32_t descent_rows;    // longest step (in rows) of the walk back to the start row
  int32_t brute;           // 1: brute-force candidate scans
};
}

namespace orc {

// Forward-mode dual number: value and derivative along one direction.
struct Dual {
  double v = 0.0, d = 0.0;
  Dual() = default;
  Dual(double x) : v(x), d(0.0) {}  // NOLINT: constants promote implicitly
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator==(Dual a, Dual b) { return a.v == b.v; }
inline Dual sqrt(Dual a) {
  const double s = std::sqrt(a.v);
  return {s, a.d * 0.5 / s};
}
inline Dual fabs(Dual a) { return a.v < 0.0 ? -a : a; }
inline double value(double x) { return x; }
inline double value(float x) { return double(x); }
inline double value(Dual x) { return x.v; }


template <class T>
struct Consts {
  T kappa, sy2, sz2, wy, wz, d2max, chi2max, smax, umax, cww0;
};

template <class T>
Consts<T> make_consts(const OrcParams& p) {
  Consts<T> c;
  // kappa = c[GeV/(T cm)] * Bz: the rate of change of sin(phi) per cm and per
  // unit of q/pT.  Computed in double, then rounded once to T.
  c.kappa = T(2.99792458e-3 * double(p.bz));
  c.sy2 = T(p.sigma_y) * T(p.sigma_y);
  c.sz2 = T(p.sigma_z) * T(p.sigma_z);
  c.wy = T(p.win_y);
  c.wz = T(p.win_z);
  c.d2max = T(p.d2_max);
  c.chi2max = T(p.chi2_max);
  c.smax = T(p.sinphi_max);
  c.umax = T(p.u_max);
  c.cww0 = T(p.cww0);
  return c;
}

// asin(u)/u: the ratio of arc length to chord for a chord of half-length u*R.
inline float arc_over_chord(float u) {
  const float a1 = float(1.0 / 6.0);
  const float a2 = float(3.0 / 40.0);
  float u2 = u * u;
  return 1.0f + u2 * (a1 + u2 * a2);
}
inline double arc_over_chord(double u) { return u > 0.0 ? std::asin(u) / u : 1.0; }
// asin(u)/u and its derivative d/du = (u / sqrt(1 - u^2) - asin(u)) / u^2
// (series near 0, where the closed form cancels).
inline Dual arc_over_chord(Dual u) {
  const double x = u.v;
  double f, df;
  if (std::fabs(x) < 1e-3) {
    const double x2 = x * x;
    f = 1.0 + x2 * (1.0 / 6.0 + x2 * (3.0 / 40.0 + x2 * (5.0 / 112.0)));
    df = x * (1.0 / 3.0 + x2 * (3.0 / 10.0 + x2 * (15.0 / 56.0)));
  } else {
    const double as = std::asin(x);
    f = as / x;
    df = (x / std::sqrt(1.0 - x * x) - as) / (x * x);
  }
  return {f, df * u.d};
}

// Track state at the plane x: (y, z, s = sin(phi), t = dz/ds_xy, w = q/pT) and
// the two diagonal blocks of the covariance, (y, s, w) and (z, t).
template <class T>
struct State {
  T x, y, z, s, t, w;
  T cyy, csy, css, cwy, cws, cww;
  T czz, ctz, ctt;
};

// Propagate to the plane x1 along the circle of curvature -kappa*w.  Returns
// false (state untouched) when |sin(phi)| would reach smax or the chord is too
// long for the arc-length series.
template <class T>
bool propagate(State<T>& st, T x1, const Consts<T>& c) {
  using std::fabs;
  using std::sqrt;
  T dx = x1 - st.x;
  T k = c.kappa * st.w;
  T s1 = st.s - k * dx;
  if (!(fabs(s1) < c.smax)) return false;
  T c0 = sqrt(T(1) - st.s * st.s);
  T c1 = sqrt(T(1) - s1 * s1);
  T cc = c0 + c1;
  T ss = st.s + s1;
  T icc = T(1) / cc;
  T tg = ss * icc;
  T dy = dx * tg;
  T dl = sqrt(dx * dx + dy * dy);
  T u = (fabs(k) * dl) * T(0.5);
  if (!(u <= c.umax)) return false;
  T dS = dl * arc_over_chord(u);
  if (dx < T(0)) dS = -dS;
  // Jacobian of (y, s) with respect to (s, w); z couples to t only.
  T r0 = st.s / c0;
  T r1 = s1 / c1;
  T icc2 = icc * icc;
  T a = dx * ((T(2) * cc + ss * (r0 + r1)) * icc2);
  T e = -(c.kappa * dx);
  T b = (dx * e) * ((cc + ss * r1) * icc2);
  // C' = J C J^T, y-block
  T Py = (st.cyy + a * st.csy) + b * st.cwy;
  T Ps = (st.csy + a * st.css) + b * st.cws;
  T Pw = (st.cwy + a * st.cws) + b * st.cww;
  T Qy = st.csy + e * st.cwy;
  T Qs = st.css + e * st.cws;
  T Qw = st.cws + e * st.cww;
  st.cyy = (Py + a * Ps) + b * Pw;
  st.csy = (Qy + a * Qs) + b * Qw;
  st.cwy = Pw;
  st.css = Qs + e * Qw;
  st.cws = Qw;
  // z-block
  T Rz = st.czz + dS * st.ctz;
  T Rt = st.ctz + dS * st.ctt;
  st.czz = Rz + dS * Rt;
  st.ctz = Rt;
  // state
  st.y = st.y + dy;
  st.z = st.z + st.t * dS;
  st.s = s1;
  st.x = x1;
  return true;
}

// chi2 of the cluster (my, mz): squared residuals times the inverse
// residual variances (cluster error plus track error).
template <class T>
T chi2_of(const State<T>& st, T my, T mz, const Consts<T>& c) {
  T ry = my - st.y;
  T rz = mz - st.z;
  T iSy = T(1) / (st.cyy + c.sy2);
  T iSz = T(1) / (st.czz + c.sz2);
  return (ry * ry) * iSy + (rz * rz) * iSz;
}

// Kalman update with the cluster (my, mz); returns the cluster's chi2.
template <class T>
T update(State<T>& st, T my, T mz, const Consts<T>& c) {
  T ry = my - st.y;
  T rz = mz - st.z;
  T iSy = T(1) / (st.cyy + c.sy2);
  T iSz = T(1) / (st.czz + c.sz2);
  T chi2 = (ry * ry) * iSy + (rz * rz) * iSz;
  T k0 = st.cyy * iSy, k1 = st.csy * iSy, k2 = st.cwy * iSy;
  st.y = st.y + k0 * ry;
  st.s = st.s + k1 * ry;
  st.w = st.w + k2 * ry;
  T cyy = st.cyy, csy = st.csy, cwy = st.cwy;
  st.cyy = cyy - k0 * cyy;
  st.csy = csy - k1 * cyy;
  st.cwy = cwy - k2 * cyy;
  st.css = st.css - k1 * csy;
  st.cws = st.cws - k2 * csy;
  st.cww = st.cww - k2 * cwy;
  T kz0 = st.czz * iSz, kz1 = st.ctz * iSz;
  st.z = st.z + kz0 * rz;
  st.t = st.t + kz1 * rz;
  T czz = st.czz, ctz = st.ctz;
  st.czz = czz - kz0 * czz;
  st.ctz = ctz - kz1 * czz;
  st.ctt = st.ctt - kz1 * ctz;
  return chi2;
}


}  // namespace orc
