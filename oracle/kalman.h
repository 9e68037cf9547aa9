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
// the two diagonal blocks of the covariance, (y, s, w) and (z, t), each held
// as a U D U^T factorisation (U unit upper triangular, D diagonal; Bierman,
// "Factorization Methods for Discrete Sequential Estimation", 1977):
//   (y, s, w):  U = [[1, uys, uyw], [0, 1, usw], [0, 0, 1]],  D = diag(dy, ds, dw)
//   (z, t):     U = [[1, uzt], [0, 1]],                       D = diag(dz, dt)
// The transport Jacobians are unit upper triangular, so the transport only
// adds to U, and the measurement update forms no difference of nearly equal
// covariances (the textbook C - K H C loses about log2(C_yy / sigma^2) bits
// in float when the predicted variance of y is far above the cluster error).
template <class T>
struct State {
  T x, y, z, s, t, w;
  T uys, uyw, usw, dy, ds, dw;
  T uzt, dz, dt;
};

// Covariance entries of a state, lower triangle of each block.
template <class T>
struct Cov9 {
  T cyy, csy, css, cwy, cws, cww, czz, ctz, ctt;
};

template <class T>
Cov9<T> covariance(const State<T>& st) {
  Cov9<T> c;
  c.cww = st.dw;
  c.cws = st.usw * st.dw;
  c.cwy = st.uyw * st.dw;
  c.css = st.ds + st.usw * c.cws;
  c.csy = st.uys * st.ds + st.uyw * c.cws;
  c.cyy = (st.dy + st.uys * (st.uys * st.ds)) + st.uyw * c.cwy;
  c.ctt = st.dt;
  c.ctz = st.uzt * st.dt;
  c.czz = st.dz + st.uzt * c.ctz;
  return c;
}

// The factorisation of given covariance blocks (positive definite).
template <class T>
void set_covariance(State<T>& st, const Cov9<T>& c) {
  st.dw = c.cww;
  st.uyw = c.cwy / st.dw;
  st.usw = c.cws / st.dw;
  st.ds = c.css - st.usw * st.usw * st.dw;
  st.uys = (c.csy - st.uyw * st.usw * st.dw) / st.ds;
  st.dy = c.cyy - st.uys * st.uys * st.ds - st.uyw * st.uyw * st.dw;
  st.dt = c.ctt;
  st.uzt = c.ctz / st.dt;
  st.dz = c.czz - st.uzt * st.uzt * st.dt;
}

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
  // Jacobian of (y, s, w): [[1, a, b], [0, 1, e], [0, 0, 1]]; of (z, t):
  // [[1, dS], [0, 1]] (z couples to t only).
  T r0 = st.s / c0;
  T r1 = s1 / c1;
  T icc2 = icc * icc;
  T a = dx * ((T(2) * cc + ss * (r0 + r1)) * icc2);
  T e = -(c.kappa * dx);
  T b = (dx * e) * ((cc + ss * r1) * icc2);
  // C' = J U D U^T J^T = (J U) D (J U)^T: J U is unit upper triangular again
  st.uyw = (st.uyw + a * st.usw) + b;
  st.uys = st.uys + a;
  st.usw = st.usw + e;
  st.uzt = st.uzt + dS;
  // state
  st.y = st.y + dy;
  st.z = st.z + st.t * dS;
  st.s = s1;
  st.x = x1;
  return true;
}

// Residual variances of a cluster measurement, S_y = C_yy + sy^2 and
// S_z = C_zz + sz^2, as sums of non-negative terms of the factorisation; the
// partial sums a1, a2 (and z1) are the ones the update needs.
template <class T>
struct Innov {
  T v2, v3, a1, a2, sy;  // sy = S_y
  T vz, z1, sz;          // sz = S_z
};

template <class T>
Innov<T> innovation(const State<T>& st, const Consts<T>& c) {
  Innov<T> q;
  q.v2 = st.ds * st.uys;
  q.v3 = st.dw * st.uyw;
  q.a1 = c.sy2 + st.dy;
  q.a2 = q.a1 + q.v2 * st.uys;
  q.sy = q.a2 + q.v3 * st.uyw;
  q.vz = st.dt * st.uzt;
  q.z1 = c.sz2 + st.dz;
  q.sz = q.z1 + q.vz * st.uzt;
  return q;
}

// chi2 of the cluster (my, mz): squared residuals times the inverse
// residual variances (cluster error plus track error).
template <class T>
T chi2_of(const State<T>& st, T my, T mz, const Consts<T>& c) {
  const Innov<T> q = innovation(st, c);
  T ry = my - st.y;
  T rz = mz - st.z;
  T iSy = T(1) / q.sy;
  T iSz = T(1) / q.sz;
  return (ry * ry) * iSy + (rz * rz) * iSz;
}

// Kalman update with the cluster (my, mz); returns the cluster's chi2.
// Measurement of the first component of each block, processed as in
// Bierman's scalar update: with f = U^T h = (1, uys, uyw) and v = D f, the
// partial sums a1 = sy^2 + dy, a2 = a1 + v2 uys, S_y = a2 + v3 uyw give
//   D' = (dy sy^2/a1, ds a1/a2, dw a2/S_y),
//   uys' = uys sy^2/a1, uyw' = uyw sy^2/a2, usw' = usw - v2 uyw/a2,
// and the gain S_y^-1 (C_yy, C_sy, C_wy) with C_yy = dy + uys v2 + uyw v3,
// C_sy = v2 + usw v3, C_wy = v3 (the first column of the prior covariance).
// The (z, t) block is the same with two components.
template <class T>
T update(State<T>& st, T my, T mz, const Consts<T>& c) {
  const Innov<T> q = innovation(st, c);
  T ry = my - st.y;
  T rz = mz - st.z;
  T iSy = T(1) / q.sy;
  T iSz = T(1) / q.sz;
  T chi2 = (ry * ry) * iSy + (rz * rz) * iSz;
  T i1 = T(1) / q.a1;
  T i2 = T(1) / q.a2;
  T b1 = (st.dy + st.uys * q.v2) + st.uyw * q.v3;
  T b2 = q.v2 + st.usw * q.v3;
  T g = ry * iSy;
  st.y = st.y + b1 * g;
  st.s = st.s + b2 * g;
  st.w = st.w + q.v3 * g;
  T f1 = c.sy2 * i1;
  st.usw = st.usw - q.v2 * (st.uyw * i2);
  st.uyw = st.uyw * (c.sy2 * i2);
  st.uys = st.uys * f1;
  st.dw = st.dw * (q.a2 * iSy);
  st.ds = st.ds * (q.a1 * i2);
  st.dy = st.dy * f1;
  T j1 = T(1) / q.z1;
  T bz1 = st.dz + st.uzt * q.vz;
  T gz = rz * iSz;
  st.z = st.z + bz1 * gz;
  st.t = st.t + q.vz * gz;
  T fz = c.sz2 * j1;
  st.uzt = st.uzt * fz;
  st.dt = st.dt * (q.z1 * iSz);
  st.dz = st.dz * fz;
  return chi2;
}

// The 2-point seed's covariance for a chord of length dl (1/dl = idl)
// between two clusters of errors sy, sz: C_yy = sy^2, C_sy = sy^2/dl,
// C_ss = 2 sy^2/dl^2 (likewise for z, t), var(q/pT) = cww0, no other
// correlation.  Factorised: uys = dl/2, dy = sy^2/2, ds = C_ss.
template <class T>
void seed_covariance(State<T>& st, T dl, T idl, const Consts<T>& c) {
  T idl2 = idl * idl;
  st.uys = dl * T(0.5);
  st.uyw = T(0);
  st.usw = T(0);
  st.dy = c.sy2 * T(0.5);
  st.ds = (c.sy2 + c.sy2) * idl2;
  st.dw = c.cww0;
  st.uzt = dl * T(0.5);
  st.dz = c.sz2 * T(0.5);
  st.dt = (c.sz2 + c.sz2) * idl2;
}

// A diagonal covariance diag(vy, vz, vs, vt, vw).
template <class T>
void diagonal_covariance(State<T>& st, T vy, T vz, T vs, T vt, T vw) {
  st.uys = T(0);
  st.uyw = T(0);
  st.usw = T(0);
  st.dy = vy;
  st.ds = vs;
  st.dw = vw;
  st.uzt = T(0);
  st.dz = vz;
  st.dt = vt;
}


}  // namespace orc
