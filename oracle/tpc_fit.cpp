// TEST INFRASTRUCTURE ONLY -- the checking implementation ("oracle") of the
// three-iteration track fit with interpolation-based cluster rejection.
//
// The paper (Section 2, track fit) fits every track three times, inwards,
// outwards, inwards: the first iteration gives the later ones good initial
// parameters; the cluster chi2 cut is taken against the interpolation of two
// iterations' states at each pad row (position and covariance stored in
// reduced precision by one iteration, combined with the current one in the
// next), because a chi2 cut inside a single iteration cannot use the whole
// track and is unstable while the uncertainties are large.  Section 3
// (Phase I) moves the interpolation one iteration earlier: the first, inward
// iteration stores the position and covariance, the second, outward
// iteration interpolates and takes the chi2 cut, and the rejection is applied
// in the third.  This build's reading, per track (clusters sorted by row,
// innermost first, at least 3):
//
//   origin    y and z of the state are relative to the outermost cluster.
//   iter 1    (inwards) start from the tracking result at x_ref, propagated
//             without updates through the clusters' planes to the outermost
//             one; there y, z are replaced by that cluster's, the covariance
//             by diag(sy^2, sz^2, vs, vt, vw).  At every further cluster
//             (outer to inner): propagate, store the predicted residual
//             (y - m_y, z - m_z) and predicted variances (C_yy, C_zz) as
//             bfloat16 (round to nearest even), update.
//   iter 2    (outwards) start at the innermost cluster: y, z of the cluster,
//             sin(phi), dz/ds, q/pT of iteration 1's final state, the same
//             diagonal covariance.  At every cluster: the outward prediction
//             (none at the innermost) is combined with the stored inward one
//             (none at the outermost) by inverse-variance weighting per
//             coordinate, r = -(d_in C_out + d_out C_in) / (C_in + C_out),
//             C = C_in C_out / (C_in + C_out); chi2 = r_y^2/(C_y + sy^2) +
//             r_z^2/(C_z + sz^2); the cluster is rejected when chi2 >
//             chi2_cut; then the update with the cluster (all clusters).
//   iter 3    (inwards) from iteration 2's final state, propagated back to
//             the outermost kept cluster, whose y, z it takes, diagonal
//             covariance; then every further kept cluster: propagate,
//             update, chi2 += cluster chi2.  Result: the state after the last
//             update (the innermost kept cluster), chi2, ndf = 2 n_kept - 5.
//   fails     when a propagation guard stops a step or fewer than 3 clusters
//             are kept; a failed fit rejects no cluster.
//
// One template for float (decisions) and double (reference); replay mode
// takes the rejection flags as given and runs iteration 3 only.
#include <algorithm>
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

// bfloat16 storage: round a float to its 16 high bits (nearest, ties to even).
float to_bf16(float v) {
  uint32_t b;
  std::memcpy(&b, &v, 4);
  b = (b + 0x7FFFu + ((b >> 16) & 1u)) & 0xFFFF0000u;
  float r;
  std::memcpy(&r, &b, 4);
  return r;
}
double to_bf16(double v) { return double(to_bf16(float(v))); }

struct FitParams {
  float chi2_cut;  // interpolation chi2 cut (2 degrees of freedom)
  float vs, vt, vw;  // seed variances of sin(phi), dz/ds, q/pT
};

template <class T>
struct FitOut {
  State<T> st;
  T chi2;
  int n_kept;
  bool ok;
};

template <class T>
void reset_cov(State<T>& st, const Consts<T>& c, const FitParams& f) {
  diagonal_covariance(st, c.sy2, c.sz2, T(f.vs), T(f.vt), T(f.vw));
}

// Propagate through the planes xs[from .. to] (inclusive, in that order).
template <class T>
bool walk(State<T>& st, const T* xs, int from, int to, const Consts<T>& c) {
  const int step = to >= from ? 1 : -1;
  for (int i = from;; i += step) {
    if (!(st.x == xs[i]) && !propagate(st, xs[i], c)) return false;
    if (i == to) break;
  }
  return true;
}

// The fit of one track.  x, my, mz: clusters innermost first (my, mz absolute);
// seed: tracking result (y, z, s, t, w) at x_ref.  decide: iteration 2 writes
// the rejection flags; otherwise they are read (the FP64 replay of given
// decisions).
template <class T>
FitOut<T> fit_track(int n, const T* x, const float* my, const float* mz, T x_ref, const float* seed,
                    const Consts<T>& c, const FitParams& f, uint8_t* reject, bool decide) {
  FitOut<T> out{};
  out.ok = false;
  if (n < 3) return out;
  const T oy = T(my[n - 1]), oz = T(mz[n - 1]);
  std::vector<T> ry(n), rz(n);
  for (int i = 0; i < n; ++i) {
    ry[i] = T(my[i]) - oy;
    rz[i] = T(mz[i]) - oz;
  }
  // iteration 1: inwards, storing the predictions
  State<T> st{};
  st.x = x_ref;
  st.y = T(seed[0]) - oy;
  st.z = T(seed[1]) - oz;
  st.s = T(seed[2]);
  st.t = T(seed[3]);
  st.w = T(seed[4]);
  reset_cov(st, c, f);
  int first = 0;  // from x_ref outwards through the planes beyond it
  while (first < n && !(x[first] > x_ref)) ++first;
  if (first < n && !walk(st, x, first, n - 1, c)) return out;
  if (!(st.x == x[n - 1]) && !propagate(st, x[n - 1], c)) return out;
  st.y = ry[n - 1];
  st.z = rz[n - 1];
  reset_cov(st, c, f);
  std::vector<T> din(n), ein(n), cin(n), kin(n);
  for (int i = n - 2; i >= 0; --i) {
    if (!propagate(st, x[i], c)) return out;
    const Cov9<T> cv = covariance(st);
    din[i] = to_bf16(st.y - ry[i]);
    ein[i] = to_bf16(st.z - rz[i]);
    cin[i] = to_bf16(cv.cyy);
    kin[i] = to_bf16(cv.czz);
    update(st, ry[i], rz[i], c);
  }
  // iteration 2: outwards, interpolation and chi2 cut
  const T s1 = st.s, t1 = st.t, w1 = st.w;
  st = State<T>{};
  st.x = x[0];
  st.y = ry[0];
  st.z = rz[0];
  st.s = s1;
  st.t = t1;
  st.w = w1;
  reset_cov(st, c, f);
  for (int i = 0; i < n; ++i) {
    T dy, dz, vy, vz;  // interpolated residual (prediction - cluster) and variance
    if (i > 0 && !propagate(st, x[i], c)) return out;
    if (i == 0) {
      dy = din[0];
      dz = ein[0];
      vy = cin[0];
      vz = kin[0];
    } else {
      const Cov9<T> cv = covariance(st);
      const T dout = st.y - ry[i], eout = st.z - rz[i];
      if (i == n - 1) {
        dy = dout;
        dz = eout;
        vy = cv.cyy;
        vz = cv.czz;
      } else {
        const T iy = T(1) / (cin[i] + cv.cyy);
        const T iz = T(1) / (kin[i] + cv.czz);
        dy = (din[i] * cv.cyy + dout * cin[i]) * iy;
        dz = (ein[i] * cv.czz + eout * kin[i]) * iz;
        vy = (cin[i] * cv.cyy) * iy;
        vz = (kin[i] * cv.czz) * iz;
      }
    }
    if (decide) {
      const T chi2 = (dy * dy) / (vy + c.sy2) + (dz * dz) / (vz + c.sz2);
      reject[i] = chi2 > T(f.chi2_cut) ? 1 : 0;
    }
    if (i > 0) update(st, ry[i], rz[i], c);
  }
  // iteration 3: inwards over the kept clusters, from iteration 2's state
  int j = n - 1;
  while (j >= 0 && reject[j]) --j;
  if (j < 2) return out;
  for (int i = n - 2; i >= j; --i)
    if (!propagate(st, x[i], c)) return out;
  st.y = ry[j];
  st.z = rz[j];
  reset_cov(st, c, f);
  T chi2 = T(0);
  int kept = 1;
  State<T> last = st;
  for (int i = j - 1; i >= 0; --i) {
    if (!propagate(st, x[i], c)) return out;
    if (reject[i]) continue;
    chi2 = chi2 + update(st, ry[i], rz[i], c);
    ++kept;
    last = st;
  }
  if (kept < 3) return out;
  last.y = oy + last.y;
  last.z = oz + last.z;
  out.st = last;
  out.chi2 = chi2;
  out.n_kept = kept;
  out.ok = true;
  return out;
}

}  // namespace

extern "C" {

// The fit of n_tracks tracks (hit lists as in the refit: hit_begin
// [n_tracks+1], hit_id, hit_row, innermost first); seed [n][5] and x_ref [n]
// from the tracking.  precision 32 takes the rejection decisions (written to
// reject[hits]); precision 64 with decide = 0 replays given decisions.
// Writes param [n][5] (y, z absolute) at x_out [n], cov [n][15], chi2 [n],
// n_kept [n] and ok [n].
void orc_fit(int precision, int decide, const float* row_x, const OrcParams* p, float chi2_cut,
             float vs, float vt, float vw, int64_t n_tracks, const int64_t* hit_begin,
             const int32_t* hit_id, const uint8_t* hit_row, const float* seed, const float* x_ref,
             const float* y, const float* z, uint8_t* reject, double* param, double* cov,
             double* chi2, double* x_out, int32_t* n_kept, int32_t* ok) {
  const FitParams f{chi2_cut, vs, vt, vw};
  auto go = [&](auto tag) {
    using T = decltype(tag);
    const Consts<T> c = make_consts<T>(*p);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t t = 0; t < n_tracks; ++t) {
      const int64_t b = hit_begin[t];
      const int n = int(hit_begin[t + 1] - b);
      std::vector<T> xs(n);
      std::vector<float> my(n), mz(n);
      for (int i = 0; i < n; ++i) {
        xs[i] = T(row_x[hit_row[b + i]]);
        my[i] = y[hit_id[b + i]];
        mz[i] = z[hit_id[b + i]];
      }
      const FitOut<T> o = fit_track<T>(n, xs.data(), my.data(), mz.data(), T(x_ref[t]), seed + 5 * t, c, f,
                                       reject + b, decide != 0);
      ok[t] = o.ok ? 1 : 0;
      if (!o.ok && decide) std::memset(reject + b, 0, size_t(n));  // a failed fit rejects nothing
      n_kept[t] = o.ok ? o.n_kept : 0;
      chi2[t] = o.ok ? double(o.chi2) : 0.0;
      x_out[t] = o.ok ? double(o.st.x) : 0.0;
      const double pv[5] = {double(o.st.y), double(o.st.z), double(o.st.s), double(o.st.t), double(o.st.w)};
      const Cov9<T> cv = covariance(o.st);
      const double cvv[15] = {double(cv.cyy), 0.0, double(cv.czz), double(cv.csy), 0.0, double(cv.css),
                              0.0, double(cv.ctz), 0.0, double(cv.ctt), double(cv.cwy), 0.0,
                              double(cv.cws), 0.0, double(cv.cww)};
      for (int k = 0; k < 5; ++k) param[5 * t + k] = o.ok ? pv[k] : 0.0;
      for (int k = 0; k < 15; ++k) cov[15 * t + k] = o.ok ? cvv[k] : 0.0;
    }
  };
  if (precision == 64)
    go(0.0);
  else
    go(0.0f);
}

}  // extern "C"
