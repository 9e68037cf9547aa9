// TEST INFRASTRUCTURE ONLY -- the checking implementation ("oracle") of the
// track merging.
//
// The paper (Section 2, track merging) merges the track segments found by the
// sector tracking first inside a sector, then between adjacent sectors of one
// TPC half, then across the central electrode.  It names no matching
// criterion.  This build's reading:
//
//   views    every track's state (y, z, sin(phi), dz/ds, q/pT at the plane of
//            its innermost cluster, in its sector's frame) is carried to the
//            plane x = x_m (a fixed radius between the pad rows) in three
//            frames: its own (view 0), the frame of the boundary with the
//            next sector of its half (its x axis on the boundary line, the
//            state rotated by -h, h = half the sector opening; view 1) and the
//            frame of the boundary with the previous sector (rotated by +h;
//            view 2).  The rotation turns (x, y) about the beam axis and adds
//            the angle to phi; the carrying is the tracking's own circle step.
//            A view is missing when |sin(phi)|, before or after the rotation,
//            or a step hits the propagation guards.
//   pairs    a (inner) and b (outer) may merge when a's outermost row is below
//            b's innermost one and they are in the same unit (views 0, 0),
//            in the units of the same azimuth on the two sides of the central
//            electrode (views 0, 0; when enabled), or in adjacent sectors
//            (a's view 1 against b's view 2 when b's sector is a's next one,
//            a's view 2 against b's view 1 when it is the previous one).
//   chi2     sum over the five parameters of (difference / tolerance)^2, in
//            that order, IEEE binary32 (the decisions' precision);
//            candidates with chi2 <= cut.
//   links    a's outer partner is its candidate with the smallest (chi2,
//            index); b's inner partner likewise; a and b are linked when each
//            is the other's choice.  Linked tracks form chains (rows strictly
//            increase along a chain, so there are no cycles); root = the
//            chain's innermost track.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

#include "kalman.h"

extern "C" {
struct OrcMergeParams {
  float x_m;                 // plane of the views [cm]
  float cos_h, sin_h;        // cos and sin of half the sector opening (rounded once)
  float tol[5];              // tolerances of y, z, sin(phi), dz/ds, q/pT
  float chi2_cut;
  int32_t cross_electrode;   // 1: merge across the central electrode
};
}

namespace {

using namespace orc;

// View v of a track: 5 numbers, or false when missing.
template <class T>
bool merge_view(const float* prm, float x_ref, int v, const OrcMergeParams& mp, const Consts<T>& c, T out[5]) {
  State<T> st{};
  st.x = T(x_ref);
  st.y = T(prm[0]);
  st.z = T(prm[1]);
  st.s = T(prm[2]);
  st.t = T(prm[3]);
  st.w = T(prm[4]);
  {
    using std::fabs;
    if (!(fabs(st.s) < c.smax)) return false;
  }
  if (v != 0) {
    using std::sqrt;
    using std::fabs;
    const T ch = T(mp.cos_h);
    const T sh = v == 1 ? -T(mp.sin_h) : T(mp.sin_h);
    const T cphi = sqrt(T(1) - st.s * st.s);
    const T x1 = st.x * ch - st.y * sh;
    const T y1 = st.x * sh + st.y * ch;
    const T s1 = st.s * ch + cphi * sh;
    st.x = x1;
    st.y = y1;
    st.s = s1;
    if (!(fabs(st.s) < c.smax)) return false;
  }
  // carried in equal steps of at most 10 cm (the arc-length series of one
  // step is good for short chords only)
  const T x0 = st.x, xm = T(mp.x_m);
  if (!(x0 == xm)) {
    using std::fabs;
    using std::ceil;
    const int n = int(ceil(fabs(xm - x0) * T(0.1)));
    const T dxs = (xm - x0) / T(n);
    for (int k = 1; k < n; ++k)
      if (!propagate(st, x0 + T(k) * dxs, c)) return false;
    if (!propagate(st, xm, c)) return false;
  }
  out[0] = st.y;
  out[1] = st.z;
  out[2] = st.s;
  out[3] = st.t;
  out[4] = st.w;
  return true;
}

template <class T>
T merge_chi2(const T* a, const T* b, const T* itol2) {
  T c2 = T(0);
  for (int i = 0; i < 5; ++i) {
    const T d = a[i] - b[i];
    c2 = c2 + (d * d) * itol2[i];
  }
  return c2;
}

}  // namespace

extern "C" {

// Views of every track in FP64 (pins) or FP32: views[t][v][5], ok[t][v].
int orc_merge_views(const OrcParams* p, const OrcMergeParams* mp, int precision, int64_t n_tracks,
                    const float* param, const float* x_ref, double* views, uint8_t* ok) {
  for (int64_t t = 0; t < n_tracks; ++t) {
    for (int v = 0; v < 3; ++v) {
      bool good;
      double* o = views + (t * 3 + v) * 5;
      if (precision == 64) {
        const Consts<double> c = make_consts<double>(*p);
        good = merge_view<double>(param + 5 * t, x_ref[t], v, *mp, c, o);
      } else {
        const Consts<float> c = make_consts<float>(*p);
        float f[5];
        good = merge_view<float>(param + 5 * t, x_ref[t], v, *mp, c, f);
        for (int i = 0; i < 5; ++i) o[i] = good ? double(f[i]) : 0.0;
      }
      if (!good)
        for (int i = 0; i < 5; ++i) o[i] = 0.0;
      ok[t * 3 + v] = good ? 1 : 0;
    }
  }
  return 0;
}

// Track merging (FP32 decisions).  Tracks in unit order; unit_nbr[u][3] =
// (next sector's unit, previous sector's unit, the unit across the central
// electrode), -1 where there is none.  Outputs prev/next (-1: none) and root.
int orc_merge(const OrcParams* p, const OrcMergeParams* mp, int64_t n_tracks, int32_t n_units,
              const int32_t* unit, const float* param, const float* x_ref, const int32_t* r_in,
              const int32_t* r_out, const int32_t* unit_nbr, int32_t* prev, int32_t* next, int32_t* root) {
  const Consts<float> c = make_consts<float>(*p);
  std::vector<float> view(size_t(n_tracks) * 15, 0.0f);
  std::vector<uint8_t> ok(size_t(n_tracks) * 3, 0);
  for (int64_t t = 0; t < n_tracks; ++t)
    for (int v = 0; v < 3; ++v)
      ok[t * 3 + v] = merge_view<float>(param + 5 * t, x_ref[t], v, *mp, c, &view[(t * 3 + v) * 5]) ? 1 : 0;
  // the tracks of every unit
  std::vector<int64_t> ub(size_t(n_units) + 1, 0);
  for (int64_t t = 0; t < n_tracks; ++t) ub[unit[t] + 1]++;
  for (int u = 0; u < n_units; ++u) ub[u + 1] += ub[u];
  float itol2[5];
  for (int i = 0; i < 5; ++i) itol2[i] = 1.0f / (mp->tol[i] * mp->tol[i]);
  std::vector<float> out_c(n_tracks, 0.0f), in_c(n_tracks, 0.0f);
  std::vector<int32_t> out_b(n_tracks, -1), in_b(n_tracks, -1);
  auto better = [](float c2, int32_t j, float bc, int32_t bj) { return bj < 0 || c2 < bc || (c2 == bc && j < bj); };
  for (int64_t a = 0; a < n_tracks; ++a) {
    const int ua = unit[a];
    // (partner unit, view of a, view of b)
    int rel[4][3] = {{ua, 0, 0}, {unit_nbr[3 * ua + 2], 0, 0}, {unit_nbr[3 * ua + 0], 1, 2}, {unit_nbr[3 * ua + 1], 2, 1}};
    if (!mp->cross_electrode) rel[1][0] = -1;
    for (int k = 0; k < 4; ++k) {
      const int ub2 = rel[k][0], va = rel[k][1], vb = rel[k][2];
      if (ub2 < 0 || !ok[a * 3 + va]) continue;
      for (int64_t b = ub[ub2]; b < ub[ub2 + 1]; ++b) {
        if (b == a || !ok[b * 3 + vb] || !(r_out[a] < r_in[b])) continue;
        const float c2 = merge_chi2<float>(&view[(a * 3 + va) * 5], &view[(b * 3 + vb) * 5], itol2);
        if (!(c2 <= mp->chi2_cut)) continue;
        if (better(c2, int32_t(b), out_c[a], out_b[a])) {
          out_c[a] = c2;
          out_b[a] = int32_t(b);
        }
        if (better(c2, int32_t(a), in_c[b], in_b[b])) {
          in_c[b] = c2;
          in_b[b] = int32_t(a);
        }
      }
    }
  }
  for (int64_t t = 0; t < n_tracks; ++t) {
    next[t] = (out_b[t] >= 0 && in_b[out_b[t]] == int32_t(t)) ? out_b[t] : -1;
    prev[t] = (in_b[t] >= 0 && out_b[in_b[t]] == int32_t(t)) ? in_b[t] : -1;
  }
  for (int64_t t = 0; t < n_tracks; ++t) {
    int32_t r = int32_t(t);
    while (prev[r] >= 0) r = prev[r];
    root[t] = r;
  }
  return 0;
}

}  // extern "C"
