// TEST INFRASTRUCTURE ONLY -- the checking implementation ("oracle") of the
// track rebuild of the fit (Phase II).
//
// The paper (Section 3, Phase II) rebuilds the cluster-to-track attachment
// during iterations 2 and 3 of the fit: instead of a chi2 cut, iteration 2
// queries the sector tracking's cluster search grid for all clusters
// compatible with the chi2 cut against the interpolation and writes every
// candidate with its residual to temporary storage; after iteration 2 of all
// tracks a second ambiguity solving assigns candidates to tracks by rank
// (global chi2 and length), a track that does not get its best candidate
// remaining eligible for its second, and so on; iteration 3 then fits the
// new tracks with a plain chi2 cut (no interpolation).  This build's reading
// (per track of one unit, its clusters innermost first, rows r_in .. r_out):
//
//   iter 1   from the tracking result at x_ref out to the outermost
//            cluster (its y, z; diagonal covariance), then row by row inwards
//            to r_in: at every row store the predicted y, z (binary32,
//            relative to the outermost cluster) and C_yy, C_zz (bfloat16),
//            then update with the track's own cluster of that row, if any.
//   iter 2   restart at the innermost cluster (its y, z; sin(phi), dz/ds,
//            q/pT of iteration 1; diagonal covariance), row by row outwards
//            to r_out: the outward prediction and the stored inward one are
//            combined by inverse-variance weighting (one of them alone at
//            r_in and r_out); every cluster of the row with chi2 against that
//            interpolation <= chi2_cut is a candidate; the K best by (chi2,
//            cluster id) are kept; the state is updated with the best one
//            (not at r_in, where the state already sits on a cluster).
//   assign   ranks as in the ambiguity solving (chi2/ndf, then length, then
//            order in the unit) of the tracking result; R rounds of
//            proposals: every (track, row) proposes its current candidate,
//            each cluster is held by its best-ranked proposer so far, and a
//            (track, row) whose candidate is held by another moves to its
//            next one.  After R rounds a (track, row) gets its candidate if it
//            holds it.  No cluster is shared.
//   iter 3   from iteration 2's final state back to the outermost assigned
//            row (its cluster's y, z; diagonal covariance), then inwards
//            over the assigned rows: a cluster whose filter chi2 exceeds
//            chi2_final is dropped, the others update.  Result at the
//            innermost kept cluster; ndf = 2 n_kept - 5.
//   fails    on a propagation guard or fewer than 3 kept clusters.
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

float bf16(float v) {
  uint32_t b;
  std::memcpy(&b, &v, 4);
  b = (b + 0x7FFFu + ((b >> 16) & 1u)) & 0xFFFF0000u;
  float r;
  std::memcpy(&r, &b, 4);
  return r;
}
double bf16(double v) { return double(bf16(float(v))); }

struct RebuildParams {
  float chi2_cut, chi2_final, vs, vt, vw;
  int k_max, rounds;
  int extrapolate;    // Phase III: candidates also beyond the track's ends
  float chi2_extrap;  // their chi2 cut
};

template <class T>
void diag(State<T>& st, const Consts<T>& c, const RebuildParams& f) {
  diagonal_covariance(st, c.sy2, c.sz2, T(f.vs), T(f.vt), T(f.vw));
}

struct Cand {
  int32_t id;
  float chi2;
};

// Per track: candidates of every row r_lo .. r_hi (r_in .. r_out, extended
// beyond the track's ends by the extrapolation) after iteration 2, and the
// final state of iteration 2 (at r_hi).
template <class T>
struct Pass2 {
  bool ok = false;
  int r_lo = 0, r_hi = 0;
  T oy{}, oz{};
  State<T> st{};
  std::vector<std::vector<Cand>> cand;  // [r_out - r_in + 1]
};

// The candidates of one row against the prediction (iy, iz) with variances
// (vy, vz): chi2 <= cut, the k_max best by (chi2, id).
template <class T>
void row_candidates(std::vector<Cand>& L, int64_t j0, int64_t j1, const float* y, const float* z, T oy, T oz, T iy,
                    T iz, T vy, T vz, const Consts<T>& c, float cut, int k_max) {
  const T sy = vy + c.sy2, sz = vz + c.sz2;
  for (int64_t j = j0; j < j1; ++j) {
    const T dy = (T(y[j]) - oy) - iy, dz = (T(z[j]) - oz) - iz;
    const T ch = (dy * dy) / sy + (dz * dz) / sz;
    if (ch <= T(cut)) L.push_back({int32_t(j), float(ch)});
  }
  std::sort(L.begin(), L.end(), [](const Cand& a, const Cand& b) {
    return a.chi2 < b.chi2 || (a.chi2 == b.chi2 && a.id < b.id);
  });
  if (int(L.size()) > k_max) L.resize(k_max);
}

template <class T>
Pass2<T> pass12(int n, const int32_t* hits, const uint8_t* rows, const float* seed, T x_ref, const T* xr,
                int n_rows, const int64_t* rb, const float* y, const float* z, const Consts<T>& c,
                const RebuildParams& f) {
  Pass2<T> P;
  if (n < 3) return P;
  const int r_in = rows[0], r_out = rows[n - 1];
  std::vector<int32_t> own(n_rows, -1);
  for (int i = 0; i < n; ++i) own[rows[i]] = hits[i];
  P.oy = T(y[hits[n - 1]]);
  P.oz = T(z[hits[n - 1]]);
  const T oy = P.oy, oz = P.oz;
  // iteration 1
  State<T> st{};
  st.x = x_ref;
  st.y = T(seed[0]) - oy;
  st.z = T(seed[1]) - oz;
  st.s = T(seed[2]);
  st.t = T(seed[3]);
  st.w = T(seed[4]);
  diag(st, c, f);
  for (int i = 0; i < n; ++i) {
    const T xi = xr[rows[i]];
    if (xi > x_ref && !(st.x == xi) && !propagate(st, xi, c)) return P;
  }
  if (!(st.x == xr[r_out]) && !propagate(st, xr[r_out], c)) return P;
  st.y = T(0);
  st.z = T(0);
  diag(st, c, f);
  std::vector<T> py(n_rows), pz(n_rows), cy(n_rows), cz(n_rows);
  for (int r = r_out - 1; r >= r_in; --r) {
    if (!propagate(st, xr[r], c)) return P;
    const Cov9<T> cv = covariance(st);
    py[r] = st.y;
    pz[r] = st.z;
    cy[r] = bf16(cv.cyy);
    cz[r] = bf16(cv.czz);
    const int32_t h = own[r];
    if (h >= 0) update(st, T(y[h]) - oy, T(z[h]) - oz, c);
  }
  const T s1 = st.s, t1 = st.t, w1 = st.w;
  // Phase III inwards: the state of r_in carried further in, row by row,
  // without updates, until the first row or a propagation guard
  int r_lo = r_in;
  if (f.extrapolate) {
    State<T> ex = st;
    for (int r = r_in - 1; r >= 0; --r) {
      if (!propagate(ex, xr[r], c)) break;
      const Cov9<T> cv = covariance(ex);
      py[r] = ex.y;
      pz[r] = ex.z;
      cy[r] = bf16(cv.cyy);
      cz[r] = bf16(cv.czz);
      r_lo = r;
    }
  }
  // iteration 2
  st = State<T>{};
  st.x = xr[r_in];
  st.y = T(y[hits[0]]) - oy;
  st.z = T(z[hits[0]]) - oz;
  st.s = s1;
  st.t = t1;
  st.w = w1;
  diag(st, c, f);
  std::vector<std::vector<Cand>> cand(n_rows);
  // rows below the track: the inward extrapolation alone
  for (int r = r_lo; r < r_in; ++r)
    row_candidates(cand[r], rb[r], rb[r + 1], y, z, oy, oz, py[r], pz[r], cy[r], cz[r], c, f.chi2_extrap, f.k_max);
  for (int r = r_in; r <= r_out; ++r) {
    if (r > r_in && !propagate(st, xr[r], c)) return P;
    T iy, iz, vy, vz;
    if (r == r_in) {
      iy = py[r];
      iz = pz[r];
      vy = cy[r];
      vz = cz[r];
    } else {
      const Cov9<T> cv = covariance(st);
      if (r == r_out) {
        iy = st.y;
        iz = st.z;
        vy = cv.cyy;
        vz = cv.czz;
      } else {
        const T wy = T(1) / (cy[r] + cv.cyy);
        const T wz = T(1) / (cz[r] + cv.czz);
        iy = (py[r] * cv.cyy + st.y * cy[r]) * wy;
        iz = (pz[r] * cv.czz + st.z * cz[r]) * wz;
        vy = (cy[r] * cv.cyy) * wy;
        vz = (cz[r] * cv.czz) * wz;
      }
    }
    std::vector<Cand>& L = cand[r];
    row_candidates(L, rb[r], rb[r + 1], y, z, oy, oz, iy, iz, vy, vz, c, f.chi2_cut, f.k_max);
    if (r > r_in && !L.empty()) update(st, T(y[L[0].id]) - oy, T(z[L[0].id]) - oz, c);
  }
  // Phase III outwards: the final state carried further out, without
  // updates, until the last row or a propagation guard
  int r_hi = r_out;
  if (f.extrapolate) {
    for (int r = r_out + 1; r < n_rows; ++r) {
      State<T> nx = st;
      if (!propagate(nx, xr[r], c)) break;
      st = nx;
      const Cov9<T> cv = covariance(st);
      row_candidates(cand[r], rb[r], rb[r + 1], y, z, oy, oz, st.y, st.z, cv.cyy, cv.czz, c, f.chi2_extrap,
                     f.k_max);
      r_hi = r;
    }
  }
  P.r_lo = r_lo;
  P.r_hi = r_hi;
  P.cand.assign(cand.begin() + r_lo, cand.begin() + r_hi + 1);
  P.st = st;
  P.ok = true;
  return P;
}

// 64-bit rank key as in the ambiguity solving: larger ranks higher.
uint64_t rank_key(float chi2, int32_t ndf, int32_t n, int64_t local) {
  const float q = chi2 / float(ndf);
  uint32_t b;
  std::memcpy(&b, &q, 4);
  const int64_t cap = (int64_t(1) << 24) - 1;
  return (uint64_t(~b) << 32) | (uint64_t(std::min(n, 255)) << 24) | uint64_t(cap - std::min(local, cap));
}

}  // namespace

extern "C" {

// The rebuild of n_tracks tracks (unit [n], hit lists innermost first, seed
// [n][5], x_ref [n], chi2 [n] and ndf [n] of the tracking result for the
// rank) against the clusters of their units (row_begin [n_units * n_rows + 1],
// y, z).  Writes assigned [n][n_rows] (the cluster kept at each row after
// iteration 3, -1 for none), param [n][5], cov [n][15], chi2_out [n], x_out
// [n], n_kept [n], ok [n].
void orc_rebuild(int precision, const float* row_x, int n_rows, const OrcParams* p, float chi2_cut,
                 float chi2_final, float vs, float vt, float vw, int32_t k_max, int32_t rounds,
                 int32_t extrapolate, float chi2_extrap, int32_t n_units, int64_t n_tracks, const int32_t* unit, const int64_t* hit_begin,
                 const int32_t* hit_id,
                 const uint8_t* hit_row, const float* seed, const float* x_ref, const float* t_chi2,
                 const int32_t* t_ndf, const int64_t* row_begin, const float* y, const float* z,
                 int32_t* assigned, double* param, double* cov, double* chi2_out, double* x_out,
                 int32_t* n_kept, int32_t* ok) {
  const RebuildParams f{chi2_cut, chi2_final, vs, vt, vw, k_max, rounds, extrapolate, chi2_extrap};
  auto go = [&](auto tag) {
    using T = decltype(tag);
    const Consts<T> c = make_consts<T>(*p);
    std::vector<T> xr(n_rows);
    for (int r = 0; r < n_rows; ++r) xr[r] = T(row_x[r]);
    std::vector<Pass2<T>> P(n_tracks);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t t = 0; t < n_tracks; ++t) {
      const int64_t b = hit_begin[t];
      const int n = int(hit_begin[t + 1] - b);
      P[t] = pass12<T>(n, hit_id + b, hit_row + b, seed + 5 * t, T(x_ref[t]), xr.data(), n_rows,
                       row_begin + int64_t(unit[t]) * n_rows, y, z, c, f);
    }
    // ranks and proposal rounds (a cluster belongs to one unit)
    std::vector<uint64_t> key(n_tracks);
    for (int64_t t = 0, local = 0; t < n_tracks; ++t) {
      local = (t > 0 && unit[t] == unit[t - 1]) ? local + 1 : 0;
      key[t] = rank_key(t_chi2[t], t_ndf[t], int32_t(hit_begin[t + 1] - hit_begin[t]), local);
    }
    std::vector<uint64_t> holder(size_t(row_begin[int64_t(n_units) * n_rows]), 0);
    std::vector<std::vector<int>> ptr(n_tracks);
    for (int64_t t = 0; t < n_tracks; ++t) ptr[t].assign(P[t].cand.size(), 0);
    for (int round = 0; round < f.rounds; ++round) {
      for (int64_t t = 0; t < n_tracks; ++t) {
        if (!P[t].ok) continue;
        for (size_t q = 0; q < P[t].cand.size(); ++q) {
          const int k = ptr[t][q];
          if (k < int(P[t].cand[q].size())) {
            uint64_t& h = holder[P[t].cand[q][k].id];
            h = std::max(h, key[t]);
          }
        }
      }
      for (int64_t t = 0; t < n_tracks; ++t) {
        if (!P[t].ok) continue;
        for (size_t q = 0; q < P[t].cand.size(); ++q) {
          int& k = ptr[t][q];
          if (k < int(P[t].cand[q].size()) && holder[P[t].cand[q][k].id] != key[t]) ++k;
        }
      }
    }
    // iteration 3
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t t = 0; t < n_tracks; ++t) {
      int32_t* as = assigned + t * n_rows;
      for (int r = 0; r < n_rows; ++r) as[r] = -1;
      ok[t] = 0;
      n_kept[t] = 0;
      chi2_out[t] = 0.0;
      x_out[t] = 0.0;
      for (int k = 0; k < 5; ++k) param[5 * t + k] = 0.0;
      for (int k = 0; k < 15; ++k) cov[15 * t + k] = 0.0;
      const Pass2<T>& Q = P[t];
      if (!Q.ok) continue;
      const int nr = Q.r_hi - Q.r_lo + 1;
      std::vector<int32_t> got(nr, -1);
      for (int q = 0; q < nr; ++q) {
        const int k = ptr[t][q];
        if (k < int(Q.cand[q].size()) && holder[Q.cand[q][k].id] == key[t]) got[q] = Q.cand[q][k].id;
      }
      int j = nr - 1;
      while (j >= 0 && got[j] < 0) --j;
      if (j < 2) continue;
      State<T> st = Q.st;
      bool good = true;
      for (int q = nr - 2; q >= j && good; --q) good = propagate(st, xr[Q.r_lo + q], c);
      if (!good) continue;
      st.y = T(y[got[j]]) - Q.oy;
      st.z = T(z[got[j]]) - Q.oz;
      diag(st, c, f);
      std::vector<int32_t> keep(nr, -1);
      keep[j] = got[j];
      T chi2 = T(0);
      int kept = 1;
      State<T> last = st;
      for (int q = j - 1; q >= 0 && good; --q) {
        if (got[q] < 0) continue;
        if (!propagate(st, xr[Q.r_lo + q], c)) {
          good = false;
          break;
        }
        const T my = T(y[got[q]]) - Q.oy, mz = T(z[got[q]]) - Q.oz;
        const T ch = chi2_of(st, my, mz, c);
        if (!(ch <= T(f.chi2_final))) continue;
        chi2 = chi2 + update(st, my, mz, c);
        keep[q] = got[q];
        ++kept;
        last = st;
      }
      if (!good || kept < 3) continue;
      for (int q = 0; q < nr; ++q) as[Q.r_lo + q] = keep[q];
      ok[t] = 1;
      n_kept[t] = kept;
      chi2_out[t] = double(chi2);
      x_out[t] = double(last.x);
      const double pv[5] = {double(Q.oy + last.y), double(Q.oz + last.z), double(last.s), double(last.t),
                            double(last.w)};
      const Cov9<T> cv = covariance(last);
      const double cvv[15] = {double(cv.cyy), 0.0, double(cv.czz), double(cv.csy), 0.0, double(cv.css),
                              0.0, double(cv.ctz), 0.0, double(cv.ctt), double(cv.cwy), 0.0,
                              double(cv.cws), 0.0, double(cv.cww)};
      for (int k = 0; k < 5; ++k) param[5 * t + k] = pv[k];
      for (int k = 0; k < 15; ++k) cov[15 * t + k] = cvv[k];
    }
  };
  if (precision == 64)
    go(0.0);
  else
    go(0.0f);
}

}  // extern "C"
