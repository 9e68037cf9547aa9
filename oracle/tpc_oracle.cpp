// TEST INFRASTRUCTURE ONLY -- the checking implementation ("oracle") of the
// per-sector TPC track finding.  Only the tests, the smoke check and the CPU
// baseline of the benchmark load it; the GPU library never does.
//
// A plain, slow, deliberately unoptimised CPU implementation of what the
// paper's sector tracking computes (Section 2): a combinatorial seeding based
// on a cellular automaton (neighbour finder over adjacent pad rows, link
// cleaning, start hits), then track following that fits each seed with a
// Kalman filter and picks up further clusters row by row under a chi2 cut.
// Tracks are found several times; all instances are kept (ambiguity solving is
// a later step of the paper's chain, not part of this one).
//
// The paper gives the algorithm in words only; every formula below is the
// reading recorded with this implementation's documentation: an exact circle
// propagation in the bending plane, a block-diagonal covariance, a 2-point
// seed, greedy nearest-chi2 attachment with ties broken by the cluster index.
//
// The code is one template instantiated twice:
//   float  -- every operation in IEEE binary32, round to nearest, no fused
//             multiply-add (compile with -ffp-contract=off), correctly rounded
//             divide and square root.  This precision takes the decisions, as
//             the tracking kernels do (deterministic mode, Section 5).
//   double -- the FP64 reference: runs the same steps, or replays the float
//             decisions, to bound the rounding error of the float results.
//
// Candidate searches come in two forms that must give identical results: a
// brute scan over every cluster of a row, and a scan of a z-sorted index over
// a conservatively widened z window followed by the same exact predicate.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

#include "kalman.h"

namespace {

using namespace orc;

constexpr int kFlagDescentFailed = 1;

// ---------------------------------------------------------------------------
// one unit (sector): rows with their clusters, and a z-sorted index per row
// ---------------------------------------------------------------------------
struct RowIndex {
  std::vector<int64_t> by_z;  // cluster indices sorted by (z, index)
};

struct Unit {
  int n_rows;
  const int64_t* rb;  // rb[r] .. rb[r+1]
  const float* y;
  const float* z;
  std::vector<RowIndex> idx;
  void build() {
    idx.resize(n_rows);
    for (int r = 0; r < n_rows; ++r) {
      auto& v = idx[r].by_z;
      v.clear();
      for (int64_t i = rb[r]; i < rb[r + 1]; ++i) v.push_back(i);
      // (is NaN, z, index): a strict weak order also with NaN coordinates,
      // which go last (they pass no window test)
      std::sort(v.begin(), v.end(), [&](int64_t a, int64_t b) {
        const bool na = std::isnan(z[a]), nb = std::isnan(z[b]);
        if (na != nb) return nb;
        if (na) return a < b;
        return z[a] < z[b] || (z[a] == z[b] && a < b);
      });
    }
  }
  // Calls fn(i) for every cluster of row r whose z lies in [lo, hi] (exact,
  // double) -- a superset of every cluster the caller's exact predicate can
  // accept when the window was widened conservatively.  Brute mode visits the
  // whole row.
  template <class F>
  void scan(int r, bool brute, double lo, double hi, F&& fn) const {
    if (brute) {
      for (int64_t i = rb[r]; i < rb[r + 1]; ++i) fn(i);
      return;
    }
    const auto& v = idx[r].by_z;
    auto it = std::lower_bound(v.begin(), v.end(), lo,
                               [&](int64_t a, double val) { return double(z[a]) < val; });
    for (; it != v.end() && double(z[*it]) <= hi; ++it) fn(*it);
  }
};

// Widening of search windows: every cluster passing an exact predicate
// computed in float or double lies inside the window widened by this much.
constexpr double kPadAbs = 1e-3;   // cm
constexpr double kPadRel = 1e-4;

// ---------------------------------------------------------------------------
// neighbour finder, cleaning, start hits
// ---------------------------------------------------------------------------
template <class T>
void find_neighbours(const Unit& un, const std::vector<T>& xr, bool brute, const Consts<T>& c,
                     int32_t* link_up, int32_t* link_down, int64_t* n_pairs) {
  const int R = un.n_rows;
  for (int r = 0; r < R; ++r)
    for (int64_t h = un.rb[r]; h < un.rb[r + 1]; ++h) link_up[h] = link_down[h] = -1;
  for (int r = 1; r + 1 < R; ++r) {
    // fraction of the way from row r-1 to row r+1 at which row r lies
    T f = (xr[r] - xr[r - 1]) / (xr[r + 1] - xr[r - 1]);
    std::vector<int64_t> U, D;
    for (int64_t h = un.rb[r]; h < un.rb[r + 1]; ++h) {
      T yh = T(un.y[h]), zh = T(un.z[h]);
      U.clear();
      D.clear();
      double lo = double(un.z[h]) - double(c.wz) - kPadAbs, hi = double(un.z[h]) + double(c.wz) + kPadAbs;
      un.scan(r + 1, brute, lo, hi, [&](int64_t u) {
        if (std::fabs(T(un.y[u]) - yh) <= c.wy && std::fabs(T(un.z[u]) - zh) <= c.wz) U.push_back(u);
      });
      un.scan(r - 1, brute, lo, hi, [&](int64_t d) {
        if (std::fabs(T(un.y[d]) - yh) <= c.wy && std::fabs(T(un.z[d]) - zh) <= c.wz) D.push_back(d);
      });
      T bestD = T(0);
      int64_t bu = -1, bd = -1;
      for (int64_t u : U) {
        for (int64_t d : D) {
          T yu = T(un.y[u]), zu = T(un.z[u]), yd = T(un.y[d]), zd = T(un.z[d]);
          T ey = yh - (yd + (yu - yd) * f);
          T ez = zh - (zd + (zu - zd) * f);
          T D2 = ey * ey + ez * ez;
          ++*n_pairs;
          if (!(D2 <= c.d2max)) continue;
          bool better = bu < 0 || D2 < bestD || (D2 == bestD && (u < bu || (u == bu && d < bd)));
          if (better) {
            bestD = D2;
            bu = u;
            bd = d;
          }
        }
      }
      link_up[h] = int32_t(bu);
      link_down[h] = int32_t(bd);
    }
  }
}

// Keep a link only when the linked cluster links back.
void clean_links(int64_t b, int64_t e, const int32_t* up, const int32_t* down, int32_t* cup,
                 int32_t* cdown) {
  for (int64_t h = b; h < e; ++h) {
    int32_t u = up[h], d = down[h];
    cup[h] = (u >= 0 && down[u] == h) ? u : -1;
    cdown[h] = (d >= 0 && up[d] == h) ? d : -1;
  }
}

// ---------------------------------------------------------------------------
// tracklet constructor
// ---------------------------------------------------------------------------
template <class T>
struct Tracklet {
  int64_t start;
  int32_t unit, r0, n, flags, row_ref;
  State<T> st;
  T chi2;
  std::vector<int32_t> hits;  // sorted by row
  std::vector<uint8_t> rows;
  // work counters
  int64_t n_prop = 0, n_search = 0, n_box = 0, n_chain = 0, n_cand = 0;
};

template <class T>
struct Searcher {
  const Unit& un;
  bool brute;
  const Consts<T>& c;
  // margin check (see orc_margins): when set, candidates whose chi2 lies
  // within eps of the cut or of the best one are marked
  uint8_t* margin_flags = nullptr;
  double eps = 0.0;
  double eps_gap = 0.0;  // margin of the best-vs-second chi2 gap
  // Best cluster of row r by (chi2, index) among those with chi2 <= chi2max.
  // n_box counts the clusters scanned; n_cand those inside the chi2 box
  // |dy| <= sqrt(chi2max Sy), |dz| <= sqrt(chi2max Sz), which any
  // implementation must examine (a work measure, not part of the result).
  // The state's y and z are relative to the tracklet's origin (oy, oz).
  int64_t best(const State<T>& st, T oy, T oz, int r, T* chi2_out, int64_t* n_box, int64_t* n_cand) const {
    const Innov<T> iv = innovation(st, c);
    double sz = std::sqrt(double(c.chi2max) * double(iv.sz));
    double sy = std::sqrt(double(c.chi2max) * double(iv.sy));
    double hw = sz * (1.0 + kPadRel) + kPadAbs;
    const double cy = double(oy) + double(st.y), cz = double(oz) + double(st.z);
    double lo = cz - hw, hi = cz + hw;
    int64_t bi = -1, si = -1;
    T bc = T(0), sc = T(0);
    const double mc = eps * std::max(1.0, double(c.chi2max));
    un.scan(r, brute, lo, hi, [&](int64_t i) {
      ++*n_box;
      if (std::fabs(double(un.y[i]) - cy) <= sy && std::fabs(double(un.z[i]) - cz) <= sz)
        ++*n_cand;
      T ch = chi2_of(st, T(un.y[i]) - oy, T(un.z[i]) - oz, c);
      if (margin_flags && std::fabs(double(ch) - double(c.chi2max)) <= mc) margin_flags[i] = 1;
      if (!(ch <= c.chi2max)) return;
      if (bi < 0 || ch < bc || (ch == bc && i < bi)) {
        si = bi;
        sc = bc;
        bi = i;
        bc = ch;
      } else if (si < 0 || ch < sc) {
        si = i;
        sc = ch;
      }
    });
    if (margin_flags && si >= 0 && double(sc) - double(bc) <= eps_gap * std::max(1.0, double(bc)))
      margin_flags[bi] = margin_flags[si] = 1;
    *chi2_out = bc;
    return bi;
  }
};

// Propagate from row `from` down to row `to` (< from) in steps of at most
// `step` rows, with prop(st, x) (a propagation).  False if a step fails.
template <class T, class Prop>
bool descend(State<T>& st, const std::vector<T>& xr, int from, int to, int step, Prop&& prop,
             int64_t* n_prop) {
  for (int rr = from; rr > to;) {
    const int next = std::max(to, rr - step);
    ++*n_prop;
    if (!prop(st, xr[next])) return false;
    rr = next;
  }
  return true;
}

// Whether a propagation of st to x1 evaluates one of its guards within eps of
// the threshold: |sin(phi)| against smax, or the chord's u = |C| dl / 2
// against umax (the same quantities propagate() tests).
template <class T>
bool guard_near(const State<T>& st, T x1, const Consts<T>& c, double eps) {
  const double dx = double(x1) - double(st.x);
  const double k = double(c.kappa) * double(st.w);
  const double s0 = double(st.s), s1 = s0 - k * dx;
  const double smax = double(c.smax), umax = double(c.umax);
  if (std::fabs(std::fabs(s1) - smax) <= eps * std::max(1.0, smax)) return true;
  if (!(std::fabs(s1) < smax)) return false;
  const double c0 = std::sqrt(1.0 - s0 * s0), c1 = std::sqrt(1.0 - s1 * s1);
  const double dy = dx * (s0 + s1) / (c0 + c1);
  const double u = 0.5 * std::fabs(k) * std::sqrt(dx * dx + dy * dy);
  return std::fabs(u - umax) <= eps * std::max(1.0, umax);
}

template <class T>
Tracklet<T> construct(const Unit& un, int unit_id, const std::vector<T>& xr, const int32_t* cup,
                      int64_t h0, int r0, bool brute, const Consts<T>& c, int max_misses,
                      int descent_rows, uint8_t* margin_flags = nullptr, double eps = 0.0,
                      double eps_gap = 0.0) {
  const int R = un.n_rows;
  Tracklet<T> tk;
  tk.start = h0;
  tk.unit = unit_id;
  tk.r0 = r0;
  tk.flags = 0;
  Searcher<T> se{un, brute, c, margin_flags, eps, eps_gap};
  std::vector<std::pair<int, int32_t>> att;  // (row, cluster)

  // with margin_flags set: a propagation guard evaluated within eps of its
  // threshold marks the cluster attached last (it fixed the state)
  auto prop = [&](State<T>& s, T x1) {
    if (margin_flags && !att.empty() && guard_near(s, x1, c, eps)) margin_flags[att.back().second] = 1;
    return propagate(s, x1, c);
  };

  std::vector<int64_t> chain{h0};
  while (cup[chain.back()] >= 0) chain.push_back(cup[chain.back()]);
  tk.n_chain = int64_t(chain.size());

  // 2-point seed at the second chain cluster
  int64_t c0 = chain[0], c1 = chain[1];
  State<T> st;
  T dx = xr[r0 + 1] - xr[r0];
  T dy = T(un.y[c1]) - T(un.y[c0]);
  T dz = T(un.z[c1]) - T(un.z[c0]);
  T dl = std::sqrt(dx * dx + dy * dy);
  T idl = T(1) / dl;
  // y and z of the state are kept relative to the seed cluster c1: their
  // rounding then scales with the distance travelled, not with the absolute
  // coordinate (z reaches thousands of cm in a time frame)
  const T oy = T(un.y[c1]), oz = T(un.z[c1]);
  st.x = xr[r0 + 1];
  st.y = T(0);
  st.z = T(0);
  st.s = dy * idl;
  st.t = dz * idl;
  st.w = T(0);
  seed_covariance(st, dl, idl, c);
  T chi2 = T(0);
  int n = 2;
  att.push_back({r0, int32_t(c0)});
  att.push_back({r0 + 1, int32_t(c1)});
  int row = r0 + 1;

  // the rest of the chain, attached without a cut
  bool up_ok = true;
  for (size_t j = 2; j < chain.size(); ++j) {
    int rr = r0 + int(j);
    ++tk.n_prop;
    if (!prop(st, xr[rr])) {
      up_ok = false;
      break;
    }
    chi2 = chi2 + update(st, T(un.y[chain[j]]) - oy, T(un.z[chain[j]]) - oz, c);
    ++n;
    att.push_back({rr, int32_t(chain[j])});
    row = rr;
  }
  State<T> best = st;
  int best_row = row;

  // following outwards
  if (up_ok) {
    int misses = 0;
    for (int rr = row + 1; rr < R; ++rr) {
      ++tk.n_prop;
      if (!prop(st, xr[rr])) break;
      ++tk.n_search;
      T ch;
      int64_t hi = se.best(st, oy, oz, rr, &ch, &tk.n_box, &tk.n_cand);
      if (hi >= 0) {
        chi2 = chi2 + update(st, T(un.y[hi]) - oy, T(un.z[hi]) - oz, c);
        ++n;
        att.push_back({rr, int32_t(hi)});
        best = st;
        best_row = rr;
        misses = 0;
      } else if (++misses == max_misses) {
        break;
      }
    }
  }

  // back to the start row (no search, steps of at most descent_rows rows),
  // then following inwards
  st = best;
  bool down_ok = descend(st, xr, best_row, r0, descent_rows, prop, &tk.n_prop);
  State<T> out = best;
  int out_row = best_row;
  if (!down_ok) {
    tk.flags |= kFlagDescentFailed;
  } else {
    out = st;
    out_row = r0;
    int misses = 0;
    for (int rr = r0 - 1; rr >= 0; --rr) {
      ++tk.n_prop;
      if (!prop(st, xr[rr])) break;
      ++tk.n_search;
      T ch;
      int64_t hi = se.best(st, oy, oz, rr, &ch, &tk.n_box, &tk.n_cand);
      if (hi >= 0) {
        chi2 = chi2 + update(st, T(un.y[hi]) - oy, T(un.z[hi]) - oz, c);
        ++n;
        att.push_back({rr, int32_t(hi)});
        out = st;
        out_row = rr;
        misses = 0;
      } else if (++misses == max_misses) {
        break;
      }
    }
  }

  std::sort(att.begin(), att.end());
  for (auto& a : att) {
    tk.hits.push_back(a.second);
    tk.rows.push_back(uint8_t(a.first));
  }
  tk.n = n;
  out.y = oy + out.y;
  out.z = oz + out.z;
  tk.st = out;
  tk.row_ref = out_row;
  tk.chi2 = chi2;
  return tk;
}

// Re-run the constructor's arithmetic with the attachment decisions forced:
// hits sorted by row, the start row r0, and whether the descent failed.
// Returns false when a propagation fails where the decisions say it did not.
template <class T>
bool replay(const std::vector<T>& xr, const float* y, const float* z, const int32_t* hits,
            const uint8_t* rows, int n, int r0, int flags, int descent_rows, const Consts<T>& c,
            State<T>* out_st, int* out_row, T* out_chi2, double* out_smax = nullptr) {
  // the largest |sin(phi)| the replayed trajectory reaches (a conditioning
  // measure: near |sin(phi)| = 1 the step's dy/d(sin phi) grows as 1/cos^3)
  double smax = 0.0;
  auto prop = [&](State<T>& s, T x1) {
    const bool ok = propagate(s, x1, c);
    if (ok) smax = std::max(smax, std::fabs(value(s.s)));
    if (out_smax) *out_smax = smax;
    return ok;
  };
  int k0 = -1;  // first hit at or above r0
  for (int i = 0; i < n; ++i)
    if (rows[i] == r0) {
      k0 = i;
      break;
    }
  if (k0 < 0 || k0 + 1 >= n || rows[k0 + 1] != r0 + 1) return false;
  int32_t c0 = hits[k0], c1 = hits[k0 + 1];
  State<T> st;
  T dx = xr[r0 + 1] - xr[r0];
  T dy = T(y[c1]) - T(y[c0]);
  T dz = T(z[c1]) - T(z[c0]);
  T dl = std::sqrt(dx * dx + dy * dy);
  T idl = T(1) / dl;
  const T oy = T(y[c1]), oz = T(z[c1]);
  st.x = xr[r0 + 1];
  st.y = T(0);
  st.z = T(0);
  st.s = dy * idl;
  st.t = dz * idl;
  st.w = T(0);
  seed_covariance(st, dl, idl, c);
  T chi2 = T(0);
  int row = r0 + 1;
  for (int i = k0 + 2; i < n; ++i) {
    for (int rr = row + 1; rr <= rows[i]; ++rr)
      if (!prop(st, xr[rr])) return false;
    chi2 = chi2 + update(st, T(y[hits[i]]) - oy, T(z[hits[i]]) - oz, c);
    row = rows[i];
  }
  State<T> best = st;
  int best_row = row;
  best.y = oy + best.y;
  best.z = oz + best.z;
  if (flags & kFlagDescentFailed) {
    *out_st = best;
    *out_row = best_row;
    *out_chi2 = chi2;
    return k0 == 0;
  }
  int64_t np = 0;
  if (!descend(st, xr, best_row, r0, descent_rows, prop, &np)) return false;
  row = r0;
  State<T> out = st;
  int orow = r0;
  for (int i = k0 - 1; i >= 0; --i) {
    for (int rr = row - 1; rr >= rows[i]; --rr)
      if (!prop(st, xr[rr])) return false;
    chi2 = chi2 + update(st, T(y[hits[i]]) - oy, T(z[hits[i]]) - oz, c);
    row = rows[i];
    out = st;
    orow = row;
  }
  out.y = oy + out.y;
  out.z = oz + out.z;
  *out_st = out;
  *out_row = orow;
  *out_chi2 = chi2;
  return true;
}

// 15 lower-triangle entries (row-major) of the 5x5 covariance of (y,z,s,t,w).
template <class T>
void cov15(const State<T>& st, double* o) {
  const Cov9<T> s = covariance(st);
  const double v[15] = {double(s.cyy), 0.0, double(s.czz), double(s.csy), 0.0, double(s.css),
                        0.0, double(s.ctz), 0.0, double(s.ctt), double(s.cwy), 0.0, double(s.cws),
                        0.0, double(s.cww)};
  std::memcpy(o, v, sizeof v);
}

// ---------------------------------------------------------------------------
// whole-input driver
// ---------------------------------------------------------------------------
struct Result {
  std::vector<int32_t> link_up, link_down, clean_up, clean_down;
  std::vector<int64_t> starts;
  // one entry per start hit
  std::vector<int64_t> t_start, t_hit_begin;
  std::vector<int32_t> t_unit, t_r0, t_n, t_flags, t_row_ref, t_ndf, t_hits;
  std::vector<uint8_t> t_rows;
  std::vector<double> t_param, t_cov, t_chi2, t_xref;
  std::vector<int64_t> counters;  // n_pairs, n_prop, n_search, n_box, n_attached, n_chain, n_cand
};

template <class T>
Result* run(const float* row_x, int n_rows, const OrcParams& p, int n_units,
            const int64_t* row_begin, const float* y, const float* z, int unit_lo, int unit_hi,
            int n_threads, uint8_t* margin_flags = nullptr, double eps = 0.0,
            double eps_gap = 0.0) {
  Consts<T> c = make_consts<T>(p);
  std::vector<T> xr(n_rows);
  for (int r = 0; r < n_rows; ++r) xr[r] = T(row_x[r]);
  const int64_t N = row_begin[int64_t(n_units) * n_rows];
  auto* res = new Result;
  res->link_up.assign(N, -1);
  res->link_down.assign(N, -1);
  res->clean_up.assign(N, -1);
  res->clean_down.assign(N, -1);
  if (unit_lo < 0) unit_lo = 0;
  if (unit_hi > n_units || unit_hi < 0) unit_hi = n_units;
  int nu = std::max(0, unit_hi - unit_lo);
  std::vector<std::vector<int64_t>> starts(nu);
  std::vector<std::vector<Tracklet<T>>> tks(nu);
  std::vector<int64_t> pairs(nu, 0);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int k = 0; k < nu; ++k) {
    int u = unit_lo + k;
    Unit un;
    un.n_rows = n_rows;
    un.rb = row_begin + int64_t(u) * n_rows;
    un.y = y;
    un.z = z;
    un.build();
    find_neighbours<T>(un, xr, p.brute != 0, c, res->link_up.data(), res->link_down.data(), &pairs[k]);
    clean_links(un.rb[0], un.rb[n_rows], res->link_up.data(), res->link_down.data(),
                res->clean_up.data(), res->clean_down.data());
    const int32_t* cup = res->clean_up.data();
    const int32_t* cdn = res->clean_down.data();
    for (int r = 0; r < n_rows; ++r)
      for (int64_t h = un.rb[r]; h < un.rb[r + 1]; ++h) {
        int32_t uu = cup[h];
        if (cdn[h] < 0 && uu >= 0 && cup[uu] >= 0) starts[k].push_back(h);
      }
    for (int64_t h : starts[k]) {
      int r0 = 0;
      while (!(h >= un.rb[r0] && h < un.rb[r0 + 1])) ++r0;
      tks[k].push_back(construct<T>(un, u, xr, cup, h, r0, p.brute != 0, c, p.max_misses, p.descent_rows,
                                    margin_flags, eps, eps_gap));
    }
  }
  int64_t np = 0, nprop = 0, nsearch = 0, nbox = 0, natt = 0, nchain = 0, ncand = 0;
  for (int k = 0; k < nu; ++k) {
    np += pairs[k];
    for (int64_t h : starts[k]) res->starts.push_back(h);
    for (auto& tk : tks[k]) {
      res->t_start.push_back(tk.start);
      res->t_unit.push_back(tk.unit);
      res->t_r0.push_back(tk.r0);
      res->t_n.push_back(tk.n);
      res->t_flags.push_back(tk.flags);
      res->t_row_ref.push_back(tk.row_ref);
      res->t_ndf.push_back(2 * tk.n - 5);
      res->t_hit_begin.push_back(int64_t(res->t_hits.size()));
      for (size_t i = 0; i < tk.hits.size(); ++i) {
        res->t_hits.push_back(tk.hits[i]);
        res->t_rows.push_back(tk.rows[i]);
      }
      const double pv[5] = {double(tk.st.y), double(tk.st.z), double(tk.st.s), double(tk.st.t),
                            double(tk.st.w)};
      res->t_param.insert(res->t_param.end(), pv, pv + 5);
      double cv[15];
      cov15(tk.st, cv);
      res->t_cov.insert(res->t_cov.end(), cv, cv + 15);
      res->t_chi2.push_back(double(tk.chi2));
      res->t_xref.push_back(double(tk.st.x));
      nprop += tk.n_prop;
      nsearch += tk.n_search;
      nbox += tk.n_box;
      natt += tk.n;
      nchain += tk.n_chain;
      ncand += tk.n_cand;
    }
  }
  res->t_hit_begin.push_back(int64_t(res->t_hits.size()));
  res->counters = {np, nprop, nsearch, nbox, natt, nchain, ncand};
  return res;
}

template <class V>
int64_t vlen(const V& v) {
  return int64_t(v.size());
}

// ---------------------------------------------------------------------------
// neighbour-finder predicates near their thresholds (input check for the
// comparison of float and double decisions)
// ---------------------------------------------------------------------------
// Marks h when, evaluated in double, one of its decisions lies within
// eps * max(1, threshold) of going the other way: a window test |dy| <= wy or
// |dz| <= wz against a cluster of rows r +- 1, a pair's D <= d2max, or the gap
// between its smallest and second-smallest accepted D.
int64_t nf_margins_unit(const Unit& un, const std::vector<double>& xr, const OrcParams& p, double eps,
                        uint8_t* flags) {
  const int R = un.n_rows;
  const double wy = p.win_y, wz = p.win_z, d2 = p.d2_max;
  const double mw = eps * std::max(1.0, std::max(wy, wz)), md = eps * std::max(1.0, d2);
  int64_t n = 0;
  for (int r = 1; r + 1 < R; ++r) {
    const double f = (xr[r] - xr[r - 1]) / (xr[r + 1] - xr[r - 1]);
    std::vector<int64_t> U, D;
    for (int64_t h = un.rb[r]; h < un.rb[r + 1]; ++h) {
      const double yh = un.y[h], zh = un.z[h];
      bool near = false;
      U.clear();
      D.clear();
      const double lo = zh - wz - kPadAbs - mw, hi = zh + wz + kPadAbs + mw;
      auto window = [&](int64_t c, std::vector<int64_t>& L) {
        const double dy = std::fabs(double(un.y[c]) - yh), dz = std::fabs(double(un.z[c]) - zh);
        if (dy > wy + mw || dz > wz + mw) return;
        if (std::fabs(dy - wy) <= mw || std::fabs(dz - wz) <= mw) near = true;
        if (dy <= wy && dz <= wz) L.push_back(c);
      };
      un.scan(r + 1, false, lo, hi, [&](int64_t c) { window(c, U); });
      un.scan(r - 1, false, lo, hi, [&](int64_t c) { window(c, D); });
      double b1 = std::numeric_limits<double>::infinity(), b2 = b1;
      for (int64_t u : U)
        for (int64_t d : D) {
          const double yu = un.y[u], zu = un.z[u], yd = un.y[d], zd = un.z[d];
          const double ey = yh - (yd + (yu - yd) * f), ez = zh - (zd + (zu - zd) * f);
          const double v = ey * ey + ez * ez;
          if (std::fabs(v - d2) <= md) near = true;
          if (v > d2) continue;
          if (v < b1) {
            b2 = b1;
            b1 = v;
          } else if (v < b2) {
            b2 = v;
          }
        }
      if (std::isfinite(b2) && b2 - b1 <= eps * std::max(1.0, b1)) near = true;
      if (near) {
        flags[h] = 1;
        ++n;
      }
    }
  }
  return n;
}

}  // namespace

extern "C" {

// precision: 32 (float, decisions) or 64 (double).  Units [unit_lo, unit_hi)
// are processed (-1 for all); links of other units stay -1.
void* orc_track(int precision, const float* row_x, int n_rows, const OrcParams* p, int n_units,
                const int64_t* row_begin, const float* y, const float* z, int unit_lo, int unit_hi,
                int n_threads) {
  if (precision == 64)
    return run<double>(row_x, n_rows, *p, n_units, row_begin, y, z, unit_lo, unit_hi, n_threads);
  return run<float>(row_x, n_rows, *p, n_units, row_begin, y, z, unit_lo, unit_hi, n_threads);
}

// Neighbour-finder decisions within eps of their thresholds, in double:
// flags[h] = 1 for every such cluster (flags has n_clusters entries, zeroed by
// the caller); returns their number.
int64_t orc_nf_margins(const float* row_x, int n_rows, const OrcParams* p, int n_units,
                       const int64_t* row_begin, const float* y, const float* z, double eps,
                       uint8_t* flags) {
  std::vector<double> xr(row_x, row_x + n_rows);
  int64_t total = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
#endif
  for (int u = 0; u < n_units; ++u) {
    Unit un;
    un.n_rows = n_rows;
    un.rb = row_begin + int64_t(u) * n_rows;
    un.y = y;
    un.z = z;
    un.build();
    total += nf_margins_unit(un, xr, *p, eps, flags);
  }
  return total;
}

// The margin check of both stages: orc_nf_margins, then the double-precision
// tracklet constructor, marking every candidate whose chi2 lies within
// eps * max(1, chi2max) of the cut, the best and second-best candidates of a
// search when their chi2 differ by at most eps_gap * max(1, best) (an argmin
// between two clusters is decided on a state that float carries with a
// relative error of up to ~1e-4 after many steps, so its margin is wider than
// that of a fixed threshold), and the cluster
// attached last before a propagation whose sin(phi) or chord guard lies within
// eps * max(1, threshold) of its threshold.  Returns the number of marked
// clusters.
int64_t orc_margins(const float* row_x, int n_rows, const OrcParams* p, int n_units,
                    const int64_t* row_begin, const float* y, const float* z, double eps,
                    double eps_gap, uint8_t* flags) {
  orc_nf_margins(row_x, n_rows, p, n_units, row_begin, y, z, eps, flags);
  delete run<double>(row_x, n_rows, *p, n_units, row_begin, y, z, -1, -1, 0, flags, eps, eps_gap);
  const int64_t N = row_begin[int64_t(n_units) * n_rows];
  int64_t n = 0;
  for (int64_t i = 0; i < N; ++i) n += flags[i] ? 1 : 0;
  return n;
}

void orc_free(void* h) { delete static_cast<Result*>(h); }

// Length (in elements) of a named result array, or -1.
int64_t orc_len(void* h, const char* name) {
  auto* r = static_cast<Result*>(h);
  std::string n(name);
  if (n == "link_up") return vlen(r->link_up);
  if (n == "link_down") return vlen(r->link_down);
  if (n == "clean_up") return vlen(r->clean_up);
  if (n == "clean_down") return vlen(r->clean_down);
  if (n == "starts") return vlen(r->starts);
  if (n == "t_start") return vlen(r->t_start);
  if (n == "t_hit_begin") return vlen(r->t_hit_begin);
  if (n == "t_unit") return vlen(r->t_unit);
  if (n == "t_r0") return vlen(r->t_r0);
  if (n == "t_n") return vlen(r->t_n);
  if (n == "t_flags") return vlen(r->t_flags);
  if (n == "t_row_ref") return vlen(r->t_row_ref);
  if (n == "t_ndf") return vlen(r->t_ndf);
  if (n == "t_hits") return vlen(r->t_hits);
  if (n == "t_rows") return vlen(r->t_rows);
  if (n == "t_param") return vlen(r->t_param);
  if (n == "t_cov") return vlen(r->t_cov);
  if (n == "t_chi2") return vlen(r->t_chi2);
  if (n == "t_xref") return vlen(r->t_xref);
  if (n == "counters") return vlen(r->counters);
  return -1;
}

// Copies a named result array into dst (caller sized it with orc_len).
int orc_get(void* h, const char* name, void* dst) {
  auto* r = static_cast<Result*>(h);
  std::string n(name);
  auto cp = [&](const auto& v) {
    if (!v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
    return 0;
  };
  if (n == "link_up") return cp(r->link_up);
  if (n == "link_down") return cp(r->link_down);
  if (n == "clean_up") return cp(r->clean_up);
  if (n == "clean_down") return cp(r->clean_down);
  if (n == "starts") return cp(r->starts);
  if (n == "t_start") return cp(r->t_start);
  if (n == "t_hit_begin") return cp(r->t_hit_begin);
  if (n == "t_unit") return cp(r->t_unit);
  if (n == "t_r0") return cp(r->t_r0);
  if (n == "t_n") return cp(r->t_n);
  if (n == "t_flags") return cp(r->t_flags);
  if (n == "t_row_ref") return cp(r->t_row_ref);
  if (n == "t_ndf") return cp(r->t_ndf);
  if (n == "t_hits") return cp(r->t_hits);
  if (n == "t_rows") return cp(r->t_rows);
  if (n == "t_param") return cp(r->t_param);
  if (n == "t_cov") return cp(r->t_cov);
  if (n == "t_chi2") return cp(r->t_chi2);
  if (n == "t_xref") return cp(r->t_xref);
  if (n == "counters") return cp(r->counters);
  return -1;
}

// FP64 (or float) replay of given tracklets.  hit_begin has n_tracks+1
// entries into hits/rows.  Writes params [5], cov [15], chi2, x_ref and a
// status (1 ok, 0 a propagation failed) per tracklet.
void orc_replay(int precision, const float* row_x, int n_rows, const OrcParams* p, const float* y,
                const float* z, int64_t n_tracks, const int64_t* hit_begin, const int32_t* hits,
                const uint8_t* rows, const int32_t* r0, const int32_t* flags, double* param,
                double* cov, double* chi2, double* xref, int32_t* ok, double* smax) {
  auto go = [&](auto tag) {
    using T = decltype(tag);
    Consts<T> c = make_consts<T>(*p);
    std::vector<T> xr(n_rows);
    for (int r = 0; r < n_rows; ++r) xr[r] = T(row_x[r]);
    for (int64_t i = 0; i < n_tracks; ++i) {
      State<T> st{};
      int orow = 0;
      T ch = T(0);
      int64_t b = hit_begin[i];
      int n = int(hit_begin[i + 1] - b);
      bool good = replay<T>(xr, y, z, hits + b, rows + b, n, r0[i], flags[i], p->descent_rows, c, &st,
                             &orow, &ch, smax ? smax + i : nullptr);
      ok[i] = good ? 1 : 0;
      const double pv[5] = {double(st.y), double(st.z), double(st.s), double(st.t), double(st.w)};
      std::memcpy(param + 5 * i, pv, sizeof pv);
      cov15(st, cov + 15 * i);
      chi2[i] = double(ch);
      xref[i] = double(st.x);
    }
  };
  if (precision == 64)
    go(0.0);
  else
    go(0.0f);
}

// Single propagation step (for closed-form pins).  state: x,y,z,s,t,w then
// the 9 covariance numbers (yy, sy, ss, wy, ws, ww, zz, tz, tt), factorised on
// entry and multiplied out on exit.  Returns 1 on
// success, 0 when a guard stops it.
int orc_propagate(int precision, const OrcParams* p, double* state, double x1) {
  auto go = [&](auto tag) {
    using T = decltype(tag);
    Consts<T> c = make_consts<T>(*p);
    State<T> st{};
    st.x = T(state[0]);
    st.y = T(state[1]);
    st.z = T(state[2]);
    st.s = T(state[3]);
    st.t = T(state[4]);
    st.w = T(state[5]);
    set_covariance(st, Cov9<T>{T(state[6]), T(state[7]), T(state[8]), T(state[9]), T(state[10]),
                               T(state[11]), T(state[12]), T(state[13]), T(state[14])});
    bool ok = propagate(st, T(x1), c);
    const Cov9<T> cv = covariance(st);
    const double v[15] = {double(st.x), double(st.y), double(st.z), double(st.s), double(st.t),
                          double(st.w), double(cv.cyy), double(cv.csy), double(cv.css),
                          double(cv.cwy), double(cv.cws), double(cv.cww), double(cv.czz),
                          double(cv.ctz), double(cv.ctt)};
    std::memcpy(state, v, sizeof v);
    return ok ? 1 : 0;
  };
  return precision == 64 ? go(0.0) : go(0.0f);
}

// Single Kalman update (for closed-form pins); same state layout.  Returns chi2.
double orc_update(int precision, const OrcParams* p, double* state, double my, double mz) {
  auto go = [&](auto tag) {
    using T = decltype(tag);
    Consts<T> c = make_consts<T>(*p);
    State<T> st{};
    st.x = T(state[0]);
    st.y = T(state[1]);
    st.z = T(state[2]);
    st.s = T(state[3]);
    st.t = T(state[4]);
    st.w = T(state[5]);
    set_covariance(st, Cov9<T>{T(state[6]), T(state[7]), T(state[8]), T(state[9]), T(state[10]),
                               T(state[11]), T(state[12]), T(state[13]), T(state[14])});
    T ch = update(st, T(my), T(mz), c);
    const Cov9<T> cv = covariance(st);
    const double v[15] = {double(st.x), double(st.y), double(st.z), double(st.s), double(st.t),
                          double(st.w), double(cv.cyy), double(cv.csy), double(cv.css),
                          double(cv.cwy), double(cv.cws), double(cv.cww), double(cv.czz),
                          double(cv.ctz), double(cv.ctt)};
    std::memcpy(state, v, sizeof v);
    return double(ch);
  };
  return precision == 64 ? go(0.0) : go(0.0f);
}

}  // extern "C"
