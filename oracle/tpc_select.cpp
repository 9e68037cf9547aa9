// TEST INFRASTRUCTURE ONLY -- the checking implementation ("oracle") of the
// ambiguity solving that follows the sector tracking.
//
// The paper (Section 2) states what the step does: tracks are found several
// times, so it identifies the best instance of each track, assigns the
// clusters to it and removes the clones, while a configurable fraction of a
// track's clusters (10% by default; 20% after the loosening described in
// Section 2) may be shared with other tracks.  Section 3 (Phase I) fixes the
// competition and the counting: among tracks competing for a cluster the one
// with the smaller global chi2 has priority, the track length weighing less;
// shared clusters are counted starting from the outermost pad row.  The
// definition below is this build's reading of those statements:
//
//   priority  q = chi2 / ndf (IEEE binary32 quotient of the tracklet's float
//             chi2 and ndf); a tracklet ranks above another when its q is
//             smaller, then when it has more clusters, then when it comes
//             first in its unit (start-hit order).
//   owner     every cluster belongs to the highest-ranked tracklet that
//             contains it.
//   select    a tracklet is kept when, walking its clusters from the
//             outermost row inwards, after every step k the number s(k) of
//             clusters seen so far that belong to another tracklet satisfies
//             s(k) <= f k, with f = num / den (compared in integers:
//             den s(k) <= num k).  Otherwise it is a clone (or a fragment
//             whose outer clusters belong to a better track) and is removed.
//   assign    every cluster is assigned to the highest-ranked kept tracklet
//             that contains it (-1 when none does).
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// true when tracklet a ranks above tracklet b
bool ranks_above(float qa, int na, int64_t ia, float qb, int nb, int64_t ib) {
  if (qa != qb) return qa < qb;
  if (na != nb) return na > nb;
  return ia < ib;
}

}  // namespace

extern "C" {

// Tracklets t = 0 .. n_tracks-1 (kept tracking output, in start-hit order,
// units contiguous): unit[t], n[t] clusters hit_id[hit_begin[t] ..] sorted by
// row (innermost first), chi2[t], ndf[t].  n_clusters bounds the cluster ids.
// Writes keep[t] (1: selected) and assign[c] for every cluster c; returns the
// number of selected tracklets.
int64_t orc_select(int64_t n_tracks, const int32_t* unit, const int32_t* n, const int64_t* hit_begin,
                   const int32_t* hit_id, const float* chi2, const int32_t* ndf, int64_t n_clusters,
                   int32_t shared_num, int32_t shared_den, uint8_t* keep, int32_t* assign) {
  std::vector<float> q(n_tracks);
  std::vector<int64_t> local(n_tracks);
  for (int64_t t = 0; t < n_tracks; ++t) {
    q[t] = chi2[t] / float(ndf[t]);
    local[t] = (t > 0 && unit[t] == unit[t - 1]) ? local[t - 1] + 1 : 0;
  }
  auto above = [&](int64_t a, int64_t b) {
    return ranks_above(q[a], n[a], local[a], q[b], n[b], local[b]);
  };
  // owner of every cluster among all tracklets
  std::vector<int64_t> owner(n_clusters, -1);
  for (int64_t t = 0; t < n_tracks; ++t)
    for (int64_t j = hit_begin[t]; j < hit_begin[t] + n[t]; ++j) {
      const int32_t c = hit_id[j];
      if (owner[c] < 0 || above(t, owner[c])) owner[c] = t;
    }
  // selection: shared clusters counted from the outermost row inwards
  int64_t n_keep = 0;
  for (int64_t t = 0; t < n_tracks; ++t) {
    int64_t seen = 0, shared = 0;
    bool ok = true;
    for (int64_t j = hit_begin[t] + n[t] - 1; j >= hit_begin[t]; --j) {
      ++seen;
      if (owner[hit_id[j]] != t) ++shared;
      if (int64_t(shared_den) * shared > int64_t(shared_num) * seen) {
        ok = false;
        break;
      }
    }
    keep[t] = ok ? 1 : 0;
    n_keep += ok ? 1 : 0;
  }
  // assignment among the selected tracklets
  std::vector<int64_t> best(n_clusters, -1);
  for (int64_t t = 0; t < n_tracks; ++t) {
    if (!keep[t]) continue;
    for (int64_t j = hit_begin[t]; j < hit_begin[t] + n[t]; ++j) {
      const int32_t c = hit_id[j];
      if (best[c] < 0 || above(t, best[c])) best[c] = t;
    }
  }
  for (int64_t c = 0; c < n_clusters; ++c) assign[c] = int32_t(best[c]);
  return n_keep;
}

}  // extern "C"
