// Ambiguity solving after the sector tracking (paper, Section 2: tracks are
// found several times; the best instance of each track keeps the clusters,
// the clones are removed, and a configurable fraction of a track's clusters
// may be shared; Section 3, Phase I: among tracks competing for a cluster
// the smaller global chi2 has priority, the track length weighing less, and
// shared clusters are counted from the outermost pad row).
//
// Rank of a tracklet: smaller q = chi2/ndf (IEEE binary32 quotient), then
// more clusters, then earlier in its unit (start-hit order), packed into one
// 64-bit key, larger = better:
//   bits 63..32  ~bits(q)   (q >= 0: the bit pattern orders like the value)
//   bits 31..24  n          (at most 255 clusters)
//   bits 23..0   2^24 - 1 - index in the unit
// so an atomic maximum over the keys of the tracklets containing a cluster
// names its owner, whatever the order of the atomics.
//   claim    every tracklet raises owner[c] to its key for each cluster c
//            (in bands of chi2/ndf, best first, each claim only where the
//            owner word is below the tracklet's key);
//   decide   a tracklet is kept when, walking its clusters from the outermost
//            row inwards, after every step k the count s(k) of clusters owned
//            by another tracklet satisfies den s(k) <= num k;
//   reclaim  each kept tracklet replaces owner[c] by its key where the
//            holder is a rejected tracklet or a kept one with a smaller key
//            (compare-and-swap; where a kept tracklet holds the largest key
//            of all, the common case, nothing is written), so owner[c] ends
//            as the largest kept key, or a rejected key when no kept
//            tracklet contains c;
//   assign   each cluster goes to the kept tracklet whose key it holds (-1
//            when none): at once, in the reclaim, where that is the largest
//            key of all claimants; else by a pass over the tracklets that won
//            a swap.
#pragma once

#include "tpcx_common.h"

namespace tpcx {

constexpr int64_t kSelectMaxPerUnit = int64_t(1) << 24;

struct SelectIn {
  int64_t cap_tracks;
  const int64_t* counts;  // tpcx_tracks counts: [1] tracklets, [3] status
  const int32_t* unit;
  const int32_t* n_hits;
  const int64_t* hit_begin;
  const int32_t* hit_id;
  const float* chi2;
  const int32_t* ndf;
};

// Tracklets to consider: none when the tracking overflowed a capacity.
__device__ __forceinline__ int64_t select_count(const SelectIn& in) {
  if ((in.counts[3] & kStOverflow) != 0) return 0;
  return in.counts[1] < in.cap_tracks ? in.counts[1] : in.cap_tracks;
}

__device__ __forceinline__ uint64_t select_key(const SelectIn& in, const int64_t* first, int64_t t) {
  const float q = in.chi2[t] / float(in.ndf[t]);
  const int64_t local = t - first[in.unit[t]];
  const uint32_t lo = uint32_t(min(in.n_hits[t], 255)) << 24 |
                      uint32_t(kSelectMaxPerUnit - 1 - min(local, kSelectMaxPerUnit - 1));
  return uint64_t(~__float_as_uint(q)) << 32 | lo;
}

// first[u] = index of the first tracklet of unit u (tracklets are in unit
// order); status bit 1 when a unit holds more tracklets than the key's
// 24-bit index can order.
__global__ void k_select_first(SelectIn in, int64_t* __restrict__ first, int64_t* __restrict__ status) {
  const int64_t n = select_count(in);
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int32_t u = in.unit[t];
    if (t == 0 || in.unit[t - 1] != u) first[u] = t;
    if (t + 1 == n || in.unit[t + 1] != u) {
      // last of its unit: the unit's count must fit the key
      int64_t lo = 0, hi = t;  // first tracklet of u, by binary search (t is the last)
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (in.unit[mid] < u) lo = mid + 1; else hi = mid;
      }
      if (t - lo + 1 > kSelectMaxPerUnit) atomicOr(reinterpret_cast<unsigned long long*>(status), 1ull);
    }
  }
}

// owner[c] = max over the tracklets containing c of their keys, in passes
// over bands of q = chi2/ndf (best first: q <= 0.5, <= 1, <= 2, the rest;
// the upper 32 key bits are ~bits(q)); a tracklet claims a cluster only
// where owner[c] is below its key (a larger value read stays larger: the
// maximum only grows).  A cluster claimed in an earlier band holds a larger
// key than any of a later one, so the claims of the many clones of a good
// track end as reads.  One lane per tracklet.
constexpr int kClaimPasses = 4;
__device__ __forceinline__ uint32_t claim_band_floor(int pass) {
  // ~bits of 0.5, 1, 2: a key's upper half at least this is in bands 0 .. pass
  return pass == 0 ? ~0x3F000000u : pass == 1 ? ~0x3F800000u : ~0x40000000u;
}

__global__ void k_select_claim(SelectIn in, const int64_t* __restrict__ first, int pass,
                               unsigned long long* __restrict__ owner) {
  const int64_t n = select_count(in);
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x) {
    const unsigned long long key = select_key(in, first, t);
    const uint32_t hi = uint32_t(key >> 32);
    const bool mine = (pass == kClaimPasses - 1 || hi >= claim_band_floor(pass)) &&
                      (pass == 0 || hi < claim_band_floor(pass - 1));
    if (!mine) continue;
    const int64_t b = in.hit_begin[t];
    const int m = in.n_hits[t];
    for (int j = 0; j < m; ++j) {
      unsigned long long* o = owner + in.hit_id[b + j];
      if (__hip_atomic_load(o, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= key) continue;
      atomicMax(o, key);
    }
  }
}

// The holder of owner word `cur` of a cluster of unit u (first[u] its first
// tracklet): the tracklet whose key it is.
__device__ __forceinline__ int64_t select_holder(unsigned long long cur, int64_t first_u, int64_t n) {
  const int64_t t = first_u + (kSelectMaxPerUnit - 1 - int64_t(cur & (kSelectMaxPerUnit - 1)));
  return t < n ? t : n - 1;  // (a unit of more than 2^24 tracklets is reported and its keys collide)
}

// owner[c] = the largest key of the kept tracklets containing c, where one
// does; one lane per kept tracklet.  A kept tracklet that holds the largest
// key of all claimants of c assigns c at once (no other tracklet writes
// that word); one that wins a swap is marked (keep 3) for the assign pass.
__global__ void k_select_reclaim(SelectIn in, const int64_t* __restrict__ first, uint8_t* __restrict__ keep,
                                 unsigned long long* __restrict__ owner, int32_t* __restrict__ assign) {
  const int64_t n = select_count(in);
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x) {
    if (!keep[t]) continue;
    const unsigned long long key = select_key(in, first, t);
    const int64_t fu = first[in.unit[t]];
    const int64_t b = in.hit_begin[t];
    const int m = in.n_hits[t];
    bool swapped = false;
    for (int j = 0; j < m; ++j) {
      const int32_t c = in.hit_id[b + j];
      unsigned long long* o = owner + c;
      unsigned long long cur = __hip_atomic_load(o, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (cur == key) {  // the largest key of all: only this tracklet wrote it
        assign[c] = int32_t(t);
        continue;
      }
      while (true) {
        if (cur > key && keep[select_holder(cur, fu, n)]) break;
        const unsigned long long seen = atomicCAS(o, cur, key);
        if (seen == cur) {
          swapped = true;
          break;
        }
        cur = seen;
      }
    }
    if (swapped) keep[t] = 3;
  }
}

// keep[t] from the outer-first shared count; n_sel[0] += kept tracklets.
__global__ void k_select_decide(SelectIn in, const int64_t* __restrict__ first,
                                const unsigned long long* __restrict__ owner, int32_t num, int32_t den,
                                uint8_t* __restrict__ keep, int64_t* __restrict__ n_sel) {
  const int64_t n = select_count(in);
  int64_t kept = 0;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x) {
    const unsigned long long key = select_key(in, first, t);
    const int64_t b = in.hit_begin[t];
    const int m = in.n_hits[t];
    int64_t shared = 0;
    bool ok = true;
    for (int k = 1; k <= m; ++k) {
      if (owner[in.hit_id[b + m - k]] != key) ++shared;
      if (int64_t(den) * shared > int64_t(num) * k) {
        ok = false;
        break;
      }
    }
    keep[t] = ok ? 1 : 0;
    kept += ok ? 1 : 0;
  }
  // one atomic per wavefront
  for (int d = kWave / 2; d > 0; d >>= 1) kept += __shfl_xor(kept, d, kWave);
  if (lane_id() == 0 && kept) atomicAdd(reinterpret_cast<unsigned long long*>(n_sel),
                                        static_cast<unsigned long long>(kept));
}

// assign[c] = t for every cluster whose owner key is tracklet t's, for the
// tracklets the reclaim marked; their mark is cleared (keep 1).
__global__ void k_select_assign(SelectIn in, const int64_t* __restrict__ first, uint8_t* __restrict__ keep,
                                const unsigned long long* __restrict__ owner, int32_t* __restrict__ assign) {
  const int64_t n = select_count(in);
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x) {
    if (keep[t] != 3) continue;
    keep[t] = 1;
    const unsigned long long key = select_key(in, first, t);
    const int64_t b = in.hit_begin[t];
    const int m = in.n_hits[t];
    for (int j = 0; j < m; ++j) {
      const int32_t c = in.hit_id[b + j];
      if (owner[c] == key) assign[c] = int32_t(t);
    }
  }
}

// keep = 0 for the tracklets beyond the count (whole capacity).
__global__ void k_select_clear(int64_t cap, uint8_t* __restrict__ keep) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < cap;
       t += int64_t(gridDim.x) * blockDim.x)
    keep[t] = 0;
}

}  // namespace tpcx
