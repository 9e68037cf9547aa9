// Track following (paper, Section 2): every seed is fitted and propagated
// through the sector with a Kalman filter that picks up the nearest
// compatible cluster row by row.  One lane per start hit; lanes fetch start
// hits from a device work queue, 64 at a time per wavefront, so uneven
// tracklet lengths do not stall whole blocks.
//
// Arithmetic: IEEE binary32, no contraction, correctly rounded divide and
// square root, in exactly the operation order documented for the method, so
// the results match a CPU evaluation bit for bit.
#pragma once

#include "tpcx_common.h"

namespace tpcx {

// State at plane x: (y, z, s = sin(phi), t = dz/ds, w = q/pT) and the
// covariance blocks (y, s, w) and (z, t), each as U D U^T with U unit upper
// triangular and D diagonal:
//   (y, s, w): U = [[1, uys, uyw], [0, 1, usw], [0, 0, 1]], D = diag(dy, ds, dw)
//   (z, t):    U = [[1, uzt], [0, 1]],                      D = diag(dz, dt)
// The transport multiplies U by the unit upper triangular Jacobian; the
// measurement update (Bierman's scalar form) forms no difference of nearly
// equal covariances, which the form C - K H C does in float when the
// predicted variance of y is far above the cluster error.  In the tracklet
// constructor y and z are relative to the seed cluster.
struct KState {
  float x, y, z, s, t, w;
  float uys, uyw, usw, dy, ds, dw;
  float uzt, dz, dt;
};

// asin(u)/u to third order in u^2 (u <= 0.1 keeps the dropped term < 5e-8).
__device__ __forceinline__ float arc_chord_ratio(float u) {
  const float a1 = 0.16666667f;   // 1/6 rounded to float
  const float a2 = 0.075f;        // 3/40 rounded to float
  const float u2 = u * u;
  return 1.0f + u2 * (a1 + u2 * a2);
}

// Square root, reciprocal and quotient: IEEE correctly rounded, or (Fast) the
// hardware approximations (within 1 ulp), used where no decision of the method
// depends on the last bit (the refit).
template <bool Fast>
__device__ __forceinline__ float k_sqrt(float x) {
  if constexpr (Fast) return __builtin_amdgcn_sqrtf(x);
  else return sqrtf(x);
}
template <bool Fast>
__device__ __forceinline__ float k_rcp(float x) {
  if constexpr (Fast) return __builtin_amdgcn_rcpf(x);
  else return 1.0f / x;
}
template <bool Fast>
__device__ __forceinline__ float k_div(float a, float b) {
  if constexpr (Fast) return a * __builtin_amdgcn_rcpf(b);
  else return a / b;
}

// Exact circle step to the plane x1 with the linearised covariance transport.
// Returns false (state unchanged) when |sin(phi)| would reach smax or the
// chord is too long.  (c_prev, r_prev) = (sqrt(1 - s^2), s / that) of the
// current s when `cached` (the previous step ended at this s): the values are
// the ones the step would compute itself, bit for bit.
template <bool Fast = false>
__device__ __forceinline__ bool kf_propagate(KState& q, float x1, const DevParams& p, float& c_prev,
                                             float& r_prev, bool& cached) {
  const float dx = x1 - q.x;
  const float k = p.kappa * q.w;
  const float s1 = q.s - k * dx;
  if (!(fabsf(s1) < p.smax)) return false;
  float c0, r0;
  if (cached) {
    c0 = c_prev;
    r0 = r_prev;
  } else {
    c0 = k_sqrt<Fast>(1.0f - q.s * q.s);
    r0 = k_div<Fast>(q.s, c0);
  }
  const float c1 = k_sqrt<Fast>(1.0f - s1 * s1);
  const float cc = c0 + c1;
  const float ss = q.s + s1;
  const float icc = k_rcp<Fast>(cc);
  const float tg = ss * icc;
  const float dy = dx * tg;
  const float dl = k_sqrt<Fast>(dx * dx + dy * dy);
  const float u = (fabsf(k) * dl) * 0.5f;
  if (!(u <= p.umax)) return false;
  float dS = dl * arc_chord_ratio(u);
  if (dx < 0.0f) dS = -dS;
  const float r1 = k_div<Fast>(s1, c1);
  const float icc2 = icc * icc;
  const float a = dx * ((2.0f * cc + ss * (r0 + r1)) * icc2);
  const float e = -(p.kappa * dx);
  const float b = (dx * e) * ((cc + ss * r1) * icc2);
  // U' = J U with J = [[1, a, b], [0, 1, e], [0, 0, 1]] and [[1, dS], [0, 1]]
  q.uyw = (q.uyw + a * q.usw) + b;
  q.uys = q.uys + a;
  q.usw = q.usw + e;
  q.uzt = q.uzt + dS;
  q.y = q.y + dy;
  q.z = q.z + q.t * dS;
  q.s = s1;
  q.x = x1;
  c_prev = c1;
  r_prev = r1;
  cached = true;
  return true;
}

// Residual variances of a measurement, S_y = C_yy + sy^2 and S_z = C_zz +
// sz^2, as sums of non-negative terms of the factorisation, with the partial
// sums the update needs (v = D U^T h for h selecting y, resp. z).
struct KInnov {
  float v2, v3, a1, a2, sy;
  float vz, z1, sz;
};

__device__ __forceinline__ KInnov kf_innov(const KState& q, const DevParams& p) {
  KInnov n;
  n.v2 = q.ds * q.uys;
  n.v3 = q.dw * q.uyw;
  n.a1 = p.sy2 + q.dy;
  n.a2 = n.a1 + n.v2 * q.uys;
  n.sy = n.a2 + n.v3 * q.uyw;
  n.vz = q.dt * q.uzt;
  n.z1 = p.sz2 + q.dz;
  n.sz = n.z1 + n.vz * q.uzt;
  return n;
}

// Kalman update with the cluster (my, mz) (in the state's coordinates),
// given the partial sums of kf_innov and iSy = 1/S_y, iSz = 1/S_z; returns
// the chi2.  Bierman's scalar update, per block: D' = (dy sy^2/a1, ds a1/a2,
// dw a2/S_y), uys' = uys sy^2/a1, uyw' = uyw sy^2/a2, usw' = usw - v2 uyw/a2,
// gain S_y^-1 (C_yy, C_sy, C_wy) from the prior's first column.
template <bool Fast = false>
__device__ __forceinline__ float kf_update(KState& q, float my, float mz, const KInnov& n, float iSy,
                                           float iSz, const DevParams& p) {
  const float ry = my - q.y;
  const float rz = mz - q.z;
  const float chi2 = (ry * ry) * iSy + (rz * rz) * iSz;
  const float i1 = k_rcp<Fast>(n.a1);
  const float i2 = k_rcp<Fast>(n.a2);
  const float b1 = (q.dy + q.uys * n.v2) + q.uyw * n.v3;
  const float b2 = n.v2 + q.usw * n.v3;
  const float g = ry * iSy;
  q.y = q.y + b1 * g;
  q.s = q.s + b2 * g;
  q.w = q.w + n.v3 * g;
  const float f1 = p.sy2 * i1;
  q.usw = q.usw - n.v2 * (q.uyw * i2);
  q.uyw = q.uyw * (p.sy2 * i2);
  q.uys = q.uys * f1;
  q.dw = q.dw * (n.a2 * iSy);
  q.ds = q.ds * (n.a1 * i2);
  q.dy = q.dy * f1;
  const float j1 = k_rcp<Fast>(n.z1);
  const float bz1 = q.dz + q.uzt * n.vz;
  const float gz = rz * iSz;
  q.z = q.z + bz1 * gz;
  q.t = q.t + n.vz * gz;
  const float fz = p.sz2 * j1;
  q.uzt = q.uzt * fz;
  q.dt = q.dt * (n.z1 * iSz);
  q.dz = q.dz * fz;
  return chi2;
}

// The search box of one lane: z bins zb0..zb1 (taken in pairs), y bins
// yb0..yb1, in the row whose first bin is `base` (ny y bins per z bin).  The
// box |dy| <= 4 sqrt(Sy), |dz| <= 4 sqrt(Sz) around the predicted position
// (cy, cz) is widened so that it holds every cluster the float chi2 cut can
// accept; the hardware square root (within 1 ulp) is enough, the 1e-3
// relative margin covers its error and the rounding of (cy, cz).
struct SearchBox {
  int64_t base;
  int ny, zb0, zb1, yb0, yb1;
};

__device__ __forceinline__ SearchBox kf_box(const RowView& rv, float cy, float cz, const KInnov& n,
                                            const DevParams& p) {
  const float hy = __builtin_amdgcn_sqrtf(p.chi2max * n.sy) * 1.001f + box_pad(cy);
  const float hz = __builtin_amdgcn_sqrtf(p.chi2max * n.sz) * 1.001f + box_pad(cz);
  SearchBox b;
  b.base = rv.base;
  b.ny = rv.ri.ny;
  b.zb0 = rv.zbin(cz - hz);
  b.zb1 = rv.zbin(cz + hz);
  b.yb0 = rv.ybin(cy - hy);
  b.yb1 = rv.ybin(cy + hy);
  return b;
}

// Order-preserving map of a float chi2 to an unsigned key (-0 counts as +0).
__device__ __forceinline__ uint32_t chi2_key(float ch) {
  const uint32_t u = __float_as_uint(ch == 0.0f ? 0.0f : ch);
  return (u >> 31) ? ~u : (u | 0x80000000u);
}

// Best cluster of the search box by (chi2, caller id) among chi2 <= chi2max,
// or -1, for every lane of the wavefront with `searching` set.  The
// candidates of all lanes are spread over all 64 lanes (a lane's own box
// holds 5 candidates on average, the largest box of a wavefront ~17): the
// candidate ranges of one z-bin pair are numbered by a prefix sum over the
// lanes, and lane l evaluates candidates l, l + 64, l + 128, ... of that
// numbering (kSearchSub per round), for their owner lane's state.  A
// candidate's owner is the last lane whose range starts at or before it:
// each lane marks its start in an LDS window of the round's positions and a
// maximum scan over the window carries the marks forward.  The owners' states
// and ranges are read from LDS.  The minimum per owner is an LDS atomic on
// the 64-bit key (chi2, caller id); after each round the lane holding an
// owner's current minimum stores its coordinates.  The result does not
// depend on which lane evaluates which candidate.  Must be called with all
// 64 lanes active.
constexpr int kSearchSub = 2;

struct SearchLds {
  uint64_t best[kWave];
  float2 coord[kWave];
  float4 state[kWave];  // origin and state: oy, qy, oz, qz
  float4 inv[kWave];    // 1/Sy, 1/Sz, second range start (bits)
  int4 range[kWave];    // first candidate number, count, length and start of the first range
  int32_t mark[kSearchSub * kWave];
};

__device__ __forceinline__ int32_t kf_search_wave(const Grid& g, const SearchBox& b, bool searching,
                                                  float oy, float oz, float qy, float qz, float iSy,
                                                  float iSz, float chi2max, SearchLds& L,
                                                  float* out_my, float* out_mz) {
  const int lane = lane_id();
  L.best[lane] = ~0ull;
  L.state[lane] = make_float4(oy, qy, oz, qz);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  for (int zb = b.zb0;; zb += 2) {
    const bool act = searching && zb <= b.zb1;
    if (__ballot(act) == 0ull) break;
    int32_t a0 = 0, alen = 0, b0 = 0, n = 0;
    if (act) {
      const bool z2 = zb + 1 <= b.zb1;
      const int64_t ra = b.base + int64_t(zb) * b.ny;
      const int64_t rb = z2 ? ra + b.ny : ra;
      const int32_t j0 = g.bin_start[ra + b.yb0], j1 = g.bin_start[ra + b.yb1 + 1];
      const int32_t k0 = g.bin_start[rb + b.yb0], k1 = g.bin_start[rb + b.yb1 + 1];
      a0 = j0;
      alen = j1 - j0;
      b0 = k0;
      n = alen + (z2 ? k1 - k0 : 0);
    }
    const int incl = wave_scan_add(n);
    const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
    if (total == 0) continue;
    const int excl = incl - n;
    L.range[lane] = make_int4(excl, n, alen, a0);
    L.inv[lane] = make_float4(iSy, iSz, __int_as_float(b0), 0.0f);
    int carry = -1;  // owner of the position before the round
    for (int t0 = 0; t0 < total; t0 += kSearchSub * kWave) {
#pragma unroll
      for (int j = 0; j < kSearchSub; ++j) L.mark[j * kWave + lane] = -1;
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      const int rel = excl - t0;
      if (n > 0 && rel >= 0 && rel < kSearchSub * kWave) L.mark[rel] = lane;
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      int own[kSearchSub];
      bool ok[kSearchSub];
      float4 m[kSearchSub];
#pragma unroll
      for (int j = 0; j < kSearchSub; ++j) {
        const int o = max(wave_scan_max(L.mark[j * kWave + lane]), carry);
        carry = __builtin_amdgcn_readlane(o, kWave - 1);
        own[j] = o & (kWave - 1);
      }
      // candidate positions (an invalid slot reads position 0, which exists
      // whenever there are candidates), all gathers issued before any use
#pragma unroll
      for (int j = 0; j < kSearchSub; ++j) {
        const int t = t0 + j * kWave + lane;
        const int4 r = L.range[own[j]];
        const int u = t - r.x;
        ok[j] = (t < total) & (u >= 0) & (u < r.y);
        const int pb = __float_as_int(L.inv[own[j]].z) + (u - r.z);
        const int pos = u < r.z ? r.w + u : pb;
        m[j] = g.pts[ok[j] ? pos : 0];
      }
#pragma unroll
      for (int j = 0; j < kSearchSub; ++j) {
        // residuals in the owner's coordinates: (cluster - origin) - state
        const float4 st = L.state[own[j]];
        const float4 iv = L.inv[own[j]];
        const float ry = (m[j].x - st.x) - st.y;
        const float rz = (m[j].y - st.z) - st.w;
        const float ch = (ry * ry) * iv.x + (rz * rz) * iv.y;
        ok[j] = ok[j] && ch <= chi2max;
        const uint64_t k = (uint64_t(chi2_key(ch)) << 32) | uint32_t(__float_as_int(m[j].z));
        if (ok[j]) atomicMin(&L.best[own[j]], (unsigned long long)k);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (ok[j] && __hip_atomic_load(&L.best[own[j]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) == k)
          L.coord[own[j]] = make_float2(m[j].x, m[j].y);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
      }
    }
  }
  const uint64_t key = __hip_atomic_load(&L.best[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  if (!searching || key == ~0ull) return -1;
  const float2 cc = L.coord[lane];
  *out_my = cc.x;
  *out_mz = cc.y;
  return int32_t(uint32_t(key));
}

// Per-start-hit results before compaction.  One 128-byte record per slot:
//   words 0-15  x_ref, y, z, s, t, w, uys, uyw, usw, dy, ds, dw, uzt, dz, dt, chi2 (float;
//               y, z absolute, the covariance factorised as in KState)
//   words 16-19 n, n_up, flags, unit (int)
//   words 20-24 mask of the rows with an attached cluster (rows 0..159)
// and `stride` hit slots with the cluster ids in attachment order: the
// outward phase in ascending rows, then the inward phase in descending rows.
constexpr int kRecWords = 32;
constexpr int kRecN = 16, kRecNUp = 17, kRecFlags = 18, kRecUnit = 19, kRecMask = 20;
constexpr int kMaskWords = 5;

struct TrackletTmp {
  int64_t cap;
  int32_t stride;  // hit slots per record, n_rows rounded up to a multiple of 16
  uint32_t* rec;   // [cap][kRecWords]
  int32_t* hit;    // [cap][stride]
};

constexpr int kFlagDescentFailed = 1;

struct TrackInputs {
  const float4* pts;         // sorted clusters (y, z, caller id, cleaned up-link)
  const int32_t* start_pos;  // sorted position of every start hit
  const int32_t* start_k;    // its unit * n_rows + row
  const int32_t* order;      // slots in sorted-position order (used when all start hits fit)
  const float* row_x;        // [n_rows]
};

// Phases of a tracklet: the chain of the seed (clusters attached without a
// cut), following outwards, the walk back to the start row, following inwards.
enum : int { kChain = 0, kUp = 1, kDescend = 2, kDown = 3, kIdle = 4 };

constexpr int kConstructBlock = 256;

// Every lane runs one tracklet at a time as a sequence of row steps (one
// propagation each); the four phases share the step so that lanes of a
// wavefront in different phases still execute together.  Idle lanes take new
// start hits from the device queue in batches; they take part in the
// wavefront's cluster search, which spreads the candidates of all searching
// lanes over all 64 lanes.  Results depend only on the start hit: the order
// in which lanes pick them up is irrelevant.
// Attached cluster ids are staged per lane in LDS and written 16 at a time
// (one full 64-byte line), the row mask is kept in LDS too; the record is
// written once, as whole lines, when the tracklet ends.
constexpr int kHitBuf = 16;
constexpr int kConstructWaves = kConstructBlock / kWave;

__global__ void __launch_bounds__(kConstructBlock, 4) k_construct(
    const int64_t* __restrict__ counts, int64_t cap_start, int32_t* __restrict__ queue, int refill,
    TrackInputs in, Grid g, DevParams p, TrackletTmp out) {
  __shared__ int32_t hbuf[kConstructWaves][kHitBuf][kWave];
  __shared__ uint32_t rmask[kConstructWaves][kMaskWords][kWave];
  __shared__ SearchLds slds[kConstructWaves];
  const int64_t n_start = counts[0] < cap_start ? counts[0] : cap_start;
  const bool ordered = counts[0] <= cap_start;
  const int R = g.n_rows;
  const int lane = lane_id();
  const int wv = threadIdx.x / kWave;
  int nbuf = 0, nflushed = 0;
  int64_t slot = 0;
  auto flush = [&]() {
    int32_t* dst = out.hit + slot * out.stride + nflushed;
    if (nbuf == kHitBuf) {
#pragma unroll
      for (int j = 0; j < kHitBuf; j += 4)
        *reinterpret_cast<int4*>(dst + j) =
            make_int4(hbuf[wv][j][lane], hbuf[wv][j + 1][lane], hbuf[wv][j + 2][lane], hbuf[wv][j + 3][lane]);
    } else {
      for (int j = 0; j < nbuf; ++j) dst[j] = hbuf[wv][j][lane];
    }
    nflushed += nbuf;
    nbuf = 0;
  };
  KState q{}, best{};
  float oy = 0.0f, oz = 0.0f;  // origin of the state's y and z: the seed cluster
  float c_prev = 0.0f, r_prev = 0.0f, chi2 = 0.0f;
  bool cached = false;
  int kbase = 0, r0 = 0, row = 0, best_row = 0, phase = kIdle, misses = 0, n_up = 0, n_dn = 0,
      flags = 0;
  int32_t next_c = -1;
  int64_t extra_begin = 0, extra_end = 0;
  // wavefront-private pool [pool, pool_end) of start slots, refilled kWave
  // slots at a time from one device queue that hands out the start list in
  // order: the whole GPU works on neighbouring units at a time, which then
  // share the Infinity Cache (faster here than giving each XCD its own part).
  int64_t pool = 0, pool_end = 0;
  bool exhausted = false;
  auto grab = [&](int64_t& lo, int64_t& hi) {
    int32_t base = 0;
    if (lane == 0) base = atomicAdd(queue, kWave);
    base = __builtin_amdgcn_readfirstlane(base);
    lo = min(int64_t(base), n_start);
    hi = min(int64_t(base) + kWave, n_start);
    exhausted = hi >= n_start;
  };

  while (true) {
    // ---- hand start slots to idle lanes
    const uint64_t idle = __ballot(phase == kIdle);
    const int nidle = __popcll(idle);
    if (nidle == kWave && exhausted && pool == pool_end) break;
    if (nidle > 0 && (nidle >= refill || nidle == kWave) && !(exhausted && pool == pool_end)) {
      if (pool_end - pool < nidle && !exhausted) {
        // keep the rest of the pool (consumed first), then a fresh chunk
        int64_t lo, hi;
        grab(lo, hi);
        if (pool == pool_end) {
          pool = lo;
          pool_end = hi;
        } else {
          extra_begin = lo;
          extra_end = hi;
        }
      }
      const int rank = __popcll(idle & lanes_below());
      const int from_pool = int(min(int64_t(nidle), pool_end - pool));
      int64_t sidx = -1;
      if (phase == kIdle) {
        if (rank < from_pool)
          sidx = pool + rank;
        else if (rank - from_pool < extra_end - extra_begin)
          sidx = extra_begin + (rank - from_pool);
      }
      const int from_extra = int(min(int64_t(nidle - from_pool), extra_end - extra_begin));
      pool += from_pool;
      if (pool == pool_end && extra_end > extra_begin) {
        pool = extra_begin + from_extra;
        pool_end = extra_end;
        extra_begin = extra_end = 0;
      }
      if (phase == kIdle) {
        if (sidx >= 0) {
          // 2-point seed at the second cluster of the chain
          slot = ordered ? in.order[sidx] : sidx;
          const float4 P0 = in.pts[in.start_pos[slot]];
          const int kk = in.start_k[slot];
          r0 = kk % R;
          kbase = kk - r0;
          const float4 P1 = in.pts[__float_as_int(P0.w)];
          const int32_t c0 = __float_as_int(P0.z), c1 = __float_as_int(P1.z);
          const float dx = in.row_x[r0 + 1] - in.row_x[r0];
          const float dy = P1.x - P0.x;
          const float dz = P1.y - P0.y;
          const float dl = sqrtf(dx * dx + dy * dy);
          const float idl = 1.0f / dl;
          const float idl2 = idl * idl;
          oy = P1.x;
          oz = P1.y;
          q.x = in.row_x[r0 + 1];
          q.y = 0.0f;
          q.z = 0.0f;
          q.s = dy * idl;
          q.t = dz * idl;
          q.w = 0.0f;
          // C_yy = sy^2, C_sy = sy^2/dl, C_ss = 2 sy^2/dl^2 (z, t alike), var(q/pT) = cww0
          q.uys = dl * 0.5f;
          q.uyw = 0.0f;
          q.usw = 0.0f;
          q.dy = p.sy2 * 0.5f;
          q.ds = (p.sy2 + p.sy2) * idl2;
          q.dw = p.cww0;
          q.uzt = dl * 0.5f;
          q.dz = p.sz2 * 0.5f;
          q.dt = (p.sz2 + p.sz2) * idl2;
          cached = false;
          chi2 = 0.0f;
#pragma unroll
          for (int w = 0; w < kMaskWords; ++w) rmask[wv][w][lane] = 0u;
          hbuf[wv][0][lane] = c0;
          hbuf[wv][1][lane] = c1;
          nbuf = 2;
          nflushed = 0;
          rmask[wv][r0 >> 5][lane] |= 1u << (r0 & 31);
          rmask[wv][(r0 + 1) >> 5][lane] |= 1u << ((r0 + 1) & 31);
          n_up = 2;
          n_dn = 0;
          flags = 0;
          misses = 0;
          row = r0 + 1;
          best = q;
          best_row = row;
          next_c = __float_as_int(P1.w);
          phase = next_c >= 0 ? kChain : kUp;
        }
      }
    }
    // ---- one row step (idle lanes take part in the search only)
    const bool live = phase != kIdle;
    bool finish = false, to_descend = false, attach = false, searching = false;
    int target = 0;
    float iSy = 0.0f, iSz = 0.0f, my = 0.0f, mz = 0.0f;
    KInnov inn{};
    int32_t c = -1, chain_next = -1;
    SearchBox box{0, 1, 0, -1, 0, -1};
    if (live) {
      const bool outward = phase <= kUp;
      target = outward ? row + 1 : (phase == kDescend ? max(r0, row - p.descent_rows) : row - 1);
      bool ok = target >= 0 && target < R;
      // the target row's binning does not depend on the propagation: load it first
      const int trow = min(max(target, 0), R - 1);
      const RowView rv(g, kbase + trow, trow);
      if (ok) ok = kf_propagate(q, in.row_x[target], p, c_prev, r_prev, cached);
      if (phase == kDescend) {
        if (!ok) {
          flags |= kFlagDescentFailed;
          finish = true;
        } else {
          row = target;
          if (row == r0) {
            best = q;
            best_row = row;
            misses = 0;
            phase = kDown;
          }
        }
      } else if (!ok) {
        if (phase == kDown)
          finish = true;
        else
          to_descend = true;
      } else {
        inn = kf_innov(q, p);
        iSy = 1.0f / inn.sy;
        iSz = 1.0f / inn.sz;
        attach = true;
        if (phase == kChain) {
          const float4 P = in.pts[next_c];
          my = P.x;
          mz = P.y;
          c = __float_as_int(P.z);
          chain_next = __float_as_int(P.w);
        } else {
          searching = true;
          box = kf_box(rv, oy + q.y, oz + q.z, inn, p);
        }
      }
    }
    if (__ballot(searching) != 0ull) {
      float sy = 0.0f, sz = 0.0f;
      const int32_t sc = kf_search_wave(g, box, searching, oy, oz, q.y, q.z, iSy, iSz, p.chi2max,
                                        slds[wv], &sy, &sz);
      if (searching) {
        c = sc;
        my = sy;
        mz = sz;
      }
    }
    if (attach) {
      row = target;
      if (c >= 0) {
        chi2 = chi2 + kf_update(q, my - oy, mz - oz, inn, iSy, iSz, p);
        cached = false;
        if (phase == kDown)
          ++n_dn;
        else
          ++n_up;
        hbuf[wv][nbuf][lane] = c;
        rmask[wv][row >> 5][lane] |= 1u << (row & 31);
        if (++nbuf == kHitBuf) flush();
        best = q;
        best_row = row;
        misses = 0;
        if (phase == kChain) {
          next_c = chain_next;
          if (next_c < 0) phase = kUp;
        }
      } else if (++misses == p.max_misses) {
        if (phase == kDown)
          finish = true;
        else
          to_descend = true;
      }
    }
    if (to_descend) {
      q = best;
      row = best_row;
      cached = false;
      phase = kDescend;
    }
    if (finish) {
      flush();
      uint4* rec = reinterpret_cast<uint4*>(out.rec + slot * kRecWords);
      rec[0] = make_uint4(__float_as_uint(best.x), __float_as_uint(oy + best.y),
                          __float_as_uint(oz + best.z), __float_as_uint(best.s));
      rec[1] = make_uint4(__float_as_uint(best.t), __float_as_uint(best.w), __float_as_uint(best.uys),
                          __float_as_uint(best.uyw));
      rec[2] = make_uint4(__float_as_uint(best.usw), __float_as_uint(best.dy),
                          __float_as_uint(best.ds), __float_as_uint(best.dw));
      rec[3] = make_uint4(__float_as_uint(best.uzt), __float_as_uint(best.dz),
                          __float_as_uint(best.dt), __float_as_uint(chi2));
      rec[4] = make_uint4(uint32_t(n_up + n_dn), uint32_t(n_up), uint32_t(flags), uint32_t(kbase / R));
      rec[5] = make_uint4(rmask[wv][0][lane], rmask[wv][1][lane], rmask[wv][2][lane], rmask[wv][3][lane]);
      rec[6] = make_uint4(rmask[wv][4][lane], 0u, 0u, 0u);
      rec[7] = make_uint4(0u, 0u, 0u, 0u);
      phase = kIdle;
    }
  }
}

// ---------------------------------------------------------------------------
// ordered compaction of the kept tracklets (n >= min_hits)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void chunk_of(int64_t n, int64_t* b, int64_t* e) {
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  *b = min(n, per * int64_t(blockIdx.x));
  *e = min(n, *b + per);
}

__global__ void k_keep_count(const int64_t* __restrict__ counts, int64_t cap_start,
                             const uint32_t* __restrict__ rec, int min_hits,
                             int64_t* __restrict__ part) {
  __shared__ int64_t lds[1024 / kWave];
  const int64_t n_start = counts[0] < cap_start ? counts[0] : cap_start;
  int64_t b, e;
  chunk_of(n_start, &b, &e);
  int64_t ct = 0, ch = 0;
  for (int64_t s = b + threadIdx.x; s < e; s += blockDim.x) {
    const int32_t n = int32_t(rec[s * kRecWords + kRecN]);
    if (n >= min_hits) {
      ++ct;
      ch += n;
    }
  }
  int64_t tot_t, tot_h;
  block_exclusive_scan(ct, lds, &tot_t);
  block_exclusive_scan(ch, lds, &tot_h);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = tot_t;
    part[2 * blockIdx.x + 1] = tot_h;
  }
}

// Exclusive scan of the per-block (tracklet, hit) counts, one block of
// kKeepScanThreads threads, each taking a run of consecutive blocks.
constexpr int kKeepScanThreads = 1024;

__global__ void __launch_bounds__(kKeepScanThreads) k_keep_scan(int64_t* __restrict__ part, int nb,
                                                                int64_t* __restrict__ counts,
                                                                int64_t cap_tracks, int64_t cap_hits) {
  __shared__ int64_t lds[kKeepScanThreads / kWave];
  const int per = (nb + kKeepScanThreads - 1) / kKeepScanThreads;
  const int i0 = min(nb, int(threadIdx.x) * per), i1 = min(nb, i0 + per);
  int64_t t = 0, h = 0;
  for (int i = i0; i < i1; ++i) {
    t += part[2 * i];
    h += part[2 * i + 1];
  }
  int64_t tt, th;
  int64_t pt = block_exclusive_scan(t, lds, &tt);
  int64_t ph = block_exclusive_scan(h, lds, &th);
  for (int i = i0; i < i1; ++i) {
    const int64_t a = part[2 * i], c = part[2 * i + 1];
    part[2 * i] = pt;
    part[2 * i + 1] = ph;
    pt += a;
    ph += c;
  }
  if (threadIdx.x == 0) {
    counts[1] = tt;
    counts[2] = th;
    unsigned long long st = 0;
    if (tt > cap_tracks) st |= 2ull;
    if (th > cap_hits) st |= 4ull;
    if (st) atomicOr((unsigned long long*)&counts[3], st);
  }
}

struct TrackOut {
  int64_t cap_tracks, cap_hits;
  int32_t* unit;
  int32_t* start;
  int32_t* n_hits;
  int64_t* hit_begin;
  int32_t* hit_id;
  uint8_t* hit_row;
  float* x_ref;
  float* param;
  float* cov;
  float* chi2;
  int32_t* ndf;
};

// Writes the kept tracklets in start-hit order.  Per tile of 256 slots a
// block scan gives every kept tracklet its output index and hit offset; one
// thread writes each record, then the wavefronts copy the hit lists, one
// tracklet per wavefront at a time, lanes over the hits (coalesced).
constexpr int kKeepBlock = 256;

__global__ void __launch_bounds__(kKeepBlock) k_keep_write(
    const int64_t* __restrict__ counts, int64_t cap_start, const int32_t* __restrict__ starts,
    TrackletTmp tmp, int min_hits, const int64_t* __restrict__ part, TrackOut o) {
  __shared__ int64_t lds[kKeepBlock / kWave];
  __shared__ int64_t s_hb[kKeepBlock];
  __shared__ int32_t s_slot[kKeepBlock];
  __shared__ int32_t s_n[kKeepBlock];
  __shared__ int32_t s_nu[kKeepBlock];
  __shared__ uint32_t s_mask[kMaskWords][kKeepBlock];
  const int64_t n_start = counts[0] < cap_start ? counts[0] : cap_start;
  int64_t b, e;
  chunk_of(n_start, &b, &e);
  int64_t t_run = part[2 * blockIdx.x], h_run = part[2 * blockIdx.x + 1];
  const int wid = threadIdx.x / kWave, nw = kKeepBlock / kWave;
  for (int64_t s0 = b; s0 < e; s0 += kKeepBlock) {
    const int64_t s = s0 + threadIdx.x;
    int32_t n = 0;
    bool keep = false;
    if (s < e) {
      n = int32_t(tmp.rec[s * kRecWords + kRecN]);
      keep = n >= min_hits;
    }
    int64_t tt, th;
    const int64_t pt = block_exclusive_scan(keep ? 1 : 0, lds, &tt);
    const int64_t ph = block_exclusive_scan(keep ? n : 0, lds, &th);
    if (keep) {
      const int64_t ti = t_run + pt, hb = h_run + ph;
      const bool fits = ti < o.cap_tracks && hb + n <= o.cap_hits;
      const uint4* r4 = reinterpret_cast<const uint4*>(tmp.rec + s * kRecWords);
      const uint4 a0 = r4[0], a1 = r4[1], a2 = r4[2], a3 = r4[3], a4 = r4[4], a5 = r4[5], a6 = r4[6];
      if (fits) {
        o.unit[ti] = int32_t(a4.w);
        o.start[ti] = starts[s];
        o.n_hits[ti] = n;
        o.hit_begin[ti] = hb;
        o.ndf[ti] = 2 * n - 5;
        o.x_ref[ti] = __uint_as_float(a0.x);
        float* pp = o.param + ti * 5;
        pp[0] = __uint_as_float(a0.y);
        pp[1] = __uint_as_float(a0.z);
        pp[2] = __uint_as_float(a0.w);
        pp[3] = __uint_as_float(a1.x);
        pp[4] = __uint_as_float(a1.y);
        // covariance blocks multiplied out: C = U D U^T
        const float uys = __uint_as_float(a1.z), uyw = __uint_as_float(a1.w);
        const float usw = __uint_as_float(a2.x), dy = __uint_as_float(a2.y);
        const float ds = __uint_as_float(a2.z), dw = __uint_as_float(a2.w);
        const float uzt = __uint_as_float(a3.x), dz = __uint_as_float(a3.y);
        const float dt = __uint_as_float(a3.z);
        const float cww = dw;
        const float cws = usw * dw;
        const float cwy = uyw * dw;
        const float css = ds + usw * cws;
        const float csy = uys * ds + uyw * cws;
        const float cyy = (dy + uys * (uys * ds)) + uyw * cwy;
        const float ctt = dt;
        const float ctz = uzt * dt;
        const float czz = dz + uzt * ctz;
        const float cv[15] = {cyy, 0.0f, czz, csy, 0.0f, css, 0.0f, ctz,
                              0.0f, ctt, cwy, 0.0f, cws, 0.0f, cww};
        for (int j = 0; j < 15; ++j) o.cov[ti * 15 + j] = cv[j];
        o.chi2[ti] = __uint_as_float(a3.w);
      }
      s_slot[pt] = fits ? int32_t(s - s0) : -1;
      s_hb[pt] = hb;
      s_n[pt] = n;
      s_nu[pt] = int32_t(a4.y);
      s_mask[0][pt] = a5.x;
      s_mask[1][pt] = a5.y;
      s_mask[2][pt] = a5.z;
      s_mask[3][pt] = a5.w;
      s_mask[4][pt] = a6.x;
    }
    __syncthreads();
    // Hit lists sorted by row: the inward phase reversed, then the outward
    // phase; the row of the j-th hit is the j-th set bit of the row mask.
    for (int q = wid; q < int(tt); q += nw) {
      const int32_t sl = s_slot[q];
      if (sl < 0) continue;
      const int64_t ss = s0 + sl;
      const int nn = s_n[q], nu = s_nu[q], nd = nn - nu;
      const int64_t hb = s_hb[q];
      const int32_t* hs = tmp.hit + ss * tmp.stride;
      for (int j = lane_id(); j < nn; j += kWave) {
        const int src = j < nd ? nu + (nd - 1 - j) : j - nd;
        o.hit_id[hb + j] = hs[src];
      }
      uint32_t m[kMaskWords];
      int below[kMaskWords];
      int acc = 0;
#pragma unroll
      for (int w = 0; w < kMaskWords; ++w) {
        m[w] = s_mask[w][q];
        below[w] = acc;
        acc += __popc(m[w]);
      }
#pragma unroll
      for (int w = 0; w < kMaskWords; w += 2) {
        // lanes 0-31 take word w, lanes 32-63 word w+1
        const int ww = w + (lane_id() >> 5);
        if (ww < kMaskWords) {
          const int bit = lane_id() & 31;
          const uint32_t mw = ww == 0 ? m[0] : ww == 1 ? m[1] : ww == 2 ? m[2] : ww == 3 ? m[3] : m[4];
          const int bw = ww == 0 ? below[0] : ww == 1 ? below[1] : ww == 2 ? below[2] : ww == 3 ? below[3] : below[4];
          if ((mw >> bit) & 1u) {
            const int rank = bw + __popc(mw & ((1u << bit) - 1u));
            o.hit_row[hb + rank] = uint8_t(ww * 32 + bit);
          }
        }
      }
    }
    __syncthreads();
    t_run += tt;
    h_run += th;
  }
}

}  // namespace tpcx
