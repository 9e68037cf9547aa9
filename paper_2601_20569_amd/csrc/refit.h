// Track refit through a space-charge-distortion correction map, and its
// hand-written adjoint.
//
// The paper names the space-charge-distortion correction maps as a main source
// of track-quality problems (Abstract, Section 2) and describes the track fit
// as a Kalman filter over the attached clusters (Section 2).  Here a map is a
// tensor-product uniform cubic B-spline (36 phi x 17 r x 20 z nodes, three
// components: delta r, delta r*phi, delta z); a cluster measured at (x, y, z)
// in its sector frame (radius r, global azimuth phi) moves by delta r along
// (x, y)/r, by delta r*phi along (-y, x)/r and by delta z along z.  The refit
// runs outwards from the innermost cluster: y, z from that cluster, sin(phi),
// dz/ds, q/pT from the tracking result, covariance diag(sy^2, sz^2, 1e-2, 1e-2,
// 1); it propagates to every further cluster's own corrected x and updates,
// without rejection.  chi2 of a track = sum of the updates' chi2.
//
// The refit takes no decision that depends on the last bit of a result, so it
// uses the hardware square root and reciprocal (within 1 ulp) instead of the
// correctly rounded ones the tracking needs.
//
// The backward pass gives d(sum_t dL/dchi2_t * chi2_t)/d(map coefficients).
// The forward stores the filter state every kCkpt clusters; the backward
// recomputes one segment at a time from its checkpoint into a per-lane scratch
// area and runs the reverse sweep of every step (update, then propagation).
// Coefficient gradients are summed in 64-bit fixed point (2^-32), so the sum
// does not depend on the order of the additions: first in an LDS window of
// phi nodes around the block's tracks, then into global memory.
#pragma once

#include "tpcx_common.h"
#include "tracklet.h"

namespace tpcx {

constexpr int kMapNPhi = 36, kMapNR = 17, kMapNZ = 20, kMapComp = 3;
constexpr int kMapNCoef = kMapComp * kMapNPhi * kMapNR * kMapNZ;
constexpr float kMapDPhi = 6.28318530717958647692f / kMapNPhi;
constexpr float kMapR0 = 85.0f, kMapDR = 10.0f;
constexpr float kMapZ0 = -250.0f, kMapDZ = 500.0f / 19.0f;
constexpr int kCkpt = 16;            // clusters per checkpoint segment
constexpr int kCkptFloats = 16;      // 15 state numbers + padding
constexpr int kRefitBlock = 256;
constexpr int kWinPhi = 8;           // phi nodes held in the LDS accumulation window
constexpr double kFixScale = 4294967296.0;  // 2^32

__device__ __forceinline__ int map_index(int comp, int i, int j, int k) {
  return ((comp * kMapNPhi + i) * kMapNR + j) * kMapNZ + k;
}

// 1-D weights of the four nodes around a coordinate; node index of the first.
struct Weights4 {
  int first;
  float w[4];
};

// Weights of the uniform cubic B-spline at the four nodes first .. first+3
// around u (node spacing 1), from the fractional part f of u: (1-f)^3/6,
// (3f^3 - 6f^2 + 4)/6, (-3f^3 + 3f^2 + 3f + 1)/6, f^3/6.
__device__ __forceinline__ Weights4 weights_frac(float u) {
  const float fl = floorf(u);
  const float f = u - fl, g = 1.0f - f;
  const float f2 = f * f, f3 = f2 * f;
  Weights4 W;
  W.first = int(fl) - 1;
  W.w[0] = g * g * g * (1.0f / 6.0f);
  W.w[1] = (3.0f * f3 - 6.0f * f2 + 4.0f) * (1.0f / 6.0f);
  W.w[2] = (-3.0f * f3 + 3.0f * f2 + 3.0f * f + 1.0f) * (1.0f / 6.0f);
  W.w[3] = f3 * (1.0f / 6.0f);
  return W;
}

// phi nodes: periodic, u = phi / 10 degrees wrapped into [0, 36)
__device__ __forceinline__ Weights4 weights_phi(float phi) {
  float u = phi * (1.0f / kMapDPhi);
  u = u - float(kMapNPhi) * floorf(u * (1.0f / kMapNPhi));
  return weights_frac(u);
}

// r or z nodes x0 + i dx, i = 0 .. n-1; nodes outside have weight 0
__device__ __forceinline__ Weights4 weights_lin(float x, float x0, float inv_dx, int n) {
  Weights4 W = weights_frac((x - x0) * inv_dx);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = W.first + a;
    if (i < 0 || i >= n) W.w[a] = 0.0f;
  }
  return W;
}

// Corrected position of a measured cluster (x_m, y_m, z_m) in a sector whose
// centre lies at azimuth alpha.
struct HitGeom {
  float xm, ym, zm, inv_r, phi;
};

__device__ __forceinline__ HitGeom hit_geom(float xm, float ym, float zm, float alpha, float* r) {
  HitGeom h;
  h.xm = xm;
  h.ym = ym;
  h.zm = zm;
  *r = k_sqrt<true>(xm * xm + ym * ym);
  h.inv_r = k_rcp<true>(*r);
  h.phi = alpha + atan2f(ym, xm);
  return h;
}

// Map coefficients of node (i, j, k), the three components as one float4,
// read from the coefficient array itself.
struct ThetaGlobal {
  const float* __restrict__ theta;
  __device__ __forceinline__ float4 operator()(int i, int j, int k) const {
    return make_float4(theta[map_index(0, i, j, k)], theta[map_index(1, i, j, k)],
                       theta[map_index(2, i, j, k)], 0.0f);
  }
};

// The same from a block-local copy in LDS of kStageNPhi x kStageNR x kMapNZ
// nodes starting at phi node i_lo (periodic) and r node j_lo.
constexpr int kStageNPhi = 8, kStageNR = 6;
constexpr int kStageNodes = kStageNPhi * kStageNR * kMapNZ;

struct ThetaStaged {
  const float4* lds;
  int i_lo, j_lo;
  __device__ __forceinline__ float4 operator()(int i, int j, int k) const {
    const int si = (i - i_lo + kMapNPhi) % kMapNPhi;
    return lds[(si * kStageNR + (j - j_lo)) * kMapNZ + k];
  }
  // whether every node of a cluster with these first indices is in the copy
  __device__ __forceinline__ bool covers(int phi_first, int r_first) const {
    const int si = ((phi_first - i_lo) % kMapNPhi + kMapNPhi) % kMapNPhi;
    const int j0 = min(max(r_first, 0), kMapNR - 1), j1 = min(max(r_first + 3, 0), kMapNR - 1);
    return si + 3 < kStageNPhi && j0 >= j_lo && j1 < j_lo + kStageNR;
  }
};

// Map displacement (delta r, delta r*phi, delta z) at a cluster: the sum over
// the 4 x 4 x 4 nodes around it of the coefficients times the product of the
// three 1-D weights, summed z first, then r, then phi.  Nodes outside the r or
// z range have weight 0 (their index is clamped into the table).
template <class Theta>
__device__ __forceinline__ void map_displacement(const Theta& th, const Weights4& wp, const Weights4& wr,
                                                 const Weights4& wz, float d[3]) {
  d[0] = d[1] = d[2] = 0.0f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = ((wp.first + a) % kMapNPhi + kMapNPhi) % kMapNPhi;
    float e0 = 0.0f, e1 = 0.0f, e2 = 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = min(max(wr.first + b, 0), kMapNR - 1);
      float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k = min(max(wz.first + c, 0), kMapNZ - 1);
        const float4 v = th(i, j, k);
        f0 = __builtin_fmaf(v.x, wz.w[c], f0);
        f1 = __builtin_fmaf(v.y, wz.w[c], f1);
        f2 = __builtin_fmaf(v.z, wz.w[c], f2);
      }
      e0 = __builtin_fmaf(f0, wr.w[b], e0);
      e1 = __builtin_fmaf(f1, wr.w[b], e1);
      e2 = __builtin_fmaf(f2, wr.w[b], e2);
    }
    d[0] = __builtin_fmaf(e0, wp.w[a], d[0]);
    d[1] = __builtin_fmaf(e1, wp.w[a], d[1]);
    d[2] = __builtin_fmaf(e2, wp.w[a], d[2]);
  }
}

// The same with the z sums already formed: for a map evaluated at one fixed
// z, th(i, j) holds, per component, the sum over the four z nodes of the
// coefficients times the z weights, accumulated in the order above, so the
// result equals map_displacement's bit for bit.
template <class ThetaZ>
__device__ __forceinline__ void map_displacement_zsum(const ThetaZ& th, const Weights4& wp, const Weights4& wr,
                                                      float d[3]) {
  d[0] = d[1] = d[2] = 0.0f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = ((wp.first + a) % kMapNPhi + kMapNPhi) % kMapNPhi;
    float e0 = 0.0f, e1 = 0.0f, e2 = 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = min(max(wr.first + b, 0), kMapNR - 1);
      const float4 f = th(i, j);
      e0 = __builtin_fmaf(f.x, wr.w[b], e0);
      e1 = __builtin_fmaf(f.y, wr.w[b], e1);
      e2 = __builtin_fmaf(f.z, wr.w[b], e2);
    }
    d[0] = __builtin_fmaf(e0, wp.w[a], d[0]);
    d[1] = __builtin_fmaf(e1, wp.w[a], d[1]);
    d[2] = __builtin_fmaf(e2, wp.w[a], d[2]);
  }
}

// z sums (see map_displacement_zsum) of the staged kStageNPhi x kStageNR
// (phi, r) nodes, in LDS.
struct ThetaZStaged {
  const float4* lds;
  int i_lo, j_lo;
  __device__ __forceinline__ float4 operator()(int i, int j) const {
    const int si = (i - i_lo + kMapNPhi) % kMapNPhi;
    return lds[si * kStageNR + (j - j_lo)];
  }
};

// Corrected cluster as (x_c, y_c, z_m, delta z): z_c = z_m + delta z is not
// formed here, because z_m can be large (drift coordinate in a time frame)
// and the refit works in z relative to its first cluster (rel_z).
__device__ __forceinline__ float4 apply_displacement(const HitGeom& h, const float d[3]) {
  return make_float4(h.xm + (d[0] * h.xm - d[1] * h.ym) * h.inv_r,
                     h.ym + (d[0] * h.ym + d[1] * h.xm) * h.inv_r, h.zm, d[2]);
}

// z_c of a corrected cluster relative to the measured z of the track's first
// cluster, z_ref: (z_m - z_ref) is exact for clusters of one track, so no
// digit of delta z is lost to the magnitude of z_m.
__device__ __forceinline__ float rel_z(const float4& h, float z_ref) { return (h.z - z_ref) + h.w; }

// Corrected cluster (see apply_displacement); theta == nullptr means no map.
// The coefficients must be finite.
__device__ __forceinline__ float4 correct_cluster(const float* __restrict__ theta, float xm, float ym,
                                                  float zm, float alpha) {
  float r;
  const HitGeom h = hit_geom(xm, ym, zm, alpha, &r);
  float d[3] = {0.0f, 0.0f, 0.0f};
  if (theta)
    map_displacement(ThetaGlobal{theta}, weights_phi(h.phi), weights_lin(r, kMapR0, 1.0f / kMapDR, kMapNR),
                     weights_lin(h.zm, kMapZ0, 1.0f / kMapDZ, kMapNZ), d);
  return apply_displacement(h, d);
}

struct RefitIn {
  int64_t n_tracks;            // capacity of the track arrays
  const int64_t* n_tracks_dev; // if set: the track count is min(n_tracks, *n_tracks_dev)
  const int64_t* status_dev;   // if set and non-zero: nothing is refitted
  const int32_t* n_hit;        // if set: clusters per track; else hit_begin[t + 1] - hit_begin[t]
  int32_t min_hits;            // tracks with fewer clusters are not refitted (ok = 0)
  const int64_t* hit_begin;
  const int32_t* hit_id;
  const uint8_t* hit_row;
  const int32_t* unit;
  const float* seed;  // [n][5]
  const float* y;
  const float* z;
  const float* unit_alpha;
  const float* row_x;
};

struct RefitWs {
  float* xyz;       // [n_hits][4] corrected x, y, z (+pad) from the forward pass
  float* ckpt;      // checkpoints, kCkptFloats each
  float* scratch;   // [lanes][kCkpt][kCkptFloats] states of the segment in the backward
  int64_t* acc;     // [kMapNCoef] fixed-point gradient accumulators
  float* hgrad;     // [n_hits][4] adjoints of the corrected (x, y, z) of every hit (backward)
  int64_t n_lanes;
  unsigned long long* queue;  // [kXcds] track queues of the filter kernel (zeroed before each launch)
};

__device__ __forceinline__ int64_t ckpt_base(const RefitIn& in, int64_t t) {
  return in.hit_begin[t] / kCkpt + t;
}

__device__ __forceinline__ int64_t refit_count(const RefitIn& in) {
  if (in.status_dev && (*in.status_dev & kStOverflow) != 0) return 0;
  if (!in.n_tracks_dev) return in.n_tracks;
  const int64_t n = *in.n_tracks_dev;
  return n < in.n_tracks ? n : in.n_tracks;
}

__device__ __forceinline__ int track_size(const RefitIn& in, int64_t t) {
  return in.n_hit ? in.n_hit[t] : int(in.hit_begin[t + 1] - in.hit_begin[t]);
}

__device__ __forceinline__ void seed_state(KState& q, float xc, float yc, float zc, const float* sd,
                                           const DevParams& p) {
  q.x = xc;
  q.y = yc;
  q.z = zc;
  q.s = sd[2];
  q.t = sd[3];
  q.w = sd[4];
  // diag(sy^2, 1e-2, 1) and diag(sz^2, 1e-2): U = 1
  q.uys = 0.0f;
  q.uyw = 0.0f;
  q.usw = 0.0f;
  q.dy = p.sy2;
  q.ds = 1e-2f;
  q.dw = 1.0f;
  q.uzt = 0.0f;
  q.dz = p.sz2;
  q.dt = 1e-2f;
}

__device__ __forceinline__ void store_state(float* dst, const KState& q) {
  float4* d = reinterpret_cast<float4*>(dst);
  d[0] = make_float4(q.x, q.y, q.z, q.s);
  d[1] = make_float4(q.t, q.w, q.uys, q.uyw);
  d[2] = make_float4(q.usw, q.dy, q.ds, q.dw);
  d[3] = make_float4(q.uzt, q.dz, q.dt, 0.0f);
}

__device__ __forceinline__ KState load_state(const float* src) {
  const float4* s = reinterpret_cast<const float4*>(src);
  const float4 a = s[0], b = s[1], c = s[2], d = s[3];
  KState q;
  q.x = a.x; q.y = a.y; q.z = a.z; q.s = a.w;
  q.t = b.x; q.w = b.y; q.uys = b.z; q.uyw = b.w;
  q.usw = c.x; q.dy = c.y; q.ds = c.z; q.dw = c.w;
  q.uzt = d.x; q.dz = d.y; q.dt = d.z;
  return q;
}

// One refit step: propagate to the cluster's x, update with its (y, z).
__device__ __forceinline__ bool refit_step(KState& q, float xc, float yc, float zc,
                                           const DevParams& p, float* chi2) {
  float cp = 0.0f, rp = 0.0f;
  bool cached = false;
  if (!kf_propagate<true>(q, xc, p, cp, rp, cached)) return false;
  const KInnov n = kf_innov(q, p);
  const float iSy = k_rcp<true>(n.sy);
  const float iSz = k_rcp<true>(n.sz);
  *chi2 = *chi2 + kf_update<true>(q, yc, zc, n, iSy, iSz, p);
  return true;
}

// Corrected clusters, one per attached hit, for the standalone refit: a block
// takes the hits of kRefitBlock consecutive tracks (they are contiguous) and
// finds each hit's track by binary search over the block's offsets in LDS.
__global__ void __launch_bounds__(kRefitBlock) k_correct_hits(RefitIn in, const float* __restrict__ theta,
                                                              float4* __restrict__ xyz) {
  __shared__ int64_t hb[kRefitBlock + 1];
  __shared__ float al[kRefitBlock];
  const int64_t n_tr = in.n_tracks;
  const int64_t t0 = int64_t(blockIdx.x) * kRefitBlock;
  const int cnt = int(min(int64_t(kRefitBlock), n_tr - t0));
  const int tid = threadIdx.x;
  if (tid <= cnt) hb[tid] = in.hit_begin[t0 + tid];
  if (tid == 0 && cnt == kRefitBlock) hb[kRefitBlock] = in.hit_begin[t0 + kRefitBlock];
  if (tid < cnt) al[tid] = in.unit_alpha[in.unit[t0 + tid]];
  __syncthreads();
  for (int64_t q = hb[0] + tid; q < hb[cnt]; q += kRefitBlock) {
    int lo = 0, hi = cnt - 1;  // last s with hb[s] <= q
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (hb[mid] <= q) lo = mid; else hi = mid - 1;
    }
    xyz[q] = correct_cluster(theta, in.row_x[in.hit_row[q]], in.y[in.hit_id[q]], in.z[in.hit_id[q]], al[lo]);
  }
}

// Corrected clusters, one per input cluster, for the batched refit: one block
// per (unit, row), walking the row in caller order, so the reads of the input
// and the writes of the results are coalesced (the filter gathers them by
// caller index).  The block first copies into LDS the map nodes around its
// sector (phi within +-20 degrees of the centre line, the r nodes of the
// row's radius range); a cluster whose nodes lie outside that copy reads the
// coefficient array.  Both give the same arithmetic as correct_cluster.
// z_fixed: the map is evaluated at z = z_map for every cluster (time-frame
// input, whose drift coordinate is not z); the correction delta z still
// applies to the measured z.  Then the block forms the z sums of its staged
// (phi, r) nodes once, and a cluster sums 16 nodes instead of 64 (the same
// result, bit for bit).
__global__ void __launch_bounds__(kRefitBlock) k_correct_clusters(
    int n_rows, const int64_t* __restrict__ row_begin, const float* __restrict__ y,
    const float* __restrict__ z, const float* __restrict__ unit_alpha,
    const float* __restrict__ row_x, const float* __restrict__ theta, int z_fixed, float z_map,
    float4* __restrict__ corr) {
  __shared__ float4 stage[kStageNodes];
  const int64_t ur = xcd_block();
  const float alpha = unit_alpha[ur / n_rows];
  const float x = row_x[ur % n_rows];
  const int64_t e = row_begin[ur + 1];
  if (!theta) {
    const float d[3] = {0.0f, 0.0f, 0.0f};
    for (int64_t c = row_begin[ur] + threadIdx.x; c < e; c += kRefitBlock) {
      float r;
      corr[c] = apply_displacement(hit_geom(x, y[c], z[c], alpha, &r), d);
    }
    return;
  }
  ThetaStaged ts;
  ts.lds = stage;
  {
    const float two_pi = 6.28318530717958647692f;
    float ph = fmodf(alpha - 0.3490658503988659f, two_pi);  // 20 degrees below the centre line
    if (ph < 0.0f) ph += two_pi;
    ts.i_lo = (int(floorf(ph / kMapDPhi)) - 1 + kMapNPhi) % kMapNPhi;
    ts.j_lo = min(max(int(floorf((x - kMapR0) / kMapDR)) - 1, 0), kMapNR - kStageNR);
  }
  if (z_fixed) {
    // one z for every cluster: the z sums of the staged (phi, r) nodes once
    const Weights4 wz = weights_lin(z_map, kMapZ0, 1.0f / kMapDZ, kMapNZ);
    for (int q = threadIdx.x; q < kStageNPhi * kStageNR; q += kRefitBlock) {
      const int j = ts.j_lo + q % kStageNR;
      const int i = (ts.i_lo + q / kStageNR) % kMapNPhi;
      float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
#pragma unroll
      for (int cz = 0; cz < 4; ++cz) {
        const int k = min(max(wz.first + cz, 0), kMapNZ - 1);
        const float4 v = ThetaGlobal{theta}(i, j, k);
        f0 = __builtin_fmaf(v.x, wz.w[cz], f0);
        f1 = __builtin_fmaf(v.y, wz.w[cz], f1);
        f2 = __builtin_fmaf(v.z, wz.w[cz], f2);
      }
      stage[q] = make_float4(f0, f1, f2, 0.0f);
    }
    __syncthreads();
    const ThetaZStaged tz{stage, ts.i_lo, ts.j_lo};
    for (int64_t c = row_begin[ur] + threadIdx.x; c < e; c += kRefitBlock) {
      float r;
      const HitGeom h = hit_geom(x, y[c], z[c], alpha, &r);
      const Weights4 wp = weights_phi(h.phi);
      const Weights4 wr = weights_lin(r, kMapR0, 1.0f / kMapDR, kMapNR);
      float d[3];
      if (ts.covers(wp.first, wr.first))
        map_displacement_zsum(tz, wp, wr, d);
      else
        map_displacement(ThetaGlobal{theta}, wp, wr, wz, d);
      corr[c] = apply_displacement(h, d);
    }
    return;
  }
  for (int q = threadIdx.x; q < kStageNodes; q += kRefitBlock) {
    const int k = q % kMapNZ;
    const int j = ts.j_lo + (q / kMapNZ) % kStageNR;
    const int i = (ts.i_lo + q / (kMapNZ * kStageNR)) % kMapNPhi;
    stage[q] = ThetaGlobal{theta}(i, j, k);
  }
  __syncthreads();
  for (int64_t c = row_begin[ur] + threadIdx.x; c < e; c += kRefitBlock) {
    float r;
    const HitGeom h = hit_geom(x, y[c], z[c], alpha, &r);
    const Weights4 wp = weights_phi(h.phi);
    const Weights4 wr = weights_lin(r, kMapR0, 1.0f / kMapDR, kMapNR);
    const Weights4 wz = weights_lin(z_fixed ? z_map : h.zm, kMapZ0, 1.0f / kMapDZ, kMapNZ);
    float d[3];
    if (ts.covers(wp.first, wr.first))
      map_displacement(ts, wp, wr, wz, d);
    else
      map_displacement(ThetaGlobal{theta}, wp, wr, wz, d);
    corr[c] = apply_displacement(h, d);
  }
}

// Forward filter over the corrected clusters: xyz[hit_id[q]] when ByCluster,
// else xyz[q].  Persistent; every lane runs one track at a time.  Idle lanes
// take new tracks, `refill` or more at a time (all 64: the lanes step through
// rows together), from a wavefront-private chunk of kRefitChunk consecutive
// tracks refilled from kXcds device queues.  Three steps per iteration, each
// reloading, after its arithmetic, the register it used with the cluster
// three steps ahead: the loads overlap two steps of arithmetic.  Which lane
// runs a track does not change its result.  Checkpoints (every kCkpt
// clusters) are written when ckpt is set.
constexpr int kRefitChunk = 64;

template <bool ByCluster>
__global__ void __launch_bounds__(kRefitBlock) k_refit_filter(
    RefitIn in, DevParams p, const float4* __restrict__ xyz, float* __restrict__ ckpt,
    unsigned long long* __restrict__ queue, int refill, float* __restrict__ chi2_out,
    int32_t* __restrict__ ok_out) {
  const int64_t n_tr = refit_count(in);
  const int lane = lane_id();
  int64_t chunk = 0, chunk_end = 0;  // wavefront-uniform
  bool exhausted = false;            // wavefront-uniform
  const int qhome = int(blockIdx.x % kXcds);
  int qtried = 0;
  int64_t t = -1, hb = 0, cb = 0;
  int i = 0, n = 0;
  float chi2 = 0.0f, zref = 0.0f;
  KState q{};
  // Three steps per iteration, A, B and C: hA / hB / hC hold the corrected
  // clusters of the steps' hits, each reloaded at the end of its step (for
  // the hit three steps later) into the register the step has just used, so
  // no register is copied and a step waits only for loads two steps old;
  // idA / idB / idC are the cluster ids for those reloads, loaded three steps
  // before.
  float4 hA = make_float4(0.0f, 0.0f, 0.0f, 0.0f), hB = hA, hC = hA;
  int32_t idA = 0, idB = 0, idC = 0;
  auto xyz_index = [&](int64_t qh) -> int64_t { return ByCluster ? int64_t(in.hit_id[qh]) : qh; };
  while (true) {
    const int nidle = __popcll(__ballot(t < 0));
    if (nidle == kWave && exhausted) break;
    if (nidle > 0 && !exhausted && (nidle >= refill || nidle == kWave)) {
      // hand tracks to idle lanes; tracks too short to refit are finished here
      while (true) {
        const uint64_t want = __ballot(t < 0);
        if (!want) break;
        if (chunk == chunk_end) {
          // queue j hands out the j-th eighth of the tracks; the wavefront
          // starts with the queue of its own XCD
          while (qtried < kXcds) {
            const int j = (qhome + qtried) % kXcds;
            const int64_t qb = n_tr * j / kXcds, qe = n_tr * (j + 1) / kXcds;
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(queue + j, static_cast<unsigned long long>(kRefitChunk));
            base = __shfl(base, 0, kWave);
            if (qb + int64_t(base) < qe) {
              chunk = qb + int64_t(base);
              chunk_end = min(chunk + kRefitChunk, qe);
              break;
            }
            ++qtried;
          }
          if (qtried >= kXcds) {
            exhausted = true;
            break;
          }
        }
        const int rank = __popcll(want & lanes_below());
        const int64_t avail = chunk_end - chunk;
        if (t < 0 && rank < avail) {
          t = chunk + rank;
          n = track_size(in, t);
          if (n < in.min_hits || n < 2) {
            chi2_out[t] = 0.0f;
            ok_out[t] = 0;
            t = -1;
          } else {
            hb = in.hit_begin[t];
            const float4 h0 = xyz[xyz_index(hb)];
            zref = h0.z;
            seed_state(q, h0.x, h0.y, rel_z(h0, zref), in.seed + 5 * t, p);
            cb = ckpt_base(in, t);
            if (ckpt) store_state(ckpt + cb * kCkptFloats, q);
            i = 1;
            chi2 = 0.0f;
            // the lane's next step is of hit 1 and runs as A, B or C
            // depending on where the iteration stands: give all three
            hA = xyz[xyz_index(hb + 1)];
            hB = xyz[xyz_index(hb + min(2, n - 1))];
            hC = xyz[xyz_index(hb + min(3, n - 1))];
            if (ByCluster) {
              idA = in.hit_id[hb + min(4, n - 1)];
              idB = in.hit_id[hb + min(5, n - 1)];
              idC = in.hit_id[hb + min(6, n - 1)];
            }
          }
        }
        chunk += min(int64_t(__popcll(want)), avail);
      }
    }
    // every lane runs the steps (idle lanes on indices 0, without effect),
    // so the loads of each iteration are the same
    auto step = [&](float4& hc, int32_t& idc) {
      const bool act = t >= 0;
      const bool ok = refit_step(q, hc.x, hc.y, rel_z(hc, zref), p, &chi2);
      // reload for the hit three steps later (clamped into the track)
      if (ByCluster) {
        hc = xyz[int64_t(act ? idc : 0)];
        idc = in.hit_id[act ? hb + min(i + 6, n - 1) : 0];
      } else {
        hc = xyz[act ? hb + min(i + 3, n - 1) : 0];
      }
      if (act) {
        if (ok && ckpt && i % kCkpt == 0) store_state(ckpt + (cb + i / kCkpt) * kCkptFloats, q);
        ++i;
        if (!ok || i == n) {
          chi2_out[t] = ok ? chi2 : 0.0f;
          ok_out[t] = ok ? 1 : 0;
          t = -1;
        }
      }
    };
    step(hA, idA);
    step(hB, idB);
    step(hC, idC);
  }
}

// Adjoint of the filter state (same layout as KState).
struct KBar {
  float x, y, z, s, t, w;
  float uys, uyw, usw, dy, ds, dw;
  float uzt, dz, dt;
};

// Reverse of one refit step.  `q` is the state before the step; `g` holds the
// adjoint of the state after it and becomes the adjoint of the state before
// it; gchi2 is the adjoint of the step's chi2; returns the adjoints of the
// cluster's corrected (x, y, z).  The forward arithmetic (refit_step) is
// recomputed here, then every assignment is reversed in the opposite order.
__device__ void refit_step_reverse(const KState& q, float x1, float my, float mz, const DevParams& p,
                                   float gchi2, KBar& g, float* gx1, float* gmy, float* gmz) {
  // ---------------- forward: propagation
  const float dx = x1 - q.x;
  const float k = p.kappa * q.w;
  const float kd = k * dx;
  const float s1 = q.s - kd;
  const float c0 = k_sqrt<true>(1.0f - q.s * q.s);
  const float c1 = k_sqrt<true>(1.0f - s1 * s1);
  const float cc = c0 + c1;
  const float ss = q.s + s1;
  const float icc = k_rcp<true>(cc);
  const float tg = ss * icc;
  const float dy = dx * tg;
  const float dl = k_sqrt<true>(dx * dx + dy * dy);
  const float ak = fabsf(k);
  const float u = (ak * dl) * 0.5f;
  const float a1c = 0.16666667f, a2c = 0.075f;
  const float u2 = u * u;
  const float A = 1.0f + u2 * (a1c + u2 * a2c);
  const float sgn = dx < 0.0f ? -1.0f : 1.0f;
  const float dS = sgn * (dl * A);
  const float r0 = k_div<true>(q.s, c0);
  const float r1 = k_div<true>(s1, c1);
  const float icc2 = icc * icc;
  const float na = 2.0f * cc + ss * (r0 + r1);
  const float qa = na * icc2;
  const float a = dx * qa;
  const float e = -(p.kappa * dx);
  const float nb = cc + ss * r1;
  const float qb = nb * icc2;
  const float de = dx * e;
  const float b = de * qb;
  // state after the propagation (input of the update); D is unchanged
  const float py = q.y + dy, pz = q.z + q.t * dS;
  const float puyw = (q.uyw + a * q.usw) + b, puys = q.uys + a, pusw = q.usw + e, puzt = q.uzt + dS;
  const float pdy = q.dy, pds = q.ds, pdw = q.dw, pdz = q.dz, pdt = q.dt;
  // ---------------- forward: update
  const float v2 = pds * puys, v3 = pdw * puyw;
  const float a1 = p.sy2 + pdy;
  const float a2 = a1 + v2 * puys;
  const float Sy = a2 + v3 * puyw;
  const float vz = pdt * puzt;
  const float z1 = p.sz2 + pdz;
  const float Sz = z1 + vz * puzt;
  const float ry = my - py, rz = mz - pz;
  const float iSy = k_rcp<true>(Sy), iSz = k_rcp<true>(Sz);
  const float i1 = k_rcp<true>(a1), i2 = k_rcp<true>(a2), j1 = k_rcp<true>(z1);
  const float b1 = (pdy + puys * v2) + puyw * v3;
  const float b2 = v2 + pusw * v3;
  const float gg = ry * iSy;
  const float f1 = p.sy2 * i1, f2 = p.sy2 * i2, hh = puyw * i2;
  const float m2 = a1 * i2, m3 = a2 * iSy;
  const float bz1 = pdz + puzt * vz;
  const float gzz = rz * iSz;
  const float fz = p.sz2 * j1, mz1 = z1 * iSz;

  // ---------------- reverse: update, (z, t) block
  float Gpdz = 0.0f, Gpdt = 0.0f, Gpuzt = 0.0f, Gpz = 0.0f, Gpt = 0.0f;
  float Gfz = 0.0f, Gz1 = 0.0f, GiSz = 0.0f, Gvz = 0.0f, Gbz1 = 0.0f, Ggz = 0.0f, Grz = 0.0f;
  // dz' = pdz*fz ; dt' = pdt*mz1 (mz1 = z1*iSz) ; uzt' = puzt*fz
  Gpdz += g.dz * fz;
  Gfz += g.dz * pdz;
  Gpdt += g.dt * mz1;
  const float Gmz1 = g.dt * pdt;
  Gz1 += Gmz1 * iSz;
  GiSz += Gmz1 * z1;
  Gpuzt += g.uzt * fz;
  Gfz += g.uzt * puzt;
  // t' = pt + vz*gzz ; z' = pz + bz1*gzz
  Gpt += g.t;
  Gvz += g.t * gzz;
  Ggz += g.t * vz;
  Gpz += g.z;
  Gbz1 += g.z * gzz;
  Ggz += g.z * bz1;
  // fz = sz2*j1 ; j1 = 1/z1
  const float Gj1 = Gfz * p.sz2;
  Gz1 += -Gj1 * j1 * j1;
  // gzz = rz*iSz
  Grz += Ggz * iSz;
  GiSz += Ggz * rz;
  // bz1 = pdz + puzt*vz
  Gpdz += Gbz1;
  Gpuzt += Gbz1 * vz;
  Gvz += Gbz1 * puzt;

  // ---------------- reverse: update, (y, s, w) block
  float Gpdy = 0.0f, Gpds = 0.0f, Gpdw = 0.0f, Gpuys = 0.0f, Gpuyw = 0.0f, Gpusw = 0.0f;
  float Gpy = 0.0f, Gps = 0.0f, Gpw = 0.0f;
  float Gf1 = 0.0f, Gi2 = 0.0f, Ga1 = 0.0f, Ga2 = 0.0f, GiSy = 0.0f, Gv2 = 0.0f, Gv3 = 0.0f;
  float Gb1 = 0.0f, Gb2 = 0.0f, Ggg = 0.0f, Gry = 0.0f;
  // dy' = pdy*f1 ; ds' = pds*m2 ; dw' = pdw*m3
  Gpdy += g.dy * f1;
  Gf1 += g.dy * pdy;
  Gpds += g.ds * m2;
  const float Gm2 = g.ds * pds;
  Ga1 += Gm2 * i2;
  Gi2 += Gm2 * a1;
  Gpdw += g.dw * m3;
  const float Gm3 = g.dw * pdw;
  Ga2 += Gm3 * iSy;
  GiSy += Gm3 * a2;
  // uys' = puys*f1 ; uyw' = puyw*f2 (f2 = sy2*i2) ; usw' = pusw - v2*hh (hh = puyw*i2)
  Gpuys += g.uys * f1;
  Gf1 += g.uys * puys;
  Gpuyw += g.uyw * f2;
  Gi2 += g.uyw * puyw * p.sy2;
  Gpusw += g.usw;
  Gv2 += -g.usw * hh;
  const float Ghh = -g.usw * v2;
  Gpuyw += Ghh * i2;
  Gi2 += Ghh * puyw;
  // w' = pw + v3*gg ; s' = ps + b2*gg ; y' = py + b1*gg
  Gpw += g.w;
  Gv3 += g.w * gg;
  Ggg += g.w * v3;
  Gps += g.s;
  Gb2 += g.s * gg;
  Ggg += g.s * b2;
  Gpy += g.y;
  Gb1 += g.y * gg;
  Ggg += g.y * b1;
  // f1 = sy2*i1 ; i1 = 1/a1 ; i2 = 1/a2
  const float Gi1 = Gf1 * p.sy2;
  Ga1 += -Gi1 * i1 * i1;
  Ga2 += -Gi2 * i2 * i2;
  // gg = ry*iSy
  Gry += Ggg * iSy;
  GiSy += Ggg * ry;
  // b2 = v2 + pusw*v3 ; b1 = (pdy + puys*v2) + puyw*v3
  Gv2 += Gb2;
  Gpusw += Gb2 * v3;
  Gv3 += Gb2 * pusw;
  Gpdy += Gb1;
  Gpuys += Gb1 * v2;
  Gv2 += Gb1 * puys;
  Gpuyw += Gb1 * v3;
  Gv3 += Gb1 * puyw;
  // chi2 = ry^2*iSy + rz^2*iSz
  Gry += gchi2 * 2.0f * ry * iSy;
  GiSy += gchi2 * ry * ry;
  Grz += gchi2 * 2.0f * rz * iSz;
  GiSz += gchi2 * rz * rz;
  // iSy = 1/Sy ; iSz = 1/Sz
  const float GSy = -GiSy * iSy * iSy;
  const float GSz = -GiSz * iSz * iSz;
  // ry = my - py ; rz = mz - pz
  *gmy = Gry;
  Gpy += -Gry;
  *gmz = Grz;
  Gpz += -Grz;
  // Sz = z1 + vz*puzt ; z1 = sz2 + pdz ; vz = pdt*puzt
  Gz1 += GSz;
  Gvz += GSz * puzt;
  Gpuzt += GSz * vz;
  Gpdz += Gz1;
  Gpdt += Gvz * puzt;
  Gpuzt += Gvz * pdt;
  // Sy = a2 + v3*puyw ; a2 = a1 + v2*puys ; a1 = sy2 + pdy
  Ga2 += GSy;
  Gv3 += GSy * puyw;
  Gpuyw += GSy * v3;
  Ga1 += Ga2;
  Gv2 += Ga2 * puys;
  Gpuys += Ga2 * v2;
  Gpdy += Ga1;
  // v3 = pdw*puyw ; v2 = pds*puys
  Gpdw += Gv3 * puyw;
  Gpuyw += Gv3 * pdw;
  Gpds += Gv2 * puys;
  Gpuys += Gv2 * pds;

  // ---------------- reverse: propagation
  float gdS = 0.0f, gdy = 0.0f, gdx = 0.0f, ga = 0.0f, gb = 0.0f, ge = 0.0f, gs1 = 0.0f;
  float gx1v = g.x;  // x' = x1
  float oy = 0.0f, oz = 0.0f, os = 0.0f, ot = Gpt, ow = Gpw;
  float ouys = 0.0f, ouyw = 0.0f, ousw = 0.0f, ouzt = 0.0f;
  gs1 += Gps;  // s' = s1
  // puzt = uzt + dS ; pusw = usw + e ; puys = uys + a ; puyw = (uyw + a*usw) + b
  ouzt += Gpuzt;
  gdS += Gpuzt;
  ousw += Gpusw;
  ge += Gpusw;
  ouys += Gpuys;
  ga += Gpuys;
  ouyw += Gpuyw;
  ga += Gpuyw * q.usw;
  ousw += Gpuyw * a;
  gb += Gpuyw;
  // pz = z + t*dS ; py = y + dy
  oz += Gpz;
  ot += Gpz * dS;
  gdS += Gpz * q.t;
  oy += Gpy;
  gdy += Gpy;
  // b = de*qb ; de = dx*e ; qb = nb*icc2 ; nb = cc + ss*r1
  float gde = gb * qb, gqb = gb * de;
  gdx += gde * e;
  ge += gde * dx;
  float gnb = gqb * icc2, gicc2 = gqb * nb;
  float gcc = gnb, gsum = gnb * r1, gr1 = gnb * ss, gr0 = 0.0f;
  // e = -kappa*dx
  gdx += -ge * p.kappa;
  // a = dx*qa ; qa = na*icc2 ; na = 2cc + ss*(r0 + r1)
  gdx += ga * qa;
  const float gqa = ga * dx;
  const float gna = gqa * icc2;
  gicc2 += gqa * na;
  gcc += 2.0f * gna;
  gsum += gna * (r0 + r1);
  gr0 += gna * ss;
  gr1 += gna * ss;
  // icc2 = icc*icc
  float gicc = 2.0f * icc * gicc2;
  // r1 = s1/c1 ; r0 = s/c0
  const float ic1 = k_rcp<true>(c1), ic0 = k_rcp<true>(c0);
  gs1 += gr1 * ic1;
  float gc1 = -gr1 * r1 * ic1;
  os += gr0 * ic0;
  float gc0 = -gr0 * r0 * ic0;
  // dS = sgn * dl * A ; A = 1 + u2*(a1 + u2*a2) ; u2 = u*u ; u = 0.5*ak*dl
  float gdl = gdS * sgn * A;
  const float gA = gdS * sgn * dl;
  const float gu2 = gA * (a1c + 2.0f * a2c * u2);
  const float gu = 2.0f * u * gu2;
  const float gak = 0.5f * gu * dl;
  gdl += 0.5f * gu * ak;
  float gk = gak * (k < 0.0f ? -1.0f : (k > 0.0f ? 1.0f : 0.0f));
  // dl = sqrt(dx^2 + dy^2)
  if (dl > 0.0f) {
    const float idl = k_rcp<true>(dl);
    gdx += gdl * dx * idl;
    gdy += gdl * dy * idl;
  }
  // dy = dx*tg ; tg = ss*icc ; icc = 1/cc
  gdx += gdy * tg;
  const float gtg = gdy * dx;
  gsum += gtg * icc;
  gicc += gtg * ss;
  gcc += -gicc * icc * icc;
  // ss = s + s1 ; cc = c0 + c1
  os += gsum;
  gs1 += gsum;
  gc0 += gcc;
  gc1 += gcc;
  // c1 = sqrt(1 - s1^2) ; c0 = sqrt(1 - s^2)
  gs1 += gc1 * (-s1 * ic1);
  os += gc0 * (-q.s * ic0);
  // s1 = s - kd ; kd = k*dx ; k = kappa*w
  os += gs1;
  const float gkd = -gs1;
  gk += gkd * dx;
  gdx += gkd * k;
  ow += gk * p.kappa;
  // dx = x1 - x
  gx1v += gdx;
  const float ox = -gdx;

  *gx1 = gx1v;
  g.x = ox;
  g.y = oy;
  g.z = oz;
  g.s = os;
  g.t = ot;
  g.w = ow;
  g.uys = ouys;
  g.uyw = ouyw;
  g.usw = ousw;
  g.dy = Gpdy;
  g.ds = Gpds;
  g.dw = Gpdw;
  g.uzt = ouzt;
  g.dz = Gpdz;
  g.dt = Gpdt;
}

// Adds the coefficient gradient of one cluster: the adjoints of its corrected
// (x, y, z) pulled back through the correction and the basis.
__device__ __forceinline__ void add_hit_gradient(const HitGeom& h, float r, float gxc, float gyc,
                                                 float gzc, int wref, long long* win,
                                                 int64_t* __restrict__ acc) {
  const float gdr = (gxc * h.xm + gyc * h.ym) * h.inv_r;
  const float gdp = (-gxc * h.ym + gyc * h.xm) * h.inv_r;
  const float gdz = gzc;
  const Weights4 wp = weights_phi(h.phi);
  const Weights4 wr = weights_lin(r, kMapR0, 1.0f / kMapDR, kMapNR);
  const Weights4 wz = weights_lin(h.zm, kMapZ0, 1.0f / kMapDZ, kMapNZ);
  // r and z nodes clamped into the map: a node outside has weight 0, so its
  // terms are 0 and add nothing; the node loops then run without branches
  int jj[4], kk[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) jj[b] = min(max(wr.first + b, 0), kMapNR - 1);
#pragma unroll
  for (int c = 0; c < 4; ++c) kk[c] = min(max(wz.first + c, 0), kMapNZ - 1);
  constexpr int kWinComp = kWinPhi * kMapNR * kMapNZ;
  for (int a = 0; a < 4; ++a) {
    // (selected, not indexed: the weights stay in registers)
    const float wpa = a == 0 ? wp.w[0] : a == 1 ? wp.w[1] : a == 2 ? wp.w[2] : wp.w[3];
    const int i = ((wp.first + a) % kMapNPhi + kMapNPhi) % kMapNPhi;
    int rel = i - wref;
    if (rel > kMapNPhi / 2) rel -= kMapNPhi;
    if (rel <= -kMapNPhi / 2) rel += kMapNPhi;
    rel += kWinPhi / 2;
    if (rel >= 0 && rel < kWinPhi) {
      long long* wa = win + rel * (kMapNR * kMapNZ);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const float wab = wpa * wr.w[b];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float w = wab * wz.w[c];
          const float g3[3] = {gdr * w, gdp * w, gdz * w};
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const long long v = llrint(double(g3[q]) * kFixScale);
            if (v != 0)
              atomicAdd(reinterpret_cast<unsigned long long*>(&wa[q * kWinComp + jj[b] * kMapNZ + kk[c]]),
                        static_cast<unsigned long long>(v));
          }
        }
      }
    } else {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const float wab = wpa * wr.w[b];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float w = wab * wz.w[c];
          const float g3[3] = {gdr * w, gdp * w, gdz * w};
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const long long v = llrint(double(g3[q]) * kFixScale);
            if (v != 0)
              atomicAdd(reinterpret_cast<unsigned long long*>(&acc[map_index(q, i, jj[b], kk[c])]),
                        static_cast<unsigned long long>(v));
          }
        }
      }
    }
  }
}

// Backward, part 1: the reverse sweep, one lane per track in blocks of one
// wavefront (a few hundred tracks already spread over every compute unit).
// Recomputes one kCkpt-cluster segment at a time from its checkpoint into the
// lane's scratch, runs the reverse of every step and writes the adjoint of
// each hit's corrected (x, y, z) to hgrad (zero for tracks without gradient).
__global__ void __launch_bounds__(kWave) k_refit_bwd_sweep(RefitIn in, DevParams p, RefitWs ws,
                                                           const float* __restrict__ dL_dchi2,
                                                           const int32_t* __restrict__ ok_in) {
  const int64_t t = int64_t(blockIdx.x) * kWave + threadIdx.x;
  if (t >= in.n_tracks) return;
  const int64_t hb = in.hit_begin[t];
  const int n = track_size(in, t);
  float4* hg = reinterpret_cast<float4*>(ws.hgrad) + hb;
  if (!ok_in[t] || dL_dchi2[t] == 0.0f) {
    for (int i = 0; i < n; ++i) hg[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    return;
  }
  const float gchi2 = dL_dchi2[t];
  const int64_t cb = ckpt_base(in, t);
  float* scr = ws.scratch + t % ws.n_lanes * (kCkpt * kCkptFloats);
  const float4* xyz = reinterpret_cast<const float4*>(ws.xyz);
  const float zref = xyz[hb].z;
  KBar g{};
  const int nseg = (n - 2) / kCkpt + 1;  // segments covering steps 1..n-1
  for (int m = nseg - 1; m >= 0; --m) {
    const int i_lo = m * kCkpt;
    const int i_hi = min((m + 1) * kCkpt, n - 1);
    // recompute the segment's states S_{i_lo} .. S_{i_hi - 1}
    KState q = load_state(ws.ckpt + (cb + m) * kCkptFloats);
    for (int i = i_lo; i < i_hi; ++i) {
      store_state(scr + (i - i_lo) * kCkptFloats, q);
      if (i + 1 < i_hi) {
        const float4 h = xyz[hb + i + 1];
        float dummy = 0.0f;
        refit_step(q, h.x, h.y, rel_z(h, zref), p, &dummy);
      }
    }
    // reverse sweep over the segment's steps i = i_hi .. i_lo + 1
    for (int i = i_hi; i > i_lo; --i) {
      const KState prev = load_state(scr + (i - 1 - i_lo) * kCkptFloats);
      const float4 h = xyz[hb + i];
      float gx1, gmy, gmz;
      refit_step_reverse(prev, h.x, h.y, rel_z(h, zref), p, gchi2, g, &gx1, &gmy, &gmz);
      hg[i] = make_float4(gx1, gmy, gmz, 0.0f);
    }
  }
  // the first cluster seeds x, y, z of the state
  hg[0] = make_float4(g.x, g.y, g.z, 0.0f);
}

// Backward, part 2: every hit's adjoints pulled back through the correction
// and the basis onto the coefficients.  A block takes the hits of
// kScatterTracks consecutive tracks and sums in 64-bit fixed point, first in
// an LDS window of kWinPhi phi nodes around its first track's sector, then
// into the global accumulators; the sums do not depend on the order.
constexpr int kScatterTracks = 64;

__global__ void __launch_bounds__(kRefitBlock) k_refit_bwd_scatter(RefitIn in, RefitWs ws) {
  extern __shared__ long long win[];  // [3][kWinPhi][17][20]
  __shared__ int64_t hb[kScatterTracks + 1];
  __shared__ float al[kScatterTracks];
  const int nwin = kMapComp * kWinPhi * kMapNR * kMapNZ;
  for (int i = threadIdx.x; i < nwin; i += blockDim.x) win[i] = 0;
  const int64_t t0 = int64_t(blockIdx.x) * kScatterTracks;
  const int cnt = int(min(int64_t(kScatterTracks), in.n_tracks - t0));
  const int tid = threadIdx.x;
  if (tid <= cnt) hb[tid] = in.hit_begin[t0 + tid];
  if (tid < cnt) al[tid] = in.unit_alpha[in.unit[t0 + tid]];
  __syncthreads();
  // reference phi node: the sector centre of the block's first track
  float ph = fmodf(al[0], 6.28318530717958647692f);
  if (ph < 0.0f) ph += 6.28318530717958647692f;
  const int wref = int(floorf(ph / kMapDPhi));
  // the lanes of a wavefront take the hits of 64 different tracks (thread
  // tid: track tid % 64, every (blockDim / 64)-th hit of it): consecutive
  // hits of one track share most of their 64 nodes, and same-address LDS
  // atomics of one instruction are serialised
  const float4* hg = reinterpret_cast<const float4*>(ws.hgrad);
  const int trk = tid % kScatterTracks, nsub = blockDim.x / kScatterTracks;
  if (trk < cnt) {
    for (int64_t q = hb[trk] + tid / kScatterTracks; q < hb[trk + 1]; q += nsub) {
      const float4 g = hg[q];
      if (g.x == 0.0f && g.y == 0.0f && g.z == 0.0f) continue;
      float r;
      const HitGeom h = hit_geom(in.row_x[in.hit_row[q]], in.y[in.hit_id[q]], in.z[in.hit_id[q]], al[trk], &r);
      add_hit_gradient(h, r, g.x, g.y, g.z, wref, win, ws.acc);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nwin; i += blockDim.x) {
    const long long v = win[i];
    if (v == 0) continue;
    const int k = i % kMapNZ;
    const int j = (i / kMapNZ) % kMapNR;
    const int rel = (i / (kMapNZ * kMapNR)) % kWinPhi;
    const int qq = i / (kMapNZ * kMapNR * kWinPhi);
    const int ii = ((wref + rel - kWinPhi / 2) % kMapNPhi + kMapNPhi) % kMapNPhi;
    atomicAdd(reinterpret_cast<unsigned long long*>(&ws.acc[map_index(qq, ii, j, k)]),
              static_cast<unsigned long long>(v));
  }
}

__global__ void k_grad_finalize(const int64_t* __restrict__ acc, float* __restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMapNCoef) grad[i] = float(double(acc[i]) * (1.0 / kFixScale));
}

}  // namespace tpcx
