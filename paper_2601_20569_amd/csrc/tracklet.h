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

// State at plane x: (y, z, s = sin(phi), t = dz/ds, w = q/pT), covariance
// blocks (y, s, w) and (z, t).
struct KState {
  float x, y, z, s, t, w;
  float cyy, csy, css, cwy, cws, cww;
  float czz, ctz, ctt;
};

// asin(u)/u to third order in u^2 (u <= 0.1 keeps the dropped term < 5e-8).
__device__ __forceinline__ float arc_chord_ratio(float u) {
  const float a1 = 0.16666667f;   // 1/6 rounded to float
  const float a2 = 0.075f;        // 3/40 rounded to float
  const float u2 = u * u;
  return 1.0f + u2 * (a1 + u2 * a2);
}

// Exact circle step to the plane x1 with the linearised covariance transport.
// Returns false (state unchanged) when |sin(phi)| would reach smax or the
// chord is too long.
__device__ __forceinline__ bool kf_propagate(KState& q, float x1, const DevParams& p) {
  const float dx = x1 - q.x;
  const float k = p.kappa * q.w;
  const float s1 = q.s - k * dx;
  if (!(fabsf(s1) < p.smax)) return false;
  const float c0 = sqrtf(1.0f - q.s * q.s);
  const float c1 = sqrtf(1.0f - s1 * s1);
  const float cc = c0 + c1;
  const float ss = q.s + s1;
  const float tg = ss / cc;
  const float dy = dx * tg;
  const float dl = sqrtf(dx * dx + dy * dy);
  const float u = (fabsf(k) * dl) * 0.5f;
  if (!(u <= p.umax)) return false;
  float dS = dl * arc_chord_ratio(u);
  if (dx < 0.0f) dS = -dS;
  const float r0 = q.s / c0;
  const float r1 = s1 / c1;
  const float cc2 = cc * cc;
  const float a = dx * ((2.0f * cc + ss * (r0 + r1)) / cc2);
  const float e = -(p.kappa * dx);
  const float b = (dx * e) * ((cc + ss * r1) / cc2);
  const float Py = (q.cyy + a * q.csy) + b * q.cwy;
  const float Ps = (q.csy + a * q.css) + b * q.cws;
  const float Pw = (q.cwy + a * q.cws) + b * q.cww;
  const float Qy = q.csy + e * q.cwy;
  const float Qs = q.css + e * q.cws;
  const float Qw = q.cws + e * q.cww;
  q.cyy = (Py + a * Ps) + b * Pw;
  q.csy = (Qy + a * Qs) + b * Qw;
  q.cwy = Pw;
  q.css = Qs + e * Qw;
  q.cws = Qw;
  const float Rz = q.czz + dS * q.ctz;
  const float Rt = q.ctz + dS * q.ctt;
  q.czz = Rz + dS * Rt;
  q.ctz = Rt;
  q.y = q.y + dy;
  q.z = q.z + q.t * dS;
  q.s = s1;
  q.x = x1;
  return true;
}

__device__ __forceinline__ float kf_chi2(const KState& q, float my, float mz, const DevParams& p) {
  const float ry = my - q.y;
  const float rz = mz - q.z;
  const float Sy = q.cyy + p.sy2;
  const float Sz = q.czz + p.sz2;
  return (ry * ry) / Sy + (rz * rz) / Sz;
}

__device__ __forceinline__ float kf_update(KState& q, float my, float mz, const DevParams& p) {
  const float ry = my - q.y;
  const float rz = mz - q.z;
  const float Sy = q.cyy + p.sy2;
  const float Sz = q.czz + p.sz2;
  const float chi2 = (ry * ry) / Sy + (rz * rz) / Sz;
  const float k0 = q.cyy / Sy, k1 = q.csy / Sy, k2 = q.cwy / Sy;
  q.y = q.y + k0 * ry;
  q.s = q.s + k1 * ry;
  q.w = q.w + k2 * ry;
  const float cyy = q.cyy, csy = q.csy, cwy = q.cwy;
  q.cyy = cyy - k0 * cyy;
  q.csy = csy - k1 * cyy;
  q.cwy = cwy - k2 * cyy;
  q.css = q.css - k1 * csy;
  q.cws = q.cws - k2 * csy;
  q.cww = q.cww - k2 * cwy;
  const float kz0 = q.czz / Sz, kz1 = q.ctz / Sz;
  q.z = q.z + kz0 * rz;
  q.t = q.t + kz1 * rz;
  const float czz = q.czz, ctz = q.ctz;
  q.czz = czz - kz0 * czz;
  q.ctz = ctz - kz1 * czz;
  q.ctt = q.ctt - kz1 * ctz;
  return chi2;
}

// Best cluster of row r by (chi2, caller id) among chi2 <= chi2max, or -1.
// The grid box is |dy| <= 4 sqrt(Sy) (and z alike), widened to be exact.
__device__ __forceinline__ int32_t kf_search(const Grid& g, int u, int r, const KState& q,
                                             const DevParams& p, float* out_my, float* out_mz) {
  const int k = u * g.n_rows + r;
  const float Sy = q.cyy + p.sy2;
  const float Sz = q.czz + p.sz2;
  const float hy = sqrtf(p.chi2max * Sy) * 1.0001f + box_pad(q.y);
  const float hz = sqrtf(p.chi2max * Sz) * 1.0001f + box_pad(q.z);
  const int zb0 = g.zbin(k, q.z - hz), zb1 = g.zbin(k, q.z + hz);
  const int yb0 = g.ybin(r, q.y - hy), yb1 = g.ybin(r, q.y + hy);
  const int64_t base = g.row_base(k);
  const int ny = g.rows[r].ny;
  int32_t best = -1;
  float bch = 0.0f, bmy = 0.0f, bmz = 0.0f;
  for (int zb = zb0; zb <= zb1; ++zb) {
    const int32_t j0 = g.bin_start[base + zb * ny + yb0], j1 = g.bin_start[base + zb * ny + yb1 + 1];
    for (int32_t j = j0; j < j1; ++j) {
      const float my = g.sy[j], mz = g.sz[j];
      const float ch = kf_chi2(q, my, mz, p);
      if (!(ch <= p.chi2max)) continue;
      const int32_t id = g.sid[j];
      if (best < 0 || ch < bch || (ch == bch && id < best)) {
        best = id;
        bch = ch;
        bmy = my;
        bmz = mz;
      }
    }
  }
  *out_my = bmy;
  *out_mz = bmz;
  return best;
}

// Per-start-hit results before compaction (structure of arrays, cap entries).
struct TrackletTmp {
  int64_t cap;
  int32_t* n;        // clusters attached
  int32_t* n_up;     // of which at or above the start row
  int32_t* flags;    // bit 0: the walk back to the start row failed
  int32_t* unit;
  float* f;          // [16][cap]: x_ref, y, z, s, t, w, cyy, csy, css, cwy, cws, cww, czz, ctz, ctt, chi2
  int32_t* hit;      // [cap][n_rows]: up-phase ids from slot 0, down-phase from the end
  uint8_t* hrow;     // [cap][n_rows]
};

constexpr int kFlagDescentFailed = 1;

struct TrackInputs {
  const int64_t* row_begin;
  int n_units;
  const float* y;  // caller order
  const float* z;
  const int32_t* clean_up;
  const int32_t* starts;
  const float* row_x;  // [n_rows]
};

__device__ void build_tracklet(int64_t s, const TrackInputs& in, const Grid& g, const DevParams& p,
                               const TrackletTmp& out) {
  const int R = g.n_rows;
  const int32_t h0 = in.starts[s];
  const int k = upper_row(in.row_begin, in.n_units * R + 1, h0);
  const int u = k / R, r0 = k % R;
  int32_t* hits = out.hit + s * R;
  uint8_t* hrow = out.hrow + s * R;

  // 2-point seed at the second cluster of the chain
  const int32_t c0 = h0, c1 = in.clean_up[h0];
  KState q;
  const float dx = in.row_x[r0 + 1] - in.row_x[r0];
  const float dy = in.y[c1] - in.y[c0];
  const float dz = in.z[c1] - in.z[c0];
  const float dl = sqrtf(dx * dx + dy * dy);
  q.x = in.row_x[r0 + 1];
  q.y = in.y[c1];
  q.z = in.z[c1];
  q.s = dy / dl;
  q.t = dz / dl;
  q.w = 0.0f;
  q.cyy = p.sy2;
  q.csy = p.sy2 / dl;
  q.css = (p.sy2 + p.sy2) / (dl * dl);
  q.cwy = 0.0f;
  q.cws = 0.0f;
  q.cww = p.cww0;
  q.czz = p.sz2;
  q.ctz = p.sz2 / dl;
  q.ctt = (p.sz2 + p.sz2) / (dl * dl);
  float chi2 = 0.0f;
  int n_up = 0, n_dn = 0;
  hits[n_up] = c0;
  hrow[n_up++] = uint8_t(r0);
  hits[n_up] = c1;
  hrow[n_up++] = uint8_t(r0 + 1);
  int row = r0 + 1;

  // rest of the chain, attached without a cut
  bool up_ok = true;
  for (int32_t c = in.clean_up[c1]; c >= 0; c = in.clean_up[c]) {
    const int rr = row + 1;
    if (!kf_propagate(q, in.row_x[rr], p)) {
      up_ok = false;
      break;
    }
    chi2 = chi2 + kf_update(q, in.y[c], in.z[c], p);
    hits[n_up] = c;
    hrow[n_up++] = uint8_t(rr);
    row = rr;
  }
  KState best = q;
  int best_row = row;

  // outward following
  if (up_ok) {
    int misses = 0;
    for (int rr = row + 1; rr < R; ++rr) {
      if (!kf_propagate(q, in.row_x[rr], p)) break;
      float my, mz;
      const int32_t c = kf_search(g, u, rr, q, p, &my, &mz);
      if (c >= 0) {
        chi2 = chi2 + kf_update(q, my, mz, p);
        hits[n_up] = c;
        hrow[n_up++] = uint8_t(rr);
        best = q;
        best_row = rr;
        misses = 0;
      } else if (++misses == p.max_misses) {
        break;
      }
    }
  }

  // back to the start row, then inward following
  q = best;
  bool down_ok = true;
  for (int rr = best_row - 1; rr >= r0; --rr) {
    if (!kf_propagate(q, in.row_x[rr], p)) {
      down_ok = false;
      break;
    }
  }
  KState res = best;
  int flags = 0;
  if (!down_ok) {
    flags |= kFlagDescentFailed;
  } else {
    res = q;
    int misses = 0;
    for (int rr = r0 - 1; rr >= 0; --rr) {
      if (!kf_propagate(q, in.row_x[rr], p)) break;
      float my, mz;
      const int32_t c = kf_search(g, u, rr, q, p, &my, &mz);
      if (c >= 0) {
        chi2 = chi2 + kf_update(q, my, mz, p);
        hits[R - 1 - n_dn] = c;
        hrow[R - 1 - n_dn] = uint8_t(rr);
        ++n_dn;
        res = q;
        misses = 0;
      } else if (++misses == p.max_misses) {
        break;
      }
    }
  }

  const int64_t C = out.cap;
  out.n[s] = n_up + n_dn;
  out.n_up[s] = n_up;
  out.flags[s] = flags;
  out.unit[s] = u;
  const float v[16] = {res.x,   res.y,   res.z,   res.s,   res.t,   res.w,   res.cyy, res.csy,
                       res.css, res.cwy, res.cws, res.cww, res.czz, res.ctz, res.ctt, chi2};
#pragma unroll
  for (int j = 0; j < 16; ++j) out.f[j * C + s] = v[j];
}

// Work-queue driven constructor: each wavefront takes 64 start hits at a time.
__global__ void k_construct(const int64_t* __restrict__ counts, int64_t cap_start,
                            int32_t* __restrict__ queue, TrackInputs in, Grid g, DevParams p,
                            TrackletTmp out) {
  const int64_t n_start = counts[0] < cap_start ? counts[0] : cap_start;
  while (true) {
    int32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(queue, kWave);
    base = __shfl(base, 0, kWave);
    if (base >= n_start) break;
    const int64_t s = int64_t(base) + lane_id();
    if (s < n_start) build_tracklet(s, in, g, p, out);
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
                             const int32_t* __restrict__ tn, int min_hits,
                             int64_t* __restrict__ part) {
  __shared__ int64_t lds[1024 / kWave];
  const int64_t n_start = counts[0] < cap_start ? counts[0] : cap_start;
  int64_t b, e;
  chunk_of(n_start, &b, &e);
  int64_t ct = 0, ch = 0;
  for (int64_t s = b + threadIdx.x; s < e; s += blockDim.x) {
    const int32_t n = tn[s];
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

__global__ void k_keep_scan(int64_t* __restrict__ part, int nb, int64_t* __restrict__ counts,
                            int64_t cap_tracks, int64_t cap_hits) {
  if (threadIdx.x != 0) return;
  int64_t t = 0, h = 0;
  for (int i = 0; i < nb; ++i) {
    const int64_t a = part[2 * i], c = part[2 * i + 1];
    part[2 * i] = t;
    part[2 * i + 1] = h;
    t += a;
    h += c;
  }
  counts[1] = t;
  counts[2] = h;
  unsigned long long st = 0;
  if (t > cap_tracks) st |= 2ull;
  if (h > cap_hits) st |= 4ull;
  if (st) atomicOr((unsigned long long*)&counts[3], st);
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
    TrackletTmp tmp, int n_rows, int min_hits, const int64_t* __restrict__ part, TrackOut o) {
  __shared__ int64_t lds[kKeepBlock / kWave];
  __shared__ int64_t s_hb[kKeepBlock];
  __shared__ int32_t s_slot[kKeepBlock];
  __shared__ int32_t s_n[kKeepBlock];
  __shared__ int32_t s_nu[kKeepBlock];
  const int64_t n_start = counts[0] < cap_start ? counts[0] : cap_start;
  int64_t b, e;
  chunk_of(n_start, &b, &e);
  int64_t t_run = part[2 * blockIdx.x], h_run = part[2 * blockIdx.x + 1];
  const int64_t C = tmp.cap;
  const int wid = threadIdx.x / kWave, nw = kKeepBlock / kWave;
  for (int64_t s0 = b; s0 < e; s0 += kKeepBlock) {
    const int64_t s = s0 + threadIdx.x;
    int32_t n = 0;
    bool keep = false;
    if (s < e) {
      n = tmp.n[s];
      keep = n >= min_hits;
    }
    int64_t tt, th;
    const int64_t pt = block_exclusive_scan(keep ? 1 : 0, lds, &tt);
    const int64_t ph = block_exclusive_scan(keep ? n : 0, lds, &th);
    bool fits = false;
    if (keep) {
      const int64_t ti = t_run + pt, hb = h_run + ph;
      fits = ti < o.cap_tracks && hb + n <= o.cap_hits;
      if (fits) {
        o.unit[ti] = tmp.unit[s];
        o.start[ti] = starts[s];
        o.n_hits[ti] = n;
        o.hit_begin[ti] = hb;
        o.ndf[ti] = 2 * n - 5;
        o.x_ref[ti] = tmp.f[0 * C + s];
        for (int j = 0; j < 5; ++j) o.param[ti * 5 + j] = tmp.f[(1 + j) * C + s];
        const float cyy = tmp.f[6 * C + s], csy = tmp.f[7 * C + s], css = tmp.f[8 * C + s];
        const float cwy = tmp.f[9 * C + s], cws = tmp.f[10 * C + s], cww = tmp.f[11 * C + s];
        const float czz = tmp.f[12 * C + s], ctz = tmp.f[13 * C + s], ctt = tmp.f[14 * C + s];
        const float cv[15] = {cyy, 0.0f, czz, csy, 0.0f, css, 0.0f, ctz,
                              0.0f, ctt, cwy, 0.0f, cws, 0.0f, cww};
        for (int j = 0; j < 15; ++j) o.cov[ti * 15 + j] = cv[j];
        o.chi2[ti] = tmp.f[15 * C + s];
      }
      s_slot[pt] = fits ? int32_t(s - s0) : -1;
      s_hb[pt] = hb;
      s_n[pt] = n;
      s_nu[pt] = tmp.n_up[s];
    }
    __syncthreads();
    // hit lists: down-phase clusters sit at the end of the slot in ascending
    // row order, up-phase clusters at its start
    for (int q = wid; q < int(tt); q += nw) {
      const int32_t sl = s_slot[q];
      if (sl < 0) continue;
      const int64_t ss = s0 + sl;
      const int nn = s_n[q], nu = s_nu[q], nd = nn - nu;
      const int64_t hb = s_hb[q];
      const int32_t* hs = tmp.hit + ss * n_rows;
      const uint8_t* rs = tmp.hrow + ss * n_rows;
      for (int j = lane_id(); j < nn; j += kWave) {
        const int src = j < nd ? n_rows - nd + j : j - nd;
        o.hit_id[hb + j] = hs[src];
        o.hit_row[hb + j] = rs[src];
      }
    }
    __syncthreads();
    t_run += tt;
    h_run += th;
  }
}

}  // namespace tpcx
