// Track rebuild of the fit (paper, Section 3, Phase II): iteration 2 queries
// the cluster search grid for every cluster compatible with the chi2 cut
// against the interpolation and keeps the candidates with their chi2; a
// second ambiguity solving hands candidates to tracks by rank, a track that
// loses its best candidate taking its next; iteration 3 fits the result with
// a plain chi2 cut.
//
// k_rebuild_pass12: one lane per track.  Iteration 1 (from the tracking
// result out to the outermost cluster, then row by row inwards) stores the
// predicted y, z (binary32, relative to the outermost cluster) and C_yy, C_zz
// (bfloat16) of every row, updating with the track's own clusters.
// Iteration 2 (restart at the innermost cluster, row by row outwards)
// interpolates, scans the grid box of every row for clusters with chi2 <=
// cut, keeps the K best by (chi2, caller id) and updates with the best.
// k_rebuild_propose / k_rebuild_advance: R rounds of proposals; a cluster's
// holder is the atomic maximum of its proposers' 64-bit rank keys, so the
// result does not depend on the order of the atomics.  Only a (track, row)
// whose candidate changed proposes again (a key once proposed stays below
// the holder's, which only grows), and only the tracks that proposed or
// lost a cluster to a proposer (whose key the atomic returns) check what
// they hold: every other track still holds what it held.
// k_rebuild_pass3: iteration 3 over the rows whose candidate the track holds.
// IEEE binary32, no contraction, correctly rounded divide and square root.
#pragma once

#include "fit.h"
#include "select.h"
#include "tpcx_common.h"
#include "tracklet.h"

namespace tpcx {

constexpr int kRebuildK = 4;  // candidates kept per (track, row)
// ptr byte of a (track, row): the current candidate in the low bits, and
// kPtrMoved while that candidate has not been proposed yet
constexpr uint8_t kPtrMoved = 0x80;

struct RebuildIn {
  int64_t n_tracks;
  int64_t n_hits;
  int64_t n_clusters;
  int n_rows;
  int n_units;
  const int32_t* unit;
  const int64_t* hit_begin;
  const int32_t* hit_id;
  const uint8_t* hit_row;
  const float* seed;   // [n][5]
  const float* x_ref;  // [n]
  const float* chi2;   // [n] tracking result (rank)
  const int32_t* ndf;  // [n]
  const float* y;
  const float* z;
  const float* row_x;
};

struct RebuildWs {
  float4* pred;              // [n][n_rows] predicted y, z, bf16(C_yy) | bf16(C_zz) << 16, -
  int2* cand;                // [n][n_rows][kRebuildK] caller id, chi2 bits
  uint8_t* cnt;              // [n][n_rows] candidates kept
  uint8_t* ptr;              // [n][n_rows] current candidate
  float* state;              // [n][16] iteration 2's final state (KState), oy, oz
  int32_t* meta;             // [n][4] ok, r_in, r_out
  uint64_t* key;             // [n] rank key
  unsigned long long* holder;  // [n_clusters]
  int64_t* first;            // [n] first track of the track's unit
  uint8_t* active;           // [n] the track has candidates to propose this round
  uint8_t* check;            // [n] the track must check what it holds this round
};

struct RebuildOut {
  int32_t* assigned;  // [n][n_rows]
  float* param;
  float* cov;
  float* chi2;
  float* x_out;
  int32_t* n_kept;
  int32_t* ok;
};

struct RebuildConsts {
  float chi2_cut, chi2_final, vs, vt, vw;
  int rounds;
  int extrapolate;    // Phase III: candidates also beyond the track's ends
  float chi2_extrap;  // their chi2 cut
};

__device__ __forceinline__ void rb_reset(KState& q, const DevParams& p, const RebuildConsts& f) {
  q.uys = 0.0f;
  q.uyw = 0.0f;
  q.usw = 0.0f;
  q.dy = p.sy2;
  q.ds = f.vs;
  q.dw = f.vw;
  q.uzt = 0.0f;
  q.dz = p.sz2;
  q.dt = f.vt;
}

// rank key (as in the ambiguity solving) of every track; local index from
// the first track of its unit (tracks are in unit order)
__global__ void k_rebuild_keys(RebuildIn in, uint64_t* __restrict__ key, int64_t* __restrict__ first,
                               uint8_t* __restrict__ active, uint8_t* __restrict__ check) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= in.n_tracks) return;
  const int32_t u = in.unit[t];
  int64_t lo = 0, hi = t;  // first track of unit u
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (in.unit[mid] < u) lo = mid + 1; else hi = mid;
  }
  const float q = in.chi2[t] / float(in.ndf[t]);
  const int n = int(in.hit_begin[t + 1] - in.hit_begin[t]);
  const int64_t local = t - lo;
  key[t] = uint64_t(~__float_as_uint(q)) << 32 | uint64_t(uint32_t(min(n, 255)) << 24 |
                                                          uint32_t(kSelectMaxPerUnit - 1 - min(local, kSelectMaxPerUnit - 1)));
  first[t] = lo;
  active[t] = 1;
  check[t] = 0;
}

// The candidates of row r of unit row base kb against the prediction (iy,
// iz) (relative to (oy, oz)) with variances (vy, vz): chi2 <= cut, the
// kRebuildK best by (chi2, caller id) into cand; returns their number and the
// best one's id in *best (-1 if none).
__device__ __forceinline__ int rb_row_candidates(const Grid& g, const DevParams& p, int kb, int r, float oy,
                                                 float oz, float iy, float iz, float vy, float vz, float cut,
                                                 int2* cand, int32_t* best) {
  const float sy = vy + p.sy2, sz = vz + p.sz2;
  // the grid box around the interpolation, widened to hold every cluster
  // the float chi2 cut can accept
  const float cy_abs = oy + iy, cz_abs = oz + iz;
  const float hy = __builtin_amdgcn_sqrtf(cut * sy) * 1.001f + box_pad(cy_abs);
  const float hz = __builtin_amdgcn_sqrtf(cut * sz) * 1.001f + box_pad(cz_abs);
  const RowView rv(g, kb + r, r);
  const int zb0 = rv.zbin(cz_abs - hz), zb1 = rv.zbin(cz_abs + hz);
  const int yb0 = rv.ybin(cy_abs - hy), yb1 = rv.ybin(cy_abs + hy);
  // K best (chi2, id), ascending
  float bc[kRebuildK];
  int32_t bi[kRebuildK];
  int nb = 0;
  for (int zb = zb0; zb <= zb1; ++zb) {
    const int64_t ra = rv.base + int64_t(zb) * rv.ri.ny;
    const int32_t j0 = g.bin_start[ra + yb0], j1 = g.bin_start[ra + yb1 + 1];
    for (int32_t j = j0; j < j1; ++j) {
      const float4 pc = g.pts[j];
      const float dy = (pc.x - oy) - iy, dz = (pc.y - oz) - iz;
      const float ch = (dy * dy) / sy + (dz * dz) / sz;
      if (!(ch <= cut)) continue;
      const int32_t id = __float_as_int(pc.z);
      // insertion into the sorted top-K
      int pos = nb;
      while (pos > 0 && (ch < bc[pos - 1] || (ch == bc[pos - 1] && id < bi[pos - 1]))) --pos;
      if (pos >= kRebuildK) continue;
      for (int m = min(nb, kRebuildK - 1); m > pos; --m) {
        bc[m] = bc[m - 1];
        bi[m] = bi[m - 1];
      }
      bc[pos] = ch;
      bi[pos] = id;
      nb = min(nb + 1, kRebuildK);
    }
  }
  for (int m = 0; m < nb; ++m) cand[m] = make_int2(bi[m], __float_as_int(bc[m]));
  *best = nb > 0 ? bi[0] : -1;
  return nb;
}

__global__ void __launch_bounds__(kWave) k_rebuild_pass12(RebuildIn in, Grid g, DevParams p, RebuildConsts f,
                                                          RebuildWs ws) {
  const int64_t t = int64_t(blockIdx.x) * kWave + threadIdx.x;
  if (t >= in.n_tracks) return;
  const int R = in.n_rows;
  const int64_t b = in.hit_begin[t];
  const int n = int(in.hit_begin[t + 1] - b);
  int32_t* meta = ws.meta + 4 * t;
  meta[0] = 0;
  if (n < 3 || b < 0 || b + n > in.n_hits || in.unit[t] < 0 || in.unit[t] >= in.n_units) return;
  // a track whose list breaks the input contract (rows strictly ascending
  // and inside the geometry, ids inside the cluster array) fails
  for (int i = 0; i < n; ++i) {
    const int r = in.hit_row[b + i];
    const int32_t h = in.hit_id[b + i];
    if (r >= R || (i > 0 && r <= in.hit_row[b + i - 1]) || h < 0 || h >= in.n_clusters) return;
  }
  const int r_in = in.hit_row[b], r_out = in.hit_row[b + n - 1];
  float4* pred = ws.pred + t * R;
  uint8_t* cnt = ws.cnt + t * R;
  uint8_t* ptr = ws.ptr + t * R;
  int2* cand = ws.cand + t * R * kRebuildK;
  const int kb = in.unit[t] * R;
  const float oy = in.y[in.hit_id[b + n - 1]], oz = in.z[in.hit_id[b + n - 1]];
  auto X = [&](int r) { return in.row_x[r]; };
  // ---- iteration 1
  const float* sd = in.seed + 5 * t;
  const float xref = in.x_ref[t];
  KState q{};
  q.x = xref;
  q.y = sd[0] - oy;
  q.z = sd[1] - oz;
  q.s = sd[2];
  q.t = sd[3];
  q.w = sd[4];
  rb_reset(q, p, f);
  for (int i = 0; i < n; ++i) {
    const float xi = X(in.hit_row[b + i]);
    if (xi > xref && !(q.x == xi) && !fit_prop(q, xi, p)) return;
  }
  if (!(q.x == X(r_out)) && !fit_prop(q, X(r_out), p)) return;
  q.y = 0.0f;
  q.z = 0.0f;
  rb_reset(q, p, f);
  int hi = n - 2;  // next own cluster inwards
  for (int r = r_out - 1; r >= r_in; --r) {
    if (!fit_prop(q, X(r), p)) return;
    const uint32_t cc = bf16_bits(fit_cyy(q)) | (bf16_bits(fit_czz(q)) << 16);
    pred[r] = make_float4(q.y, q.z, __uint_as_float(cc), 0.0f);
    if (hi >= 0 && in.hit_row[b + hi] == r) {
      const int32_t h = in.hit_id[b + hi];
      fit_update(q, in.y[h] - oy, in.z[h] - oz, p);
      --hi;
    }
  }
  const float s1 = q.s, t1 = q.t, w1 = q.w;
  // Phase III inwards: the state of r_in carried further in, row by row,
  // without updates, until the first row or a propagation guard
  int r_lo = r_in;
  if (f.extrapolate) {
    KState ex = q;
    for (int r = r_in - 1; r >= 0; --r) {
      if (!fit_prop(ex, X(r), p)) break;
      const uint32_t cc = bf16_bits(fit_cyy(ex)) | (bf16_bits(fit_czz(ex)) << 16);
      pred[r] = make_float4(ex.y, ex.z, __uint_as_float(cc), 0.0f);
      r_lo = r;
    }
  }
  // ---- iteration 2
  // rows below the track: the inward extrapolation alone
  for (int r = r_lo; r < r_in; ++r) {
    const float4 pr = pred[r];
    const uint32_t cc = __float_as_uint(pr.z);
    int32_t best = -1;
    cnt[r] = uint8_t(rb_row_candidates(g, p, kb, r, oy, oz, pr.x, pr.y, bf16_lo(cc), bf16_hi(cc), f.chi2_extrap,
                                       cand + r * kRebuildK, &best));
    ptr[r] = kPtrMoved;
  }
  q = KState{};
  q.x = X(r_in);
  q.y = in.y[in.hit_id[b]] - oy;
  q.z = in.z[in.hit_id[b]] - oz;
  q.s = s1;
  q.t = t1;
  q.w = w1;
  rb_reset(q, p, f);
  for (int r = r_in; r <= r_out; ++r) {
    if (r > r_in && !fit_prop(q, X(r), p)) return;
    float iy, iz, vy, vz;
    if (r == r_in) {
      const float4 pr = pred[r];
      const uint32_t cc = __float_as_uint(pr.z);
      iy = pr.x;
      iz = pr.y;
      vy = bf16_lo(cc);
      vz = bf16_hi(cc);
    } else {
      const float cy = fit_cyy(q), cz = fit_czz(q);
      if (r == r_out) {
        iy = q.y;
        iz = q.z;
        vy = cy;
        vz = cz;
      } else {
        const float4 pr = pred[r];
        const uint32_t cc = __float_as_uint(pr.z);
        const float pcy = bf16_lo(cc), pcz = bf16_hi(cc);
        const float wy = 1.0f / (pcy + cy);
        const float wz = 1.0f / (pcz + cz);
        iy = (pr.x * cy + q.y * pcy) * wy;
        iz = (pr.y * cz + q.z * pcz) * wz;
        vy = (pcy * cy) * wy;
        vz = (pcz * cz) * wz;
      }
    }
    int32_t best = -1;
    const int nb = rb_row_candidates(g, p, kb, r, oy, oz, iy, iz, vy, vz, f.chi2_cut, cand + r * kRebuildK, &best);
    cnt[r] = uint8_t(nb);
    ptr[r] = kPtrMoved;
    if (r > r_in && nb > 0) fit_update(q, in.y[best] - oy, in.z[best] - oz, p);
  }
  // Phase III outwards: the final state carried further out, without
  // updates, until the last row or a propagation guard
  int r_hi = r_out;
  if (f.extrapolate) {
    for (int r = r_out + 1; r < R; ++r) {
      KState nx = q;
      if (!fit_prop(nx, X(r), p)) break;
      q = nx;
      int32_t best = -1;
      cnt[r] = uint8_t(rb_row_candidates(g, p, kb, r, oy, oz, q.y, q.z, fit_cyy(q), fit_czz(q), f.chi2_extrap,
                                         cand + r * kRebuildK, &best));
      ptr[r] = kPtrMoved;
      r_hi = r;
    }
  }
  meta[1] = r_lo;
  meta[2] = r_hi;
  float* st = ws.state + 16 * t;
  st[0] = q.x; st[1] = q.y; st[2] = q.z; st[3] = q.s; st[4] = q.t; st[5] = q.w;
  st[6] = q.uys; st[7] = q.uyw; st[8] = q.usw; st[9] = q.dy; st[10] = q.ds; st[11] = q.dw;
  st[12] = q.uzt; st[13] = q.dz; st[14] = q.dt; st[15] = 0.0f;
  meta[0] = 1;
}

__global__ void __launch_bounds__(kWave) k_rebuild_propose(RebuildIn in, RebuildWs ws) {
  const int64_t t = int64_t(blockIdx.x) * kWave + threadIdx.x;
  if (t >= in.n_tracks || !ws.active[t]) return;
  ws.active[t] = 0;
  const int32_t* meta = ws.meta + 4 * t;
  if (!meta[0]) return;
  ws.check[t] = 1;
  const int R = in.n_rows;
  const unsigned long long key = ws.key[t];
  const int64_t fu = ws.first[t];
  for (int r = meta[1]; r <= meta[2]; ++r) {
    const int v = ws.ptr[t * R + r];
    if (!(v & kPtrMoved)) continue;
    const int k = v & ~kPtrMoved;
    ws.ptr[t * R + r] = uint8_t(k);
    if (k >= ws.cnt[t * R + r]) continue;
    const unsigned long long old = atomicMax(ws.holder + ws.cand[(t * R + r) * kRebuildK + k].x, key);
    if (old != 0ull && old < key) {
      // the holder (a track of the same unit) lost the cluster
      const int64_t h = fu + (kSelectMaxPerUnit - 1 - int64_t(old & (kSelectMaxPerUnit - 1)));
      if (h < in.n_tracks) ws.check[h] = 1;
    }
  }
}

__global__ void __launch_bounds__(kWave) k_rebuild_advance(RebuildIn in, RebuildWs ws) {
  const int64_t t = int64_t(blockIdx.x) * kWave + threadIdx.x;
  if (t >= in.n_tracks || !ws.check[t]) return;
  ws.check[t] = 0;
  const int32_t* meta = ws.meta + 4 * t;
  if (!meta[0]) return;
  const int R = in.n_rows;
  const unsigned long long key = ws.key[t];
  bool moved = false;
  for (int r = meta[1]; r <= meta[2]; ++r) {
    const int k = ws.ptr[t * R + r] & ~kPtrMoved;
    if (k < ws.cnt[t * R + r] && ws.holder[ws.cand[(t * R + r) * kRebuildK + k].x] != key) {
      ws.ptr[t * R + r] = uint8_t(k + 1) | kPtrMoved;
      moved = true;
    }
  }
  if (moved) ws.active[t] = 1;
}

__global__ void __launch_bounds__(kWave) k_rebuild_pass3(RebuildIn in, DevParams p, RebuildConsts f,
                                                         RebuildWs ws, RebuildOut out) {
  const int64_t t = int64_t(blockIdx.x) * kWave + threadIdx.x;
  if (t >= in.n_tracks) return;
  const int R = in.n_rows;
  int32_t* as = out.assigned + t * R;
  for (int r = 0; r < R; ++r) as[r] = -1;
  auto fail = [&]() {
    out.ok[t] = 0;
    out.n_kept[t] = 0;
    out.chi2[t] = 0.0f;
    out.x_out[t] = 0.0f;
    for (int k = 0; k < 5; ++k) out.param[5 * t + k] = 0.0f;
    for (int k = 0; k < 15; ++k) out.cov[15 * t + k] = 0.0f;
  };
  const int32_t* meta = ws.meta + 4 * t;
  if (!meta[0]) return fail();
  const int r_in = meta[1], r_out = meta[2];
  const unsigned long long key = ws.key[t];
  auto got = [&](int r) -> int32_t {
    const int k = ws.ptr[t * R + r] & ~kPtrMoved;
    if (k >= ws.cnt[t * R + r]) return -1;
    const int32_t id = ws.cand[(t * R + r) * kRebuildK + k].x;
    return ws.holder[id] == key ? id : -1;
  };
  int j = r_out;
  while (j >= r_in && got(j) < 0) --j;
  if (j - r_in < 2) return fail();
  const float* st = ws.state + 16 * t;
  KState q;
  q.x = st[0]; q.y = st[1]; q.z = st[2]; q.s = st[3]; q.t = st[4]; q.w = st[5];
  q.uys = st[6]; q.uyw = st[7]; q.usw = st[8]; q.dy = st[9]; q.ds = st[10]; q.dw = st[11];
  q.uzt = st[12]; q.dz = st[13]; q.dt = st[14];
  const int64_t b = in.hit_begin[t];
  const int n = int(in.hit_begin[t + 1] - b);
  const float oy = in.y[in.hit_id[b + n - 1]], oz = in.z[in.hit_id[b + n - 1]];
  for (int r = r_out - 1; r >= j; --r)
    if (!fit_prop(q, in.row_x[r], p)) return fail();
  const int32_t cj = got(j);
  q.y = in.y[cj] - oy;
  q.z = in.z[cj] - oz;
  rb_reset(q, p, f);
  as[j] = cj;
  float chi2 = 0.0f;
  int kept = 1;
  KState last = q;
  for (int r = j - 1; r >= r_in; --r) {
    const int32_t c = got(r);
    if (c < 0) continue;
    if (!fit_prop(q, in.row_x[r], p)) {
      for (int rr = 0; rr < R; ++rr) as[rr] = -1;
      return fail();
    }
    const float my = in.y[c] - oy, mz = in.z[c] - oz;
    const KInnov nv = kf_innov(q, p);
    const float iSy = 1.0f / nv.sy, iSz = 1.0f / nv.sz;
    const float ry = my - q.y, rz = mz - q.z;
    const float ch = (ry * ry) * iSy + (rz * rz) * iSz;
    if (!(ch <= f.chi2_final)) continue;
    chi2 = chi2 + kf_update<false>(q, my, mz, nv, iSy, iSz, p);
    as[r] = c;
    ++kept;
    last = q;
  }
  if (kept < 3) {
    for (int rr = 0; rr < R; ++rr) as[rr] = -1;
    return fail();
  }
  out.ok[t] = 1;
  out.n_kept[t] = kept;
  out.chi2[t] = chi2;
  out.x_out[t] = last.x;
  float* pp = out.param + 5 * t;
  pp[0] = oy + last.y;
  pp[1] = oz + last.z;
  pp[2] = last.s;
  pp[3] = last.t;
  pp[4] = last.w;
  const float cww = last.dw;
  const float cws = last.usw * last.dw;
  const float cwy = last.uyw * last.dw;
  const float css = last.ds + last.usw * cws;
  const float csy = last.uys * last.ds + last.uyw * cws;
  const float cyy = (last.dy + last.uys * (last.uys * last.ds)) + last.uyw * cwy;
  const float ctt = last.dt;
  const float ctz = last.uzt * last.dt;
  const float czz = last.dz + last.uzt * ctz;
  const float cv[15] = {cyy, 0.0f, czz, csy, 0.0f, css, 0.0f, ctz, 0.0f, ctt, cwy, 0.0f, cws, 0.0f, cww};
  for (int k = 0; k < 15; ++k) out.cov[15 * t + k] = cv[k];
}

}  // namespace tpcx
