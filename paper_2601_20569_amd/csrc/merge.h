// Track merging (paper, Section 2: the segments of a track found by the
// sector tracking are merged inside a sector, between adjacent sectors of one
// TPC half and across the central electrode).  The paper names no matching
// criterion; the one here:
//
//   views   every track's state at its reference plane is carried to the
//           plane x = x_m in its own sector frame (view 0) and in the frames
//           of the boundaries with the next (view 1, rotated by -h) and the
//           previous sector (view 2, rotated by +h) of its half, h = half the
//           sector opening: rotation about the beam axis, then the tracking's
//           circle step in equal steps of at most 10 cm;
//   pairs   an inner and an outer segment (the inner one's last row below the
//           outer one's first) of the same unit (views 0, 0), of the two
//           units of one azimuth across the electrode (0, 0), or of adjacent
//           sectors (the inner one's view towards the outer one's sector
//           against the outer one's view towards the inner one's);
//   chi2    sum over y, z, sin(phi), dz/ds, q/pT of (difference / tolerance)^2
//           in that order, IEEE binary32; a pair is a candidate at chi2 <= cut;
//   links   a track's best outer and best inner candidate by (chi2, index);
//           a link where both choose each other; root = first of the chain.
//
// k_merge_views: one lane per track, the three views.
// k_merge_grid: one block per (unit, view): the unit's valid views sorted
//   into kMergeCells cells of z (each at least the z window wide, so a
//   window touches at most two cells).
// k_merge_match: one lane per track: for each related unit, the cells of
//   its window, the exact chi2 of the candidates inside the window.
// k_merge_link, k_merge_root: the mutual choices and the chain roots.
#pragma once

#include "tpcx_common.h"
#include "tracklet.h"

namespace tpcx {

constexpr int kMergeCells = 1024;
constexpr int kMergeBlock = 256;

struct MergeConsts {
  float x_m, cos_h, sin_h, chi2_cut;
  float itol2[5];
  float wy, wz;  // half-widths of the candidate window in y and z
  int cross_electrode;
};

struct MergeIn {
  int64_t n;
  int n_units;
  const int32_t* unit;
  const float* param;  // [n][5]
  const float* x_ref;
  const int32_t* r_in;
  const int32_t* r_out;
  const int32_t* unit_nbr;  // [n_units][3]: next sector, previous sector, across the electrode
};

struct MergeWs {
  float* view;          // [n][3][5]
  uint8_t* ok;          // [n][3]
  int64_t* ub;          // [n_units + 1] first track of each unit
  float4* rec;          // [3][n] per view, sorted by (unit, cell): y, z, index, rows
  int32_t* cell;        // [n_units][3][kMergeCells + 1] absolute starts in rec[v]
  float2* zcell;        // [n_units][3] (zmin, 1 / cell width)
  int32_t* best_out;    // [n]
  int32_t* best_in;     // [n]
};

// View v of track t into out[5]; false when missing.
__device__ __forceinline__ bool merge_view(const MergeIn& in, const DevParams& p, const MergeConsts& m,
                                           int64_t t, int v, float out[5]) {
  const float* prm = in.param + 5 * t;
  KState q{};
  q.x = in.x_ref[t];
  q.y = prm[0];
  q.z = prm[1];
  q.s = prm[2];
  q.t = prm[3];
  q.w = prm[4];
  if (!(fabsf(q.s) < p.smax)) return false;
  if (v != 0) {
    const float ch = m.cos_h;
    const float sh = v == 1 ? -m.sin_h : m.sin_h;
    const float cphi = sqrtf(1.0f - q.s * q.s);
    const float x1 = q.x * ch - q.y * sh;
    const float y1 = q.x * sh + q.y * ch;
    const float s1 = q.s * ch + cphi * sh;
    q.x = x1;
    q.y = y1;
    q.s = s1;
    if (!(fabsf(q.s) < p.smax)) return false;
  }
  const float x0 = q.x, xm = m.x_m;
  if (!(x0 == xm)) {
    const int n = int(ceilf(fabsf(xm - x0) * 0.1f));
    const float dxs = (xm - x0) / float(n);
    float cp = 0.0f, rp = 0.0f;
    bool cached = false;
    for (int k = 1; k < n; ++k) {
      cached = false;
      if (!kf_propagate<false>(q, x0 + float(k) * dxs, p, cp, rp, cached)) return false;
    }
    cached = false;
    if (!kf_propagate<false>(q, xm, p, cp, rp, cached)) return false;
  }
  out[0] = q.y;
  out[1] = q.z;
  out[2] = q.s;
  out[3] = q.t;
  out[4] = q.w;
  return true;
}

__global__ void __launch_bounds__(kMergeBlock) k_merge_views(MergeIn in, DevParams p, MergeConsts m, MergeWs ws) {
  const int64_t t = int64_t(blockIdx.x) * kMergeBlock + threadIdx.x;
  if (t >= in.n) return;
  // a track outside the input layout (unit out of range, rows not ordered)
  // has no views, so it links to nothing
  const bool valid = in.unit[t] >= 0 && in.unit[t] < in.n_units && in.r_in[t] >= 0 &&
                     in.r_in[t] <= in.r_out[t] && in.r_out[t] < 256;
#pragma unroll 1
  for (int v = 0; v < 3; ++v) {
    float o[5];
    const bool good = valid && merge_view(in, p, m, t, v, o);
    float* dst = ws.view + (t * 3 + v) * 5;
    for (int i = 0; i < 5; ++i) dst[i] = good ? o[i] : 0.0f;
    ws.ok[t * 3 + v] = good ? 1 : 0;
  }
}

// ub[u] = first track of unit u (tracks in ascending unit), u = 0 .. n_units.
__global__ void k_merge_units(MergeIn in, MergeWs ws) {
  const int u = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (u > in.n_units) return;
  int64_t lo = 0, hi = in.n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (in.unit[mid] < u) lo = mid + 1; else hi = mid;
  }
  ws.ub[u] = lo;
}

// One block per (unit, view): the valid views of the unit's tracks into
// cells of z, rec[v][ub[u] ..] in cell order.
__global__ void __launch_bounds__(kMergeBlock) k_merge_grid(MergeIn in, MergeConsts m, MergeWs ws) {
  __shared__ int32_t hist[kMergeCells + 1];
  __shared__ float red[kMergeBlock / kWave];
  __shared__ int64_t scan_lds[kMergeBlock / kWave];
  const int u = int(blockIdx.x) / 3, v = int(blockIdx.x) % 3;
  const int64_t b = ws.ub[u], e = ws.ub[u + 1];
  float lo = INFINITY, hi = -INFINITY;
  for (int64_t t = b + threadIdx.x; t < e; t += kMergeBlock) {
    if (!ws.ok[t * 3 + v]) continue;
    const float z = ws.view[(t * 3 + v) * 5 + 1];
    lo = fminf(lo, z);
    hi = fmaxf(hi, z);
  }
  lo = block_reduce_min(lo, red);
  hi = block_reduce_max(hi, red);
  // cells at least 2 wz wide (a window of half-width wz touches two at most)
  float inv = 0.0f;
  if (hi > lo) inv = fminf(float(kMergeCells) / (hi - lo), 0.5f / m.wz);
  if (!(lo <= hi)) lo = 0.0f;
  const int64_t seg = int64_t(u) * 3 + v;
  if (threadIdx.x == 0) ws.zcell[seg] = make_float2(lo, inv);
  for (int i = threadIdx.x; i <= kMergeCells; i += kMergeBlock) hist[i] = 0;
  __syncthreads();
  auto cell_of = [&](float z) {
    float c = (z - lo) * inv;
    c = fminf(fmaxf(c, 0.0f), float(kMergeCells - 1));
    return int(c);
  };
  for (int64_t t = b + threadIdx.x; t < e; t += kMergeBlock)
    if (ws.ok[t * 3 + v]) atomicAdd(&hist[cell_of(ws.view[(t * 3 + v) * 5 + 1])], 1);
  __syncthreads();
  // exclusive scan, each thread a run of kMergeCells / kMergeBlock cells
  constexpr int kPer = kMergeCells / kMergeBlock;
  int64_t s = 0;
  for (int i = 0; i < kPer; ++i) s += hist[threadIdx.x * kPer + i];
  int64_t tot;
  int64_t run = block_exclusive_scan(s, scan_lds, &tot) + b;
  for (int i = 0; i < kPer; ++i) {
    const int32_t c = hist[threadIdx.x * kPer + i];
    hist[threadIdx.x * kPer + i] = int32_t(run);
    run += c;
  }
  if (threadIdx.x == kMergeBlock - 1) hist[kMergeCells] = int32_t(run);
  __syncthreads();
  int32_t* cs = ws.cell + seg * (kMergeCells + 1);
  for (int i = threadIdx.x; i <= kMergeCells; i += kMergeBlock) cs[i] = hist[i];
  __syncthreads();
  float4* rec = ws.rec + int64_t(v) * in.n;
  for (int64_t t = b + threadIdx.x; t < e; t += kMergeBlock) {
    if (!ws.ok[t * 3 + v]) continue;
    const float* w = ws.view + (t * 3 + v) * 5;
    const int32_t pos = atomicAdd(&hist[cell_of(w[1])], 1);
    rec[pos] = make_float4(w[0], w[1], __int_as_float(int32_t(t)),
                           __int_as_float(in.r_in[t] | (in.r_out[t] << 8)));
  }
}

__device__ __forceinline__ bool merge_better(float c2, int32_t j, float bc, int32_t bj) {
  return bj < 0 || c2 < bc || (c2 == bc && j < bj);
}

// Candidates of track a in segment (u, vb) against a's view va: best outer
// (bo, co) and inner (bi, ci) partner so far.
__device__ __forceinline__ void merge_scan(const MergeIn& in, const MergeConsts& m, const MergeWs& ws, int64_t a,
                                           int ra_in, int ra_out, int u, int va, int vb, int32_t& bo, float& co,
                                           int32_t& bi, float& ci) {
  if (u < 0 || u >= in.n_units || !ws.ok[a * 3 + va]) return;
  const float* A = ws.view + (a * 3 + va) * 5;
  const float a0 = A[0], a1 = A[1], a2 = A[2], a3 = A[3], a4 = A[4];
  const int64_t seg = int64_t(u) * 3 + vb;
  const float2 zc = ws.zcell[seg];
  const float wz = m.wz + box_pad(a1), wy = m.wy + box_pad(a0);
  // cells of a range wider than the window: every cluster the window test
  // accepts lies in them
  float c0f = (a1 - 1.25f * wz - zc.x) * zc.y, c1f = (a1 + 1.25f * wz - zc.x) * zc.y;
  c0f = fminf(fmaxf(c0f, 0.0f), float(kMergeCells - 1));
  c1f = fminf(fmaxf(c1f, 0.0f), float(kMergeCells - 1));
  const int32_t* cs = ws.cell + seg * (kMergeCells + 1);
  const int32_t j0 = cs[int(c0f)], j1 = cs[int(c1f) + 1];
  const float4* rec = ws.rec + int64_t(vb) * in.n;
  for (int32_t j = j0; j < j1; ++j) {
    const float4 r = rec[j];
    const int32_t b = __float_as_int(r.z);
    if (b == int32_t(a)) continue;
    if (!(fabsf(r.x - a0) <= wy && fabsf(r.y - a1) <= wz)) continue;
    const int32_t rows = __float_as_int(r.w);
    const int rb_in = rows & 0xFF, rb_out = (rows >> 8) & 0xFF;
    const bool outer = ra_out < rb_in, inner = rb_out < ra_in;
    if (!outer && !inner) continue;
    const float* B = ws.view + (int64_t(b) * 3 + vb) * 5;
    float c2 = 0.0f, d;
    d = a0 - B[0];
    c2 = c2 + (d * d) * m.itol2[0];
    d = a1 - B[1];
    c2 = c2 + (d * d) * m.itol2[1];
    d = a2 - B[2];
    c2 = c2 + (d * d) * m.itol2[2];
    d = a3 - B[3];
    c2 = c2 + (d * d) * m.itol2[3];
    d = a4 - B[4];
    c2 = c2 + (d * d) * m.itol2[4];
    if (!(c2 <= m.chi2_cut)) continue;
    if (outer && merge_better(c2, b, co, bo)) {
      co = c2;
      bo = b;
    }
    if (inner && merge_better(c2, b, ci, bi)) {
      ci = c2;
      bi = b;
    }
  }
}

// Best outer and inner candidate of every track: the same unit, the unit
// across the electrode, the next and the previous sector's unit.
__global__ void __launch_bounds__(kMergeBlock) k_merge_match(MergeIn in, MergeConsts m, MergeWs ws) {
  const int64_t a = int64_t(blockIdx.x) * kMergeBlock + threadIdx.x;
  if (a >= in.n) return;
  int32_t bo = -1, bi = -1;
  float co = 0.0f, ci = 0.0f;
  if (ws.ok[a * 3] || ws.ok[a * 3 + 1] || ws.ok[a * 3 + 2]) {
    const int ua = in.unit[a];
    const int ra_in = in.r_in[a], ra_out = in.r_out[a];
    merge_scan(in, m, ws, a, ra_in, ra_out, ua, 0, 0, bo, co, bi, ci);
    if (m.cross_electrode) merge_scan(in, m, ws, a, ra_in, ra_out, in.unit_nbr[3 * ua + 2], 0, 0, bo, co, bi, ci);
    merge_scan(in, m, ws, a, ra_in, ra_out, in.unit_nbr[3 * ua + 0], 1, 2, bo, co, bi, ci);
    merge_scan(in, m, ws, a, ra_in, ra_out, in.unit_nbr[3 * ua + 1], 2, 1, bo, co, bi, ci);
  }
  ws.best_out[a] = bo;
  ws.best_in[a] = bi;
}

__global__ void k_merge_link(int64_t n, MergeWs ws, int32_t* __restrict__ prev, int32_t* __restrict__ next) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int32_t o = ws.best_out[t], i = ws.best_in[t];
  next[t] = (o >= 0 && ws.best_in[o] == int32_t(t)) ? o : -1;
  prev[t] = (i >= 0 && ws.best_out[i] == int32_t(t)) ? i : -1;
}

__global__ void k_merge_root(int64_t n, const int32_t* __restrict__ prev, int32_t* __restrict__ root) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  // rows strictly increase along a chain, so it has fewer than 256 links
  int32_t r = int32_t(t);
  for (int k = 0; k < 256 && prev[r] >= 0; ++k) r = prev[r];
  root[t] = r;
}

}  // namespace tpcx
