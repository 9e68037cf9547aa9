// Seeding by the cellular automaton (paper, Section 2): the neighbour finder
// links each cluster to the best pair of clusters in the adjacent rows, the
// cleaning keeps mutual links only, and start hits are the inner ends of the
// resulting chains of at least three clusters.
#pragma once

#include "tpcx_common.h"

namespace tpcx {

// Neighbour finder.  One thread per cluster (sorted order).  For cluster h in
// row r (1 <= r <= n_rows-2) consider every u in row r+1 and d in row r-1
// within |dy| <= wy and |dz| <= wz of h; the deviation of h from the chord d-u
// at row r is e = h - (d + (u - d) * f_r), D = ey^2 + ez^2.  The pair with the
// smallest (D, id_u, id_d) among D <= d2max gives link_up/link_down (caller
// ids), -1 if none.  f_r = (x_r - x_{r-1}) / (x_{r+1} - x_{r-1}) in float.
__global__ void k_neighbours(const int64_t* __restrict__ row_begin, int n_units, Grid g,
                             const float* __restrict__ frac, DevParams p,
                             int32_t* __restrict__ link_up, int32_t* __restrict__ link_down) {
  const int64_t n = row_begin[int64_t(n_units) * g.n_rows];
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = upper_row(row_begin, n_units * g.n_rows + 1, i);
  const int u = k / g.n_rows, r = k % g.n_rows;
  const int32_t h = g.sid[i];
  if (r == 0 || r == g.n_rows - 1) {
    link_up[h] = -1;
    link_down[h] = -1;
    return;
  }
  const float yh = g.sy[i], zh = g.sz[i];
  const float f = frac[r];
  const float wy = p.wy, wz = p.wz;
  const float pz = wz + box_pad(zh), py = wy + box_pad(yh);
  const int zb0 = g.zbin(u, zh - pz), zb1 = g.zbin(u, zh + pz);
  const int64_t bu = g.row_base(u, r + 1), bd = g.row_base(u, r - 1);
  const int nyu = g.rows[r + 1].ny, nyd = g.rows[r - 1].ny;
  const int yu0 = g.ybin(r + 1, yh - py), yu1 = g.ybin(r + 1, yh + py);
  const int yd0 = g.ybin(r - 1, yh - py), yd1 = g.ybin(r - 1, yh + py);

  float bestD = 0.0f;
  int32_t best_u = -1, best_d = -1;
  for (int zu = zb0; zu <= zb1; ++zu) {
    const int32_t ju0 = g.bin_start[bu + zu * nyu + yu0], ju1 = g.bin_start[bu + zu * nyu + yu1 + 1];
    for (int32_t ju = ju0; ju < ju1; ++ju) {
      const float yu = g.sy[ju], zuu = g.sz[ju];
      if (!(fabsf(yu - yh) <= wy && fabsf(zuu - zh) <= wz)) continue;
      const int32_t cu = g.sid[ju];
      for (int zd = zb0; zd <= zb1; ++zd) {
        const int32_t jd0 = g.bin_start[bd + zd * nyd + yd0], jd1 = g.bin_start[bd + zd * nyd + yd1 + 1];
        for (int32_t jd = jd0; jd < jd1; ++jd) {
          const float yd = g.sy[jd], zdd = g.sz[jd];
          if (!(fabsf(yd - yh) <= wy && fabsf(zdd - zh) <= wz)) continue;
          const float ey = yh - (yd + (yu - yd) * f);
          const float ez = zh - (zdd + (zuu - zdd) * f);
          const float D = ey * ey + ez * ez;
          if (!(D <= p.d2max)) continue;
          const int32_t cd = g.sid[jd];
          if (best_u < 0 || D < bestD || (D == bestD && (cu < best_u || (cu == best_u && cd < best_d)))) {
            bestD = D;
            best_u = cu;
            best_d = cd;
          }
        }
      }
    }
  }
  link_up[h] = best_u;
  link_down[h] = best_d;
}

// Mutual-link cleaning and start-hit flags, one thread per cluster (caller
// order).  A start hit has no cleaned down link, a cleaned up link u, and u has
// a cleaned up link itself (chain of >= 3).  Writes per-block start counts.
__global__ void k_clean_flags(int64_t n, const int32_t* __restrict__ up,
                              const int32_t* __restrict__ down, int32_t* __restrict__ cup,
                              int32_t* __restrict__ cdown, uint8_t* __restrict__ flag,
                              int32_t* __restrict__ blk_cnt) {
  __shared__ int32_t wcnt[1024 / kWave];
  const int64_t h = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  bool st = false;
  if (h < n) {
    const int32_t u = up[h], d = down[h];
    const int32_t cu = (u >= 0 && down[u] == h) ? u : -1;
    const int32_t cd = (d >= 0 && up[d] == h) ? d : -1;
    cup[h] = cu;
    cdown[h] = cd;
    if (cd < 0 && cu >= 0) {
      const int32_t uu = up[cu];
      st = uu >= 0 && down[uu] == cu;
    }
    flag[h] = st ? 1 : 0;
  }
  const uint64_t m = __ballot(st);
  const int wid = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
  if (lane_id() == 0) wcnt[wid] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int w = 0; w < nw; ++w) s += wcnt[w];
    blk_cnt[blockIdx.x] = s;
  }
}

// Exclusive scan of per-block counts (one block).  total -> *total_out, and
// the status bit when it exceeds cap.
__global__ void k_scan_counts(const int32_t* __restrict__ cnt, int64_t nb, int32_t* __restrict__ off,
                              int64_t* __restrict__ total_out, int64_t cap,
                              int64_t* __restrict__ status, int64_t status_bit) {
  __shared__ int64_t lds[1024 / kWave];
  int64_t run = 0;
  for (int64_t t0 = 0; t0 < nb; t0 += blockDim.x) {
    int64_t t = t0 + threadIdx.x;
    int64_t c = t < nb ? cnt[t] : 0;
    int64_t tot;
    int64_t ex = block_exclusive_scan(c, lds, &tot);
    if (t < nb) off[t] = int32_t(run + ex);
    run += tot;
  }
  if (threadIdx.x == 0) {
    *total_out = run;
    if (run > cap) atomicOr((unsigned long long*)status, (unsigned long long)status_bit);
  }
}

// Ordered compaction of the start flags: block offsets + wave ballot ranks.
__global__ void k_write_starts(int64_t n, const uint8_t* __restrict__ flag,
                               const int32_t* __restrict__ blk_off, int64_t cap,
                               int32_t* __restrict__ starts) {
  __shared__ int32_t wcnt[1024 / kWave];
  const int64_t h = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool st = h < n && flag[h] != 0;
  const uint64_t m = __ballot(st);
  const int wid = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
  if (lane_id() == 0) wcnt[wid] = __popcll(m);
  __syncthreads();
  int32_t woff = 0;
  for (int w = 0; w < wid; ++w) woff += wcnt[w];
  (void)nw;
  if (st) {
    int64_t pos = int64_t(blk_off[blockIdx.x]) + woff + __popcll(m & lanes_below());
    if (pos < cap) starts[pos] = int32_t(h);
  }
}

}  // namespace tpcx
