// Seeding by the cellular automaton (paper, Section 2): the neighbour finder
// links each cluster to the best pair of clusters in the adjacent rows, the
// cleaning keeps mutual links only, and start hits are the inner ends of the
// resulting chains of at least three clusters.
#pragma once

#include "tpcx_common.h"

namespace tpcx {

// Neighbour finder.  One block per (unit, row); threads walk the row's
// clusters in sorted order, so a wavefront works on neighbouring clusters and
// its reads of rows r-1 and r+1 hit the caches.  For cluster h in row r
// (1 <= r <= n_rows-2) every u in row r+1 and d in row r-1 within |dy| <= wy
// and |dz| <= wz of h is considered; the deviation of h from the chord d-u at
// row r is e = h - (d + (u - d) * f_r), D = ey^2 + ez^2.  The pair with the
// smallest (D, id_u, id_d) among D <= d2max gives link_up/link_down (caller
// ids), -1 if none.  f_r = (x_r - x_{r-1}) / (x_{r+1} - x_{r-1}) in float.
// The down candidates of a cluster are collected once in LDS (up to kNfD;
// more fall back to re-reading them for every up candidate).
constexpr int kNfD = 8;
constexpr int kNfBlock = 256;

__global__ void __launch_bounds__(kNfBlock) k_neighbours(const int64_t* __restrict__ row_begin, Grid g,
                                                         const float* __restrict__ frac, DevParams p,
                                                         int32_t* __restrict__ link_up,
                                                         int32_t* __restrict__ link_down) {
  __shared__ float dy_l[kNfD][kNfBlock];
  __shared__ float dz_l[kNfD][kNfBlock];
  __shared__ int32_t did_l[kNfD][kNfBlock];
  const int k = blockIdx.x;
  const int r = k % g.n_rows;
  const int64_t b = row_begin[k], e = row_begin[k + 1];
  const int t = threadIdx.x;
  if (r == 0 || r == g.n_rows - 1) {
    for (int64_t i = b + t; i < e; i += blockDim.x) {
      const int32_t h = g.sid[i];
      link_up[h] = -1;
      link_down[h] = -1;
    }
    return;
  }
  const float f = frac[r];
  const float wy = p.wy, wz = p.wz;
  const int ku = k + 1, kd = k - 1;
  const int64_t bu = g.row_base(ku), bd = g.row_base(kd);
  const int nyu = g.rows[r + 1].ny, nyd = g.rows[r - 1].ny;
  for (int64_t i = b + t; i < e; i += blockDim.x) {
    const int32_t h = g.sid[i];
    const float yh = g.sy[i], zh = g.sz[i];
    const float pz = wz + box_pad(zh), py = wy + box_pad(yh);
    const int zu0 = g.zbin(ku, zh - pz), zu1 = g.zbin(ku, zh + pz);
    const int zd0 = g.zbin(kd, zh - pz), zd1 = g.zbin(kd, zh + pz);
    const int yu0 = g.ybin(r + 1, yh - py), yu1 = g.ybin(r + 1, yh + py);
    const int yd0 = g.ybin(r - 1, yh - py), yd1 = g.ybin(r - 1, yh + py);

    // down candidates inside the window
    int nd = 0;
    for (int zb = zd0; zb <= zd1; ++zb) {
      const int32_t j0 = g.bin_start[bd + zb * nyd + yd0], j1 = g.bin_start[bd + zb * nyd + yd1 + 1];
      for (int32_t j = j0; j < j1; ++j) {
        const float yd = g.sy[j], zd = g.sz[j];
        if (!(fabsf(yd - yh) <= wy && fabsf(zd - zh) <= wz)) continue;
        if (nd < kNfD) {
          dy_l[nd][t] = yd;
          dz_l[nd][t] = zd;
          did_l[nd][t] = g.sid[j];
        }
        ++nd;
      }
    }
    float bestD = 0.0f;
    int32_t best_u = -1, best_d = -1;
    if (nd > 0) {
      for (int zb = zu0; zb <= zu1; ++zb) {
        const int32_t j0 = g.bin_start[bu + zb * nyu + yu0], j1 = g.bin_start[bu + zb * nyu + yu1 + 1];
        for (int32_t ju = j0; ju < j1; ++ju) {
          const float yu = g.sy[ju], zu = g.sz[ju];
          if (!(fabsf(yu - yh) <= wy && fabsf(zu - zh) <= wz)) continue;
          const int32_t cu = g.sid[ju];
          auto consider = [&](float yd, float zd, int32_t cd) {
            const float ey = yh - (yd + (yu - yd) * f);
            const float ez = zh - (zd + (zu - zd) * f);
            const float D = ey * ey + ez * ez;
            if (!(D <= p.d2max)) return;
            if (best_u < 0 || D < bestD || (D == bestD && (cu < best_u || (cu == best_u && cd < best_d)))) {
              bestD = D;
              best_u = cu;
              best_d = cd;
            }
          };
          if (nd <= kNfD) {
            for (int q = 0; q < nd; ++q) consider(dy_l[q][t], dz_l[q][t], did_l[q][t]);
          } else {
            for (int zb2 = zd0; zb2 <= zd1; ++zb2) {
              const int32_t k0 = g.bin_start[bd + zb2 * nyd + yd0], k1 = g.bin_start[bd + zb2 * nyd + yd1 + 1];
              for (int32_t jd = k0; jd < k1; ++jd) {
                const float yd = g.sy[jd], zd = g.sz[jd];
                if (!(fabsf(yd - yh) <= wy && fabsf(zd - zh) <= wz)) continue;
                consider(yd, zd, g.sid[jd]);
              }
            }
          }
        }
      }
    }
    link_up[h] = best_u;
    link_down[h] = best_d;
  }
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
