// Seeding by the cellular automaton (paper, Section 2): the neighbour finder
// links each cluster to the best pair of clusters in the adjacent rows, the
// cleaning keeps mutual links only, and start hits are the inner ends of the
// resulting chains of at least three clusters.
#pragma once

#include "tpcx_common.h"

namespace tpcx {

// Neighbour finder.  One block per (unit, row); threads walk the row's
// clusters in sorted order, so a wavefront works on neighbouring clusters, its
// reads of rows r-1 and r+1 hit the caches and its link writes are coalesced.
// For cluster h in row r (1 <= r <= n_rows-2) every u in row r+1 and d in row
// r-1 within |dy| <= wy and |dz| <= wz of h is considered; the deviation of h
// from the chord d-u at row r is e = h - (d + (u - d) * f_r), D = ey^2 + ez^2.
// The pair with the smallest (D, id_u, id_d) (caller ids) among D <= d2max
// gives the links (sorted positions), -1 if none.
// f_r = (x_r - x_{r-1}) / (x_{r+1} - x_{r-1}) in float.
//
// The candidates of each row inside the window are first collected in LDS
// (their sorted positions; up to kNfD per row), then the down candidates'
// coordinates are loaded into registers together and every up candidate is
// evaluated against all of them; the records are re-read from the cache, so
// the LDS stays small and occupancy high.
// Caller ids are read only to break an exact tie of D.  A cluster with more
// than kNfD candidates in a row takes the direct double scan instead.  A
// lane's clusters are software-pipelined: while one is processed, the record
// of the one after next and the bin ranges of the next are in flight.
constexpr int kNfD = 8;
constexpr int kNfBlock = 256;

__device__ __forceinline__ int32_t id_of(const float4& p) { return __float_as_int(p.z); }
__device__ __forceinline__ int32_t cup_of(const float4& p) { return __float_as_int(p.w); }

// Sorted positions of the window candidates around (yh, zh) of the index
// range j0 .. j1 appended to the lane's LDS list (up to kNfD; n counts them
// all): four records in flight at a time.
__device__ __forceinline__ void nf_take_range(const Grid& g, int32_t j0, int32_t j1, float yh, float zh, float wy,
                                              float wz, int32_t (*pos)[kNfBlock], int t, int& n) {
  const float2* yz = reinterpret_cast<const float2*>(g.pts);
  for (int32_t j = j0; j < j1; j += 4) {
    float2 v[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = yz[2 * int64_t(j + m < j1 ? j + m : j)];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if (j + m < j1 && fabsf(v[m].x - yh) <= wy && fabsf(v[m].y - zh) <= wz) {
        if (n < kNfD) pos[n][t] = j + m;
        ++n;
      }
    }
  }
}

// The same over the bin ranges of z bins zb0 .. zb1 (any number), one record
// at a time: for boxes wider than two z bins.
__device__ __forceinline__ int nf_collect(const Grid& g, int64_t kb, int ny, int zb0, int zb1, int yb0,
                                          int yb1, float yh, float zh, float wy, float wz,
                                          int32_t (*pos)[kNfBlock], int t) {
  int n = 0;
  for (int zb = zb0; zb <= zb1; ++zb) {
    const int32_t j0 = g.bin_start[kb + zb * ny + yb0], j1 = g.bin_start[kb + zb * ny + yb1 + 1];
    for (int32_t j = j0; j < j1; ++j) {
      const float4 pc = g.pts[j];
      if (!(fabsf(pc.x - yh) <= wy && fabsf(pc.y - zh) <= wz)) continue;
      if (n < kNfD) pos[n][t] = j;
      ++n;
    }
  }
  return n;
}

// (D, ju, jd) against the best so far under the order (D, id_u, id_d).
__device__ __forceinline__ bool nf_better(const Grid& g, float D, int32_t ju, int32_t jd, float bestD,
                                          int32_t best_ju, int32_t best_jd) {
  if (best_ju < 0 || D < bestD) return true;
  if (D != bestD) return false;
  const int32_t iu = id_of(g.pts[ju]), bu = id_of(g.pts[best_ju]);
  if (iu != bu) return iu < bu;
  return id_of(g.pts[jd]) < id_of(g.pts[best_jd]);
}

__global__ void __launch_bounds__(kNfBlock) k_neighbours(const int64_t* __restrict__ row_begin, Grid g,
                                                         const float* __restrict__ frac, DevParams p,
                                                         int32_t* __restrict__ up_s,
                                                         int32_t* __restrict__ down_s) {
  __shared__ int32_t d_pos[kNfD][kNfBlock];
  __shared__ int32_t u_pos[kNfD][kNfBlock];
  const int k = int(xcd_block());
  const int r = k % g.n_rows;
  const int64_t b = row_begin[k], e = row_begin[k + 1];
  const int t = threadIdx.x;
  if (r == 0 || r == g.n_rows - 1) {
    for (int64_t i = b + t; i < e; i += blockDim.x) {
      up_s[i] = -1;
      down_s[i] = -1;
    }
    return;
  }
  const float f = frac[r];
  const float wy = p.wy, wz = p.wz;
  const int ku = k + 1, kd = k - 1;
  const int64_t bu = g.row_base(ku), bd = g.row_base(kd);
  const int nyu = g.rows[r + 1].ny, nyd = g.rows[r - 1].ny;
  // Software pipeline over the lane's clusters i, i + B, i + 2B (B the block
  // size): while cluster i is processed, the record of i + 2B and the bin
  // ranges of i + B are in flight, so a cluster waits only for its candidates.
  const float2* yz = reinterpret_cast<const float2*>(g.pts);
  const int64_t B = blockDim.x;
  struct Box {
    int32_t r[8];  // bin ranges: d0s, d0e, d1s, d1e, u0s, u0e, u1s, u1e
    int mode;      // bit 0: boxes of at most two z bins; bit 1: two down z bins; bit 2: two up z bins
  };
  struct Bins {
    int zu0, zu1, zd0, zd1, yu0, yu1, yd0, yd1;
  };
  auto bins_of = [&](float yh, float zh) {
    const float pz = wz + box_pad(zh), py = wy + box_pad(yh);
    Bins q;
    q.zu0 = g.zbin(ku, zh - pz);
    q.zu1 = g.zbin(ku, zh + pz);
    q.zd0 = g.zbin(kd, zh - pz);
    q.zd1 = g.zbin(kd, zh + pz);
    q.yu0 = g.ybin(r + 1, yh - py);
    q.yu1 = g.ybin(r + 1, yh + py);
    q.yd0 = g.ybin(r - 1, yh - py);
    q.yd1 = g.ybin(r - 1, yh + py);
    return q;
  };
  auto box_of = [&](float yh, float zh, Box& x) {
    const Bins q = bins_of(yh, zh);
    const bool fast = q.zd1 - q.zd0 <= 1 && q.zu1 - q.zu0 <= 1;
    x.mode = (fast ? 1 : 0) | (q.zd1 > q.zd0 ? 2 : 0) | (q.zu1 > q.zu0 ? 4 : 0);
    if (fast) {
      // the bin ranges of both rows (at most two z bins each)
      const int64_t rd0 = bd + int64_t(q.zd0) * nyd, rd1 = bd + int64_t(q.zd1) * nyd;
      const int64_t ru0 = bu + int64_t(q.zu0) * nyu, ru1 = bu + int64_t(q.zu1) * nyu;
      x.r[0] = g.bin_start[rd0 + q.yd0];
      x.r[1] = g.bin_start[rd0 + q.yd1 + 1];
      x.r[2] = g.bin_start[rd1 + q.yd0];
      x.r[3] = g.bin_start[rd1 + q.yd1 + 1];
      x.r[4] = g.bin_start[ru0 + q.yu0];
      x.r[5] = g.bin_start[ru0 + q.yu1 + 1];
      x.r[6] = g.bin_start[ru1 + q.yu0];
      x.r[7] = g.bin_start[ru1 + q.yu1 + 1];
    }
  };
  int64_t i = b + t;
  float2 cur = i < e ? yz[2 * i] : make_float2(0.0f, 0.0f);
  float2 nxt = i + B < e ? yz[2 * (i + B)] : make_float2(0.0f, 0.0f);
  Box bx{};
  if (i < e) box_of(cur.x, cur.y, bx);
  for (; i < e; i += B) {
    const float yh = cur.x, zh = cur.y;
    const float2 nn = i + 2 * B < e ? yz[2 * (i + 2 * B)] : make_float2(0.0f, 0.0f);
    Box bn{};
    if (i + B < e) box_of(nxt.x, nxt.y, bn);
    int nd = 0, nu = 0;
    if (bx.mode & 1) {
      nf_take_range(g, bx.r[0], bx.r[1], yh, zh, wy, wz, d_pos, t, nd);
      if (bx.mode & 2) nf_take_range(g, bx.r[2], bx.r[3], yh, zh, wy, wz, d_pos, t, nd);
      if (nd > 0) {
        nf_take_range(g, bx.r[4], bx.r[5], yh, zh, wy, wz, u_pos, t, nu);
        if (bx.mode & 4) nf_take_range(g, bx.r[6], bx.r[7], yh, zh, wy, wz, u_pos, t, nu);
      }
    } else {
      const Bins q = bins_of(yh, zh);
      nd = nf_collect(g, bd, nyd, q.zd0, q.zd1, q.yd0, q.yd1, yh, zh, wy, wz, d_pos, t);
      nu = nd > 0 ? nf_collect(g, bu, nyu, q.zu0, q.zu1, q.yu0, q.yu1, yh, zh, wy, wz, u_pos, t) : 0;
    }
    float bestD = 0.0f;
    int32_t best_ju = -1, best_jd = -1;
    auto consider = [&](float yu, float zu, int32_t ju, float yd, float zd, int32_t jd) {
      const float ey = yh - (yd + (yu - yd) * f);
      const float ez = zh - (zd + (zu - zd) * f);
      const float D = ey * ey + ez * ez;
      if (!(D <= p.d2max)) return;
      if (nf_better(g, D, ju, jd, bestD, best_ju, best_jd)) {
        bestD = D;
        best_ju = ju;
        best_jd = jd;
      }
    };
    if (nd <= kNfD && nu <= kNfD) {
      // the down candidates' (y, z) into registers first (independent loads,
      // in flight together), then every up candidate against all of them;
      // the best down candidate is kept as its LDS slot
      const float2* yz = reinterpret_cast<const float2*>(g.pts);
      float ydv[kNfD], zdv[kNfD];
#pragma unroll
      for (int c = 0; c < kNfD; ++c) {
        float2 v = make_float2(0.0f, 0.0f);
        if (c < nd) v = yz[2 * int64_t(d_pos[c][t])];
        ydv[c] = v.x;
        zdv[c] = v.y;
      }
      int best_c = -1;
      int32_t ja = 0;
      float uy = 0.0f, uz = 0.0f;
      if (nu > 0) {
        ja = u_pos[0][t];
        const float2 v = yz[2 * int64_t(ja)];
        uy = v.x;
        uz = v.y;
      }
      for (int a = 0; a < nu; ++a) {
        // the next up candidate is loaded while this one is evaluated
        int32_t jn = ja;
        float ny = uy, nz = uz;
        if (a + 1 < nu) {
          jn = u_pos[a + 1][t];
          const float2 v = yz[2 * int64_t(jn)];
          ny = v.x;
          nz = v.y;
        }
#pragma unroll
        for (int c = 0; c < kNfD; ++c) {
          if (c < nd) {
            const float ey = yh - (ydv[c] + (uy - ydv[c]) * f);
            const float ez = zh - (zdv[c] + (uz - zdv[c]) * f);
            const float D = ey * ey + ez * ez;
            if (D <= p.d2max) {
              bool take = best_ju < 0 || D < bestD;
              if (!take && D == bestD) {
                // exact tie: the smaller (id_u, id_d)
                const int32_t iu = id_of(g.pts[ja]), bu = id_of(g.pts[best_ju]);
                take = iu != bu ? iu < bu : id_of(g.pts[d_pos[c][t]]) < id_of(g.pts[d_pos[best_c][t]]);
              }
              if (take) {
                bestD = D;
                best_ju = ja;
                best_c = c;
              }
            }
          }
        }
        ja = jn;
        uy = ny;
        uz = nz;
      }
      best_jd = best_c >= 0 ? d_pos[best_c][t] : -1;
    } else {
      // more candidates than LDS holds: scan both rows directly
      const Bins q = bins_of(yh, zh);
      const int zu0 = q.zu0, zu1 = q.zu1, zd0 = q.zd0, zd1 = q.zd1;
      const int yu0 = q.yu0, yu1 = q.yu1, yd0 = q.yd0, yd1 = q.yd1;
      for (int zb = zu0; zb <= zu1; ++zb) {
        const int32_t j0 = g.bin_start[bu + zb * nyu + yu0], j1 = g.bin_start[bu + zb * nyu + yu1 + 1];
        for (int32_t ju = j0; ju < j1; ++ju) {
          const float4 pu = g.pts[ju];
          if (!(fabsf(pu.x - yh) <= wy && fabsf(pu.y - zh) <= wz)) continue;
          for (int zb2 = zd0; zb2 <= zd1; ++zb2) {
            const int32_t k0 = g.bin_start[bd + zb2 * nyd + yd0], k1 = g.bin_start[bd + zb2 * nyd + yd1 + 1];
            for (int32_t jd = k0; jd < k1; ++jd) {
              const float4 pd = g.pts[jd];
              if (!(fabsf(pd.x - yh) <= wy && fabsf(pd.y - zh) <= wz)) continue;
              consider(pu.x, pu.y, ju, pd.x, pd.y, jd);
            }
          }
        }
      }
    }
    up_s[i] = best_ju;
    down_s[i] = best_jd;
    cur = nxt;
    nxt = nn;
    bx = bn;
  }
}

// Mutual-link cleaning and start-hit flags, one block per (unit, row), in
// sorted positions.  The cleaned up-link goes into the cluster record.  A start
// hit has no cleaned down link, a cleaned up link u, and u has a cleaned up
// link itself (chain of >= 3).  Writes the row's number of start hits.
__global__ void k_clean_starts(const int64_t* __restrict__ row_begin, const int32_t* __restrict__ up,
                               const int32_t* __restrict__ down, float4* __restrict__ pts,
                               uint8_t* __restrict__ flag, int32_t* __restrict__ row_cnt) {
  __shared__ int32_t wcnt[1024 / kWave];
  const int k = int(xcd_block());
  const int64_t b = row_begin[k], e = row_begin[k + 1];
  int32_t cnt = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    const int32_t u = up[i], d = down[i];
    const int32_t cu = (u >= 0 && down[u] == i) ? u : -1;
    const int32_t cd = (d >= 0 && up[d] == i) ? d : -1;
    pts[i].w = __int_as_float(cu);
    bool st = false;
    if (cd < 0 && cu >= 0) {
      const int32_t uu = up[cu];
      st = uu >= 0 && down[uu] == cu;
    }
    flag[i] = st ? 1 : 0;
    cnt += st ? 1 : 0;
  }
  for (int d = kWave / 2; d > 0; d >>= 1) cnt += __shfl_xor(cnt, d, kWave);
  const int wid = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
  if (lane_id() == 0) wcnt[wid] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int w = 0; w < nw; ++w) s += wcnt[w];
    row_cnt[k] = s;
  }
}

// Exclusive scan of per-row (or per-block) counts in one block.  total ->
// *total_out, and the status bit when it exceeds cap.
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

// Start hits of one row in ascending caller id: the row's flagged clusters
// mark their caller id in an LDS bitmap over the row's id range, and each one's
// rank is the number of marked ids below it.  Ranges longer than the bitmap
// are done in segments.  order[] lists the same slots in sorted-position
// (bin) order, the order in which the constructor takes them so that
// neighbouring lanes follow neighbouring tracks (written when all start hits
// fit the capacity).
constexpr int kSegBits = 65536;
constexpr int kSegWords = kSegBits / 32;

__global__ void k_write_starts(const int64_t* __restrict__ row_begin, const float4* __restrict__ pts,
                               const uint8_t* __restrict__ flag, const int32_t* __restrict__ row_off,
                               const int64_t* __restrict__ n_total, int64_t cap,
                               int32_t* __restrict__ starts, int32_t* __restrict__ start_pos,
                               int32_t* __restrict__ start_k, int32_t* __restrict__ order) {
  __shared__ uint32_t bits[kSegWords];
  __shared__ int32_t wpre[kSegWords];
  __shared__ int64_t scan_lds[1024 / kWave];
  const int k = int(xcd_block());
  const int64_t b = row_begin[k], e = row_begin[k + 1];
  int64_t seg_base = row_off[k];
  const bool all_fit = *n_total <= cap;
  for (int64_t lo = b; lo < e; lo += kSegBits) {
    const int64_t hi = min(e, lo + kSegBits);
    const int nw = int((hi - lo + 31) / 32);
    for (int w = threadIdx.x; w < nw; w += blockDim.x) bits[w] = 0u;
    __syncthreads();
    for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
      if (!flag[i]) continue;
      const int64_t h = id_of(pts[i]);
      if (h < lo || h >= hi) continue;
      atomicOr(&bits[(h - lo) >> 5], 1u << ((h - lo) & 31));
    }
    __syncthreads();
    const int per = (nw + blockDim.x - 1) / blockDim.x;
    const int w0 = min(nw, int(threadIdx.x) * per), w1 = min(nw, w0 + per);
    int64_t c = 0;
    for (int w = w0; w < w1; ++w) c += __popc(bits[w]);
    int64_t tot;
    int64_t run = block_exclusive_scan(c, scan_lds, &tot);
    for (int w = w0; w < w1; ++w) {
      wpre[w] = int32_t(run);
      run += __popc(bits[w]);
    }
    __syncthreads();
    // srank: the start hit's rank in sorted-position order within the row
    int64_t srun = row_off[k];
    for (int64_t i0 = b; i0 < e; i0 += blockDim.x) {
      const int64_t i = i0 + threadIdx.x;
      const bool fl = i < e && flag[i];
      int64_t ftot;
      const int64_t srank = srun + block_exclusive_scan(fl ? 1 : 0, scan_lds, &ftot);
      srun += ftot;
      if (!fl) continue;
      const int64_t h = id_of(pts[i]);
      if (h < lo || h >= hi) continue;
      const int64_t o = h - lo;
      const int64_t pos = seg_base + wpre[o >> 5] + __popc(bits[o >> 5] & ((1u << (o & 31)) - 1u));
      if (pos < cap) {
        starts[pos] = int32_t(h);
        start_pos[pos] = int32_t(i);
        start_k[pos] = k;
      }
      if (all_fit) order[srank] = int32_t(pos);
    }
    seg_base += tot;
    __syncthreads();
  }
}

// Debug view of the links in caller ids, at the caller's cluster positions
// (the cleaned down link is recomputed: mutual links only).
__global__ void k_links_to_caller(int64_t n, const float4* __restrict__ pts,
                                  const int32_t* __restrict__ up, const int32_t* __restrict__ down,
                                  int32_t* __restrict__ link_up,
                                  int32_t* __restrict__ link_down, int32_t* __restrict__ clean_up,
                                  int32_t* __restrict__ clean_down) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 p = pts[i];
  const int32_t h = id_of(p);
  auto id = [&](int32_t j) { return j >= 0 ? id_of(pts[j]) : -1; };
  if (link_up) link_up[h] = id(up[i]);
  if (link_down) link_down[h] = id(down[i]);
  if (clean_up) clean_up[h] = id(cup_of(p));
  if (clean_down) {
    const int32_t d = down[i];
    clean_down[h] = id((d >= 0 && up[d] == i) ? d : -1);
  }
}

}  // namespace tpcx
