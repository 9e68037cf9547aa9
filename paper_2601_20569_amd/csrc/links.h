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
// (their sorted positions; up to kNfD per row), then all pairs are visited in
// one flat loop, so a wavefront runs max(n_u * n_d) pair steps rather than
// (scanned up candidates) x max(n_d); the pair loop re-reads the candidates'
// records, which are in the cache, so the LDS stays small and occupancy high.
// Caller ids are read only to break an exact tie of D.  A cluster with more
// than kNfD candidates in a row takes the direct double scan instead.
constexpr int kNfD = 8;
constexpr int kNfBlock = 256;

__device__ __forceinline__ int32_t id_of(const float4& p) { return __float_as_int(p.z); }
__device__ __forceinline__ int32_t cup_of(const float4& p) { return __float_as_int(p.w); }

// Sorted positions of the window candidates of one row around (yh, zh) into
// LDS (up to kNfD); returns their number (which may exceed kNfD).  The bin
// ranges of up to kNfZ z bins are loaded in one round, then the candidates two
// at a time, so a lane has several loads in flight.
constexpr int kNfZ = 6;

__device__ __forceinline__ int nf_collect(const Grid& g, int64_t kb, int ny, int zb0, int zb1, int yb0,
                                          int yb1, float yh, float zh, float wy, float wz,
                                          int32_t (*pos)[kNfBlock], int t) {
  int n = 0;
  auto take = [&](const float4& pc, int32_t j) {
    if (!(fabsf(pc.x - yh) <= wy && fabsf(pc.y - zh) <= wz)) return;
    if (n < kNfD) pos[n][t] = j;
    ++n;
  };
  const int nzb = zb1 - zb0 + 1;
  if (nzb <= kNfZ) {
    int32_t s[kNfZ], e[kNfZ];
#pragma unroll
    for (int q = 0; q < kNfZ; ++q) {
      if (q < nzb) {
        s[q] = g.bin_start[kb + (zb0 + q) * ny + yb0];
        e[q] = g.bin_start[kb + (zb0 + q) * ny + yb1 + 1];
      } else {
        s[q] = e[q] = 0;
      }
    }
#pragma unroll
    for (int q = 0; q < kNfZ; ++q) {
      for (int32_t j = s[q]; j < e[q]; j += 2) {
        const bool two = j + 1 < e[q];
        const float4 pa = g.pts[j];
        const float4 pb = g.pts[two ? j + 1 : j];
        take(pa, j);
        if (two) take(pb, j + 1);
      }
    }
    return n;
  }
  for (int zb = zb0; zb <= zb1; ++zb) {
    const int32_t j0 = g.bin_start[kb + zb * ny + yb0], j1 = g.bin_start[kb + zb * ny + yb1 + 1];
    for (int32_t j = j0; j < j1; ++j) take(g.pts[j], j);
  }
  return n;
}

// Wavefront-cooperative form of nf_collect: the window candidates of all 64
// lanes' clusters in one row, spread over all lanes.  For each pair of z bins
// in turn (each lane's box starting at its own zb0), the lanes' candidate
// ranges are numbered by a prefix sum over the wavefront; lane l evaluates
// candidates l and l + 64 of every 128, for their owner lane's cluster, and
// appends those inside the owner's window to the owner's LDS list (an LDS
// counter per owner).  The order inside a list is free: the pair selection has
// a total order.  Returns the lane's own count (which may exceed kNfD).  All
// 64 lanes must call it; `act` marks lanes with a cluster to serve.
__device__ __forceinline__ int nf_collect_wave(const Grid& g, int64_t kb, int ny, int zb0, int zb1, int yb0,
                                               int yb1, bool act, float yh, float zh, float wy, float wz,
                                               int32_t (*pos)[kNfBlock], int32_t* cnt, int t) {
  const int lane = lane_id();
  const int wbase = t - lane;
  cnt[t] = 0;
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  for (int zb = zb0;; zb += 2) {
    const bool a = act && zb <= zb1;
    if (__ballot(a) == 0ull) break;
    int32_t a0 = 0, alen = 0, b0 = 0, n = 0;
    if (a) {
      const bool z2 = zb + 1 <= zb1;
      const int64_t ra = kb + int64_t(zb) * ny;
      const int64_t rb = z2 ? ra + ny : ra;
      const int32_t j0 = g.bin_start[ra + yb0], j1 = g.bin_start[ra + yb1 + 1];
      const int32_t k0 = g.bin_start[rb + yb0], k1 = g.bin_start[rb + yb1 + 1];
      a0 = j0;
      alen = j1 - j0;
      b0 = k0;
      n = alen + (z2 ? k1 - k0 : 0);
    }
    int incl = n;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int v = __shfl_up(incl, d, kWave);
      if (lane >= d) incl += v;
    }
    const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, kWave - 1, kWave));
    const int excl = incl - n;
    for (int t0 = 0; t0 < total; t0 += 2 * kWave) {
      const int ta = t0 + lane, tb = ta + kWave;
      int oa = 0, ob = 0;
#pragma unroll
      for (int st = kWave / 2; st > 0; st >>= 1) {
        const int va = __shfl(incl, oa + st - 1, kWave);
        const int vb = __shfl(incl, ob + st - 1, kWave);
        if (va <= ta) oa += st;
        if (vb <= tb) ob += st;
      }
      const int ua = ta - __shfl(excl, oa, kWave), ub = tb - __shfl(excl, ob, kWave);
      // every shuffle with all lanes active (a shuffle reads nothing from a
      // lane its branch has switched off)
      const int la = __shfl(alen, oa, kWave), lb = __shfl(alen, ob, kWave);
      const int aa = __shfl(a0, oa, kWave), ab = __shfl(a0, ob, kWave);
      const int ba = __shfl(b0, oa, kWave), bb = __shfl(b0, ob, kWave);
      const int pa = ua < la ? aa + ua : ba + (ua - la);
      const int pb = ub < lb ? ab + ub : bb + (ub - lb);
      const bool va = ta < total, vb = tb < total;
      float4 ca = make_float4(0.0f, 0.0f, 0.0f, 0.0f), cb = ca;
      if (va) ca = g.pts[pa];
      if (vb) cb = g.pts[pb];
      const float ya = __shfl(yh, oa, kWave), za = __shfl(zh, oa, kWave);
      const float yb = __shfl(yh, ob, kWave), zb_ = __shfl(zh, ob, kWave);
      if (va && fabsf(ca.x - ya) <= wy && fabsf(ca.y - za) <= wz) {
        const int slot = atomicAdd(&cnt[wbase + oa], 1);
        if (slot < kNfD) pos[slot][wbase + oa] = pa;
      }
      if (vb && fabsf(cb.x - yb) <= wy && fabsf(cb.y - zb_) <= wz) {
        const int slot = atomicAdd(&cnt[wbase + ob], 1);
        if (slot < kNfD) pos[slot][wbase + ob] = pb;
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  return __hip_atomic_load(&cnt[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
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
  __shared__ int32_t d_cnt[kNfBlock];
  __shared__ int32_t u_cnt[kNfBlock];
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
  // wavefront-uniform loop: every lane of a wavefront takes part in the
  // cooperative collections, lanes past the row's end without a cluster
  const int lane = lane_id();
  for (int64_t i0 = b + (t - lane); i0 < e; i0 += blockDim.x) {
    const int64_t i = i0 + lane;
    const bool act = i < e;
    const float4 ph = act ? g.pts[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float yh = ph.x, zh = ph.y;
    const float pz = wz + box_pad(zh), py = wy + box_pad(yh);
    const int zu0 = g.zbin(ku, zh - pz), zu1 = g.zbin(ku, zh + pz);
    const int zd0 = g.zbin(kd, zh - pz), zd1 = g.zbin(kd, zh + pz);
    const int yu0 = g.ybin(r + 1, yh - py), yu1 = g.ybin(r + 1, yh + py);
    const int yd0 = g.ybin(r - 1, yh - py), yd1 = g.ybin(r - 1, yh + py);

    const int nd = nf_collect_wave(g, bd, nyd, zd0, zd1, yd0, yd1, act, yh, zh, wy, wz, d_pos, d_cnt, t);
    const int nu = nf_collect_wave(g, bu, nyu, zu0, zu1, yu0, yu1, act && nd > 0, yh, zh, wy, wz, u_pos,
                                   u_cnt, t);
    if (!act) continue;
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
      // all (u, d) pairs in one loop: a = up index, c = down index
      int a = 0, c = 0;
      for (int q = nu * nd; q > 0; --q) {
        const int32_t ja = u_pos[a][t], jc = d_pos[c][t];
        const float4 U = g.pts[ja], Dn = g.pts[jc];
        consider(U.x, U.y, ja, Dn.x, Dn.y, jc);
        if (++c == nd) {
          c = 0;
          ++a;
        }
      }
    } else {
      // more candidates than LDS holds: scan both rows directly
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
