// Search grid ("fast cluster search grid" of the sector tracking, paper
// Section 3): per (unit, row) the clusters are binned on a 2-D (z, y) grid,
// z-major, and stored sorted by bin.  A box query then reads one contiguous
// range of sorted clusters per z bin.  The grid only accelerates searches:
// every query is widened so that it covers all clusters its exact predicate
// can accept, and every selection breaks ties by the caller's cluster index,
// so results do not depend on binning or on the order inside a bin.
#pragma once

#include "tpcx_common.h"

namespace tpcx {

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// One block per unit: z range of its clusters -> bin origin and scale.
__global__ void k_unit_zrange(const int64_t* __restrict__ row_begin, const float* __restrict__ z,
                              int n_rows, int nz, UnitZ* __restrict__ unit_z) {
  __shared__ float smin[1024 / kWave], smax[1024 / kWave];
  const int u = blockIdx.x;
  const int64_t b = row_begin[int64_t(u) * n_rows], e = row_begin[int64_t(u + 1) * n_rows];
  float lo = INFINITY, hi = -INFINITY;
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    float v = z[i];
    lo = fminf(lo, v);
    hi = fmaxf(hi, v);
  }
  for (int d = kWave / 2; d > 0; d >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, d, kWave));
    hi = fmaxf(hi, __shfl_xor(hi, d, kWave));
  }
  const int wid = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
  if (lane_id() == 0) {
    smin[wid] = lo;
    smax[wid] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < nw; ++w) {
      lo = fminf(lo, smin[w]);
      hi = fmaxf(hi, smax[w]);
    }
    UnitZ g;
    float span = hi - lo;
    if (!(span > 0.0f) || !isfinite(span)) {
      g.zmin = isfinite(lo) ? lo : 0.0f;
      g.inv_bz = 0.0f;
    } else {
      g.zmin = lo;
      g.inv_bz = float(nz) / span;
    }
    unit_z[u] = g;
  }
}

// One block per (unit, row): bin key of every cluster and its slot in the bin.
__global__ void k_grid_count(const int64_t* __restrict__ row_begin, const float* __restrict__ y,
                             const float* __restrict__ z, Grid g, int32_t* __restrict__ bin_cnt,
                             int32_t* __restrict__ key, int32_t* __restrict__ slot) {
  const int k = blockIdx.x;
  const int u = k / g.n_rows, r = k % g.n_rows;
  const int64_t b = row_begin[k], e = row_begin[k + 1];
  const int64_t base = g.row_base(u, r);
  const int ny = g.rows[r].ny;
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    int kk = g.zbin(u, z[i]) * ny + g.ybin(r, y[i]);
    key[i] = kk;
    slot[i] = atomicAdd(&bin_cnt[base + kk], 1);
  }
}

// One block per (unit, row): bin counts -> absolute start positions, in place,
// with the row end in the sentinel entry after the last bin.
__global__ void k_grid_scan(const int64_t* __restrict__ row_begin, Grid g,
                            int32_t* __restrict__ bins) {
  __shared__ int64_t lds[1024 / kWave];
  const int k = blockIdx.x;
  const int u = k / g.n_rows, r = k % g.n_rows;
  const int64_t base = g.row_base(u, r);
  const int nb = g.nz * g.rows[r].ny;
  int64_t run = row_begin[k];
  for (int t0 = 0; t0 < nb; t0 += blockDim.x) {
    int t = t0 + threadIdx.x;
    int64_t c = t < nb ? bins[base + t] : 0;
    int64_t tot;
    int64_t ex = block_exclusive_scan(c, lds, &tot);
    if (t < nb) bins[base + t] = int32_t(run + ex);
    run += tot;
  }
  if (threadIdx.x == 0) bins[base + nb] = int32_t(run);
}

// One block per (unit, row): move every cluster to its sorted position.
__global__ void k_grid_scatter(const int64_t* __restrict__ row_begin, const float* __restrict__ y,
                               const float* __restrict__ z, const int32_t* __restrict__ key,
                               const int32_t* __restrict__ slot, Grid g, float* __restrict__ sy,
                               float* __restrict__ sz, int32_t* __restrict__ sid) {
  const int k = blockIdx.x;
  const int u = k / g.n_rows, r = k % g.n_rows;
  const int64_t b = row_begin[k], e = row_begin[k + 1];
  const int64_t base = g.row_base(u, r);
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    int64_t pos = g.bin_start[base + key[i]] + slot[i];
    sy[pos] = y[i];
    sz[pos] = z[i];
    sid[pos] = int32_t(i);
  }
}

}  // namespace tpcx
