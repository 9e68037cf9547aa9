// Search grid ("fast cluster search grid" of the sector tracking, paper
// Section 3): per (unit, row) the clusters are binned on a 2-D (z, y) grid,
// z-major, and stored sorted by bin.  A box query then reads one contiguous
// range of sorted clusters per z bin.  The grid only accelerates searches:
// every query is widened so that it covers all clusters its exact predicate
// can accept, and every selection breaks ties by the caller's cluster index,
// so results do not depend on binning or on the order inside a bin.
//
// Every later stage works on sorted positions.  A sorted cluster is one
// 16-byte record (y, z, caller id, cleaned up-link), so a candidate test or a
// chain step reads a single line.  A row keeps the same index range in both
// orders.
//
// One block builds one row: z range (block reduction), histogram of bin keys
// in LDS, block-wide scan, then a scatter through LDS cursors.
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

__device__ __forceinline__ float block_reduce_min(float v, float* lds) {
  for (int d = kWave / 2; d > 0; d >>= 1) v = fminf(v, __shfl_xor(v, d, kWave));
  const int wid = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
  __syncthreads();
  if (lane_id() == 0) lds[wid] = v;
  __syncthreads();
  float r = lds[0];
  for (int w = 1; w < nw; ++w) r = fminf(r, lds[w]);
  return r;
}

__device__ __forceinline__ float block_reduce_max(float v, float* lds) {
  for (int d = kWave / 2; d > 0; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, kWave));
  const int wid = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
  __syncthreads();
  if (lane_id() == 0) lds[wid] = v;
  __syncthreads();
  float r = lds[0];
  for (int w = 1; w < nw; ++w) r = fmaxf(r, lds[w]);
  return r;
}

// Dynamic LDS: nz * ny + 1 int32 bin counters of the row.
// Status bit set when a coordinate is not finite (such a cluster passes no
// window or chi2 test later, so it links to and joins nothing).
constexpr unsigned long long kStNonFinite = 8;

__global__ void k_grid_build(const int64_t* __restrict__ row_begin, const float* __restrict__ y,
                             const float* __restrict__ z, Grid g, UnitZ* __restrict__ row_z,
                             int32_t* __restrict__ bins, float4* __restrict__ pts,
                             unsigned long long* __restrict__ status) {
  extern __shared__ int32_t hist[];
  __shared__ float red[1024 / kWave];
  __shared__ int64_t scan_lds[1024 / kWave];
  const int k = int(xcd_block());
  const int r = k % g.n_rows;
  const int64_t b = row_begin[k], e = row_begin[k + 1];
  const int ny = g.rows[r].ny;
  const int nb = g.nz * ny;
  const int64_t base = g.row_base(k);

  // z range of the row
  float lo = INFINITY, hi = -INFINITY;
  bool bad = false;
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    const float v = z[i];
    lo = fminf(lo, v);
    hi = fmaxf(hi, v);
    bad |= !(isfinite(v) && isfinite(y[i]));
  }
  if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(status, kStNonFinite);
  lo = block_reduce_min(lo, red);
  hi = block_reduce_max(hi, red);
  UnitZ rz;
  const float span = hi - lo;
  if (!(span > 0.0f) || !isfinite(span)) {
    rz.zmin = isfinite(lo) ? lo : 0.0f;
    rz.inv_bz = 0.0f;
  } else {
    rz.zmin = lo;
    rz.inv_bz = float(g.nz) / span;
  }
  if (threadIdx.x == 0) row_z[k] = rz;

  // histogram
  for (int t = threadIdx.x; t <= nb; t += blockDim.x) hist[t] = 0;
  __syncthreads();
  const RowInfo ri = g.rows[r];
  auto key_of = [&](float yy, float zz) {
    float vz = (zz - rz.zmin) * rz.inv_bz;
    vz = fminf(fmaxf(vz, 0.0f), float(g.nz - 1));
    float vy = (yy - ri.y0) * ri.inv_by;
    vy = fminf(fmaxf(vy, 0.0f), float(ny - 1));
    return int(vz) * ny + int(vy);
  };
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) atomicAdd(&hist[key_of(y[i], z[i])], 1);
  __syncthreads();

  // exclusive scan of the counters: each thread a contiguous chunk
  const int per = (nb + blockDim.x - 1) / blockDim.x;
  const int t0 = min(nb, int(threadIdx.x) * per), t1 = min(nb, t0 + per);
  int64_t s = 0;
  for (int t = t0; t < t1; ++t) s += hist[t];
  int64_t tot;
  int64_t run = block_exclusive_scan(s, scan_lds, &tot) + b;
  for (int t = t0; t < t1; ++t) {
    const int32_t c = hist[t];
    hist[t] = int32_t(run);
    run += c;
  }
  __syncthreads();
  // bin starts out of LDS, coalesced
  for (int t = threadIdx.x; t < nb; t += blockDim.x) bins[base + t] = hist[t];
  if (threadIdx.x == 0) bins[base + nb] = int32_t(e);
  __syncthreads();

  // scatter through the LDS cursors (order inside a bin is free)
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    const float yy = y[i], zz = z[i];
    const int32_t pos = atomicAdd(&hist[key_of(yy, zz)], 1);
    pts[pos] = make_float4(yy, zz, __int_as_float(int32_t(i)), __int_as_float(-1));
  }
}

}  // namespace tpcx
