// Shared device-side definitions of the tpcx kernels (one translation unit).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpcx {

constexpr int kWave = 64;

// Capacity-overflow bits of the status word (counts[3]): starts, tracklets, hits.
constexpr int64_t kStOverflow = 7;

// Method constants in the precision the kernels compute in.
struct DevParams {
  float kappa;   // d sin(phi) / dx per unit of q/pT
  float sy2, sz2;
  float wy, wz, d2max, chi2max, smax, umax, cww0;
  int32_t min_hits, max_misses, descent_rows;
};

// Search-grid description of one pad row (identical for every unit).
struct RowInfo {
  int32_t ny;      // bins along y
  int32_t cum_ny;  // sum of ny over the rows below
  float y0;        // lower y edge of bin 0
  float inv_by;    // bins per cm along y
};

// z binning of one (unit, row) of the search grid.
struct UnitZ {
  float zmin;
  float inv_bz;  // bins per cm along z
};

// Read-only view of the sorted, binned clusters.  k = unit * n_rows + row.
struct Grid {
  const RowInfo* rows;
  const UnitZ* row_z;        // [n_units * n_rows]
  const int32_t* bin_start;  // [n_units * btot]; absolute sorted positions
  const float4* pts;         // sorted clusters: y, z, caller id (bits), cleaned up-link (bits)
  int32_t n_rows, nz;
  int64_t btot;  // bins (+1 sentinel per row) of one unit

  __device__ __forceinline__ int64_t row_base(int k) const {
    const int u = k / n_rows, r = k - u * n_rows;
    return int64_t(u) * btot + int64_t(nz) * rows[r].cum_ny + r;
  }
  __device__ __forceinline__ int zbin(int k, float z) const {
    UnitZ g = row_z[k];
    float v = (z - g.zmin) * g.inv_bz;
    v = fminf(fmaxf(v, 0.0f), float(nz - 1));
    return int(v);
  }
  __device__ __forceinline__ int ybin(int r, float y) const {
    RowInfo ri = rows[r];
    float v = (y - ri.y0) * ri.inv_by;
    v = fminf(fmaxf(v, 0.0f), float(ri.ny - 1));
    return int(v);
  }
};

// The binning of one grid row k = unit * n_rows + r, read once: a search can
// load it before the state it searches for is known.
struct RowView {
  UnitZ uz;
  RowInfo ri;
  int64_t base;  // first bin of the row
  int nz;

  __device__ __forceinline__ RowView(const Grid& g, int k, int r) {
    uz = g.row_z[k];
    ri = g.rows[r];
    base = int64_t(k / g.n_rows) * g.btot + int64_t(g.nz) * ri.cum_ny + r;
    nz = g.nz;
  }
  __device__ __forceinline__ int zbin(float z) const {
    float v = (z - uz.zmin) * uz.inv_bz;
    v = fminf(fmaxf(v, 0.0f), float(nz - 1));
    return int(v);
  }
  __device__ __forceinline__ int ybin(float y) const {
    float v = (y - ri.y0) * ri.inv_by;
    v = fminf(fmaxf(v, 0.0f), float(ri.ny - 1));
    return int(v);
  }
};

// Widening of a search box so that it covers every cluster an exact float
// predicate can accept (absolute plus relative slack on the coordinate).
__device__ __forceinline__ float box_pad(float v) { return 1e-3f + 1e-6f * fabsf(v); }

// Largest k in [0, n) with a[k] <= v (a non-decreasing, a[0] <= v).
__device__ __forceinline__ int upper_row(const int64_t* a, int n, int64_t v) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (a[mid] <= v)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// The dispatcher hands workgroups to the 8 XCDs round-robin (workgroup b runs
// on XCD b % 8).  xcd_block() renumbers them so that each XCD gets runs of
// kXcdChunk consecutive logical blocks (neighbouring (unit, row) blocks then
// share one L2), while the 8 XCDs work on neighbouring runs at the same time
// (and share the Infinity Cache).  A bijection of [0, gridDim.x): the tail
// that does not fill 8 runs keeps its order.
constexpr int kXcds = 8;
constexpr int64_t kXcdChunk = 16;

__device__ __forceinline__ int64_t xcd_block() {
  const int64_t n = gridDim.x, b = blockIdx.x;
  const int64_t whole = n / (kXcds * kXcdChunk) * (kXcds * kXcdChunk);
  if (b >= whole) return b;
  const int64_t x = b % kXcds, i = b / kXcds;
  return (i / kXcdChunk) * (kXcds * kXcdChunk) + x * kXcdChunk + (i % kXcdChunk);
}

// Inclusive scans over the 64 lanes of a wavefront on the DPP lane network:
// inside each row of 16 lanes by shifts of 1, 2, 4 and 8 lanes, then across
// rows by broadcasting lane 15 into rows 1 and 3 and lane 31 into rows 2 and
// 3.  A lane whose source lies outside its row (or whose row is masked off)
// keeps `old`, the operation's identity.  All 64 lanes must be active.
__device__ __forceinline__ int wave_scan_add(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

// Inclusive maximum scan of values >= -1 (identity -1).
__device__ __forceinline__ int wave_scan_max(int x) {
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x111, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x112, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x114, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x118, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x142, 0xa, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x143, 0xc, 0xf, false));
  return x;
}

__device__ __forceinline__ uint64_t lanes_below() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Exclusive block-wide prefix sum of one int64 per thread; returns this
// thread's prefix and writes the block total to *total.  `lds` holds one
// entry per wave.  All threads of the block must call it.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* lds, int64_t* total) {
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  int64_t x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int64_t y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  if (lane == kWave - 1) lds[wid] = x;
  __syncthreads();
  if (wid == 0) {
    int64_t w = lane < nw ? lds[lane] : 0;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      int64_t y = __shfl_up(w, d, kWave);
      if (lane >= d) w += y;
    }
    if (lane < nw) lds[lane] = w;
  }
  __syncthreads();
  int64_t wave_off = wid > 0 ? lds[wid - 1] : 0;
  *total = lds[nw - 1];
  __syncthreads();
  return wave_off + x - v;
}

}  // namespace tpcx
