// Processing order of tracks by length, longest first, within chunks of
// kLenChunk consecutive tracks: one lane per track kernels (the
// three-iteration fit) then give a wavefront tracks of about equal length,
// so its lanes finish together instead of waiting for the longest of 64,
// while the tracks running at a time still come from one region of the
// track list (their clusters from a few sectors, which stay in the caches).
// A counting sort over min(length, 255) in each chunk, in LDS.  The order
// inside a (chunk, length) group is free: each track's result does not depend
// on when or where it runs.
#pragma once

#include "tpcx_common.h"

namespace tpcx {

constexpr int kLenBins = 256;
constexpr int kLenChunk = 8192;
constexpr int kLenThreads = 256;

__device__ __forceinline__ int len_bin(int64_t hb0, int64_t hb1) {
  const int64_t n = hb1 - hb0;
  return kLenBins - 1 - int(n < 0 ? 0 : (n > kLenBins - 1 ? kLenBins - 1 : n));
}

// order[b .. e) = the tracks b .. e of the block's chunk, longest first.
__global__ void __launch_bounds__(kLenThreads) k_len_order(int64_t n, const int64_t* __restrict__ hit_begin,
                                                           int32_t* __restrict__ order) {
  __shared__ int32_t h[kLenBins];
  __shared__ int64_t lds[kLenThreads / kWave];
  const int64_t b = int64_t(blockIdx.x) * kLenChunk;
  const int64_t e = min(n, b + kLenChunk);
  h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t t = b + threadIdx.x; t < e; t += kLenThreads) atomicAdd(&h[len_bin(hit_begin[t], hit_begin[t + 1])], 1);
  __syncthreads();
  const int32_t c = h[threadIdx.x];
  int64_t tot;
  const int64_t off = block_exclusive_scan(c, lds, &tot);
  __syncthreads();
  h[threadIdx.x] = int32_t(off);
  __syncthreads();
  for (int64_t t = b + threadIdx.x; t < e; t += kLenThreads) {
    const int32_t pos = atomicAdd(&h[len_bin(hit_begin[t], hit_begin[t + 1])], 1);
    order[b + pos] = int32_t(t);
  }
}

// order[0 .. n) from hit_begin[0 .. n]; n < 2^31.
inline void enqueue_length_order(int64_t n, const int64_t* hit_begin, int32_t* order, hipStream_t stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_len_order, dim3(int((n + kLenChunk - 1) / kLenChunk)), dim3(kLenThreads), 0, stream, n,
                     hit_begin, order);
}

}  // namespace tpcx
