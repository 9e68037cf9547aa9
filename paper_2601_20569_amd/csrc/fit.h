// Three-iteration track fit with interpolation-based cluster rejection
// (paper, Section 2, track fit: inwards, outwards, inwards; the cluster chi2
// cut against the interpolation of two iterations' states, the position and
// covariance of one iteration kept in reduced precision; Section 3, Phase I:
// the first, inward iteration stores, the second, outward one interpolates
// and cuts, the third applies the rejection).
//
// One lane per track, tracks taken longest first within chunks of
// consecutive tracks (so the lanes of a wavefront have equal work); the
// stored records are interleaved per wavefront so that its lanes read and
// write one contiguous block per step, and every step's record and row are
// loaded one step ahead.  Iteration 1 walks from the tracking result at x_ref
// out to the outermost cluster, restarts there (y, z of the cluster, diagonal
// covariance) and goes inwards; at every cluster it stores, per hit, the
// cluster relative to the track's origin (its outermost cluster) and the
// predicted residual and variances of y and z as bfloat16 (one 16-byte
// record).  Iteration 2 restarts at the innermost cluster and goes outwards;
// the inverse-variance combination of its prediction with the stored one
// gives the interpolation, whose chi2 above the cut rejects the cluster; it
// updates with every cluster.  Iteration 3 restarts at the outermost kept
// cluster and goes inwards over the kept ones.  IEEE binary32, no
// contraction, correctly rounded divide and square root: every decision is
// reproducible bit for bit.
#pragma once

#include "order.h"
#include "tpcx_common.h"
#include "tracklet.h"

namespace tpcx {

struct FitIn {
  int64_t n_tracks;
  int32_t n_rows;  // of row_x (at most 255)
  const int64_t* hit_begin;
  const int32_t* hit_id;
  const uint8_t* hit_row;
  const float* seed;   // [n][5]
  const float* x_ref;  // [n]
  const float2* yz;    // clusters' y, z side by side (one gather per hit)
  const float* row_x;
};

struct FitOut {
  float* param;   // [n][5]
  float* cov;     // [n][15]
  float* chi2;
  float* x_out;
  int32_t* n_kept;
  int32_t* ok;
  uint8_t* reject;  // [hits]
};

struct FitConsts {
  float chi2_cut, vs, vt, vw;
};

// bfloat16 storage: the float's 16 high bits, rounded to nearest (ties to even).
__device__ __forceinline__ uint32_t bf16_bits(float v) {
  const uint32_t b = __float_as_uint(v);
  return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

__device__ __forceinline__ void fit_reset_cov(KState& q, const DevParams& p, const FitConsts& f) {
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

// Propagation without a cached (cos, sin/cos) of the current state.
__device__ __forceinline__ bool fit_prop(KState& q, float x1, const DevParams& p) {
  float cp = 0.0f, rp = 0.0f;
  bool cached = false;
  return kf_propagate<false>(q, x1, p, cp, rp, cached);
}

__device__ __forceinline__ float fit_update(KState& q, float my, float mz, const DevParams& p) {
  const KInnov n = kf_innov(q, p);
  const float iSy = 1.0f / n.sy;
  const float iSz = 1.0f / n.sz;
  return kf_update<false>(q, my, mz, n, iSy, iSz, p);
}

// C_yy and C_zz of the factorised covariance (as multiplied out for output).
__device__ __forceinline__ float fit_cyy(const KState& q) {
  const float cwy = q.uyw * q.dw;
  return (q.dy + q.uys * (q.uys * q.ds)) + q.uyw * cwy;
}
__device__ __forceinline__ float fit_czz(const KState& q) {
  const float ctz = q.uzt * q.dt;
  return q.dz + q.uzt * ctz;
}

// Records of iteration 1 (and the rows of a track's clusters) in a
// workspace of `cap` slots.  When the wavefronts' records fit (every track
// shorter than 256 clusters guarantees it), wavefront w's slots start at
// wbase[w] and record i of its lane l is slot wbase[w] + 64 i + l: the 64
// lanes' records of one step are one contiguous 1 KiB (coalesced).
// Otherwise record i of a track is slot hit_begin + i.  The layout changes
// no value.
struct FitWs {
  float4* rec;
  uint8_t* rows;
  const int64_t* wbase;  // [n_waves + 1]; wbase[n_waves] = slots needed
  int64_t cap;
};

// yz[c] = (y[c], z[c]): the fit gathers one 8-byte pair per hit instead of
// two 4-byte values from separate arrays.
__global__ void k_fit_pack(int64_t n, const float* __restrict__ y, const float* __restrict__ z,
                           float2* __restrict__ yz) {
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < n; c += int64_t(gridDim.x) * blockDim.x)
    yz[c] = make_float2(y[c], z[c]);
}

// wlen[w] = 64 x the longest track of wavefront w (processing order).
__global__ void k_fit_wave_len(int64_t n, const int64_t* __restrict__ hit_begin,
                               const int32_t* __restrict__ order, int64_t* __restrict__ wlen) {
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int m = 0;
  if (gid < n) {
    const int64_t t = order[gid];
    m = int(min(hit_begin[t + 1] - hit_begin[t], int64_t(1) << 30));
  }
  for (int d = kWave / 2; d > 0; d >>= 1) m = max(m, __shfl_xor(m, d, kWave));
  if (lane_id() == 0 && gid < n) wlen[gid / kWave] = int64_t(m) * kWave;
}

// wbase[0 .. nw] = exclusive prefix sum of wlen[0 .. nw); one block of
// kFitScanThreads, each summing a contiguous run.
constexpr int kFitScanThreads = 1024;

__global__ void __launch_bounds__(kFitScanThreads) k_fit_scan(int64_t nw, const int64_t* __restrict__ wlen,
                                                             int64_t* __restrict__ wbase) {
  __shared__ int64_t lds[kFitScanThreads / kWave];
  const int64_t per = (nw + kFitScanThreads - 1) / kFitScanThreads;
  const int64_t b = min(nw, int64_t(threadIdx.x) * per), e = min(nw, b + per);
  int64_t s = 0;
  for (int64_t w = b; w < e; ++w) s += wlen[w];
  int64_t tot;
  int64_t run = block_exclusive_scan(s, lds, &tot);
  for (int64_t w = b; w < e; ++w) {
    wbase[w] = run;
    run += wlen[w];
  }
  if (threadIdx.x == 0) wbase[nw] = tot;
}

// rec slot = (cluster y, z relative to the origin, bf16 (d_y | d_z), bf16 (C_yy | C_zz));
// iteration 2 replaces the last word by the rejection flag.
__global__ void __launch_bounds__(kWave) k_fit(FitIn in, DevParams p, FitConsts f, const int32_t* __restrict__ order,
                                               FitWs ws, FitOut out) {
  __shared__ float srx[256];
  for (int r = threadIdx.x; r < 256; r += kWave) srx[r] = r < in.n_rows ? in.row_x[r] : __builtin_nanf("");
  __syncthreads();
  const int64_t gid = int64_t(blockIdx.x) * kWave + threadIdx.x;
  if (gid >= in.n_tracks) return;
  const int64_t nw = (in.n_tracks + kWave - 1) / kWave;
  const bool inter = ws.wbase[nw] <= ws.cap;
  const int64_t t = order[gid];
  const int64_t b = in.hit_begin[t];
  const int n = int(in.hit_begin[t + 1] - b);
  const int64_t s0 = inter ? ws.wbase[blockIdx.x] + threadIdx.x : b;
  const int64_t ss = inter ? kWave : 1;
  float4* R = ws.rec + s0;
  const uint8_t* rowp = inter ? ws.rows + s0 : in.hit_row + b;  // rows for iterations 2, 3
  uint8_t* rej = out.reject + b;
  bool good = n >= 3;
  int kept = 0;
  float chi2 = 0.0f;
  KState last{};
  const float2 o2 = good ? in.yz[in.hit_id[b + n - 1]] : make_float2(0.0f, 0.0f);
  const float oy = o2.x, oz = o2.y;
  auto X = [&](int i) { return srx[in.hit_row[b + i]]; };
  if (good) {
    // ---- iteration 1: inwards, storing the predictions
    const float* sd = in.seed + 5 * t;
    const float xref = in.x_ref[t];
    KState q{};
    q.x = xref;
    q.y = sd[0] - oy;
    q.z = sd[1] - oz;
    q.s = sd[2];
    q.t = sd[3];
    q.w = sd[4];
    fit_reset_cov(q, p, f);
    int first = 0;
    while (first < n && !(X(first) > xref)) ++first;
    {
      // out to the outermost cluster; the next row is loaded one step ahead
      int rn = first < n ? in.hit_row[b + first] : 0;
      for (int i = first; i < n && good; ++i) {
        const float xi = srx[rn];
        if (i + 1 < n) rn = in.hit_row[b + i + 1];
        if (!(q.x == xi)) good = fit_prop(q, xi, p);
      }
    }
    const float xo = X(n - 1);
    if (good && !(q.x == xo)) good = fit_prop(q, xo, p);
    if (good) {
      q.y = 0.0f;  // the outermost cluster is the origin
      q.z = 0.0f;
      fit_reset_cov(q, p, f);
      R[(n - 1) * ss] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (inter) ws.rows[s0 + (n - 1) * ss] = in.hit_row[b + n - 1];
      // Two register sets, A for the hits n-2, n-4, ... and B for n-3, n-5,
      // ...: a step uses its set's cluster (y, z, row) and reloads the set
      // for the hit two steps later, whose id the set loaded two steps
      // before; so no register is copied between steps, and a step waits
      // only for loads two steps old.  Every lane runs every step of the
      // wavefront's loop (its loads with indices clamped into the track, its
      // arithmetic only while active), so the loads are never conditional.
      auto hid = [&](int j) { return in.hit_id[b + max(j, 0)]; };
      float2 mA, mB;
      int rA, rB;
      int32_t idA, idB;
      {
        mA = in.yz[hid(n - 2)];
        rA = in.hit_row[b + n - 2];
        idA = hid(n - 4);
        mB = in.yz[hid(n - 3)];
        rB = in.hit_row[b + max(n - 3, 0)];
        idB = hid(n - 5);
      }
      auto step = [&](float2& mv, int& rv, int32_t& idv, int i, bool act) {
        if (act) {
          const float ry = mv.x - oy, rz = mv.y - oz;
          if (inter) ws.rows[s0 + i * ss] = uint8_t(rv);
          good = fit_prop(q, srx[rv], p);
          if (good) {
            const uint32_t dd = bf16_bits(q.y - ry) | (bf16_bits(q.z - rz) << 16);
            const uint32_t cc = bf16_bits(fit_cyy(q)) | (bf16_bits(fit_czz(q)) << 16);
            R[i * ss] = make_float4(ry, rz, __uint_as_float(dd), __uint_as_float(cc));
            fit_update(q, ry, rz, p);
          }
        }
        // the set's reload, after its use (into the same registers)
        rv = in.hit_row[b + max(i - 2, 0)];
        mv = in.yz[idv];
        idv = hid(i - 4);
      };
      for (int i = n - 2;; i -= 2) {
        const bool a0 = good && i >= 0;
        if (__ballot(a0) == 0ull) break;
        step(mA, rA, idA, i, a0);
        step(mB, rB, idB, i - 1, good && i - 1 >= 0);
      }
    }
    // ---- iteration 2: outwards, interpolation and chi2 cut
    if (good) {
      // two register sets (records and rows of the even and the odd
      // steps), each reloaded after its use for the step two later, every
      // lane running every step of the wavefront's loop (as in iteration 1)
      float4 rA = R[0], rB = R[ss];
      int xA = rowp[0], xB = rowp[ss];
      const float s1 = q.s, t1 = q.t, w1 = q.w;
      q = KState{};
      q.x = srx[xA];
      q.y = rA.x;
      q.z = rA.y;
      q.s = s1;
      q.t = t1;
      q.w = w1;
      fit_reset_cov(q, p, f);
      // rejection flags gathered per 4-byte word of rej (whole words stored
      // where they lie inside the track)
      uint32_t racc = 0;
      const uint32_t rmis = uint32_t(reinterpret_cast<uintptr_t>(rej) & 3);
      auto put_flag = [&](int i, uint32_t rj) {
        const uint32_t lb = (rmis + uint32_t(i)) & 3;
        racc |= rj << (8 * lb);
        if (lb == 3 || i == n - 1) {
          const int i0 = i - int(lb);
          if (lb == 3 && i0 >= 0) {
            *reinterpret_cast<uint32_t*>(rej + i0) = racc;
          } else {
            for (int k = max(i0, 0); k <= i; ++k) rej[k] = uint8_t(racc >> (8 * (k - i0)));
          }
          racc = 0;
        }
      };
      auto step2 = [&](float4& rv, int& xv, int i, bool act) {
        if (act) {
          if (i > 0) good = fit_prop(q, srx[xv], p);
          if (good) {
            const float4 ri = rv;
            const float ry = i == n - 1 ? 0.0f : ri.x, rz = i == n - 1 ? 0.0f : ri.y;
            float dy, dz, vy, vz;
            if (i == 0) {
              const uint32_t dd = __float_as_uint(ri.z), cc = __float_as_uint(ri.w);
              dy = bf16_lo(dd);
              dz = bf16_hi(dd);
              vy = bf16_lo(cc);
              vz = bf16_hi(cc);
            } else {
              const float cy = fit_cyy(q), cz = fit_czz(q);
              const float dout = q.y - ry, eout = q.z - rz;
              if (i == n - 1) {
                dy = dout;
                dz = eout;
                vy = cy;
                vz = cz;
              } else {
                const uint32_t dd = __float_as_uint(ri.z), cc = __float_as_uint(ri.w);
                const float din = bf16_lo(dd), ein = bf16_hi(dd), cin = bf16_lo(cc), kin = bf16_hi(cc);
                const float iy = 1.0f / (cin + cy);
                const float iz = 1.0f / (kin + cz);
                dy = (din * cy + dout * cin) * iy;
                dz = (ein * cz + eout * kin) * iz;
                vy = (cin * cy) * iy;
                vz = (kin * cz) * iz;
              }
            }
            const float c2 = (dy * dy) / (vy + p.sy2) + (dz * dz) / (vz + p.sz2);
            const uint32_t rj = c2 > f.chi2_cut ? 1u : 0u;
            put_flag(i, rj);
            reinterpret_cast<float*>(&R[i * ss])[3] = __uint_as_float(rj);
            if (i > 0) fit_update(q, ry, rz, p);
          }
        }
        const int64_t nx = min(i + 2, n - 1);
        rv = R[nx * ss];
        xv = rowp[nx * ss];
      };
      for (int i = 0;; i += 2) {
        const bool a0 = good && i < n;
        if (__ballot(a0) == 0ull) break;
        step2(rA, xA, i, a0);
        step2(rB, xB, i + 1, good && i + 1 < n);
      }
    }
    // ---- iteration 3: inwards over the kept clusters
    if (good) {
      auto flag = [&](int i) { return __float_as_uint(reinterpret_cast<const float*>(&R[i * ss])[3]) != 0u; };
      int j = n - 1;
      while (j >= 0 && flag(j)) --j;
      good = j >= 2;
      for (int i = n - 2; i >= j && good; --i) good = fit_prop(q, srx[rowp[i * ss]], p);
      if (good) {
        const float4 rj = R[j * ss];
        q.y = j == n - 1 ? 0.0f : rj.x;
        q.z = j == n - 1 ? 0.0f : rj.y;
        fit_reset_cov(q, p, f);
        kept = 1;
        last = q;
        float4 rn = j > 0 ? R[(j - 1) * ss] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        int xn = j > 0 ? rowp[(j - 1) * ss] : 0;
        for (int i = j - 1; i >= 0 && good; --i) {
          const float4 ri = rn;
          const int xi = xn;
          if (i > 0) {
            rn = R[(i - 1) * ss];
            xn = rowp[(i - 1) * ss];
          }
          good = fit_prop(q, srx[xi], p);
          if (!good || __float_as_uint(ri.w) != 0u) continue;
          chi2 = chi2 + fit_update(q, ri.x, ri.y, p);
          ++kept;
          last = q;
        }
        good = good && kept >= 3;
      }
    }
  }
  if (!good) {
    // a failed fit rejects nothing
    for (int i = 0; i < n; ++i) rej[i] = 0;
    out.ok[t] = 0;
    out.n_kept[t] = 0;
    out.chi2[t] = 0.0f;
    out.x_out[t] = 0.0f;
    for (int k = 0; k < 5; ++k) out.param[5 * t + k] = 0.0f;
    for (int k = 0; k < 15; ++k) out.cov[15 * t + k] = 0.0f;
    return;
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
