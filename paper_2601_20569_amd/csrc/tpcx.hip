// tpcx: host side of the C interface declared in include/tpcx.h, and the
// single translation unit that holds every kernel.
#include "../../include/tpcx.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "grid.h"
#include "links.h"
#include "refit.h"
#include "select.h"
#include "fit.h"
#include "rebuild.h"
#include "merge.h"
#include "tpcx_common.h"
#include "tracklet.h"

using namespace tpcx;

// Workspace of tpcx_track_static, for callers that cannot allocate device
// memory: one copy per device (reserved when the code object is loaded on
// the device, held until the process ends).  Host code never uses this name
// as an address: it resolves the device's copy with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[TPCX_STATIC_SCRATCH_BYTES];

struct tpcx_ctx {
  int device = 0;
  int n_rows = 0;
  std::vector<float> row_x;       // host copy
  std::vector<float> frac;        // neighbour-finder interpolation fractions
  float tan_half = 0.0f;
  DevParams dp{};
  tpcx_params params{};
  tpcx_tuning tuning{};
  bool tuning_fixed = false;
  std::vector<RowInfo> rows_host;
  int32_t sum_ny = 0;
  // device tables (immutable between set-ups)
  float* d_row_x = nullptr;
  float* d_frac = nullptr;
  RowInfo* d_rows = nullptr;
  int n_cu = 256;
  // bin counters of one row that fit the grid build's LDS
  int max_row_bins = 16384;
  // stage timing: (TPCX_N_STAGES + 1) events per recorded call
  std::vector<hipEvent_t> events;
  int32_t timing_max = 0, timing_used = 0;
  // batched form: the graph of the last argument set
  hipGraphExec_t graph = nullptr;
  // batched form: a second stream for the cluster correction, which needs
  // only the search grid and runs beside the tracking stages
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<unsigned char> graph_key;
  // device address of this device's `scratch` array
  void* scratch = nullptr;
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Sub-allocator over the caller's workspace.
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(int64_t n) {
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += align_up(size_t(std::max<int64_t>(n, 1)) * sizeof(T));
    return p;
  }
};

struct Layout {
  UnitZ* row_z;
  int32_t* bins;
  float4* pts;
  int32_t* up;
  int32_t* down;
  uint8_t* flag;
  int32_t* row_cnt;
  int32_t* row_off;
  int32_t* starts;
  int32_t* start_pos;
  int32_t* start_k;
  int32_t* order;
  int32_t* queue;
  int64_t* part;
  TrackletTmp tmp;
  size_t bytes;
};

// compaction blocks: one resident round on 256 CUs (5 blocks of 4 wavefronts
// per CU at the kernel's register count), so no partial last round
constexpr int kKeepBlocks = 1280;
constexpr int kGridBuildBlock = 1024;

int blocks_for(int64_t n, int b) { return int((n + b - 1) / b); }

int64_t bins_per_unit(const tpcx_ctx* c, int nz) { return int64_t(nz) * c->sum_ny + c->n_rows; }

Layout carve(const tpcx_ctx* c, void* ws, int32_t n_units, int64_t n, int64_t cap_start, int nz,
             int /*block*/) {
  Carver cv{static_cast<char*>(ws)};
  Layout L{};
  L.row_z = cv.take<UnitZ>(int64_t(n_units) * c->n_rows);
  L.bins = cv.take<int32_t>(int64_t(n_units) * bins_per_unit(c, nz));
  L.pts = cv.take<float4>(n);
  L.up = cv.take<int32_t>(n);
  L.down = cv.take<int32_t>(n);
  L.flag = cv.take<uint8_t>(n);
  L.row_cnt = cv.take<int32_t>(int64_t(n_units) * c->n_rows);
  L.row_off = cv.take<int32_t>(int64_t(n_units) * c->n_rows);
  L.starts = cv.take<int32_t>(cap_start);
  L.start_pos = cv.take<int32_t>(cap_start);
  L.start_k = cv.take<int32_t>(cap_start);
  L.order = cv.take<int32_t>(cap_start);
  L.queue = cv.take<int32_t>(1);
  L.part = cv.take<int64_t>(2 * kKeepBlocks);
  L.tmp.cap = std::max<int64_t>(cap_start, 1);
  L.tmp.stride = (c->n_rows + 15) / 16 * 16;
  L.tmp.rec = cv.take<uint32_t>(L.tmp.cap * kRecWords);
  L.tmp.hit = cv.take<int32_t>(L.tmp.cap * L.tmp.stride);
  L.bytes = cv.off;
  return L;
}

struct RefitLayout {
  RefitWs ws;
  int32_t* ok;
  size_t bytes;
};

RefitLayout carve_refit(void* base, int64_t n_tracks, int64_t n_hits) {
  Carver cv{static_cast<char*>(base)};
  RefitLayout L{};
  L.ws.xyz = cv.take<float>(4 * std::max<int64_t>(n_hits, 1));
  L.ws.ckpt = cv.take<float>(int64_t(kCkptFloats) * (n_hits / kCkpt + n_tracks + 1));
  L.ws.n_lanes = std::max<int64_t>(n_tracks, 1);
  L.ws.scratch = cv.take<float>(L.ws.n_lanes * kCkpt * kCkptFloats);
  L.ws.acc = cv.take<int64_t>(kMapNCoef);
  L.ws.hgrad = cv.take<float>(4 * std::max<int64_t>(n_hits, 1));
  L.ws.queue = cv.take<unsigned long long>(kXcds);
  L.ok = cv.take<int32_t>(n_tracks);
  L.bytes = cv.off;
  return L;
}

// Workspace of the refit inside the batched call: corrected clusters, one per
// input cluster, and the filter's queue words.
struct BatchRefitLayout {
  float4* corr;
  unsigned long long* queue;
  size_t bytes;
};

BatchRefitLayout carve_batch_refit(void* base, int64_t n_clusters) {
  Carver cv{static_cast<char*>(base)};
  BatchRefitLayout L{};
  L.corr = cv.take<float4>(n_clusters);
  L.queue = cv.take<unsigned long long>(kXcds);
  L.bytes = cv.off;
  return L;
}

// Persistent grid of the refit filter: enough blocks for the tracks, at most
// the tuning's refit_grid (0: kRefitBlocksPerCu per compute unit, the
// filter's occupancy limit).
constexpr int kRefitBlocksPerCu = 8;

int refit_filter_grid(const tpcx_ctx* c, int64_t n_tracks, int32_t refit_grid) {
  const int64_t per_block = int64_t(kRefitBlock) / kWave * kRefitChunk;
  const int64_t cap = refit_grid > 0 ? refit_grid : int64_t(kRefitBlocksPerCu) * c->n_cu;
  return int(std::max<int64_t>(1, std::min<int64_t>((n_tracks + per_block - 1) / per_block, cap)));
}

bool refit_args_ok(const tpcx_ctx* c, const tpcx_refit_in* in) {
  if (!c || !in || in->n_tracks < 0 || in->n_hits < 0) return false;
  if (in->n_tracks > 0 && (!in->hit_begin || !in->hit_id || !in->hit_row || !in->unit || !in->seed ||
                           !in->y || !in->z || !in->unit_alpha))
    return false;
  return true;
}

RefitIn refit_view(const tpcx_ctx* c, const tpcx_refit_in* in) {
  RefitIn r;
  r.n_tracks = in->n_tracks;
  r.n_tracks_dev = nullptr;
  r.status_dev = nullptr;
  r.n_hit = nullptr;
  r.min_hits = 2;
  r.hit_begin = in->hit_begin;
  r.hit_id = in->hit_id;
  r.hit_row = in->hit_row;
  r.unit = in->unit;
  r.seed = in->seed;
  r.y = in->y;
  r.z = in->z;
  r.unit_alpha = in->unit_alpha;
  r.row_x = c->d_row_x;
  return r;
}

int max_row_ny(const tpcx_ctx* c) {
  int m = 1;
  for (const RowInfo& r : c->rows_host) m = std::max(m, r.ny);
  return m;
}

tpcx_tuning effective_tuning(const tpcx_ctx* c, int32_t n_units, int64_t n) {
  tpcx_tuning t = c->tuning;
  if (!c->tuning_fixed) {
    tpcx_default_tuning(n_units, n, &t);
    t.bin_y = c->tuning.bin_y;  // the row table is built for this width
  }
  t.n_zbins = std::max(1, std::min(t.n_zbins, (c->max_row_bins - 1) / max_row_ny(c)));
  return t;
}

bool valid_tuning(const tpcx_tuning& t) {
  return t.bin_y > 0.0f && std::isfinite(t.bin_y) && t.n_zbins >= 1 && t.n_zbins <= 65536 &&
         t.block >= 64 && t.block <= 1024 && t.block % 64 == 0 && t.construct_grid >= 1 &&
         t.construct_refill >= 1 && t.construct_refill <= kWave && t.refit_grid >= 0 &&
         t.refit_refill >= 1 && t.refit_refill <= kWave;
}

// Device address of the current device's `scratch` array, resolved once per
// device and kept for the process (each device holds its own copy).
constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

tpcx_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return TPCX_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TPCX_E_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TPCX_OK;
}

tpcx_status build_rows(tpcx_ctx* c) {
  c->rows_host.resize(c->n_rows);
  int32_t cum = 0;
  for (int r = 0; r < c->n_rows; ++r) {
    const double half = double(c->row_x[r]) * double(c->tan_half);
    int ny = int(std::ceil(2.0 * half / double(c->tuning.bin_y)));
    ny = std::max(1, std::min(ny, 4096));
    RowInfo ri;
    ri.ny = ny;
    ri.cum_ny = cum;
    ri.y0 = float(-half);
    ri.inv_by = float(double(ny) / (2.0 * half));
    c->rows_host[r] = ri;
    cum += ny;
  }
  c->sum_ny = cum;
  if (hipMemcpy(c->d_rows, c->rows_host.data(), sizeof(RowInfo) * c->n_rows, hipMemcpyHostToDevice) !=
      hipSuccess)
    return TPCX_E_HIP;
  return TPCX_OK;
}

}  // namespace

extern "C" {

void tpcx_default_tuning(int32_t n_units, int64_t n_clusters, tpcx_tuning* t) {
  if (!t) return;
  t->bin_y = 2.0f;
  // about half a cluster per bin for rows ~30 y-bins wide (fewer candidates
  // per search box; finer bins than that cost more bin-range loads)
  const double per_row = double(n_clusters) / std::max(1.0, double(n_units) * 152.0);
  int nz = int(per_row / 15.0);
  t->n_zbins = std::max(4, std::min(nz, 4096));
  t->block = 256;
  t->construct_grid = 1024;  // 4 blocks of 4 wavefronts per CU, persistent
  t->construct_refill = 16;
  t->refit_grid = 0;
  // lanes refilled only when all of a wavefront's are idle: its lanes then
  // step through rows together (the filter waits on the cluster loads)
  t->refit_refill = 64;
}

tpcx_status tpcx_create(const tpcx_geometry* g, const tpcx_params* p, const tpcx_tuning* tuning,
                        tpcx_ctx** out) {
  if (!g || !p || !out || !g->row_x_host || g->n_rows < 3 || g->n_rows > 255) return TPCX_E_ARG;
  for (int r = 0; r < g->n_rows; ++r) {
    if (!std::isfinite(g->row_x_host[r]) || (r > 0 && !(g->row_x_host[r] > g->row_x_host[r - 1])))
      return TPCX_E_ARG;
  }
  if (g->n_rows > 32 * kMaskWords) return TPCX_E_ARG;
  if (!(g->tan_half_opening > 0.0f) || !std::isfinite(g->bz_tesla)) return TPCX_E_ARG;
  if (!(p->win_y >= 0.0f) || !(p->win_z >= 0.0f) || !(p->d2_max >= 0.0f) || !(p->chi2_max > 0.0f) ||
      !(p->sinphi_max > 0.0f && p->sinphi_max < 1.0f) || !(p->u_max > 0.0f && p->u_max < 1.0f) ||
      !(p->sigma_y > 0.0f) || !(p->sigma_z > 0.0f) || !(p->cww0 > 0.0f) || p->min_hits < 2 ||
      p->max_misses < 1 || p->descent_rows < 1 || p->descent_rows > 255)
    return TPCX_E_ARG;
  if (tuning && !valid_tuning(*tuning)) return TPCX_E_ARG;
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TPCX_E_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return TPCX_E_HIP;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TPCX_E_DEVICE;

  auto* c = new (std::nothrow) tpcx_ctx;
  if (!c) return TPCX_E_HIP;
  c->device = dev;
  c->n_cu = prop.multiProcessorCount;
  {
    // the grid build keeps a row's bin counters in LDS: as many as the
    // device's LDS per workgroup holds (160 KiB on gfx950)
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        lds > 65536 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_grid_build),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds - 256) == hipSuccess)
      c->max_row_bins = (lds - 256) / int(sizeof(int32_t)) - 1;
    (void)hipGetLastError();
  }
  c->n_rows = g->n_rows;
  c->row_x.assign(g->row_x_host, g->row_x_host + g->n_rows);
  c->tan_half = g->tan_half_opening;
  c->params = *p;
  // constants in the kernels' precision; kappa rounded once from double
  c->dp.kappa = float(2.99792458e-3 * double(g->bz_tesla));
  c->dp.sy2 = p->sigma_y * p->sigma_y;
  c->dp.sz2 = p->sigma_z * p->sigma_z;
  c->dp.wy = p->win_y;
  c->dp.wz = p->win_z;
  c->dp.d2max = p->d2_max;
  c->dp.chi2max = p->chi2_max;
  c->dp.smax = p->sinphi_max;
  c->dp.umax = p->u_max;
  c->dp.cww0 = p->cww0;
  c->dp.min_hits = p->min_hits;
  c->dp.max_misses = p->max_misses;
  c->dp.descent_rows = p->descent_rows;
  c->frac.assign(g->n_rows, 0.0f);
  for (int r = 1; r + 1 < g->n_rows; ++r) {
    const float a = c->row_x[r] - c->row_x[r - 1];
    const float b = c->row_x[r + 1] - c->row_x[r - 1];
    c->frac[r] = a / b;
  }
  if (tuning) {
    c->tuning = *tuning;
    c->tuning_fixed = true;
  } else {
    tpcx_default_tuning(36, 1, &c->tuning);
  }
  bool ok = hipMalloc(&c->d_row_x, sizeof(float) * c->n_rows) == hipSuccess &&
            hipMalloc(&c->d_frac, sizeof(float) * c->n_rows) == hipSuccess &&
            hipMalloc(&c->d_rows, sizeof(RowInfo) * c->n_rows) == hipSuccess &&
            hipMemcpy(c->d_row_x, c->row_x.data(), sizeof(float) * c->n_rows,
                      hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(c->d_frac, c->frac.data(), sizeof(float) * c->n_rows,
                      hipMemcpyHostToDevice) == hipSuccess &&
            hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) == hipSuccess;
  if (!ok || build_rows(c) != TPCX_OK || scratch_address(dev, &c->scratch) != TPCX_OK) {
    tpcx_destroy(c);
    return TPCX_E_HIP;
  }
  *out = c;
  return TPCX_OK;
}

void tpcx_destroy(tpcx_ctx* c) {
  if (!c) return;
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  if (c->d_row_x) (void)hipFree(c->d_row_x);
  if (c->d_frac) (void)hipFree(c->d_frac);
  if (c->d_rows) (void)hipFree(c->d_rows);
  delete c;
}

size_t tpcx_workspace_bytes(const tpcx_ctx* c, int32_t n_units, int64_t n_clusters,
                            int64_t cap_start) {
  if (!c || n_units < 1 || n_clusters < 0 || cap_start < 0) return 0;
  const tpcx_tuning t = effective_tuning(c, n_units, n_clusters);
  return carve(c, nullptr, n_units, n_clusters, cap_start, t.n_zbins, t.block).bytes;
}

}  // extern "C"

namespace {

tpcx_status check_track_args(const tpcx_ctx* c, const tpcx_clusters* in, const void* ws,
                             int64_t cap_start, const tpcx_tracks* out) {
  if (!c || !in || !out || !out->counts || in->n_units < 1 || in->n_clusters < 0 ||
      in->n_clusters >= (int64_t(1) << 31) || cap_start < 0 || cap_start >= (int64_t(1) << 31) ||
      out->cap_tracks < 0 || out->cap_hits < 0)
    return TPCX_E_ARG;
  if (in->n_clusters > 0 && (!in->row_begin || !in->y || !in->z)) return TPCX_E_ARG;
  if (!in->row_begin) return TPCX_E_ARG;
  if ((out->cap_tracks > 0 && (!out->unit || !out->start || !out->n_hits || !out->hit_begin ||
                               !out->x_ref || !out->param || !out->cov || !out->chi2 || !out->ndf)) ||
      (out->cap_hits > 0 && (!out->hit_id || !out->hit_row)))
    return TPCX_E_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return TPCX_E_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device) return TPCX_E_ARG;
  return TPCX_OK;
}

// The whole tracking sequence on `stream`.  `ev` (nullable) receives one event
// per stage boundary.  No host synchronisation and no memset, so the sequence
// can be captured into a graph.
void enqueue_track(const tpcx_ctx* c, const tpcx_clusters* in, const Layout& L, const tpcx_tuning& t,
                   int64_t cap_start, const tpcx_tracks* out, hipStream_t stream, hipEvent_t* ev,
                   hipEvent_t after_grid = nullptr) {
  const int32_t U = in->n_units;
  const int R = c->n_rows;
  const int B = t.block;
  Grid g;
  g.rows = c->d_rows;
  g.row_z = L.row_z;
  g.bin_start = L.bins;
  g.pts = L.pts;
  g.n_rows = R;
  g.nz = t.n_zbins;
  g.btot = bins_per_unit(c, t.n_zbins);
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], stream);
  };
  mark(0);
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, stream, out->counts, int64_t(4), int64_t(0));
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, stream, L.queue, int64_t(1), 0);
  const int UR = U * R;
  const size_t hist_bytes = sizeof(int32_t) * (size_t(t.n_zbins) * max_row_ny(c) + 1);
  // the row's bin counters fill most of the LDS, so one block runs per CU:
  // the largest block keeps 4 wavefronts per SIMD on the row's gathers
  hipLaunchKernelGGL(k_grid_build, dim3(UR), dim3(kGridBuildBlock), hist_bytes, stream, in->row_begin, in->y,
                     in->z, g, L.row_z, L.bins, L.pts,
                     reinterpret_cast<unsigned long long*>(out->counts + 3));
  if (after_grid) (void)hipEventRecord(after_grid, stream);
  mark(1);
  hipLaunchKernelGGL(k_neighbours, dim3(UR), dim3(kNfBlock), 0, stream, in->row_begin, g,
                     c->d_frac, c->dp, L.up, L.down);
  mark(2);
  hipLaunchKernelGGL(k_clean_starts, dim3(UR), dim3(B), 0, stream, in->row_begin, L.up, L.down,
                     L.pts, L.flag, L.row_cnt);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, stream, L.row_cnt, int64_t(UR),
                     L.row_off, out->counts, cap_start, out->counts + 3,
                     int64_t(TPCX_ST_START_OVERFLOW));
  hipLaunchKernelGGL(k_write_starts, dim3(UR), dim3(B), 0, stream, in->row_begin, L.pts, L.flag,
                     L.row_off, out->counts, cap_start, L.starts, L.start_pos, L.start_k, L.order);

  TrackInputs ti;
  ti.pts = L.pts;
  ti.start_pos = L.start_pos;
  ti.start_k = L.start_k;
  ti.order = L.order;
  ti.row_x = c->d_row_x;
  mark(3);
  hipLaunchKernelGGL(k_construct, dim3(t.construct_grid), dim3(kConstructBlock), 0, stream,
                     out->counts, cap_start, L.queue, t.construct_refill, ti, g, c->dp, L.tmp);

  TrackOut o;
  o.cap_tracks = out->cap_tracks;
  o.cap_hits = out->cap_hits;
  o.unit = out->unit;
  o.start = out->start;
  o.n_hits = out->n_hits;
  o.hit_begin = out->hit_begin;
  o.hit_id = out->hit_id;
  o.hit_row = out->hit_row;
  o.x_ref = out->x_ref;
  o.param = out->param;
  o.cov = out->cov;
  o.chi2 = out->chi2;
  o.ndf = out->ndf;
  mark(4);
  hipLaunchKernelGGL(k_keep_count, dim3(kKeepBlocks), dim3(256), 0, stream, out->counts, cap_start,
                     L.tmp.rec, c->dp.min_hits, L.part);
  hipLaunchKernelGGL(k_keep_scan, dim3(1), dim3(kKeepScanThreads), 0, stream, L.part, kKeepBlocks, out->counts,
                     out->cap_tracks, out->cap_hits);
  hipLaunchKernelGGL(k_keep_write, dim3(kKeepBlocks), dim3(kKeepBlock), 0, stream, out->counts,
                     cap_start, L.starts, L.tmp, c->dp.min_hits, L.part, o);
  mark(5);
}

// The batched refit: the cluster correction on c->aux (it needs only the input
// clusters, so it overlaps the tracking stages; it starts after the grid build,
// which is bound by HBM bandwidth), the filter on `stream` once both the
// tracking and the correction are done.  enqueue_track must have recorded
// c->ev_fork after the grid build.
void enqueue_batch_refit(const tpcx_ctx* c, const tpcx_clusters* in, const tpcx_tracks* out,
                         const tpcx_batch_refit* refit, const BatchRefitLayout& RL,
                         const tpcx_tuning& t, hipStream_t stream) {
  (void)hipStreamWaitEvent(c->aux, c->ev_fork, 0);
  const int64_t n_ur = int64_t(in->n_units) * c->n_rows;
  if (in->n_clusters > 0)
    hipLaunchKernelGGL(k_correct_clusters, dim3(unsigned(n_ur)), dim3(kRefitBlock), 0, c->aux,
                       c->n_rows, in->row_begin, in->y, in->z, refit->unit_alpha, c->d_row_x,
                       refit->theta, refit->map_z_fixed ? 1 : 0, refit->map_z, RL.corr);
  (void)hipEventRecord(c->ev_join, c->aux);

  RefitIn r;
  r.n_tracks = out->cap_tracks;
  r.n_tracks_dev = out->counts + 1;
  r.status_dev = out->counts + 3;
  r.n_hit = out->n_hits;
  r.min_hits = refit->min_hits;
  r.hit_begin = out->hit_begin;
  r.hit_id = out->hit_id;
  r.hit_row = out->hit_row;
  r.unit = out->unit;
  r.seed = out->param;
  r.y = in->y;
  r.z = in->z;
  r.unit_alpha = refit->unit_alpha;
  r.row_x = c->d_row_x;
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, stream, reinterpret_cast<int64_t*>(RL.queue),
                     int64_t(kXcds), int64_t(0));
  (void)hipStreamWaitEvent(stream, c->ev_join, 0);
  hipLaunchKernelGGL(k_refit_filter<true>, dim3(refit_filter_grid(c, out->cap_tracks, t.refit_grid)),
                     dim3(kRefitBlock), 0, stream, r, c->dp, RL.corr, static_cast<float*>(nullptr),
                     RL.queue, t.refit_refill, refit->chi2, refit->ok);
}

// Candidate values of one tuning parameter (knob) around the tuning b: the
// search-grid z bins, the block size of the per-row kernels, the grid and
// refill threshold of the constructor, the grid and refill threshold of the
// refit filter.
constexpr int kAutotuneKnobs = 6;

std::vector<tpcx_tuning> autotune_candidates(const tpcx_ctx* c, const tpcx_tuning& b, int knob) {
  std::vector<tpcx_tuning> v;
  auto add = [&](tpcx_tuning t) {
    t.n_zbins = std::max(1, std::min(t.n_zbins, (c->max_row_bins - 1) / max_row_ny(c)));
    if (!valid_tuning(t) || std::memcmp(&t, &b, sizeof t) == 0) return;
    for (const tpcx_tuning& u : v)
      if (std::memcmp(&t, &u, sizeof t) == 0) return;
    v.push_back(t);
  };
  tpcx_tuning t = b;
  switch (knob) {
    case 0:
      for (double f : {0.5, 0.7, 1.4, 2.0}) {
        t = b;
        t.n_zbins = std::max(1, int(std::lround(b.n_zbins * f)));
        add(t);
      }
      break;
    case 1:
      for (int blk : {128, 256, 512}) {
        t = b;
        t.block = blk;
        add(t);
      }
      break;
    case 2:
      // at most 4 constructor blocks are resident per CU (its register use)
      for (int per_cu : {2, 3, 4}) {
        t = b;
        t.construct_grid = per_cu * c->n_cu;
        add(t);
      }
      break;
    case 3:
      for (int r : {4, 8, 16, 32}) {
        t = b;
        t.construct_refill = r;
        add(t);
      }
      break;
    case 4:
      for (int per_cu : {4, 6, 7, 8}) {
        t = b;
        t.refit_grid = per_cu * c->n_cu;
        add(t);
      }
      break;
    case 5:
      for (int r : {4, 16, 32, 64}) {
        t = b;
        t.refit_refill = r;
        add(t);
      }
      break;
    default:
      break;
  }
  return v;
}

// One eager batched run with tuning t; TPCX_E_ARG when t needs more workspace.
tpcx_status autotune_run(const tpcx_ctx* c, const tpcx_clusters* in, void* ws, size_t ws_bytes,
                         int64_t cap_start, const tpcx_tracks* out, const tpcx_batch_refit* refit,
                         const tpcx_tuning& t, hipStream_t stream) {
  const Layout L = carve(c, ws, in->n_units, in->n_clusters, cap_start, t.n_zbins, t.block);
  const BatchRefitLayout RL = carve_batch_refit(static_cast<char*>(ws) + L.bytes, in->n_clusters);
  if (L.bytes + RL.bytes > ws_bytes) return TPCX_E_ARG;
  enqueue_track(c, in, L, t, cap_start, out, stream, nullptr, refit ? c->ev_fork : nullptr);
  if (refit) enqueue_batch_refit(c, in, out, refit, RL, t, stream);
  return hipGetLastError() == hipSuccess ? TPCX_OK : TPCX_E_HIP;
}

hipEvent_t* next_timing_slot(tpcx_ctx* c) {
  if (c->timing_used >= c->timing_max) return nullptr;
  hipEvent_t* ev = &c->events[size_t(c->timing_used) * (TPCX_N_STAGES + 1)];
  ++c->timing_used;
  return ev;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// tpcx_track on the workspace ws of ws_bytes.
tpcx_status track_on(tpcx_ctx* c, const tpcx_clusters* in, void* ws, size_t ws_bytes,
                     int64_t cap_start, const tpcx_tracks* out, const tpcx_debug* dbg,
                     hipStream_t stream) {
  const tpcx_status st = check_track_args(c, in, ws, cap_start, out);
  if (st != TPCX_OK) return st;
  const int64_t N = in->n_clusters;
  const tpcx_tuning t = effective_tuning(c, in->n_units, N);
  const Layout L = carve(c, ws, in->n_units, N, cap_start, t.n_zbins, t.block);
  if (!ws || ws_bytes < L.bytes) return TPCX_E_ARG;
  hipEvent_t* ev = next_timing_slot(c);
  enqueue_track(c, in, L, t, cap_start, out, stream, ev);
  if (ev) (void)hipEventRecord(ev[TPCX_N_STAGES], stream);  // no refit stage here
  if (dbg) {
    if (N > 0 && (dbg->link_up || dbg->link_down || dbg->clean_up || dbg->clean_down))
      hipLaunchKernelGGL(k_links_to_caller, dim3(blocks_for(N, 256)), dim3(256), 0, stream, N,
                         L.pts, L.up, L.down, dbg->link_up, dbg->link_down, dbg->clean_up,
                         dbg->clean_down);
    if (dbg->starts && cap_start)
      (void)hipMemcpyAsync(dbg->starts, L.starts, size_t(cap_start) * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, stream);
  }
  return hipGetLastError() == hipSuccess ? TPCX_OK : TPCX_E_HIP;
}

}  // namespace

extern "C" {

tpcx_status tpcx_track(tpcx_ctx* c, const tpcx_clusters* in, void* ws, size_t ws_bytes,
                       int64_t cap_start, const tpcx_tracks* out, const tpcx_debug* dbg,
                       hipStream_t stream) {
  return track_on(c, in, ws, ws_bytes, cap_start, out, dbg, stream);
}

tpcx_status tpcx_track_static(tpcx_ctx* c, const tpcx_clusters* in, int64_t cap_start,
                              const tpcx_tracks* out, const tpcx_debug* dbg, hipStream_t stream) {
  if (!c || !c->scratch) return TPCX_E_ARG;
  // the size check comes first: nothing is enqueued for an input that does not fit
  if (!in || in->n_units < 1 || in->n_clusters < 0 || cap_start < 0 ||
      tpcx_workspace_bytes(c, in->n_units, in->n_clusters, cap_start) > size_t(TPCX_STATIC_SCRATCH_BYTES))
    return TPCX_E_ARG;
  // every cleared word of the workspace is cleared by a fill kernel of the
  // sequence itself, so the array's previous contents do not matter
  return track_on(c, in, c->scratch, size_t(TPCX_STATIC_SCRATCH_BYTES), cap_start, out, dbg, stream);
}

tpcx_status tpcx_poll(tpcx_ctx* c, const tpcx_tracks* out, hipStream_t stream) {
  if (!c || !out || !out->counts) return TPCX_E_ARG;
  if (hipStreamSynchronize(stream) != hipSuccess) return TPCX_E_HIP;
  int64_t st = 0;
  if (hipMemcpy(&st, out->counts + 3, sizeof st, hipMemcpyDeviceToHost) != hipSuccess) return TPCX_E_HIP;
  if (st & (TPCX_ST_START_OVERFLOW | TPCX_ST_TRACK_OVERFLOW | TPCX_ST_HIT_OVERFLOW)) return TPCX_E_CAPACITY;
  return (st & TPCX_ST_NONFINITE) ? TPCX_E_INPUT : TPCX_OK;
}


size_t tpcx_refit_workspace_bytes(const tpcx_ctx* c, int64_t n_tracks, int64_t n_hits) {
  if (!c || n_tracks < 0 || n_hits < 0) return 0;
  return carve_refit(nullptr, n_tracks, n_hits).bytes;
}

tpcx_status tpcx_refit(tpcx_ctx* c, const tpcx_refit_in* in, const float* theta, float* chi2,
                       int32_t* ok, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!refit_args_ok(c, in) || (in->n_tracks > 0 && (!chi2 || !ok))) return TPCX_E_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return TPCX_E_ARG;
  const RefitLayout L = carve_refit(ws, in->n_tracks, in->n_hits);
  if (!ws || ws_bytes < L.bytes) return TPCX_E_ARG;
  if (in->n_tracks == 0) return TPCX_OK;
  const RefitIn rv = refit_view(c, in);
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, stream, reinterpret_cast<int64_t*>(L.ws.queue),
                     int64_t(kXcds), int64_t(0));
  hipLaunchKernelGGL(k_correct_hits, dim3(blocks_for(in->n_tracks, kRefitBlock)), dim3(kRefitBlock), 0,
                     stream, rv, theta, reinterpret_cast<float4*>(L.ws.xyz));
  hipLaunchKernelGGL(k_refit_filter<false>, dim3(refit_filter_grid(c, in->n_tracks, c->tuning.refit_grid)),
                     dim3(kRefitBlock), 0, stream, rv, c->dp, reinterpret_cast<const float4*>(L.ws.xyz),
                     L.ws.ckpt, L.ws.queue, c->tuning.refit_refill, chi2, L.ok);
  (void)hipMemcpyAsync(ok, L.ok, sizeof(int32_t) * size_t(in->n_tracks), hipMemcpyDeviceToDevice,
                       stream);
  return hipGetLastError() == hipSuccess ? TPCX_OK : TPCX_E_HIP;
}

tpcx_status tpcx_refit_backward(tpcx_ctx* c, const tpcx_refit_in* in, const float* dL_dchi2,
                                float* grad_theta, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!refit_args_ok(c, in) || !grad_theta || (in->n_tracks > 0 && !dL_dchi2)) return TPCX_E_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return TPCX_E_ARG;
  const RefitLayout L = carve_refit(ws, in->n_tracks, in->n_hits);
  if (!ws || ws_bytes < L.bytes) return TPCX_E_ARG;
  hipLaunchKernelGGL(k_fill_i64, dim3(64), dim3(256), 0, stream, L.ws.acc, int64_t(kMapNCoef),
                     int64_t(0));
  if (in->n_tracks > 0) {
    const size_t win_bytes = sizeof(long long) * kMapComp * kWinPhi * kMapNR * kMapNZ;
    const RefitIn rv = refit_view(c, in);
    hipLaunchKernelGGL(k_refit_bwd_sweep, dim3(blocks_for(in->n_tracks, kWave)), dim3(kWave), 0, stream,
                       rv, c->dp, L.ws, dL_dchi2, L.ok);
    hipLaunchKernelGGL(k_refit_bwd_scatter, dim3(blocks_for(in->n_tracks, kScatterTracks)),
                       dim3(kRefitBlock), win_bytes, stream, rv, L.ws);
  }
  hipLaunchKernelGGL(k_grad_finalize, dim3((kMapNCoef + 255) / 256), dim3(256), 0, stream, L.ws.acc,
                     grad_theta);
  return hipGetLastError() == hipSuccess ? TPCX_OK : TPCX_E_HIP;
}

size_t tpcx_batched_workspace_bytes(const tpcx_ctx* c, int32_t n_units, int64_t n_clusters,
                                    int64_t cap_start, int64_t cap_tracks, int64_t cap_hits) {
  if (!c || n_units < 1 || n_clusters < 0 || cap_start < 0 || cap_tracks < 0 || cap_hits < 0)
    return 0;
  const tpcx_tuning t = effective_tuning(c, n_units, n_clusters);
  const size_t a = carve(c, nullptr, n_units, n_clusters, cap_start, t.n_zbins, t.block).bytes;
  (void)cap_tracks;
  (void)cap_hits;
  return a + carve_batch_refit(nullptr, n_clusters).bytes;
}

tpcx_status tpcx_track_batched(tpcx_ctx* c, const tpcx_clusters* in, void* ws, size_t ws_bytes,
                               int64_t cap_start, const tpcx_tracks* out,
                               const tpcx_batch_refit* refit, hipStream_t stream) {
  tpcx_status st = check_track_args(c, in, ws, cap_start, out);
  if (st != TPCX_OK) return st;
  if (refit && (refit->min_hits < 2 || !refit->unit_alpha || !refit->chi2 || !refit->ok ||
                (refit->map_z_fixed != 0 && refit->map_z_fixed != 1) || !std::isfinite(refit->map_z)))
    return TPCX_E_ARG;
  if (!stream) return TPCX_E_ARG;  // the legacy default stream cannot be captured
  const int64_t N = in->n_clusters;
  const tpcx_tuning t = effective_tuning(c, in->n_units, N);
  const Layout L = carve(c, ws, in->n_units, N, cap_start, t.n_zbins, t.block);
  const BatchRefitLayout RL =
      carve_batch_refit(ws ? static_cast<char*>(ws) + L.bytes : nullptr, in->n_clusters);
  if (!ws || ws_bytes < L.bytes + RL.bytes) return TPCX_E_ARG;

  // the graph depends on every argument; rebuild it when one changes
  std::vector<unsigned char> key;
  auto put = [&](const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    key.insert(key.end(), b, b + n);
  };
  put(in, sizeof *in);
  put(&ws, sizeof ws);
  put(&ws_bytes, sizeof ws_bytes);
  put(&cap_start, sizeof cap_start);
  put(out, sizeof *out);
  const int has_refit = refit ? 1 : 0;
  put(&has_refit, sizeof has_refit);
  if (refit) put(refit, sizeof *refit);
  put(&t, sizeof t);
  put(&stream, sizeof stream);

  if (hipEvent_t* ev = next_timing_slot(c)) {
    // timed run: the same sequence launched directly, with stage events
    enqueue_track(c, in, L, t, cap_start, out, stream, ev, refit ? c->ev_fork : nullptr);
    if (refit) enqueue_batch_refit(c, in, out, refit, RL, t, stream);
    (void)hipEventRecord(ev[TPCX_N_STAGES], stream);
    return hipGetLastError() == hipSuccess ? TPCX_OK : TPCX_E_HIP;
  }
  if (!c->graph || key != c->graph_key) {
    if (c->graph) {
      (void)hipGraphExecDestroy(c->graph);
      c->graph = nullptr;
    }
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return TPCX_E_HIP;
    enqueue_track(c, in, L, t, cap_start, out, stream, nullptr, refit ? c->ev_fork : nullptr);
    if (refit) enqueue_batch_refit(c, in, out, refit, RL, t, stream);
    hipGraph_t g = nullptr;
    const hipError_t e1 = hipStreamEndCapture(stream, &g);
    if (e1 != hipSuccess || !g) return TPCX_E_HIP;
    const hipError_t e2 = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
      c->graph = nullptr;
      return TPCX_E_HIP;
    }
    c->graph_key = key;
  }
  return hipGraphLaunch(c->graph, stream) == hipSuccess ? TPCX_OK : TPCX_E_HIP;
}

tpcx_status tpcx_set_tuning(tpcx_ctx* c, const tpcx_tuning* t) {
  if (!c) return TPCX_E_ARG;
  if (!t) {
    const float bin_y = c->tuning.bin_y;
    tpcx_default_tuning(36, 1, &c->tuning);
    c->tuning.bin_y = bin_y;
    c->tuning_fixed = false;
    return TPCX_OK;
  }
  if (!valid_tuning(*t) || t->bin_y != c->tuning.bin_y) return TPCX_E_ARG;
  c->tuning = *t;
  c->tuning_fixed = true;
  return TPCX_OK;
}

size_t tpcx_autotune_workspace_bytes(const tpcx_ctx* c, int32_t n_units, int64_t n_clusters,
                                     int64_t cap_start, int64_t cap_tracks, int64_t cap_hits) {
  if (!c || n_units < 1 || n_clusters < 0 || cap_start < 0 || cap_tracks < 0 || cap_hits < 0)
    return 0;
  const tpcx_tuning b = effective_tuning(c, n_units, n_clusters);
  size_t most = 0;
  std::vector<tpcx_tuning> zs = autotune_candidates(c, b, 0);
  zs.push_back(b);
  for (const tpcx_tuning& z : zs) {
    std::vector<tpcx_tuning> bs = autotune_candidates(c, z, 1);
    bs.push_back(z);
    for (const tpcx_tuning& t : bs)
      most = std::max(most, carve(c, nullptr, n_units, n_clusters, cap_start, t.n_zbins, t.block).bytes);
  }
  return most + carve_batch_refit(nullptr, n_clusters).bytes;
}

tpcx_status tpcx_autotune_batched(tpcx_ctx* c, const tpcx_clusters* in, void* ws, size_t ws_bytes,
                                  int64_t cap_start, const tpcx_tracks* out,
                                  const tpcx_batch_refit* refit, int32_t reps, tpcx_tuning* best,
                                  hipStream_t stream) {
  tpcx_status st = check_track_args(c, in, ws, cap_start, out);
  if (st != TPCX_OK) return st;
  if (!ws || !best || reps < 1) return TPCX_E_ARG;
  if (refit && (refit->min_hits < 2 || !refit->unit_alpha || !refit->chi2 || !refit->ok))
    return TPCX_E_ARG;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return TPCX_E_HIP;
  }
  // A candidate is timed as the batched form runs it: its sequence captured
  // once into a graph and replayed (eager launches of the same sequence
  // rank the z-bin candidates differently); on the legacy default stream,
  // which cannot be captured, the sequence is launched directly.
  auto measure = [&](const tpcx_tuning& t, float* ms) -> tpcx_status {
    hipGraphExec_t ge = nullptr;
    if (stream) {
      const Layout L = carve(c, ws, in->n_units, in->n_clusters, cap_start, t.n_zbins, t.block);
      const BatchRefitLayout RL = carve_batch_refit(static_cast<char*>(ws) + L.bytes, in->n_clusters);
      if (L.bytes + RL.bytes > ws_bytes) return TPCX_E_ARG;
      if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return TPCX_E_HIP;
      enqueue_track(c, in, L, t, cap_start, out, stream, nullptr, refit ? c->ev_fork : nullptr);
      if (refit) enqueue_batch_refit(c, in, out, refit, RL, t, stream);
      hipGraph_t g = nullptr;
      if (hipStreamEndCapture(stream, &g) != hipSuccess || !g) return TPCX_E_HIP;
      const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) return TPCX_E_HIP;
    }
    auto run = [&]() -> tpcx_status {
      if (ge) return hipGraphLaunch(ge, stream) == hipSuccess ? TPCX_OK : TPCX_E_HIP;
      return autotune_run(c, in, ws, ws_bytes, cap_start, out, refit, t, stream);
    };
    tpcx_status r = run();  // warm-up
    if (r == TPCX_OK && hipEventRecord(e0, stream) != hipSuccess) r = TPCX_E_HIP;
    for (int i = 0; i < reps && r == TPCX_OK; ++i) r = run();
    if (r == TPCX_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(ms, e0, e1) != hipSuccess))
      r = TPCX_E_HIP;
    if (ge) {
      (void)hipStreamSynchronize(stream);
      (void)hipGraphExecDestroy(ge);
    }
    if (r != TPCX_OK) return r;
    *ms /= float(reps);
    return TPCX_OK;
  };
  tpcx_tuning b = effective_tuning(c, in->n_units, in->n_clusters);
  float best_ms = 0.0f;
  st = measure(b, &best_ms);
  if (st == TPCX_OK) {
    int64_t status = 0;
    if (hipMemcpy(&status, out->counts + 3, sizeof status, hipMemcpyDeviceToHost) != hipSuccess)
      st = TPCX_E_HIP;
    else if (status != 0)
      st = TPCX_E_CAPACITY;
  }
  for (int knob = 0; knob < kAutotuneKnobs && st == TPCX_OK; ++knob) {
    if (knob >= 4 && !refit) break;
    for (const tpcx_tuning& t : autotune_candidates(c, b, knob)) {
      float ms = 0.0f;
      const tpcx_status r = measure(t, &ms);
      if (r == TPCX_E_ARG) continue;  // does not fit the workspace
      if (r != TPCX_OK) {
        st = r;
        break;
      }
      if (ms < 0.99f * best_ms) {
        // a win is confirmed by timing both again: the two tunings' times
        // differ by about as much as one timing's noise
        float ms2 = 0.0f, base2 = 0.0f;
        tpcx_status r2 = measure(t, &ms2);
        if (r2 == TPCX_OK) r2 = measure(b, &base2);
        if (r2 != TPCX_OK) {
          st = r2;
          break;
        }
        if (ms + ms2 < 0.99f * (best_ms + base2)) {
          best_ms = 0.5f * (ms + ms2);
          b = t;
        } else {
          best_ms = 0.5f * (best_ms + base2);
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != TPCX_OK) return st;
  c->tuning = b;
  c->tuning_fixed = true;
  *best = b;
  return TPCX_OK;
}

tpcx_status tpcx_timing_enable(tpcx_ctx* c, int32_t max_calls) {
  if (!c || max_calls < 0) return TPCX_E_ARG;
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  c->events.clear();
  c->timing_max = 0;
  c->timing_used = 0;
  const size_t n = size_t(max_calls) * (TPCX_N_STAGES + 1);
  c->events.resize(n);
  for (size_t i = 0; i < n; ++i) {
    if (hipEventCreate(&c->events[i]) != hipSuccess) {
      c->events.resize(i);
      return TPCX_E_HIP;
    }
  }
  c->timing_max = max_calls;
  return TPCX_OK;
}

tpcx_status tpcx_timing_read(tpcx_ctx* c, float* ms_host, int32_t* n_calls) {
  if (!c || !ms_host || !n_calls) return TPCX_E_ARG;
  for (int s = 0; s < TPCX_N_STAGES; ++s) ms_host[s] = 0.0f;
  for (int32_t i = 0; i < c->timing_used; ++i) {
    hipEvent_t* ev = &c->events[size_t(i) * (TPCX_N_STAGES + 1)];
    if (hipEventSynchronize(ev[TPCX_N_STAGES]) != hipSuccess) return TPCX_E_HIP;
    for (int s = 0; s < TPCX_N_STAGES; ++s) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ev[s], ev[s + 1]) != hipSuccess) return TPCX_E_HIP;
      ms_host[s] += ms;
    }
  }
  *n_calls = c->timing_used;
  c->timing_used = 0;
  return TPCX_OK;
}

}  // extern "C"

namespace {

// Fit workspace: record slots for n_hits plus, per chunk of the length
// order, one wavefront's worth of the longest possible track (the slack of
// the per-wavefront layout when every track has fewer than 256 clusters),
// the rows of the slots, per-wavefront sizes and offsets, the order.
struct FitLayout {
  float2* yz;
  float4* rec;
  uint8_t* rows;
  int64_t* wlen;
  int64_t* wbase;
  int32_t* order;
  int64_t cap;
  size_t bytes;
};

FitLayout carve_fit(void* base, int64_t n_tracks, int64_t n_hits, int64_t n_clusters) {
  Carver cv{static_cast<char*>(base)};
  FitLayout L{};
  L.yz = cv.take<float2>(n_clusters);
  const int64_t nw = (n_tracks + kWave - 1) / kWave;
  L.cap = n_hits + (n_tracks + kLenChunk - 1) / kLenChunk * int64_t(kWave) * 256;
  L.rec = cv.take<float4>(L.cap);
  L.rows = cv.take<uint8_t>(L.cap);
  L.wlen = cv.take<int64_t>(nw);
  L.wbase = cv.take<int64_t>(nw + 1);
  L.order = cv.take<int32_t>(n_tracks);
  L.bytes = cv.off;
  return L;
}

}  // namespace

extern "C" {

size_t tpcx_fit_workspace_bytes(const tpcx_ctx* c, int64_t n_tracks, int64_t n_hits, int64_t n_clusters) {
  if (!c || n_tracks < 0 || n_hits < 0 || n_clusters < 0) return 0;
  return carve_fit(nullptr, n_tracks, n_hits, n_clusters).bytes;
}

tpcx_status tpcx_fit(tpcx_ctx* c, const tpcx_fit_in* in, const tpcx_fit_params* fp, const tpcx_fit_out* out,
                     void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!c || !in || !fp || !out || in->n_tracks < 0 || in->n_hits < 0 || in->n_clusters < 0) return TPCX_E_ARG;
  if (in->n_clusters > 0 && (!in->y || !in->z)) return TPCX_E_ARG;
  if (in->n_hits > 0 && in->n_clusters == 0) return TPCX_E_ARG;
  if (in->n_tracks > 0 && (!in->hit_begin || !in->seed || !in->x_ref || !out->param || !out->cov ||
                           !out->chi2 || !out->x_out || !out->n_kept || !out->ok))
    return TPCX_E_ARG;
  if (in->n_hits > 0 && (!in->hit_id || !in->hit_row || !in->y || !in->z || !out->reject)) return TPCX_E_ARG;
  if (!(fp->chi2_cut >= 0.0f) || !(fp->var_s > 0.0f) || !(fp->var_t > 0.0f) || !(fp->var_w > 0.0f))
    return TPCX_E_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return TPCX_E_ARG;
  if (in->n_tracks >= (int64_t(1) << 31)) return TPCX_E_ARG;
  const FitLayout L = carve_fit(ws, in->n_tracks, in->n_hits, in->n_clusters);
  if (!ws || ws_bytes < L.bytes) return TPCX_E_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device) return TPCX_E_ARG;
  if (in->n_tracks == 0) return TPCX_OK;
  FitIn fi;
  fi.n_tracks = in->n_tracks;
  fi.hit_begin = in->hit_begin;
  fi.hit_id = in->hit_id;
  fi.hit_row = in->hit_row;
  fi.seed = in->seed;
  fi.x_ref = in->x_ref;
  fi.yz = L.yz;
  fi.row_x = c->d_row_x;
  fi.n_rows = c->n_rows;
  FitOut fo;
  fo.param = out->param;
  fo.cov = out->cov;
  fo.chi2 = out->chi2;
  fo.x_out = out->x_out;
  fo.n_kept = out->n_kept;
  fo.ok = out->ok;
  fo.reject = out->reject;
  const FitConsts f{fp->chi2_cut, fp->var_s, fp->var_t, fp->var_w};
  if (in->n_clusters > 0)
    hipLaunchKernelGGL(k_fit_pack, dim3(std::min(blocks_for(in->n_clusters, 256), 4096)), dim3(256), 0, stream,
                       in->n_clusters, in->y, in->z, L.yz);
  enqueue_length_order(in->n_tracks, in->hit_begin, L.order, stream);
  const int64_t nw = (in->n_tracks + kWave - 1) / kWave;
  hipLaunchKernelGGL(k_fit_wave_len, dim3(blocks_for(in->n_tracks, 256)), dim3(256), 0, stream, in->n_tracks,
                     in->hit_begin, L.order, L.wlen);
  hipLaunchKernelGGL(k_fit_scan, dim3(1), dim3(kFitScanThreads), 0, stream, nw, L.wlen, L.wbase);
  const FitWs fw{L.rec, L.rows, L.wbase, L.cap};
  hipLaunchKernelGGL(k_fit, dim3(blocks_for(in->n_tracks, kWave)), dim3(kWave), 0, stream, fi, c->dp, f, L.order,
                     fw, fo);
  return hipGetLastError() == hipSuccess ? TPCX_OK : TPCX_E_HIP;
}

}  // extern "C"

namespace {

struct RebuildLayout {
  UnitZ* row_z;
  int32_t* bins;
  float4* pts;
  int64_t* status;
  RebuildWs ws;
  size_t bytes;
};

RebuildLayout carve_rebuild(const tpcx_ctx* c, void* base, int32_t n_units, int64_t n_clusters,
                            int64_t n_tracks, int nz) {
  Carver cv{static_cast<char*>(base)};
  RebuildLayout L{};
  const int64_t R = c->n_rows;
  L.row_z = cv.take<UnitZ>(int64_t(n_units) * R);
  L.bins = cv.take<int32_t>(int64_t(n_units) * bins_per_unit(c, nz));
  L.pts = cv.take<float4>(n_clusters);
  L.status = cv.take<int64_t>(1);
  L.ws.pred = cv.take<float4>(n_tracks * R);
  L.ws.cand = cv.take<int2>(n_tracks * R * kRebuildK);
  L.ws.cnt = cv.take<uint8_t>(n_tracks * R);
  L.ws.ptr = cv.take<uint8_t>(n_tracks * R);
  L.ws.state = cv.take<float>(16 * n_tracks);
  L.ws.meta = cv.take<int32_t>(4 * n_tracks);
  L.ws.key = cv.take<uint64_t>(n_tracks);
  L.ws.holder = cv.take<unsigned long long>(n_clusters);
  L.ws.first = cv.take<int64_t>(n_tracks);
  L.ws.active = cv.take<uint8_t>(n_tracks);
  L.ws.check = cv.take<uint8_t>(n_tracks);
  L.bytes = cv.off;
  return L;
}

}  // namespace

extern "C" {

namespace {

struct MergeLayout {
  MergeWs ws;
  size_t bytes;
};

MergeLayout carve_merge(void* base, int32_t n_units, int64_t n) {
  Carver cv{static_cast<char*>(base)};
  MergeLayout L{};
  L.ws.view = cv.take<float>(15 * n);
  L.ws.ok = cv.take<uint8_t>(3 * n);
  L.ws.ub = cv.take<int64_t>(int64_t(n_units) + 1);
  L.ws.rec = cv.take<float4>(3 * n);
  L.ws.cell = cv.take<int32_t>(int64_t(n_units) * 3 * (kMergeCells + 1));
  L.ws.zcell = cv.take<float2>(int64_t(n_units) * 3);
  L.ws.best_out = cv.take<int32_t>(n);
  L.ws.best_in = cv.take<int32_t>(n);
  L.bytes = cv.off;
  return L;
}

}  // namespace

size_t tpcx_merge_workspace_bytes(const tpcx_ctx* c, int32_t n_units, int64_t n_tracks) {
  if (!c || n_units < 1 || n_tracks < 0) return 0;
  return carve_merge(nullptr, n_units, n_tracks).bytes;
}

tpcx_status tpcx_merge(tpcx_ctx* c, const tpcx_merge_in* in, const tpcx_merge_params* mp, const tpcx_merge_out* out,
                       void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!c || !in || !mp || !out || in->n_tracks < 0 || in->n_tracks >= (int64_t(1) << 31) || in->n_units < 1)
    return TPCX_E_ARG;
  if (in->n_tracks > 0 && (!in->unit || !in->param || !in->x_ref || !in->r_in || !in->r_out || !in->unit_nbr ||
                           !out->prev || !out->next || !out->root))
    return TPCX_E_ARG;
  if (!std::isfinite(mp->x_m) || !(mp->chi2_cut >= 0.0f) || !std::isfinite(mp->chi2_cut) ||
      !(std::fabs(mp->cos_h) <= 1.0f) || !(std::fabs(mp->sin_h) <= 1.0f))
    return TPCX_E_ARG;
  for (int i = 0; i < 5; ++i)
    if (!(mp->tol[i] > 0.0f) || !std::isfinite(mp->tol[i])) return TPCX_E_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return TPCX_E_ARG;
  const MergeLayout L = carve_merge(ws, in->n_units, in->n_tracks);
  if (!ws || ws_bytes < L.bytes) return TPCX_E_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device) return TPCX_E_ARG;
  if (in->n_tracks == 0) return TPCX_OK;
  MergeIn mi;
  mi.n = in->n_tracks;
  mi.n_units = in->n_units;
  mi.unit = in->unit;
  mi.param = in->param;
  mi.x_ref = in->x_ref;
  mi.r_in = in->r_in;
  mi.r_out = in->r_out;
  mi.unit_nbr = in->unit_nbr;
  MergeConsts m;
  m.x_m = mp->x_m;
  m.cos_h = mp->cos_h;
  m.sin_h = mp->sin_h;
  m.chi2_cut = mp->chi2_cut;
  for (int i = 0; i < 5; ++i) m.itol2[i] = 1.0f / (mp->tol[i] * mp->tol[i]);
  // the window holds every pair the chi2 cut can accept (with a margin for
  // the rounding of the float chi2)
  const float rc = std::sqrt(mp->chi2_cut);
  m.wy = mp->tol[0] * rc * 1.001f;
  m.wz = std::max(mp->tol[1] * rc * 1.001f, 1e-6f);
  m.cross_electrode = mp->cross_electrode ? 1 : 0;
  const int64_t n = in->n_tracks;
  hipLaunchKernelGGL(k_merge_views, dim3(blocks_for(n, kMergeBlock)), dim3(kMergeBlock), 0, stream, mi, c->dp, m,
                     L.ws);
  hipLaunchKernelGGL(k_merge_units, dim3(blocks_for(int64_t(in->n_units) + 1, 256)), dim3(256), 0, stream, mi, L.ws);
  hipLaunchKernelGGL(k_merge_grid, dim3(in->n_units * 3), dim3(kMergeBlock), 0, stream, mi, m, L.ws);
  hipLaunchKernelGGL(k_merge_match, dim3(blocks_for(n, kMergeBlock)), dim3(kMergeBlock), 0, stream, mi, m, L.ws);
  hipLaunchKernelGGL(k_merge_link, dim3(blocks_for(n, 256)), dim3(256), 0, stream, n, L.ws, out->prev, out->next);
  hipLaunchKernelGGL(k_merge_root, dim3(blocks_for(n, 256)), dim3(256), 0, stream, n, out->prev, out->root);
  return hipGetLastError() == hipSuccess ? TPCX_OK : TPCX_E_HIP;
}

size_t tpcx_rebuild_workspace_bytes(const tpcx_ctx* c, int32_t n_units, int64_t n_clusters, int64_t n_tracks) {
  if (!c || n_units < 1 || n_clusters < 0 || n_tracks < 0) return 0;
  const tpcx_tuning t = effective_tuning(c, n_units, n_clusters);
  return carve_rebuild(c, nullptr, n_units, n_clusters, n_tracks, t.n_zbins).bytes;
}

tpcx_status tpcx_rebuild(tpcx_ctx* c, const tpcx_clusters* cl, const tpcx_rebuild_in* in,
                         const tpcx_rebuild_params* rp, const tpcx_rebuild_out* out, void* ws, size_t ws_bytes,
                         hipStream_t stream) {
  if (!c || !cl || !in || !rp || !out || cl->n_units < 1 || cl->n_clusters < 0 ||
      cl->n_clusters >= (int64_t(1) << 31) || !cl->row_begin || in->n_tracks < 0 || in->n_hits < 0)
    return TPCX_E_ARG;
  if (cl->n_clusters > 0 && (!cl->y || !cl->z)) return TPCX_E_ARG;
  if (in->n_tracks > 0 && (!in->unit || !in->hit_begin || !in->seed || !in->x_ref || !in->chi2 || !in->ndf ||
                           !out->assigned || !out->param || !out->cov || !out->chi2 || !out->x_out ||
                           !out->n_kept || !out->ok))
    return TPCX_E_ARG;
  if (in->n_hits > 0 && (!in->hit_id || !in->hit_row)) return TPCX_E_ARG;
  if (!(rp->chi2_cut >= 0.0f) || !(rp->chi2_final >= 0.0f) || !(rp->var_s > 0.0f) || !(rp->var_t > 0.0f) ||
      !(rp->var_w > 0.0f) || rp->rounds < 0 || rp->rounds > 64 || !(rp->chi2_extrap >= 0.0f))
    return TPCX_E_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return TPCX_E_ARG;
  const tpcx_tuning t = effective_tuning(c, cl->n_units, cl->n_clusters);
  const RebuildLayout L = carve_rebuild(c, ws, cl->n_units, cl->n_clusters, in->n_tracks, t.n_zbins);
  if (!ws || ws_bytes < L.bytes) return TPCX_E_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device) return TPCX_E_ARG;
  if (in->n_tracks == 0) return TPCX_OK;
  Grid g;
  g.rows = c->d_rows;
  g.row_z = L.row_z;
  g.bin_start = L.bins;
  g.pts = L.pts;
  g.n_rows = c->n_rows;
  g.nz = t.n_zbins;
  g.btot = bins_per_unit(c, t.n_zbins);
  const int UR = cl->n_units * c->n_rows;
  const size_t hist_bytes = sizeof(int32_t) * (size_t(t.n_zbins) * max_row_ny(c) + 1);
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, stream, L.status, int64_t(1), int64_t(0));
  hipLaunchKernelGGL(k_grid_build, dim3(UR), dim3(t.block), hist_bytes, stream, cl->row_begin, cl->y, cl->z, g,
                     L.row_z, L.bins, L.pts, reinterpret_cast<unsigned long long*>(L.status));
  RebuildIn ri;
  ri.n_tracks = in->n_tracks;
  ri.n_hits = in->n_hits;
  ri.n_clusters = cl->n_clusters;
  ri.n_rows = c->n_rows;
  ri.n_units = cl->n_units;
  ri.unit = in->unit;
  ri.hit_begin = in->hit_begin;
  ri.hit_id = in->hit_id;
  ri.hit_row = in->hit_row;
  ri.seed = in->seed;
  ri.x_ref = in->x_ref;
  ri.chi2 = in->chi2;
  ri.ndf = in->ndf;
  ri.y = cl->y;
  ri.z = cl->z;
  ri.row_x = c->d_row_x;
  const RebuildConsts f{rp->chi2_cut,    rp->chi2_final, rp->var_s,      rp->var_t,
                       rp->var_w,       rp->rounds,     rp->extrapolate ? 1 : 0, rp->chi2_extrap};
  RebuildOut ro;
  ro.assigned = out->assigned;
  ro.param = out->param;
  ro.cov = out->cov;
  ro.chi2 = out->chi2;
  ro.x_out = out->x_out;
  ro.n_kept = out->n_kept;
  ro.ok = out->ok;
  const dim3 gw(blocks_for(in->n_tracks, kWave));
  hipLaunchKernelGGL(k_rebuild_keys, dim3(blocks_for(in->n_tracks, 256)), dim3(256), 0, stream, ri, L.ws.key,
                     L.ws.first, L.ws.active, L.ws.check);
  hipLaunchKernelGGL(k_rebuild_pass12, gw, dim3(kWave), 0, stream, ri, g, c->dp, f, L.ws);
  if (cl->n_clusters > 0)
    hipLaunchKernelGGL(k_fill_i64, dim3(std::max(1, std::min(blocks_for(cl->n_clusters, 256), 4096))), dim3(256),
                       0, stream, reinterpret_cast<int64_t*>(L.ws.holder), cl->n_clusters, int64_t(0));
  for (int round = 0; round < rp->rounds; ++round) {
    hipLaunchKernelGGL(k_rebuild_propose, gw, dim3(kWave), 0, stream, ri, L.ws);
    hipLaunchKernelGGL(k_rebuild_advance, gw, dim3(kWave), 0, stream, ri, L.ws);
  }
  hipLaunchKernelGGL(k_rebuild_pass3, gw, dim3(kWave), 0, stream, ri, c->dp, f, L.ws, ro);
  return hipGetLastError() == hipSuccess ? TPCX_OK : TPCX_E_HIP;
}

size_t tpcx_select_workspace_bytes(const tpcx_ctx* c, int32_t n_units, int64_t n_clusters) {
  if (!c || n_units < 1 || n_clusters < 0) return 0;
  Carver cv{nullptr};
  cv.take<unsigned long long>(n_clusters);
  cv.take<int64_t>(n_units);
  return cv.off;
}

tpcx_status tpcx_select(tpcx_ctx* c, const tpcx_tracks* tracks, int32_t n_units, int64_t n_clusters,
                        int32_t shared_num, int32_t shared_den, uint8_t* keep, int32_t* assign,
                        int64_t* sel_counts, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!c || !tracks || !tracks->counts || n_units < 1 || n_clusters < 0 ||
      n_clusters >= (int64_t(1) << 31) || shared_num < 0 || shared_den < 1 || !sel_counts ||
      tracks->cap_tracks < 0 || tracks->cap_hits < 0)
    return TPCX_E_ARG;
  if (tracks->cap_tracks > 0 && (!keep || !tracks->unit || !tracks->n_hits || !tracks->hit_begin ||
                                 !tracks->chi2 || !tracks->ndf))
    return TPCX_E_ARG;
  if (tracks->cap_hits > 0 && !tracks->hit_id) return TPCX_E_ARG;
  if (n_clusters > 0 && !assign) return TPCX_E_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return TPCX_E_ARG;
  Carver cv{static_cast<char*>(ws)};
  auto* owner = cv.take<unsigned long long>(n_clusters);
  auto* first = cv.take<int64_t>(n_units);
  if (!ws || ws_bytes < cv.off) return TPCX_E_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device) return TPCX_E_ARG;
  SelectIn in;
  in.cap_tracks = tracks->cap_tracks;
  in.counts = tracks->counts;
  in.unit = tracks->unit;
  in.n_hits = tracks->n_hits;
  in.hit_begin = tracks->hit_begin;
  in.hit_id = tracks->hit_id;
  in.chi2 = tracks->chi2;
  in.ndf = tracks->ndf;
  const int grid_t = int(std::max<int64_t>(1, std::min<int64_t>(blocks_for(tracks->cap_tracks, 256),
                                                                 int64_t(8) * c->n_cu)));
  const int grid_c = int(std::max<int64_t>(1, std::min<int64_t>(blocks_for(n_clusters, 256),
                                                                 int64_t(16) * c->n_cu)));
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, stream, sel_counts, int64_t(2), int64_t(0));
  if (tracks->cap_tracks > 0)
    hipLaunchKernelGGL(k_select_clear, dim3(grid_t), dim3(256), 0, stream, tracks->cap_tracks, keep);
  if (n_clusters > 0) {
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_c), dim3(256), 0, stream,
                       reinterpret_cast<int64_t*>(owner), n_clusters, int64_t(0));
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_c), dim3(256), 0, stream, assign, n_clusters, -1);
  }
  if (tracks->cap_tracks == 0 || n_clusters == 0) return hipGetLastError() == hipSuccess ? TPCX_OK : TPCX_E_HIP;
  hipLaunchKernelGGL(k_select_first, dim3(grid_t), dim3(256), 0, stream, in, first, sel_counts + 1);
  for (int pass = 0; pass < kClaimPasses; ++pass)
    hipLaunchKernelGGL(k_select_claim, dim3(grid_t), dim3(256), 0, stream, in, first, pass, owner);
  hipLaunchKernelGGL(k_select_decide, dim3(grid_t), dim3(256), 0, stream, in, first, owner, shared_num,
                     shared_den, keep, sel_counts);
  hipLaunchKernelGGL(k_select_reclaim, dim3(grid_t), dim3(256), 0, stream, in, first, keep, owner, assign);
  hipLaunchKernelGGL(k_select_assign, dim3(grid_t), dim3(256), 0, stream, in, first, keep, owner, assign);
  return hipGetLastError() == hipSuccess ? TPCX_OK : TPCX_E_HIP;
}

const char* tpcx_strerror(tpcx_status s) {
  switch (s) {
    case TPCX_OK: return "ok";
    case TPCX_E_ARG: return "invalid argument";
    case TPCX_E_CAPACITY: return "a device capacity was exceeded; counts hold the required sizes";
    case TPCX_E_HIP: return "HIP runtime error";
    case TPCX_E_DEVICE: return "device is not gfx950";
    case TPCX_E_INPUT: return "some cluster coordinates are not finite (those clusters were ignored)";
    default: return "unknown status";
  }
}

}  // extern "C"
