/*
 * tpcx -- per-sector TPC track finding on AMD Instinct MI355X (gfx950).
 *
 * The operation is the sector tracking of the ALICE TPC reconstruction
 * (arXiv 2601.20569, Section 2): clusters organised by sector and pad row go
 * in; a cellular-automaton seeding (neighbour finder over adjacent rows,
 * mutual-link cleaning, start hits) is followed by a Kalman-filter track
 * following that picks up clusters row by row under a chi2 cut; track
 * candidates ("tracklets") with their cluster ids, helix parameters,
 * covariances and chi2 come out.  As the paper states, one particle usually
 * yields several candidates; all are returned (no ambiguity solving here).
 *
 * Conventions (the paper fixes none of them; they are this library's):
 *   - a "unit" is one sector of one event or time-frame slice; units are
 *     independent.  Each unit has n_rows pad rows, planes at local x = row_x[r].
 *   - a cluster is (y, z) in the unit's local frame: y along the pad row, z the
 *     drift coordinate.  Cluster id = its index in the caller's arrays.
 *   - track state at plane x: (y, z, sin(phi), dz/ds_xy, q/pT [(GeV/c)^-1]);
 *     sin(phi) changes by -kappa * q/pT per cm of x, kappa = 2.99792458e-3 * Bz.
 *   - every floating-point operation that takes a decision is IEEE binary32,
 *     round-to-nearest, without contraction, so that results are reproducible
 *     bit for bit (the paper's deterministic mode, Section 5).
 *
 * Memory: every pointer is a device (HIP) address unless its name ends in
 * _host.  The caller owns all inputs, outputs and the workspace; the context
 * owns only immutable tables built at creation.  No call allocates device
 * memory.  Calls enqueue work on the given stream and return; a context may be
 * used by one stream at a time.
 *
 * Errors: argument errors are returned at once and nothing is enqueued.
 * Conditions found on the device (a capacity too small) are written to
 * counts[3] of the output (bit set) with the REQUIRED sizes in counts[0..2];
 * outputs are then truncated but consistent, and the caller may resize and
 * call again.  No C++ exception crosses this interface.
 */
#ifndef TPCX_H_
#define TPCX_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tpcx_status;
#define TPCX_OK 0
#define TPCX_E_ARG (-1)      /* invalid argument; nothing enqueued */
#define TPCX_E_CAPACITY (-2) /* reported by tpcx_poll: a device capacity was exceeded */
#define TPCX_E_HIP (-3)      /* a HIP runtime call failed */
#define TPCX_E_DEVICE (-4)   /* current device is not gfx950 */
#define TPCX_E_INPUT (-5)    /* reported by tpcx_poll: some cluster coordinates were not finite */

/* device status bits, counts[3] of tpcx_tracks */
#define TPCX_ST_START_OVERFLOW 1 /* more start hits than cap_start */
#define TPCX_ST_TRACK_OVERFLOW 2 /* more tracklets than cap_tracks */
#define TPCX_ST_HIT_OVERFLOW 4   /* more attached clusters than cap_hits */
#define TPCX_ST_NONFINITE 8      /* a cluster's y or z is not finite: it joins nothing; results otherwise complete */

typedef struct tpcx_ctx tpcx_ctx;

/* Detector description: the pad-row planes of a sector (Section 2: two halves
 * of 18 trapezoidal sectors, each with pad rows). */
typedef struct {
  int32_t n_rows;            /* 3 .. 160 */
  const float* row_x_host;   /* [n_rows] strictly increasing plane distances, cm */
  float tan_half_opening;    /* half-width of a row = row_x * tan_half_opening (tan 10 deg) */
  float bz_tesla;            /* solenoid field */
} tpcx_geometry;

/* Method parameters (Section 2 describes the steps; the values are readings). */
typedef struct {
  float win_y, win_z;   /* neighbour finder: |dy|, |dz| window to the adjacent rows, cm */
  float d2_max;         /* neighbour finder: cut on the squared chord deviation, cm^2 */
  float chi2_max;       /* following: attach a cluster if its chi2 <= chi2_max */
  float sinphi_max;     /* propagation stops when |sin(phi)| would reach this */
  float u_max;          /* propagation stops when |curvature| * chord / 2 exceeds this */
  float sigma_y, sigma_z; /* cluster errors, cm */
  float cww0;           /* seed variance of q/pT, (GeV/c)^-2 */
  int32_t min_hits;     /* tracklets with fewer clusters are dropped */
  int32_t max_misses;   /* consecutive rows without a cluster that end following */
  int32_t descent_rows; /* longest step (rows) of the walk back to the start row */
} tpcx_params;

/* Launch, work-queue and search-grid tuning.  Never changes results. */
typedef struct {
  float bin_y;          /* search-grid bin width along the pad row, cm (fixed per context) */
  int32_t n_zbins;      /* search-grid bins along z per unit (z range taken from data) */
  int32_t block;        /* threads per block of the per-cluster kernels (64..1024) */
  int32_t construct_grid;   /* blocks of 256 lanes of the persistent tracklet constructor */
  int32_t construct_refill; /* idle lanes of a constructor wavefront that trigger a refill (1..64) */
  int32_t refit_grid;       /* blocks of 256 lanes of the persistent refit filter; 0: 7 per CU */
  int32_t refit_refill;     /* idle lanes of a refit wavefront that trigger a refill (1..64) */
} tpcx_tuning;

/* Clusters grouped by (unit, row): those of unit u, row r are the index range
 * [row_begin[u*n_rows + r], row_begin[u*n_rows + r + 1]).  Order inside a
 * range is free.  n_clusters = row_begin[n_units*n_rows] < 2^31. */
typedef struct {
  int32_t n_units;
  int64_t n_clusters;
  const int64_t* row_begin; /* [n_units*n_rows + 1] */
  const float* y;           /* [n_clusters] */
  const float* z;           /* [n_clusters] */
} tpcx_clusters;

/* Tracklets, in the order of their start hits (ascending cluster index). */
typedef struct {
  int64_t cap_tracks;   /* capacity of the per-tracklet arrays */
  int64_t cap_hits;     /* capacity of hit_id / hit_row */
  int64_t* counts;      /* [4]: n_start, n_tracks, n_hits (required sizes), status bits */
  int32_t* unit;        /* [cap_tracks] unit of the tracklet */
  int32_t* start;       /* [cap_tracks] start-hit cluster id */
  int32_t* n_hits;      /* [cap_tracks] clusters attached */
  int64_t* hit_begin;   /* [cap_tracks] offset of the tracklet's clusters in hit_id */
  int32_t* hit_id;      /* [cap_hits] cluster ids, sorted by row within a tracklet */
  uint8_t* hit_row;     /* [cap_hits] their rows */
  float* x_ref;         /* [cap_tracks] plane of the parameters: innermost attached row */
  float* param;         /* [cap_tracks][5] y, z, sin(phi), dz/ds, q/pT */
  float* cov;           /* [cap_tracks][15] lower triangle of the 5x5 covariance, row-major */
  float* chi2;          /* [cap_tracks] */
  int32_t* ndf;         /* [cap_tracks] 2*n_hits - 5 */
} tpcx_tracks;

/* Optional intermediate results (each pointer may be NULL). */
typedef struct {
  int32_t* link_up;     /* [n_clusters] neighbour finder: best cluster in row r+1, or -1 */
  int32_t* link_down;   /* [n_clusters] best cluster in row r-1, or -1 */
  int32_t* clean_up;    /* [n_clusters] after keeping only mutual links */
  int32_t* clean_down;  /* [n_clusters] */
  int32_t* starts;      /* [cap_start] start hits, ascending */
} tpcx_debug;

/* Fill *t with the default tuning for a workload of this size. */
void tpcx_default_tuning(int32_t n_units, int64_t n_clusters, tpcx_tuning* t);

/* Create a context on the current HIP device.  tuning may be NULL (defaults
 * chosen per call from the input size).  Returns TPCX_E_DEVICE on a device
 * that is not gfx950. */
tpcx_status tpcx_create(const tpcx_geometry* g, const tpcx_params* p, const tpcx_tuning* tuning,
                        tpcx_ctx** out);
void tpcx_destroy(tpcx_ctx* ctx);

/* Bytes of workspace tpcx_track needs for this input size and start-hit
 * capacity (cap_start <= n_clusters/3 + 1 can never overflow: every start hit
 * owns a chain of at least three clusters). */
size_t tpcx_workspace_bytes(const tpcx_ctx* ctx, int32_t n_units, int64_t n_clusters,
                            int64_t cap_start);

/* Sector tracking of every unit of `in` (Section 2: seeding by the cellular
 * automaton, then track following with the Kalman filter).  ws must hold
 * tpcx_workspace_bytes(ctx, in->n_units, in->n_clusters, cap_start) bytes,
 * 256-byte aligned.  out->counts is written on the device. */
tpcx_status tpcx_track(tpcx_ctx* ctx, const tpcx_clusters* in, void* ws, size_t ws_bytes,
                       int64_t cap_start, const tpcx_tracks* out, const tpcx_debug* dbg,
                       hipStream_t stream);

/* Workspace of tpcx_track_static: 64 MiB per device. */
#define TPCX_STATIC_SCRATCH_BYTES (64u << 20)

/* tpcx_track for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * workspace is a library-owned array of TPCX_STATIC_SCRATCH_BYTES on each
 * device (reserved when the library's code is loaded on the device, held
 * until the process ends; its address is resolved in tpcx_create), so the
 * call allocates nothing; inputs, outputs and results are those of
 * tpcx_track.  Returns TPCX_E_ARG, with nothing enqueued, when
 * tpcx_workspace_bytes(ctx, in->n_units, in->n_clusters, cap_start) exceeds
 * TPCX_STATIC_SCRATCH_BYTES (a single sector or event of a few 10^5 clusters
 * with cap_start near its start-hit count fits).  Every call on a device
 * shares that device's array and the array keeps the last call's contents
 * (each call clears what it needs itself): calls that overlap in time on one
 * device -- other streams, contexts or threads -- race and give wrong
 * results. */
tpcx_status tpcx_track_static(tpcx_ctx* ctx, const tpcx_clusters* in, int64_t cap_start,
                              const tpcx_tracks* out, const tpcx_debug* dbg, hipStream_t stream);

/* Waits for the stream and returns TPCX_E_CAPACITY if the last tpcx_track on
 * it overflowed a capacity, else TPCX_E_INPUT if some cluster coordinate was
 * not finite, TPCX_E_HIP on a runtime error, else TPCX_OK. */
tpcx_status tpcx_poll(tpcx_ctx* ctx, const tpcx_tracks* out, hipStream_t stream);

const char* tpcx_strerror(tpcx_status s);

/* ------------------------------------------------------------------------
 * Track refit through a space-charge-distortion correction map, and its
 * gradient with respect to the map (paper: correction maps for the TPC
 * space-charge distortions, Abstract and Section 2; the track fit is a Kalman
 * filter over the attached clusters, Section 2).
 *
 * Map: three components (delta r, delta r*phi, delta z) [cm], each a
 * tensor-product uniform cubic B-spline over 36 phi nodes (every 10 deg,
 * periodic, node 0 at phi = 0), 17 r nodes (85 + 10 j cm) and 20 z nodes
 * (-250 + k 500/19 cm); theta[((c*36 + i)*17 + j)*20 + k], float32.  A cluster
 * measured at (x, y, z) in its sector frame (radius r, azimuth
 * alpha_unit + atan2(y, x)) moves by delta r along (x, y)/r, by delta r*phi
 * along (-y, x)/r and by delta z along z.
 * Refit: outwards from the track's innermost cluster; y, z from that cluster,
 * sin(phi), dz/ds, q/pT from `seed`, covariance diag(sy^2, sz^2, 1e-2, 1e-2,
 * 1); propagate to every further cluster's own corrected x and update, no
 * rejection; chi2 = sum of the updates' chi2.  A track whose propagation is
 * stopped by a guard gets ok = 0, chi2 = 0 and no gradient.
 * ------------------------------------------------------------------------ */
#define TPCX_MAP_NCOEF 36720

typedef struct {
  int64_t n_tracks;
  int64_t n_hits;            /* host copy of hit_begin[n_tracks] (sizes the workspace) */
  const int64_t* hit_begin;  /* [n_tracks + 1] offsets into hit_id / hit_row */
  const int32_t* hit_id;     /* cluster ids (indices into y, z), ascending rows per track */
  const uint8_t* hit_row;    /* rows of those clusters */
  const int32_t* unit;       /* [n_tracks] unit of each track */
  const float* seed;         /* [n_tracks][5] y, z, sin(phi), dz/ds, q/pT (tracking result) */
  const float* y;            /* clusters, as given to tpcx_track */
  const float* z;
  const float* unit_alpha;   /* [n_units] azimuth of each unit's sector centre line, rad */
} tpcx_refit_in;

/* Workspace of tpcx_refit + tpcx_refit_backward (shared by the pair).  Both
 * calls enqueue and return without waiting: the hit count comes from
 * in->n_hits. */
size_t tpcx_refit_workspace_bytes(const tpcx_ctx* ctx, int64_t n_tracks, int64_t n_hits);

/* Forward refit: chi2[n_tracks], ok[n_tracks].  theta may be NULL (no
 * correction).  Keeps the corrected clusters and the filter state every 16
 * clusters in ws for tpcx_refit_backward. */
tpcx_status tpcx_refit(tpcx_ctx* ctx, const tpcx_refit_in* in, const float* theta, float* chi2,
                       int32_t* ok, void* ws, size_t ws_bytes, hipStream_t stream);

/* Backward: grad_theta[TPCX_MAP_NCOEF] (overwritten) = d(sum_t dL_dchi2[t] *
 * chi2[t]) / d theta, at the theta of the preceding tpcx_refit with the same
 * `in` and ws.  Recomputes the filter states one 16-cluster segment at a
 * time from the stored states and runs the reverse sweep; sums in 64-bit fixed
 * point (2^-32), so the result does not depend on scheduling. */
tpcx_status tpcx_refit_backward(tpcx_ctx* ctx, const tpcx_refit_in* in, const float* dL_dchi2,
                                float* grad_theta, void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched form: many events or time-frame slices at once.  Their units are
 * packed unit-major into one tpcx_clusters (tracklets carry their unit, so a
 * slice's tracklets are those of its unit range).  The whole tracking sequence
 * and the refit of every tracklet with at least refit->min_hits clusters run
 * as one HIP graph: captured on the first call with a given set of arguments,
 * replayed by later calls with the same arguments.  In a time frame the
 * drift coordinate of a cluster mixes its z with its collision's time, which
 * the tracking does not know; for such input the map is evaluated at one
 * fixed z (map_z_fixed = 1), i.e. only its dependence on r and phi acts.
 * The stream must be one
 * that can be captured (not the legacy default stream).  The correction of
 * the clusters for the refit needs only the search grid: it runs on a second
 * stream owned by the context, forked after the grid build and joined before
 * the refit filter (both branches are in the graph).  The persistent
 * kernels (tracklet constructor, refit) take their work counts from the
 * device, so a replay needs no host synchronisation.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t min_hits;         /* refit tracklets with at least this many clusters (>= 2) */
  int32_t map_z_fixed;      /* 0: map evaluated at each cluster's measured z; 1: at z = map_z */
  float map_z;              /* cm; the z of the map evaluation when map_z_fixed (a time frame) */
  const float* theta;       /* map coefficients [TPCX_MAP_NCOEF], or NULL for no correction */
  const float* unit_alpha;  /* [n_units] azimuth of each unit's sector centre line, rad */
  float* chi2;              /* [cap_tracks] refit chi2 (0 when not refitted) */
  int32_t* ok;              /* [cap_tracks] 1 when refitted */
} tpcx_batch_refit;

size_t tpcx_batched_workspace_bytes(const tpcx_ctx* ctx, int32_t n_units, int64_t n_clusters,
                                    int64_t cap_start, int64_t cap_tracks, int64_t cap_hits);

/* The batched form of the sector tracking (paper, Section 2), over many
 * units at once, with the autotuned launch shapes of Section 5's tuning:
 * tracking of every unit of `in` plus the refit (refit may be NULL).
 * Outputs as tpcx_track; an overflow bit in out->counts[3] means no
 * tracklet is refitted. */
tpcx_status tpcx_track_batched(tpcx_ctx* ctx, const tpcx_clusters* in, void* ws, size_t ws_bytes,
                               int64_t cap_start, const tpcx_tracks* out,
                               const tpcx_batch_refit* refit, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Ambiguity solving (paper, Section 2: tracks are found several times; the
 * best instance of each track keeps its clusters and the clones are removed,
 * a configurable fraction of a track's clusters -- 10 % by default, 20 %
 * after the loosening the paper describes -- may be shared with other
 * tracks; Section 3, Phase I: among tracks competing for a cluster the one
 * with the smaller global chi2 has priority, the track length weighing less,
 * and shared clusters are counted starting at the outermost pad row).
 *
 * Rank: a tracklet ranks above another when its q = chi2/ndf (binary32
 * quotient) is smaller, then when it has more clusters, then when it comes
 * first in its unit.  Every cluster is owned by the highest-ranked tracklet
 * containing it.  A tracklet is kept when, walking its clusters from the
 * outermost row inwards, after every step k the number s(k) of clusters seen
 * that another tracklet owns satisfies shared_den * s(k) <= shared_num * k.
 * Every cluster is then assigned to the highest-ranked kept tracklet that
 * contains it.
 * ------------------------------------------------------------------------ */

/* Workspace of tpcx_select (8 bytes per cluster and per unit). */
size_t tpcx_select_workspace_bytes(const tpcx_ctx* ctx, int32_t n_units, int64_t n_clusters);

/* Ambiguity solving of the tracklets a tpcx_track or tpcx_track_batched call
 * wrote to `tracks` (unit, n_hits, hit_begin, hit_id, chi2, ndf and counts
 * are read; the tracklet count is counts[1]; nothing is selected when
 * counts[3] reports an overflow).  n_units and n_clusters are those of the
 * tracking input.  Writes keep[cap_tracks] (1: kept; 0 for a clone and for
 * every slot beyond the count), assign[n_clusters] (index of the kept
 * tracklet a cluster is assigned to, or -1) and sel_counts[2] on the device:
 * [0] kept tracklets, [1] status (1: a unit holds more than 2^24 tracklets,
 * beyond the rank's index field).  shared_num / shared_den is the allowed
 * shared fraction (shared_den >= 1).  ws: tpcx_select_workspace_bytes bytes,
 * 256-byte aligned.  Enqueues and returns. */
tpcx_status tpcx_select(tpcx_ctx* ctx, const tpcx_tracks* tracks, int32_t n_units, int64_t n_clusters,
                        int32_t shared_num, int32_t shared_den, uint8_t* keep, int32_t* assign,
                        int64_t* sel_counts, void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Three-iteration track fit with interpolation-based cluster rejection
 * (paper, Section 2, track fit: three iterations, inwards, outwards,
 * inwards, the cluster chi2 cut taken against the interpolation between one
 * iteration's state and the position and covariance another iteration stored
 * per pad row in reduced precision; Section 3, Phase I: the first, inward
 * iteration stores, the second, outward one interpolates and cuts, the third
 * applies the rejection).
 *
 * Per track (clusters innermost first, y and z relative to the outermost):
 *   1. from the tracking result at x_ref, propagate out to the outermost
 *      cluster, take its y, z and a diagonal covariance (sy^2, sz^2, var_s,
 *      var_t, var_w), then inwards: at every cluster store the predicted
 *      residual (y - m_y, z - m_z) and predicted C_yy, C_zz as bfloat16
 *      (round to nearest even), update;
 *   2. restart at the innermost cluster (its y, z; sin(phi), dz/ds, q/pT of
 *      iteration 1; diagonal covariance), outwards: per coordinate the
 *      inverse-variance combination r = (d_in C_out + d_out C_in) / (C_in +
 *      C_out), C = C_in C_out / (C_in + C_out) of the outward prediction and
 *      the stored inward one (one of them alone at the two ends); reject the
 *      cluster when r_y^2/(C_y + sy^2) + r_z^2/(C_z + sz^2) > chi2_cut; update
 *      with every cluster;
 *   3. from iteration 2's state, propagate back to the outermost kept
 *      cluster, take its y, z and the diagonal covariance, then inwards over
 *      the kept clusters.  Result at the innermost kept cluster; chi2 of the
 *      kept clusters' updates; ndf = 2 n_kept - 5.
 * A fit fails (ok = 0, zero results, nothing rejected) when a propagation
 * guard stops a step or fewer than 3 clusters are kept.
 * ------------------------------------------------------------------------ */
typedef struct {
  float chi2_cut;              /* interpolation chi2 cut (2 degrees of freedom) */
  float var_s, var_t, var_w;   /* restart variances of sin(phi), dz/ds, q/pT */
} tpcx_fit_params;

typedef struct {
  int64_t n_tracks;
  int64_t n_hits;              /* host copy of hit_begin[n_tracks] */
  const int64_t* hit_begin;    /* [n_tracks + 1] */
  const int32_t* hit_id;       /* cluster ids, rows ascending per track */
  const uint8_t* hit_row;
  const float* seed;           /* [n_tracks][5] tracking result y, z, sin(phi), dz/ds, q/pT */
  const float* x_ref;          /* [n_tracks] its plane */
  const float* y;              /* clusters */
  const float* z;
  int64_t n_clusters;          /* length of y and z */
} tpcx_fit_in;

typedef struct {
  float* param;     /* [n_tracks][5] at x_out */
  float* cov;       /* [n_tracks][15] lower triangle */
  float* chi2;      /* [n_tracks] */
  float* x_out;     /* [n_tracks] plane of the innermost kept cluster */
  int32_t* n_kept;  /* [n_tracks] */
  int32_t* ok;      /* [n_tracks] */
  uint8_t* reject;  /* [n_hits] 1: cluster rejected */
} tpcx_fit_out;

/* Workspace of tpcx_fit: 17 bytes per record slot (the stored iteration-1
 * record and its row), n_hits slots plus 16384 per 8192 tracks (the slack of
 * the per-wavefront interleaved layout; a track of 256 or more clusters may
 * make the fit fall back to one record per hit in track order, same results),
 * 16 bytes per 64 tracks, 4 bytes per track (the processing order: longest
 * tracks first within chunks of 8192 consecutive tracks) and 8 bytes per
 * cluster (y and z side by side: one gather per hit).  n_tracks < 2^31. */
size_t tpcx_fit_workspace_bytes(const tpcx_ctx* ctx, int64_t n_tracks, int64_t n_hits, int64_t n_clusters);

/* Enqueues the fit of every track of `in`; ws 256-byte aligned. */
tpcx_status tpcx_fit(tpcx_ctx* ctx, const tpcx_fit_in* in, const tpcx_fit_params* params,
                     const tpcx_fit_out* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Track rebuild (paper, Section 3, Phase II: during the fit the attachment
 * is redone; iteration 2 queries the sector tracking's cluster search grid
 * for every cluster compatible with the chi2 cut against the interpolation
 * and stores the candidates with their residuals; a second ambiguity solving
 * assigns candidates by rank, a track that does not get its best candidate
 * staying eligible for the next; iteration 3 applies a plain chi2 cut).
 *
 * Per track of one unit (clusters innermost first, rows r_in .. r_out, y and
 * z relative to the outermost cluster):
 *   1. from the tracking result at x_ref out to the outermost cluster (its
 *      y, z; diagonal covariance), then row by row inwards to r_in: store the
 *      predicted y, z (binary32) and C_yy, C_zz (bfloat16) of every row,
 *      update with the track's own cluster of the row;
 *   2. restart at the innermost cluster, row by row outwards: combine the
 *      outward prediction with the stored one by inverse-variance weighting
 *      (one alone at r_in and r_out); every cluster of the row with chi2 <=
 *      chi2_cut against that interpolation is a candidate; the 4 best by
 *      (chi2, caller id) are kept; update with the best (not at r_in);
 *   3. rank of a track as in tpcx_select, from the given chi2, ndf and
 *      length; `rounds` rounds in which every (track, row) proposes its
 *      current candidate, a cluster is held by its best-ranked proposer so
 *      far, and a (track, row) whose candidate another holds moves to its
 *      next; a (track, row) gets its candidate if it holds it; no sharing;
 *   4. from step 2's final state back to the outermost assigned row (its
 *      cluster's y, z; diagonal covariance), then inwards over the assigned
 *      rows: a cluster whose filter chi2 exceeds chi2_final is dropped.
 *      Result at the innermost kept cluster; ndf = 2 n_kept - 5.
 * Phase III (paper, Section 3: the rebuild extended by extrapolating the
 * tracks inwards and outwards; candidates found so go through the same
 * ambiguity solving, optionally with a stricter cut), when extrapolate is
 * set: after step 1 the state of r_in is carried further in row by row
 * (no updates) until row 0 or a propagation guard, and after step 2 its
 * final state further out until the last row or a guard; those rows' clusters
 * with chi2 <= chi2_extrap against the extrapolation alone are candidates,
 * and steps 3 and 4 run over the extended rows.  Not across sector
 * boundaries.
 * A rebuild fails (ok = 0, nothing assigned) on a propagation guard, with
 * fewer than 3 kept clusters, or when its input breaks the layout below
 * (unit outside 0 .. n_units - 1, rows not strictly ascending or outside
 * the geometry, cluster ids outside the cluster array, offsets outside
 * 0 .. n_hits): such input is never read out of bounds.
 * ------------------------------------------------------------------------ */
typedef struct {
  float chi2_cut;              /* candidate chi2 cut against the interpolation */
  float chi2_final;            /* chi2 cut of the last iteration */
  float var_s, var_t, var_w;   /* restart variances of sin(phi), dz/ds, q/pT */
  int32_t rounds;              /* proposal rounds of the assignment (0 .. 64) */
  int32_t extrapolate;         /* 1: Phase III, candidates also beyond the track's ends */
  float chi2_extrap;           /* chi2 cut of those candidates */
} tpcx_rebuild_params;

typedef struct {
  int64_t n_tracks;            /* tracks in unit order */
  int64_t n_hits;              /* host copy of hit_begin[n_tracks] */
  const int32_t* unit;         /* [n_tracks] */
  const int64_t* hit_begin;    /* [n_tracks + 1] */
  const int32_t* hit_id;       /* clusters, rows ascending per track */
  const uint8_t* hit_row;
  const float* seed;           /* [n_tracks][5] tracking result */
  const float* x_ref;          /* [n_tracks] */
  const float* chi2;           /* [n_tracks] tracking chi2 (rank) */
  const int32_t* ndf;          /* [n_tracks] */
} tpcx_rebuild_in;

typedef struct {
  int32_t* assigned;  /* [n_tracks][n_rows] cluster kept at each row, -1 for none */
  float* param;       /* [n_tracks][5] */
  float* cov;         /* [n_tracks][15] */
  float* chi2;        /* [n_tracks] */
  float* x_out;       /* [n_tracks] */
  int32_t* n_kept;    /* [n_tracks] */
  int32_t* ok;        /* [n_tracks] */
} tpcx_rebuild_out;

/* Workspace of tpcx_rebuild: the search grid of the clusters, ~50 bytes per
 * track and row, 8 bytes per cluster. */
size_t tpcx_rebuild_workspace_bytes(const tpcx_ctx* ctx, int32_t n_units, int64_t n_clusters,
                                    int64_t n_tracks);

/* Enqueues the rebuild of the tracks `in` against the clusters `clusters`
 * (the tracking input: its search grid is built here); ws 256-byte aligned. */
tpcx_status tpcx_rebuild(tpcx_ctx* ctx, const tpcx_clusters* clusters, const tpcx_rebuild_in* in,
                         const tpcx_rebuild_params* params, const tpcx_rebuild_out* out, void* ws,
                         size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Track merging (paper, Section 2: the track segments of the sector tracking
 * are merged inside a sector, between adjacent sectors of one TPC half and
 * across the central electrode).  The paper gives no matching criterion;
 * this one:
 *   views  each track's state (param at x_ref, in its sector frame) is
 *          carried to the plane x = x_m in its own frame (view 0) and in the
 *          frames of the boundaries with the next (view 1: rotated by -h
 *          about the beam axis, h = half the sector opening) and the
 *          previous sector of its half (view 2: +h), with the tracking's
 *          circle step in equal steps of at most 10 cm; a view is missing
 *          when |sin(phi)| (before or after the rotation) or a step meets the
 *          tracking's propagation guards;
 *   pairs  a (inner) and b (outer), r_out[a] < r_in[b], in the same unit
 *          (views 0, 0), in the units of one azimuth across the electrode
 *          (0, 0; when cross_electrode), or in adjacent sectors (a's view
 *          towards b's sector against b's view towards a's: 1 against 2 when
 *          b's unit is a's next, 2 against 1 when it is the previous);
 *   chi2   sum over (y, z, sin(phi), dz/ds, q/pT) of (difference)^2 /
 *          tol^2, in this order, IEEE binary32; candidates at chi2 <= cut;
 *   links  a's best outer candidate and b's best inner candidate by (chi2,
 *          track index); a and b are linked when each is the other's.
 * Outputs per track: next (its outer partner), prev (its inner partner), -1
 * for none, and root (the first track of its chain).  A track whose unit is
 * outside 0 .. n_units - 1 or whose rows are not 0 <= r_in <= r_out < 256
 * links to nothing.
 * ------------------------------------------------------------------------ */
typedef struct {
  float x_m;              /* plane of the views [cm] */
  float cos_h, sin_h;     /* cos and sin of half the sector opening */
  float tol[5];           /* tolerances of y, z [cm], sin(phi), dz/ds, q/pT [(GeV/c)^-1] */
  float chi2_cut;
  int32_t cross_electrode;
} tpcx_merge_params;

typedef struct {
  int64_t n_tracks;          /* < 2^31 */
  int32_t n_units;
  const int32_t* unit;       /* [n_tracks], ascending */
  const float* param;        /* [n_tracks][5] at x_ref, sector frame */
  const float* x_ref;        /* [n_tracks] */
  const int32_t* r_in;       /* [n_tracks] first row */
  const int32_t* r_out;      /* [n_tracks] last row */
  const int32_t* unit_nbr;   /* [n_units][3]: unit of the next sector of the same half,
                                of the previous one, across the electrode; -1: none */
} tpcx_merge_in;

typedef struct {
  int32_t* prev;  /* [n_tracks] */
  int32_t* next;  /* [n_tracks] */
  int32_t* root;  /* [n_tracks] */
} tpcx_merge_out;

/* Workspace of tpcx_merge: 128 bytes per track and 12 KiB per unit. */
size_t tpcx_merge_workspace_bytes(const tpcx_ctx* ctx, int32_t n_units, int64_t n_tracks);

/* Enqueues the merging of the tracks `in` (device arrays); ws 256-byte
 * aligned. */
tpcx_status tpcx_merge(tpcx_ctx* ctx, const tpcx_merge_in* in, const tpcx_merge_params* params,
                       const tpcx_merge_out* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Tuning and autotuning.  No tuning changes any result (every selection of
 * the method has a total order), only the speed.
 * ------------------------------------------------------------------------ */

/* Make *t the context's tuning for later calls (NULL: back to the defaults,
 * chosen by workload size).  t->bin_y must equal the context's.  A batched
 * graph captured with another tuning is captured again on its next call. */
tpcx_status tpcx_set_tuning(tpcx_ctx* ctx, const tpcx_tuning* t);

/* Workspace that fits every tuning tpcx_autotune_batched tries. */
size_t tpcx_autotune_workspace_bytes(const tpcx_ctx* ctx, int32_t n_units, int64_t n_clusters,
                                     int64_t cap_start, int64_t cap_tracks, int64_t cap_hits);

/* Autotuner of the batched form (paper, Section 5: launch parameters are
 * tuned automatically per GPU).  Times the batched sequence (tracking, plus
 * the refit when refit is set) on the caller's input for candidate tunings,
 * one parameter at a time in a fixed order: z bins of the search grid, block
 * size of the per-row kernels, grid and refill threshold of the persistent
 * constructor, grid and refill threshold of the persistent refit filter.  A
 * candidate replaces the current best when it is at least 1% faster (one
 * warm-up run, then the mean of reps >= 1 runs, each a replay of the
 * candidate's sequence captured into a graph as the batched form runs it;
 * directly launched on the legacy default stream), confirmed by timing both
 * once more (the sums of the two timings must differ by 1%); a candidate
 * whose workspace exceeds ws_bytes is skipped.  The best tuning becomes the context's
 * tuning and is written to *best.  Synchronises the stream.  Returns
 * TPCX_E_CAPACITY if the output capacities are too small for the input. */
tpcx_status tpcx_autotune_batched(tpcx_ctx* ctx, const tpcx_clusters* in, void* ws, size_t ws_bytes,
                                  int64_t cap_start, const tpcx_tracks* out,
                                  const tpcx_batch_refit* refit, int32_t reps, tpcx_tuning* best,
                                  hipStream_t stream);

/* Stage timing (profiling aid).  Stages of one tpcx_track call, in order. */
#define TPCX_STAGE_GRID 0       /* search-grid build */
#define TPCX_STAGE_NEIGHBOURS 1 /* neighbour finder */
#define TPCX_STAGE_STARTS 2     /* cleaning, start flags, ordered compaction */
#define TPCX_STAGE_CONSTRUCT 3  /* tracklet constructor */
#define TPCX_STAGE_COMPACT 4    /* ordered compaction of the kept tracklets */
#define TPCX_STAGE_REFIT 5      /* refit filter, from the end of the compaction (batched form only) */
#define TPCX_N_STAGES 6

/* Record HIP events on the call's stream around every stage of the next
 * max_calls tpcx_track / tpcx_track_batched calls (max_calls = 0 switches
 * timing off).  While timing slots are left, tpcx_track_batched launches its
 * sequence directly (same kernels and launch shapes) instead of replaying the
 * graph.  Creates the events; call it outside timed or captured regions. */
tpcx_status tpcx_timing_enable(tpcx_ctx* ctx, int32_t max_calls);

/* Waits for the recorded events and writes, per stage, the summed elapsed
 * milliseconds over the recorded calls to ms_host[TPCX_N_STAGES] and their
 * number to *n_calls; then starts a new recording. */
tpcx_status tpcx_timing_read(tpcx_ctx* ctx, float* ms_host, int32_t* n_calls);

#ifdef __cplusplus
}
#endif

#endif /* TPCX_H_ */
