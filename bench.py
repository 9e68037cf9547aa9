#!/usr/bin/env python3
"""Throughput of per-sector TPC track finding on one MI355X.

Default workload ("batched"): 16 synthetic time-frame slices (32-160 Pb-Pb
collisions each, overlapped in drift time, radial space-charge distortion),
all 576 sector units tracked plus the refit of every tracklet with at least 20
clusters through a distortion-correction map, as one HIP graph.  One step is
one replay of that graph with the inputs resident in HBM.

The JSON line also carries: the plain form (one tpcx_track call per slice,
and one per sector unit), the adjoint refit (forward + hand-written backward) on a central event, the
roofline position of the dominant kernel (HIP events recorded by the library
on its stream around every stage), and the CPU oracle timed on a bounded
sample of the same input.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload batched|timeframe|central|single]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TPC clusters/s tracked (1 GPU, % HBM roofline); batched & adjoint vs plain"
HBM_PEAK_GBS = 8000.0

# algorithmic bytes: the compulsory traffic of the method's own passes (each
# array read once and written once; data-dependent counts from the oracle's
# counters), per pass of the hot path
B_GRID_PER_CLUSTER = 24        # read y, z, id (12 B); write sorted y, z, perm (12 B)
B_NF_PER_CLUSTER = 16          # read y, z (8 B; neighbour rows reused); write up, down links (8 B)
B_STARTS_PER_CLUSTER = 16      # read two links (8 B), write two cleaned links (8 B)
B_STARTS_PER_START = 8         # write the start hit (id and position)
B_CON_PER_TRACKLET = 104       # tracklet record: x_ref, 5 parameters, covariance, chi2, n, ndf, offsets
B_CON_PER_CHAIN_HIT = 12       # chain step: the link (4 B) and y, z (8 B) of the next chain cluster
B_CON_PER_SEARCH = 8           # following step: the bin offsets of the search box
B_CON_PER_CANDIDATE = 8        # y, z of every cluster inside the chi2 box of a searched row
B_CON_PER_ATTACHED = 5         # write id and row of every attached cluster
B_OUT_PER_TRACK = 2 * 104      # read the tracklet record, write the kept one
B_OUT_PER_HIT = 2 * 5          # read and write id + row of every kept cluster
B_REFIT_PER_TRACK = 104        # refitted tracklet: its record (seed, offsets) and result
B_REFIT_PER_HIT = 12           # refitted cluster: id, y, z
B_SEL_PER_TRACK = 25           # ambiguity solving: unit, n, offset, chi2, ndf read; kept flag written
B_SEL_PER_HIT = 4              # the cluster id of every attached cluster
B_SEL_PER_CLUSTER = 20         # owner key written and read (8 + 8), assignment written (4)
B_RB_PER_TRACK = 160           # rebuild: seed, rank inputs, offsets read; results written
B_RB_PER_HIT = 5               # id + row of every input cluster
B_RB_PER_CLUSTER = 32          # grid build (24) and the holder word (8) of every cluster
B_MERGE_PER_TRACK = 48        # merging: unit, param, x_ref, first and last row read; prev, next, root written
B_FIT_PER_TRACK = 128          # fit: seed, x_ref, offsets read; parameters, covariance, chi2, counts written
B_FIT_PER_HIT = 62             # id, row, y, z read; 16-byte record written once and read twice; flag written


# kernels of each stage, for the recorded HBM traffic (profiles/)
STAGE_KERNELS = {"grid": ["k_grid_build"], "neighbours": ["k_neighbours"],
                 "starts": ["k_clean_starts", "k_write_starts"], "construct": ["k_construct"],
                 "compact": ["k_keep_count", "k_keep_write"], "refit": ["k_correct_clusters", "k_refit_filter<true>"]}


def source_sha256():
    """Hash of the kernel sources, as recorded in the counter summaries."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2601_20569_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_valu(stage, workload):
    """Per-kernel VALU issue rate per CU-cycle, active lanes, waiting fraction
    and L2 hit rate of a stage's kernels from the committed counter summary,
    or None when it is missing or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"valu_{workload}.md")
    if not os.path.exists(path):
        return None
    rec, sha = {}, None
    for line in open(path):
        line = line.strip()
        if line.startswith("source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith("valu "):
            k, v = line[len("valu "):].split(":", 1)
            rec[k.strip()] = {kv.split("=")[0]: float(kv.split("=")[1]) for kv in v.split()}
    if sha != source_sha256():
        return None
    ks = [k for k in STAGE_KERNELS.get(stage, []) if k in rec]
    return {k: rec[k] for k in ks} or None


def recorded_traffic(stage, workload):
    """HBM bytes per launch of a stage's kernels from the committed counter
    summary, or None when it is missing or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    rec, sha = {}, None
    for line in open(path):
        line = line.strip()
        if line.startswith("source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith("traffic_bytes_per_launch "):
            k, v = line[len("traffic_bytes_per_launch "):].split(":")
            rec[k.strip()] = int(v)
    if sha != source_sha256():
        return None
    ks = STAGE_KERNELS.get(stage, [])
    if not ks or any(k not in rec for k in ks):
        return None
    return sum(rec[k] for k in ks)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sync():
    import torch
    torch.cuda.synchronize()


def gen_batch(device):
    """16 slices, generated one at a time, packed unit-major on the device."""
    import numpy as np
    import torch

    import synth
    ncoll = synth.slice_batch_collisions(seed=4000, n_slices=16)
    ys, zs, rbs, sectors, sizes, first = [], [], [], [], [], None
    off = 0
    for i, nc in enumerate(ncoll):
        cs = synth.timeframe_slice(seed=4000 + i, n_collisions=nc, device=device, truth=(i == 0))
        if i == 0:
            first = cs
        ys.append(torch.as_tensor(cs.y, device=device))
        zs.append(torch.as_tensor(cs.z, device=device))
        rbs.append(cs.row_begin[:-1] + off)
        sectors.append(cs.unit_sector)
        sizes.append((off, cs.n_clusters, cs.row_begin.copy()))
        off += cs.n_clusters
        log(f"slice {i}: {nc} collisions, {cs.n_clusters} clusters")
    rb = np.concatenate(rbs + [np.array([off], np.int64)])
    y = torch.cat(ys)
    z = torch.cat(zs)
    del ys, zs
    return dict(rb=torch.as_tensor(rb, device=device), y=y, z=z, n=off,
                n_units=len(rb) - 1 - 0, sectors=np.concatenate(sectors), slices=sizes,
                first=first, ncoll=ncoll)


def cached_batch(device, cache):
    """gen_batch, stored under `cache` on its first use and read back on the
    next ones (profiling passes of the same input); the first slice's
    cluster set is not stored (None when read back)."""
    import numpy as np
    import torch
    meta = os.path.join(cache, "batch.json")
    if os.path.exists(meta):
        m = json.load(open(meta))
        arr = np.load(os.path.join(cache, "batch_index.npz"))
        y = torch.from_numpy(np.load(os.path.join(cache, "batch_y.npy"))).to(device)
        z = torch.from_numpy(np.load(os.path.join(cache, "batch_z.npy"))).to(device)
        slices = [(int(o), int(n), arr[f"rb{i}"]) for i, (o, n) in enumerate(m["slices"])]
        log(f"input read from {cache}")
        return dict(rb=torch.as_tensor(arr["rb"], device=device), y=y, z=z, n=m["n"], n_units=m["n_units"],
                    sectors=arr["sectors"], slices=slices, first=None, ncoll=m["ncoll"])
    B = gen_batch(device)
    os.makedirs(cache, exist_ok=True)
    np.save(os.path.join(cache, "batch_y.npy"), B["y"].cpu().numpy())
    np.save(os.path.join(cache, "batch_z.npy"), B["z"].cpu().numpy())
    np.savez(os.path.join(cache, "batch_index.npz"), rb=B["rb"].cpu().numpy(), sectors=B["sectors"],
             **{f"rb{i}": sl[2] for i, sl in enumerate(B["slices"])})
    json.dump(dict(n=int(B["n"]), n_units=int(B["n_units"]), ncoll=[int(c) for c in B["ncoll"]],
                   slices=[(int(sl[0]), int(sl[1])) for sl in B["slices"]]), open(meta, "w"))
    log(f"input stored under {cache}")
    return B


def order_rows_by_z(rb, y, z):
    """The same clusters with each (unit, row) range sorted by z (stable)."""
    import torch
    counts = rb[1:] - rb[:-1]
    key = torch.repeat_interleave(torch.arange(len(counts), device=y.device), counts)
    o1 = torch.sort(z, stable=True).indices
    order = o1[torch.sort(key[o1], stable=True).indices]
    del o1, key
    return y[order].contiguous(), z[order].contiguous()


def make_tracker(n_units, n, bin_y=None):
    import paper_2601_20569_amd as px
    from synth import geometry as G
    tuning = px.default_tuning(n_units, n)
    if bin_y is not None:  # the grid's y-bin width is fixed when the context is made
        tuning.bin_y = float(bin_y)
    return px.SectorTracker(G.row_x(), G.tan_half_opening(), G.BZ_TESLA, tuning=tuning)


def size_run(tr, rb, y, z, n_units):
    """Required capacities from one tracking call (retries on overflow)."""
    n = int(y.numel())
    res = tr.track(rb, y, z, n_units, cap_start=max(1024, n // 16), cap_tracks=max(1024, n // 16),
                   cap_hits=max(4096, 3 * n))
    out = (res["n_start"], len(res["n_hits"]), len(res["hit_id"]))
    del res
    return out


def cpu_baseline(cs, n_units_sample, threads, where="the input"):
    """The oracle (float decisions) on the first units of the same input."""
    import oracle
    from synth import geometry as G
    lo, hi = 0, min(cs.n_units, n_units_sample)
    n = int(cs.row_begin[hi * G.N_ROWS] - cs.row_begin[lo * G.N_ROWS])
    t0 = time.perf_counter()
    res = oracle.track(cs, units=(lo, hi), n_threads=threads)
    dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="clusters/s", cores=threads, kind="oracle",
                sample=f"sectors {lo}-{hi - 1} of {where}: {n} clusters, {dt:.1f} s"), res


def timed(fn, steps, stream=None, per_step=None):
    """Mean ms per call of fn over `steps` calls, between events on `stream`.
    per_step (a list): receives each call's own ms (events between calls)."""
    import torch
    s = stream or torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    sync()
    ev[0].record(s)
    for i in range(steps):
        fn()
        ev[i + 1].record(s)
    sync()
    if per_step is not None:
        per_step.extend(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    return ev[0].elapsed_time(ev[steps]) / steps


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """GB/s of a plain device-to-device copy (read + write), same run."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ms = timed(lambda: dst.copy_(src), reps)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def next_steps(tr, bufs, n_units, n_clusters, n_tracks, n_hits, y, z, steps, stream, row_begin_t, unit_sector,
               unit_group, cross_electrode):
    """The steps after the sector tracking on its output: ambiguity solving
    (every tracklet of the batch), the rebuild of the kept tracklets of the
    first slice, and the three-iteration fit with interpolation rejection
    (every tracklet of the batch), each timed on its own, with its
    algorithmic bytes against the HBM peak."""
    import torch
    res = {}
    o = bufs["out"]
    row_begin_h = row_begin_t.cpu().numpy()
    sel = tr.allocate_select(n_units, n_clusters, bufs["cap_tracks"])
    with torch.cuda.stream(stream):
        tr.select_into(bufs, n_units, n_clusters, sel, stream=stream)
        sync()
        ms = timed(lambda: tr.select_into(bufs, n_units, n_clusters, sel, stream=stream), steps, stream)
    kept = int(sel["counts"][0])
    b = B_SEL_PER_TRACK * n_tracks + B_SEL_PER_HIT * n_hits + B_SEL_PER_CLUSTER * n_clusters
    res["select"] = dict(ms=round(ms, 3), tracklets=n_tracks, kept=kept, shared="10%", alg_bytes=int(b),
                         GBs=round(b / (ms * 1e-3) / 1e9, 2), frac=round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5))
    log(f"ambiguity solving: {ms:.3f} ms, {kept} of {n_tracks} tracklets kept")
    # merging of the kept tracklets of the whole batch (units of one slice)
    import paper_2601_20569_amd as px
    kidx = sel["keep"][:n_tracks].bool().nonzero().squeeze(1)
    hb0 = o["hit_begin"][:n_tracks][kidx]
    margs = (o["unit"][:n_tracks][kidx].contiguous(), o["param"][:n_tracks][kidx].contiguous(),
             o["x_ref"][:n_tracks][kidx].contiguous(), o["hit_row"][hb0].to(torch.int32).contiguous(),
             o["hit_row"][hb0 + o["n_hits"][:n_tracks][kidx].to(torch.int64) - 1].to(torch.int32).contiguous(),
             torch.as_tensor(px.unit_neighbours(unit_sector, unit_group), device=y.device), n_units)
    del hb0
    with torch.cuda.stream(stream):
        r = tr.merge(*margs, cross_electrode=cross_electrode, stream=stream)
        sync()
        del r
        ms = timed(lambda: tr.merge(*margs, cross_electrode=cross_electrode, stream=stream), steps, stream)
        r = tr.merge(*margs, cross_electrode=cross_electrode, stream=stream)
        sync()
    nk = len(kidx)
    b = B_MERGE_PER_TRACK * nk
    links = int((r["next"] >= 0).sum())
    res["merge"] = dict(ms=round(ms, 3), tracks=nk, links=links, cross_electrode=cross_electrode, alg_bytes=int(b),
                        GBs=round(b / (ms * 1e-3) / 1e9, 2), frac=round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5))
    log(f"merging: {ms:.3f} ms, {nk} tracks, {links} links")
    del r, margs, kidx
    # the rebuild (Phase II) of the kept tracklets of the first slice (36 units)
    u1 = min(n_units, 36)
    keep = sel["keep"][:n_tracks].bool() & (o["unit"][:n_tracks] < u1)
    idx = keep.nonzero().squeeze(1)
    del sel
    torch.cuda.empty_cache()
    cnt = o["n_hits"][:n_tracks][idx].to(torch.int64)
    hb = torch.zeros(len(idx) + 1, dtype=torch.int64, device=y.device)
    hb[1:] = torch.cumsum(cnt, 0)
    src = torch.repeat_interleave(o["hit_begin"][:n_tracks][idx], cnt) + (
        torch.arange(int(hb[-1]), device=y.device) - torch.repeat_interleave(hb[:-1], cnt))
    n1 = int(row_begin_h[u1 * 152])
    rargs = (row_begin_t[:u1 * 152 + 1].contiguous(), y[:n1], z[:n1], u1, o["unit"][:n_tracks][idx].contiguous(), hb,
             o["hit_id"][src].contiguous(), o["hit_row"][src].contiguous(), o["param"][:n_tracks][idx].contiguous(),
             o["x_ref"][:n_tracks][idx].contiguous(), o["chi2"][:n_tracks][idx].contiguous(),
             o["ndf"][:n_tracks][idx].contiguous())
    del src
    with torch.cuda.stream(stream):
        r = tr.rebuild(*rargs, stream=stream)
        sync()
        del r
        ms = timed(lambda: tr.rebuild(*rargs, stream=stream), steps, stream)
        r = tr.rebuild(*rargs, stream=stream)
        sync()
    nt1, nh1 = len(idx), int(hb[-1])
    b = B_RB_PER_TRACK * nt1 + B_RB_PER_HIT * nh1 + B_RB_PER_CLUSTER * n1
    res["rebuild"] = dict(ms=round(ms, 3), workload=f"kept tracklets of the first {u1} units", clusters=n1,
                          tracks=nt1, input_hits=nh1, ok=int(r["ok"].sum()), kept_hits=int(r["n_kept"].sum()),
                          alg_bytes=int(b), GBs=round(b / (ms * 1e-3) / 1e9, 2),
                          frac=round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5))
    log(f"rebuild: {ms:.3f} ms, {nt1} tracks of the first slice, {res['rebuild']['kept_hits']} clusters kept")
    del r
    # the same with Phase III's extrapolation beyond the tracks' ends
    with torch.cuda.stream(stream):
        r = tr.rebuild(*rargs, extrapolate=True, stream=stream)
        sync()
        del r
        ms = timed(lambda: tr.rebuild(*rargs, extrapolate=True, stream=stream), steps, stream)
        r = tr.rebuild(*rargs, extrapolate=True, stream=stream)
        sync()
    res["rebuild_phase3"] = dict(ms=round(ms, 3), ok=int(r["ok"].sum()), kept_hits=int(r["n_kept"].sum()),
                                 alg_bytes=int(b), GBs=round(b / (ms * 1e-3) / 1e9, 2),
                                 frac=round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5))
    log(f"rebuild with extrapolation: {ms:.3f} ms, {res['rebuild_phase3']['kept_hits']} clusters kept")
    del r, rargs
    torch.cuda.empty_cache()
    # every kept tracklet (their hits are contiguous in the output)
    hb = torch.empty(n_tracks + 1, dtype=torch.int64, device=y.device)
    hb[:n_tracks] = o["hit_begin"][:n_tracks]
    hb[n_tracks] = n_hits
    args = (hb, o["hit_id"][:n_hits], o["hit_row"][:n_hits], o["param"][:n_tracks].contiguous(),
            o["x_ref"][:n_tracks], y, z)
    with torch.cuda.stream(stream):
        r = tr.fit(*args, stream=stream)
        sync()
        del r
        ms = timed(lambda: tr.fit(*args, stream=stream), steps, stream)
        r = tr.fit(*args, stream=stream)
        sync()
    nt, nhf = n_tracks, n_hits
    b = B_FIT_PER_TRACK * nt + B_FIT_PER_HIT * nhf
    res["fit"] = dict(ms=round(ms, 3), tracks=nt, clusters=nhf, ok=int(r["ok"].sum()),
                      rejected=int(r["reject"].sum()), alg_bytes=int(b), GBs=round(b / (ms * 1e-3) / 1e9, 2),
                      frac=round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5))
    log(f"three-iteration fit: {ms:.3f} ms, {nt} tracks, {res['fit']['rejected']} clusters rejected")
    del r, args
    torch.cuda.empty_cache()
    return res


def adjoint_form(steps):
    """Refit forward + hand-written backward on the distorted central event."""
    import numpy as np
    import torch

    import paper_2601_20569_amd as px
    import synth
    from synth import geometry as G
    dev = torch.device("cuda", 0)
    cs = synth.central_event(seed=5, distortion=synth.RadialDistortion(), device="cuda")
    tr = make_tracker(cs.n_units, cs.n_clusters)
    y = torch.as_tensor(cs.y, device=dev)
    z = torch.as_tensor(cs.z, device=dev)
    res = tr.track(torch.as_tensor(cs.row_begin, device=dev), y, z, cs.n_units)
    keep = (res["n_hits"] >= 20).nonzero().squeeze(1)
    n_hits = res["n_hits"][keep].to(torch.int64)
    hb = torch.zeros(len(keep) + 1, dtype=torch.int64, device=dev)
    hb[1:] = torch.cumsum(n_hits, 0)
    src = torch.repeat_interleave(res["hit_begin"][keep], n_hits) + (
        torch.arange(int(hb[-1]), device=dev) - torch.repeat_interleave(hb[:-1], n_hits))
    job = px.RefitJob(tr, hb, res["hit_id"][src].contiguous(), res["hit_row"][src].contiguous(),
                      res["unit"][keep].contiguous(), res["param"][keep].contiguous(), y, z,
                      torch.as_tensor(G.sector_alpha(cs.unit_sector).astype(np.float32), device=dev))
    theta = torch.as_tensor(np.random.default_rng(1).normal(0.0, 0.05, px.MAP_NCOEF).astype(np.float32),
                            device=dev)
    job.forward(theta)
    w = job.ok[:job.n_tracks].float()
    job.backward(w)
    fwd = timed(lambda: job.forward(theta), steps)
    bwd = timed(lambda: job.backward(w), steps)
    return dict(workload="central-event+distortion", tracks=job.n_tracks, hits=job.n_hits,
                forward_ms=round(fwd, 4), backward_ms=round(bwd, 4),
                backward_over_forward=round(bwd / fwd, 3))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched", choices=["batched", "timeframe", "central", "single"])
    ap.add_argument("--cpu-units", type=int, default=0, help="sectors in the oracle sample (0: one per thread)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-forms", action="store_true", help="skip the plain and adjoint comparisons")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tuning")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the ambiguity solving and three-iteration fit legs")
    ap.add_argument("--tuning", default=None,
                    help="fixed tuning as JSON (the dict an autotuned run prints); skips the autotuner")
    ap.add_argument("--in-row-order", default="generated", choices=["generated", "z"],
                    help="order of the clusters inside each row of the batch: as generated "
                         "(random), or by z as a pad/time-ordered cluster finder delivers them")
    ap.add_argument("--input-cache", default=None,
                    help="directory holding the generated batch: written on the first run, read on later ones")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with one plain 1 GiB device-to-device copy kernel (reference for HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: units (sectors x time-frame slices) are independent, "
              "so more GPUs would each track their own share; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from synth import geometry as G

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    if args.workload == "batched":
        log("generating 16 time-frame slices on the GPU")
        B = cached_batch("cuda", args.input_cache) if args.input_cache else gen_batch("cuda")
        rb, y, z, N, U = B["rb"], B["y"], B["z"], B["n"], len(B["sectors"])
        first = B["first"]
        cfg = dict(workload="timeframe-slice-batch", slices=16, collisions=int(sum(B["ncoll"])),
                   seeds="4000-4015", form="batched graph: tracking + refit of tracklets >= 20 clusters")
        if args.in_row_order == "z":
            y, z = order_rows_by_z(rb, y, z)
            B["y"], B["z"] = y, z
            cfg["in_row_order"] = "z"
            log("clusters ordered by z inside each row")
    else:
        gen = {"timeframe": lambda: synth.timeframe_slice(seed=3000, device="cuda"),
               "central": lambda: synth.central_event(seed=2, device="cuda"),
               "single": lambda: synth.single_sector(seed=1, device="cuda")}[args.workload]
        first = gen()
        rb = torch.as_tensor(first.row_begin, device=dev)
        y = torch.as_tensor(first.y, device=dev)
        z = torch.as_tensor(first.z, device=dev)
        N, U = first.n_clusters, first.n_units
        cfg = dict(workload=first.meta["workload"], seed=first.meta["seed"],
                   form="batched graph: tracking + refit of tracklets >= 20 clusters")
        B = dict(sectors=first.unit_sector, slices=[(0, N, first.row_begin.copy())])
    log(f"input: {N} clusters in {U} sector units ({time.perf_counter() - t0:.1f} s)")

    fixed = json.loads(args.tuning) if args.tuning else None
    tr = make_tracker(U, N, fixed.get("bin_y") if fixed else None)
    n_start, n_tracks, n_hits = size_run(tr, rb, y, z, U)
    log(f"tracklets: {n_start} start hits, {n_tracks} kept, {n_hits} attached clusters")
    alpha = torch.as_tensor(G.sector_alpha(B["sectors"]).astype(np.float32), device=dev)
    theta = torch.as_tensor(np.random.default_rng(1).normal(0.0, 0.05, 36720).astype(np.float32),
                            device=dev)
    # time frames: the drift coordinate is not z, so the map is evaluated at a
    # fixed z (its r and phi dependence acts); single events: at the cluster's z
    map_z = 0.0 if cfg["workload"].startswith("timeframe") else None
    cfg["map_z"] = "0 cm (time frame)" if map_z is not None else "measured z"
    stream = torch.cuda.Stream()
    tuning = None
    if args.tuning:
        tuning = json.loads(args.tuning)
        tr.set_tuning(tuning)
        log(f"fixed tuning {tuning}")
    bufs = tr.allocate_batched(U, N, cap_start=n_start + 1, cap_tracks=n_tracks + 1, cap_hits=n_hits + 1,
                               autotune=not (args.no_autotune or args.tuning))
    if not (args.no_autotune or args.tuning):
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            tuning = tr.autotune_batched(rb, y, z, U, bufs, stream, unit_alpha=alpha, theta=theta, reps=3,
                                         map_z=map_z)
        log(f"autotuned in {time.perf_counter() - t0:.1f} s: {tuning}")
    log(f"workspace {bufs['ws_bytes'] / 2**30:.1f} GiB; capturing the graph")

    def step():
        tr.track_batched_into(rb, y, z, U, bufs, stream, unit_alpha=alpha, theta=theta, map_z=map_z)

    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup)):
            step()
        sync()
        counts = bufs["out"]["counts"].cpu().tolist()
        assert counts[3] == 0 and counts[0] == n_start and counts[1] == n_tracks, counts
        nh = bufs["out"]["n_hits"][:n_tracks]
        sel = nh >= 20
        n_refit, n_refit_hits = int(sel.sum()), int(nh[sel].to(torch.int64).sum())
        n_refit_ok = int(bufs["refit_ok"][:n_tracks].sum())
        log(f"warm-up done; {n_refit} tracklets refitted ({n_refit_hits} clusters, {n_refit_ok} ok)")
        replay_ms = []
        ms = timed(step, args.steps, stream, per_step=replay_ms)
        log(f"timed {args.steps} graph replays: {ms:.3f} ms/step (median {np.median(replay_ms):.3f}, "
            f"min {min(replay_ms):.3f}, max {max(replay_ms):.3f})")
        # per-stage kernel times: the same sequence launched directly with events
        tr.timing_enable(args.steps)
        for _ in range(args.steps):
            step()
        sync()
    stage_ms, ncalls = tr.timing_read()
    stage_ms = {k: v / max(ncalls, 1) for k, v in stage_ms.items()}
    log("stages (ms): " + ", ".join(f"{k} {v:.3f}" for k, v in stage_ms.items()))

    forms = {}
    if not args.no_extra_forms:
        # the same graph without the refit: tracking only, for the plain comparison
        def step_track():
            tr.track_batched_into(rb, y, z, U, bufs, stream)

        with torch.cuda.stream(stream):
            step_track()
            sync()
            track_ms = timed(step_track, args.steps, stream)
        forms["batched_ms"] = round(ms, 3)
        forms["batched_tracking_only_ms"] = round(track_ms, 3)
        log(f"batched graph without the refit: {track_ms:.3f} ms/step")
    if not args.no_next:
        groups = None
        if len(B["slices"]) > 1:
            per = [len(sl[2]) - 1 for sl in B["slices"]]  # rows of each slice
            groups = np.repeat(np.arange(len(per)), np.array(per) // G.N_ROWS)
        # a time frame's drift coordinate is not z: no merging across the electrode
        forms.update(next_steps(tr, bufs, U, N, n_tracks, n_hits, y, z, args.steps, stream, rb, B["sectors"],
                                groups, not cfg["workload"].startswith("timeframe")))
    del bufs
    torch.cuda.empty_cache()

    if not args.no_extra_forms:
        # plain form: one tpcx_track call per slice
        slices = B["slices"]
        if len(slices) > 1:
            caps = []
            views = []
            for off, n, rb_s in slices:
                rbt = torch.as_tensor(rb_s, device=dev)
                views.append((rbt, y[off:off + n], z[off:off + n]))
            mx = max(n for _, n, _ in slices)
            pbufs = tr.allocate(36, mx, cap_start=n_start + 1, cap_tracks=n_tracks + 1,
                                cap_hits=n_hits + 1)

            def plain_all():
                for rbt, ys, zs in views:
                    tr.track_into(rbt, ys, zs, 36, pbufs)

            plain_all()
            plain_ms = timed(plain_all, args.steps)
            forms["plain_per_slice_ms"] = round(plain_ms, 3)
            forms["batched_speedup_vs_plain"] = round(plain_ms / track_ms, 3)
            log(f"plain, one call per slice: {plain_ms:.3f} ms per batch (tracking only)")
            del pbufs, views
            torch.cuda.empty_cache()
        # plain form per sector: one tpcx_track call per unit
        rb_h = rb.cpu().numpy()
        R = G.N_ROWS
        uviews = []
        for u in range(U):
            lo, hi = int(rb_h[u * R]), int(rb_h[(u + 1) * R])
            uviews.append((torch.as_tensor(rb_h[u * R:(u + 1) * R + 1] - lo, device=dev), y[lo:hi], z[lo:hi]))
        mxu = max(int(v[1].numel()) for v in uviews)
        ubufs = tr.allocate(1, mxu, cap_start=mxu, cap_tracks=mxu, cap_hits=8 * mxu)

        def plain_units():
            for rbt, ys, zs in uviews:
                tr.track_into(rbt, ys, zs, 1, ubufs)

        plain_units()
        unit_ms = timed(plain_units, 1)
        assert int(ubufs["out"]["counts"][3]) == 0, "per-sector capacity overflow"
        forms["plain_per_sector_ms"] = round(unit_ms, 3)
        forms["batched_speedup_vs_plain_per_sector"] = round(unit_ms / track_ms, 3)
        log(f"plain, one call per sector ({U} calls): {unit_ms:.3f} ms per batch (tracking only)")
        del ubufs, uviews
        torch.cuda.empty_cache()
        adj = adjoint_form(args.steps)
        forms["adjoint"] = adj
        log(f"adjoint refit: forward {adj['forward_ms']} ms, backward {adj['backward_ms']} ms "
            f"({adj['tracks']} tracks)")

    copy_gbs = copy_bandwidth()
    log(f"device copy: {copy_gbs:.1f} GB/s (read + write)")

    # ----- CPU baseline (oracle) on a bounded sample of the same input
    cpu = None
    per_start_con = None
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        nu = args.cpu_units or threads
        log(f"oracle on {nu} sectors with {threads} threads")
        if first is None:  # input read from the cache: the first slice again, from its seed
            import synth
            first = synth.timeframe_slice(seed=4000, n_collisions=int(B["ncoll"][0]), device="cuda", truth=True)
        where = "the first slice" if args.workload == "batched" else "the input"
        cpu, ores = cpu_baseline(first, nu, threads, where)
        one, _ = cpu_baseline(first, 1, 1, where)
        cpu["one_core"] = dict(value=one["value"], sample=one["sample"])
        cpu["cpu_model"] = cpu_model()
        cpu["host_cpus"] = os.cpu_count()
        c = ores["counters"]
        s = max(len(ores["starts"]), 1)
        per_start_con = (B_CON_PER_TRACKLET * s + B_CON_PER_CHAIN_HIT * c["chain"] +
                         B_CON_PER_SEARCH * c["searches"] + B_CON_PER_CANDIDATE * c["box_candidates"] +
                         B_CON_PER_ATTACHED * c["attached"]) / s
        log(f"oracle: {cpu['value']:.3e} clusters/s ({cpu['sample']}); "
            f"constructor bytes per start hit {per_start_con:.1f}")

    # ----- algorithmic bytes per stage and the roofline of the dominant one
    stage_bytes = {
        "grid": B_GRID_PER_CLUSTER * N,
        "neighbours": B_NF_PER_CLUSTER * N,
        "starts": B_STARTS_PER_CLUSTER * N + B_STARTS_PER_START * n_start,
        "construct": (per_start_con * n_start) if per_start_con else None,
        "compact": B_OUT_PER_TRACK * n_tracks + B_OUT_PER_HIT * n_hits,
        "refit": B_REFIT_PER_TRACK * n_refit + B_REFIT_PER_HIT * n_refit_hits,
    }
    dom = max(stage_ms, key=stage_ms.get)
    b = stage_bytes.get(dom)
    roof = None
    if b is not None:
        gbs = b / (stage_ms[dom] * 1e-3) / 1e9
        tr_b = recorded_traffic(dom, cfg["workload"])
        roof = dict(bound="hbm", achieved=round(gbs, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(gbs / HBM_PEAK_GBS, 5), traffic=tr_b,
                    copy_GBs=round(copy_gbs, 1), frac_of_copy=round(gbs / copy_gbs, 5), kernel=dom,
                    kernels=STAGE_KERNELS.get(dom), kernel_ms=round(stage_ms[dom], 4), alg_bytes=int(b),
                    valu=recorded_valu(dom, cfg["workload"]))

    known = [k for k in stage_ms if stage_bytes.get(k) is not None]
    # every stage against HBM: algorithmic bytes over its measured time, and
    # the counted traffic of its kernels where a current summary holds it
    stages_roof = {k: dict(alg_bytes=int(stage_bytes[k]),
                           GBs=round(stage_bytes[k] / (stage_ms[k] * 1e-3) / 1e9, 2),
                           frac=round(stage_bytes[k] / (stage_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                           traffic=recorded_traffic(k, cfg["workload"]),
                           valu=recorded_valu(k, cfg["workload"]))
                   for k in known if stage_ms[k] > 0}
    path = None
    if len(known) == len(stage_ms):
        tot_b = sum(stage_bytes[k] for k in known)
        path = dict(alg_bytes=int(tot_b), GBs=round(tot_b / (ms * 1e-3) / 1e9, 2),
                    frac=round(tot_b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                    frac_of_copy=round(tot_b / (ms * 1e-3) / 1e9 / copy_gbs, 5))

    line = dict(metric=METRIC, value=N / (ms * 1e-3), unit="clusters/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=round(ms, 4),
                replay_ms=dict(median=round(float(np.median(replay_ms)), 4),
                               min=round(min(replay_ms), 4), max=round(max(replay_ms), 4)),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
                data="synthetic",
                config=dict(cfg, clusters=N, units=U, start_hits=n_start, tracklets=n_tracks,
                            attached=n_hits, refitted=n_refit, refitted_clusters=n_refit_hits,
                            tuning=tuning or "default"),
                roofline=roof, cpu_baseline=cpu,
                stages_ms={k: round(v, 4) for k, v in stage_ms.items()}, stages_roofline=stages_roof,
                path_roofline=path,
                forms=forms)
    print(json.dumps(line), flush=True)
    if args.copy_calibration:
        n = 1 << 28
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        sync()
        dst.copy_(src)
        sync()
        log(f"copy calibration: {4 * n} bytes read, {4 * n} bytes written")


if __name__ == "__main__":
    main()
