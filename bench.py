#!/usr/bin/env python3
"""Throughput of per-sector TPC track finding on one MI355X.

One step is one pass of the whole tracking path (search-grid build, neighbour
finder, cleaning and start hits, tracklet constructor, output compaction) over
one synthetic input already resident in HBM.  Prints one JSON line with the
clusters/s, the roofline position of the dominant stage (timed with HIP events
recorded by the library on its stream) and the CPU oracle timed on a bounded
sample of the same input.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload timeframe|central|single]
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

# algorithmic bytes (compulsory traffic of the method's own passes)
B_GRID_PER_CLUSTER = 24        # read y, z (+ row range); write sorted y, z, id
B_NF_PER_CLUSTER = 20          # read own y, z, id; write two links (neighbour rows via cache)
B_STARTS_PER_CLUSTER = 17      # read two links, write two cleaned links and a flag
B_STARTS_PER_START = 4         # write the start id
B_CON_PER_START = 88           # read start id, write the tracklet record (x, 5 p, 9 cov, chi2, counts)
B_CON_PER_CHAIN_HIT = 12       # link, y, z of every chain cluster
B_CON_PER_CANDIDATE = 12       # y, z, id of every cluster inside the chi2 box of a searched row
B_CON_PER_ATTACHED = 5         # write id and row of every attached cluster
B_OUT_PER_START = 4            # read n
B_OUT_PER_TRACK = 88 + 104     # read the record, write the output record
B_OUT_PER_HIT = 10             # read and write id + row


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_input(workload, device):
    import synth
    if workload == "timeframe":
        return synth.timeframe_slice(seed=3000, device=device), dict(
            workload="timeframe-slice", collisions=128, seed=3000)
    if workload == "central":
        return synth.central_event(seed=2, device=device), dict(workload="central-event", seed=2)
    return synth.single_sector(seed=1, device=device), dict(workload="single-sector", seed=1)


def cpu_baseline(cs, n_units_sample, threads):
    """The oracle (float decisions) on the first units of the same input."""
    import oracle
    lo, hi = 0, min(cs.n_units, n_units_sample)
    from synth import geometry as G
    n = int(cs.row_begin[hi * G.N_ROWS] - cs.row_begin[lo * G.N_ROWS])
    t0 = time.perf_counter()
    res = oracle.track(cs, units=(lo, hi), n_threads=threads)
    dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="clusters/s", cores=threads, kind="oracle",
                sample=f"sectors {lo}-{hi - 1} of the same input: {n} clusters, {dt:.1f} s"), res, n


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="timeframe", choices=["timeframe", "central", "single"])
    ap.add_argument("--cpu-units", type=int, default=0, help="sectors in the oracle sample (0: one per thread)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: units (sectors x time-frame slices) are independent, "
              "so more GPUs would each track their own share; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2601_20569_amd as px
    from synth import geometry as G

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"generating {args.workload} input on {dev}")
    t0 = time.perf_counter()
    cs, cfg = make_input(args.workload, "cuda")
    N = cs.n_clusters
    log(f"input: {N} clusters in {cs.n_units} sectors ({time.perf_counter() - t0:.1f} s)")
    rb = torch.as_tensor(cs.row_begin, device=dev)
    y = torch.as_tensor(cs.y, device=dev)
    z = torch.as_tensor(cs.z, device=dev)

    tuning = px.default_tuning(cs.n_units, N)
    tr = px.SectorTracker(G.row_x(), G.tan_half_opening(), G.BZ_TESLA, tuning=tuning)
    # size the outputs from one call, then reuse the buffers for every step
    first = tr.track(rb, y, z, cs.n_units)
    n_start, n_tracks, n_hits = first["n_start"], len(first["n_hits"]), len(first["hit_id"])
    del first
    bufs = tr.allocate(cs.n_units, N, cap_start=max(n_start, 1), cap_tracks=max(n_tracks, 1),
                       cap_hits=max(n_hits, 1))
    log(f"tracklets: {n_start} start hits, {n_tracks} kept, {n_hits} attached clusters; "
        f"workspace {bufs['ws_bytes'] / 2**30:.2f} GiB")
    for _ in range(args.warmup):
        tr.track_into(rb, y, z, cs.n_units, bufs)
    torch.cuda.synchronize()
    log(f"warm-up done ({args.warmup} steps)")

    tr.timing_enable(args.steps)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        tr.track_into(rb, y, z, cs.n_units, bufs)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    stage_ms, ncalls = tr.timing_read()
    stage_ms = {k: v / max(ncalls, 1) for k, v in stage_ms.items()}
    counts = bufs["out"]["counts"].cpu().tolist()
    assert counts[3] == 0 and counts[0] == n_start, counts
    log(f"timed {args.steps} steps: {ms:.3f} ms/step; stages (ms) " +
        ", ".join(f"{k} {v:.3f}" for k, v in stage_ms.items()))

    # ----- CPU baseline (oracle) on a bounded sample of the same input
    cpu = None
    per_start_con = None
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        nu = args.cpu_units or threads
        log(f"oracle on {nu} sectors with {threads} threads")
        cpu, ores, n_sample = cpu_baseline(cs, nu, threads)
        c = ores["counters"]
        s = max(len(ores["starts"]), 1)
        per_start_con = (B_CON_PER_START * s + B_CON_PER_CHAIN_HIT * c["chain"] +
                         B_CON_PER_CANDIDATE * c["box_candidates"] +
                         B_CON_PER_ATTACHED * c["attached"]) / s
        log(f"oracle: {cpu['value']:.3e} clusters/s ({cpu['sample']}); "
            f"constructor bytes per start hit {per_start_con:.1f}")

    # ----- algorithmic bytes per stage and the roofline of the dominant one
    stage_bytes = {
        "grid": B_GRID_PER_CLUSTER * N,
        "neighbours": B_NF_PER_CLUSTER * N,
        "starts": B_STARTS_PER_CLUSTER * N + B_STARTS_PER_START * n_start,
        "construct": (per_start_con * n_start) if per_start_con else None,
        "compact": B_OUT_PER_START * n_start + B_OUT_PER_TRACK * n_tracks + B_OUT_PER_HIT * n_hits,
    }
    dom = max(stage_ms, key=stage_ms.get)
    b = stage_bytes[dom]
    roof = None
    if b is not None:
        gbs = b / (stage_ms[dom] * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=round(gbs, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(gbs / HBM_PEAK_GBS, 5), traffic=None, kernel=dom,
                    kernel_ms=round(stage_ms[dom], 4), alg_bytes=int(b))

    line = dict(metric=METRIC, value=N / (ms * 1e-3), unit="clusters/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=round(ms, 4),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
                data="synthetic",
                config=dict(cfg, form="plain", clusters=N, units=cs.n_units, start_hits=n_start,
                            tracklets=n_tracks, attached=n_hits),
                roofline=roof, cpu_baseline=cpu,
                stages_ms={k: round(v, 4) for k, v in stage_ms.items()})
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
