"""Batched form (many slices + refits in one captured HIP graph) against the
plain per-slice form and the standalone refit: bit-identical per unit.

Graph replays are checked one by one, with eager device work between them.
"""
import numpy as np
import pytest

import synth
from synth import geometry as G

from gpu_helpers import make_tracker, run_gpu

pytestmark = pytest.mark.gpu


def pack(sets):
    """Concatenate cluster sets unit-major (what the batched call takes)."""
    rbs, ys, zs, sectors = [], [], [], []
    off = 0
    for cs in sets:
        rbs.append(cs.row_begin[:-1] + off)
        ys.append(cs.y)
        zs.append(cs.z)
        sectors.append(cs.unit_sector)
        off += cs.n_clusters
    rb = np.concatenate(rbs + [np.array([off], np.int64)])
    return rb, np.concatenate(ys), np.concatenate(zs), np.concatenate(sectors)


def _sets():
    return [synth.timeframe_slice(seed=4000 + i, n_collisions=3 + 2 * i, mean_primaries=400.0)
            for i in range(3)] + [synth.central_event(seed=9, n_primaries=800)]


def _run_batched(tr, rb, y, z, n_units, alpha, theta, replays=1):
    import torch
    dev = torch.device("cuda")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    rb_t, y_t, z_t = T(rb, torch.int64), T(y, torch.float32), T(z, torch.float32)
    alpha_t = T(alpha, torch.float32)
    theta_t = T(theta, torch.float32) if theta is not None else None
    probe = tr.track(rb_t, y_t, z_t, n_units)
    bufs = tr.allocate_batched(n_units, len(y), max(probe["n_start"], 1), max(len(probe["n_hits"]), 1),
                               max(len(probe["hit_id"]), 1))
    s = torch.cuda.Stream()
    outs = []
    for rep in range(replays):
        with torch.cuda.stream(s):
            tr.track_batched_into(rb_t, y_t, z_t, n_units, bufs, s, unit_alpha=alpha_t, theta=theta_t)
        s.synchronize()
        # eager work between replays
        junk = torch.randn(1 << 20, device=dev).sum()
        torch.cuda.synchronize()
        del junk
        o = bufs["out"]
        counts = o["counts"].cpu().numpy()
        nt, nh = int(counts[1]), int(counts[2])
        outs.append(dict(counts=counts, unit=o["unit"][:nt].cpu().numpy(), start=o["start"][:nt].cpu().numpy(),
                         n_hits=o["n_hits"][:nt].cpu().numpy(), hit_id=o["hit_id"][:nh].cpu().numpy(),
                         hit_row=o["hit_row"][:nh].cpu().numpy(), param=o["param"][:nt].cpu().numpy(),
                         cov=o["cov"][:nt].cpu().numpy(), chi2=o["chi2"][:nt].cpu().numpy(),
                         refit_chi2=bufs["refit_chi2"][:nt].cpu().numpy(),
                         refit_ok=bufs["refit_ok"][:nt].cpu().numpy()))
    return outs


def test_batched_equals_plain_per_slice_and_replays_agree():
    sets = _sets()
    rb, y, z, sectors = pack(sets)
    n_units = len(sectors)
    alpha = G.sector_alpha(sectors)
    print(f"case: {len(sets)} sets, {n_units} units, {len(y)} clusters", flush=True)
    tr = make_tracker()
    theta = np.random.default_rng(1).normal(0.0, 0.05, 36720)
    outs = _run_batched(tr, rb, y, z, n_units, alpha, theta, replays=3)
    a = outs[0]
    assert a["counts"][3] == 0
    for b in outs[1:]:
        for k in a:
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"replay differs in {k}")
    # plain, one slice at a time
    unit_off, clus_off = 0, 0
    pos = 0
    hpos = 0
    for cs in sets:
        p = run_gpu(cs, tr, debug=False)
        n = len(p["n_hits"])
        sl = slice(pos, pos + n)
        np.testing.assert_array_equal(a["unit"][sl], p["unit"] + unit_off)
        np.testing.assert_array_equal(a["start"][sl], p["start"] + clus_off)
        np.testing.assert_array_equal(a["n_hits"][sl], p["n_hits"])
        nh = len(p["hit_id"])
        np.testing.assert_array_equal(a["hit_id"][hpos:hpos + nh], p["hit_id"] + clus_off)
        np.testing.assert_array_equal(a["hit_row"][hpos:hpos + nh], p["hit_row"])
        for k in ("param", "cov", "chi2"):
            np.testing.assert_array_equal(a[k][sl], p[k])
        pos += n
        hpos += nh
        unit_off += cs.n_units
        clus_off += cs.n_clusters
    assert pos == len(a["unit"])


def test_batched_refit_equals_standalone_refit():
    import torch

    import paper_2601_20569_amd as px
    sets = _sets()[:2]
    rb, y, z, sectors = pack(sets)
    n_units = len(sectors)
    alpha = G.sector_alpha(sectors).astype(np.float32)
    tr = make_tracker()
    theta = np.random.default_rng(2).normal(0.0, 0.05, 36720).astype(np.float32)
    a = _run_batched(tr, rb, y, z, n_units, alpha, theta)[0]
    keep = a["n_hits"] >= 20
    assert keep.sum() > 100
    assert (a["refit_ok"][~keep] == 0).all() and (a["refit_chi2"][~keep] == 0).all()
    sel = np.nonzero(keep)[0]
    hb = np.zeros(len(a["n_hits"]) + 1, np.int64)
    hb[1:] = np.cumsum(a["n_hits"])
    hits = np.concatenate([a["hit_id"][hb[i]:hb[i + 1]] for i in sel])
    rows = np.concatenate([a["hit_row"][hb[i]:hb[i + 1]] for i in sel])
    nb = np.zeros(len(sel) + 1, np.int64)
    nb[1:] = np.cumsum(a["n_hits"][sel])
    dev = torch.device("cuda")
    T = lambda v, dt: torch.as_tensor(np.ascontiguousarray(v), dtype=dt, device=dev)
    job = px.RefitJob(tr, T(nb, torch.int64), T(hits, torch.int32), T(rows, torch.uint8),
                      T(a["unit"][sel], torch.int32), T(a["param"][sel], torch.float32),
                      T(y, torch.float32), T(z, torch.float32), T(alpha, torch.float32))
    chi2 = job.forward(T(theta, torch.float32)).cpu().numpy()
    ok = job.ok[:job.n_tracks].cpu().numpy()
    np.testing.assert_array_equal(chi2, a["refit_chi2"][sel])
    np.testing.assert_array_equal(ok, a["refit_ok"][sel])


def test_autotuned_batched_equals_default_tuning():
    """The autotuner may pick any tuning; the results must not change."""
    import torch
    sets = _sets()[:3]
    rb, y, z, sectors = pack(sets)
    n_units = len(sectors)
    alpha = G.sector_alpha(sectors).astype(np.float32)
    theta = np.random.default_rng(4).normal(0.0, 0.05, 36720)
    tr = make_tracker()
    want = _run_batched(tr, rb, y, z, n_units, alpha, theta)[0]
    print(f"case: autotune on {n_units} units, {len(y)} clusters", flush=True)
    dev = torch.device("cuda")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    rb_t, y_t, z_t = T(rb, torch.int64), T(y, torch.float32), T(z, torch.float32)
    tr2 = make_tracker()
    c = want["counts"]
    bufs = tr2.allocate_batched(n_units, len(y), int(c[0]) + 1, int(c[1]) + 1, int(c[2]) + 1, autotune=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        best = tr2.autotune_batched(rb_t, y_t, z_t, n_units, bufs, s, unit_alpha=T(alpha, torch.float32),
                                    theta=T(theta, torch.float32), reps=1)
    s.synchronize()
    print("tuning:", best)
    assert 1 <= best["construct_refill"] <= 64 and 1 <= best["refit_refill"] <= 64
    got = _run_batched(tr2, rb, y, z, n_units, alpha, theta)[0]
    for k in want:
        np.testing.assert_array_equal(want[k], got[k], err_msg=f"autotuned run differs in {k}")


def test_batched_overflow_skips_refit_and_empty_input_runs():
    import torch

    import paper_2601_20569_amd as px
    dev = torch.device("cuda")
    sets = _sets()[:1]
    rb, y, z, sectors = pack(sets)
    n_units = len(sectors)
    alpha = torch.as_tensor(G.sector_alpha(sectors).astype(np.float32), device=dev)
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    print("case: batched with too few hit slots", flush=True)
    tr = make_tracker()
    bufs = tr.allocate_batched(n_units, len(y), cap_start=len(y), cap_tracks=len(y), cap_hits=100)
    bufs["refit_chi2"].fill_(-1.0)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tr.track_batched_into(T(rb, torch.int64), T(y, torch.float32), T(z, torch.float32), n_units, bufs, s,
                              unit_alpha=alpha)
    s.synchronize()
    counts = bufs["out"]["counts"].cpu().numpy()
    assert counts[3] & px.ST_HIT_OVERFLOW and counts[2] > 100
    assert (bufs["refit_chi2"].cpu().numpy() == -1.0).all()  # no tracklet refitted
    print("case: batched on units without clusters", flush=True)
    rb0 = torch.zeros(n_units * G.N_ROWS + 1, dtype=torch.int64, device=dev)
    e = torch.zeros(0, dtype=torch.float32, device=dev)
    tr2 = make_tracker()
    b2 = tr2.allocate_batched(n_units, 0, 1, 1, 1)
    with torch.cuda.stream(s):
        tr2.track_batched_into(rb0, e, e, n_units, b2, s, unit_alpha=alpha)
    s.synchronize()
    assert (b2["out"]["counts"].cpu().numpy() == 0).all()
