"""A full-size time-frame slice (128 collisions, ~57M clusters) through the
batched form, in the launch configuration the benchmark times (one captured
graph: tracking plus refit of tracklets with >= 20 clusters), checked against
the oracle on sampled sector units: the oracle tracks one unit of this input
in about a second.

Per sampled unit: the kept tracklets (start hit, clusters, rows) bit for bit
against the float oracle, their parameters, covariances and chi2 bit for bit
too, and the refit chi2 within 1e-3 (relative) of the FP64 oracle refit for
tracklets that fit (chi2/ndf <= 10), within 5e-3 for the rest.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import geometry as G

from gpu_helpers import make_tracker

pytestmark = pytest.mark.gpu


def test_full_timeframe_slice_batched_on_sampled_units():
    import torch
    cs = synth.timeframe_slice(seed=3000, device="cuda", truth=False)
    print(f"case: time-frame slice seed 3000, {cs.n_clusters} clusters, batched graph", flush=True)
    dev = torch.device("cuda")
    rb = torch.as_tensor(cs.row_begin, device=dev)
    y = torch.as_tensor(cs.y, device=dev)
    z = torch.as_tensor(cs.z, device=dev)
    U = cs.n_units
    tr = make_tracker()
    probe = tr.track(rb, y, z, U)
    ns, nt, nh = probe["n_start"], len(probe["n_hits"]), len(probe["hit_id"])
    del probe
    bufs = tr.allocate_batched(U, cs.n_clusters, ns + 1, nt + 1, nh + 1)
    alpha = torch.as_tensor(G.sector_alpha(cs.unit_sector).astype(np.float32), device=dev)
    theta = np.random.default_rng(11).normal(0.0, 0.05, oracle.map_ncoef())
    theta_t = torch.as_tensor(theta, dtype=torch.float32, device=dev)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tr.track_batched_into(rb, y, z, U, bufs, s, unit_alpha=alpha, theta=theta_t)
    s.synchronize()
    o = bufs["out"]
    counts = o["counts"].cpu().numpy()
    assert counts[3] == 0 and counts[1] == nt and counts[2] == nh
    g = {k: o[k][:nt].cpu().numpy() for k in ("unit", "start", "n_hits", "hit_begin", "param", "cov", "chi2")}
    g["hit_id"] = o["hit_id"][:nh].cpu().numpy()
    g["hit_row"] = o["hit_row"][:nh].cpu().numpy()
    rchi2 = bufs["refit_chi2"][:nt].cpu().numpy()
    rok = bufs["refit_ok"][:nt].cpu().numpy().astype(bool)
    del bufs
    torch.cuda.empty_cache()

    for u in sorted(np.random.default_rng(0).choice(U, 3, replace=False)):
        print(f"unit {u}", flush=True)
        ref = oracle.track(cs, units=(int(u), int(u) + 1), n_threads=16)
        k = oracle.kept_tracklets(ref)
        gi = np.nonzero(g["unit"] == u)[0]
        assert len(gi) == len(k["n"]) and len(gi) > 1000
        np.testing.assert_array_equal(g["start"][gi], k["start"].astype(np.int32))
        np.testing.assert_array_equal(g["n_hits"][gi], k["n"])
        hits = np.concatenate([g["hit_id"][g["hit_begin"][i]:g["hit_begin"][i] + g["n_hits"][i]] for i in gi])
        rows = np.concatenate([g["hit_row"][g["hit_begin"][i]:g["hit_begin"][i] + g["n_hits"][i]] for i in gi])
        np.testing.assert_array_equal(hits, k["hits"])
        np.testing.assert_array_equal(rows, k["rows"])
        np.testing.assert_array_equal(g["param"][gi].astype(np.float64), k["param"])
        np.testing.assert_array_equal(g["cov"][gi].astype(np.float64), k["cov"])
        np.testing.assert_array_equal(g["chi2"][gi].astype(np.float64), k["chi2"])
        # refit of the tracklets with >= 20 clusters against the FP64 oracle
        tk = oracle.select_tracks(k, 20)
        want, ok_ref = oracle.refit(cs, tk, theta)
        sel = gi[g["n_hits"][gi] >= 20]
        assert len(sel) == len(want)
        ok = rok[sel]
        assert (ok == ok_ref).mean() > 0.999
        both = ok & ok_ref
        rel = np.abs(rchi2[sel][both] - want[both]) / np.maximum(want[both], 1.0)
        # tracklets that fit (chi2/ndf <= 10) within 1e-3; those with wrong
        # clusters (chi2/ndf in the hundreds, |sin phi| near the guard) lose
        # ~1e-3 to FP32 rounding whatever the divide and square root
        fits = want[both] <= 10.0 * (2 * g["n_hits"][sel][both] - 5)
        print(f"refit: {fits.sum()} fitting tracks, max rel {rel[fits].max():.2e}; "
              f"{(~fits).sum()} others, max rel {rel[~fits].max() if (~fits).any() else 0:.2e}", flush=True)
        assert fits.mean() > 0.9
        assert rel[fits].max() < 1e-3, rel[fits].max()
        assert rel.max() < 5e-3, rel.max()
        assert (rchi2[sel][~ok] == 0).all()


def test_full_batch_of_16_slices_on_sampled_units():
    """The benchmark's workload: 16 time-frame slices (32-160 collisions each,
    ~843M clusters, 576 units) through the batched graph; 4 sampled units of
    different slices against the oracle, as above."""
    from types import SimpleNamespace

    import torch
    dev = torch.device("cuda")
    ncoll = synth.slice_batch_collisions(seed=4000, n_slices=16)
    ys, zs, rbs, sectors = [], [], [], []
    off = 0
    for i, nc in enumerate(ncoll):
        cs = synth.timeframe_slice(seed=4000 + i, n_collisions=nc, device="cuda", truth=False)
        ys.append(torch.as_tensor(cs.y, device=dev))
        zs.append(torch.as_tensor(cs.z, device=dev))
        rbs.append(cs.row_begin[:-1] + off)
        sectors.append(cs.unit_sector)
        off += cs.n_clusters
        del cs
    rb_h = np.concatenate(rbs + [np.array([off], np.int64)])
    sectors = np.concatenate(sectors)
    y, z = torch.cat(ys), torch.cat(zs)
    del ys, zs
    U = len(sectors)
    print(f"case: 16-slice batch, {off} clusters, {U} units, batched graph", flush=True)
    rb = torch.as_tensor(rb_h, device=dev)
    tr = make_tracker()
    probe = tr.track(rb, y, z, U)
    ns, nt, nh = probe["n_start"], len(probe["n_hits"]), len(probe["hit_id"])
    del probe
    torch.cuda.empty_cache()
    bufs = tr.allocate_batched(U, off, ns + 1, nt + 1, nh + 1)
    alpha_h = G.sector_alpha(sectors).astype(np.float32)
    theta = np.random.default_rng(12).normal(0.0, 0.05, oracle.map_ncoef())
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tr.track_batched_into(rb, y, z, U, bufs, s, unit_alpha=torch.as_tensor(alpha_h, device=dev),
                              theta=torch.as_tensor(theta, dtype=torch.float32, device=dev))
    s.synchronize()
    o = bufs["out"]
    counts = o["counts"].cpu().numpy()
    assert counts[3] == 0 and counts[1] == nt and counts[2] == nh
    unit = o["unit"][:nt].cpu().numpy()
    for u in sorted(np.random.default_rng(1).choice(U, 4, replace=False)):
        lo, hi = int(rb_h[u * G.N_ROWS]), int(rb_h[(u + 1) * G.N_ROWS])
        print(f"unit {u}: clusters {lo}..{hi}", flush=True)
        cu = SimpleNamespace(n_units=1, row_begin=rb_h[u * G.N_ROWS:(u + 1) * G.N_ROWS + 1] - lo,
                             y=y[lo:hi].cpu().numpy(), z=z[lo:hi].cpu().numpy())
        ref = oracle.track(cu, n_threads=16)
        k = oracle.kept_tracklets(ref)
        gi = np.nonzero(unit == u)[0]
        assert len(gi) == len(k["n"]) and len(gi) > 100
        sel = torch.as_tensor(gi, device=dev)
        n_hits = o["n_hits"][sel].cpu().numpy()
        np.testing.assert_array_equal(o["start"][sel].cpu().numpy() - lo, k["start"].astype(np.int32))
        np.testing.assert_array_equal(n_hits, k["n"])
        hb = o["hit_begin"][sel].cpu().numpy()
        h0, h1 = int(hb[0]), int(hb[-1] + n_hits[-1])  # a unit's tracklets are contiguous
        np.testing.assert_array_equal(o["hit_id"][h0:h1].cpu().numpy() - lo, k["hits"])
        np.testing.assert_array_equal(o["hit_row"][h0:h1].cpu().numpy(), k["rows"])
        np.testing.assert_array_equal(o["param"][sel].cpu().numpy().astype(np.float64), k["param"])
        np.testing.assert_array_equal(o["cov"][sel].cpu().numpy().astype(np.float64), k["cov"])
        np.testing.assert_array_equal(o["chi2"][sel].cpu().numpy().astype(np.float64), k["chi2"])
        tk = oracle.select_tracks(k, 20)
        tk["unit"] = np.zeros_like(tk["unit"])
        want, ok_ref = oracle.refit(cu, tk, theta, unit_alpha=alpha_h[u:u + 1])
        gsel = gi[n_hits >= 20]
        rchi2 = bufs["refit_chi2"][torch.as_tensor(gsel, device=dev)].cpu().numpy()
        rok = bufs["refit_ok"][torch.as_tensor(gsel, device=dev)].cpu().numpy().astype(bool)
        assert len(gsel) == len(want)
        assert (rok == ok_ref).mean() > 0.999
        both = rok & ok_ref
        rel = np.abs(rchi2[both] - want[both]) / np.maximum(want[both], 1.0)
        fits = want[both] <= 10.0 * (2 * tk["n"][both] - 5)
        print(f"refit: {fits.sum()} fitting tracks, max rel {rel[fits].max():.2e}; max rel {rel.max():.2e}",
              flush=True)
        assert rel[fits].max() < 1e-3 and rel.max() < 5e-3
        assert (rchi2[~rok] == 0).all()
