"""A full-size time-frame slice (128 collisions, ~57M clusters) through the
batched form, in the launch configuration the benchmark times (one captured
graph: tracking plus refit of tracklets with >= 20 clusters, the map evaluated
at z = 0 as for every time frame), checked against the oracle on sampled
sector units: the oracle tracks one unit of this input in about a second.

Per sampled unit: the kept tracklets (start hit, clusters, rows) bit for bit
against the float oracle, their parameters, covariances and chi2 bit for bit
too; the same numbers within tolerance of the FP64 replay; the refit ok flags
equal to the FP64 oracle refit's and every refit chi2 within 1e-3 (relative)
of it.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import geometry as G

from gpu_helpers import make_tracker
from tolerances import NEAR_GUARD, chi2_bad, cov_bad, param_bad, refit_chi2_bad

pytestmark = pytest.mark.gpu


def check_against_fp64_replay(cs, k, param, cov, chi2):
    """Parameters, covariances and chi2 of kept tracklets within the
    tolerances of the FP64 replay of their decisions."""
    rp = oracle.replay(cs, k)
    assert rp["ok"].all()
    near = rp["smax"] >= NEAR_GUARD
    plain = param_bad(param.astype(np.float64), rp["param"]).any(1)
    print(f"FP64 replay: {len(near)} tracklets, {near.sum()} near the sin(phi) guard, "
          f"{plain.sum()} beyond the plain bound (all near the guard: {bool((plain <= near).all())})",
          flush=True)
    assert near.mean() < 0.1
    assert not param_bad(param.astype(np.float64), rp["param"], rp["smax"]).any()
    assert not cov_bad(cov.astype(np.float64), rp["cov"], rp["smax"]).any()
    assert not chi2_bad(chi2.astype(np.float64), rp["chi2"]).any()


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
        tr.track_batched_into(rb, y, z, U, bufs, s, unit_alpha=alpha, theta=theta_t, map_z=0.0)
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
        check_against_fp64_replay(cs, k, g["param"][gi], g["cov"][gi], g["chi2"][gi])
        # refit of the tracklets with >= 20 clusters against the FP64 oracle
        tk = oracle.select_tracks(k, 20)
        want, ok_ref = oracle.refit(cs, tk, theta, map_z=0.0)
        sel = gi[g["n_hits"][gi] >= 20]
        assert len(sel) == len(want)
        ok = rok[sel]
        np.testing.assert_array_equal(ok, ok_ref)
        rel = np.abs(rchi2[sel][ok] - want[ok]) / np.maximum(want[ok], 1.0)
        print(f"refit: {ok.sum()} tracks, max rel {rel.max():.2e}", flush=True)
        assert not refit_chi2_bad(rchi2[sel][ok].astype(np.float64), want[ok]).any(), rel.max()
        assert (rchi2[sel][~ok] == 0).all()


@pytest.mark.timeout(900)
def test_full_batch_of_16_slices_on_sampled_units():
    """The benchmark's workload: 16 time-frame slices (32-160 collisions each,
    ~843M clusters, 576 units) through the batched graph; one random unit of
    each of the first 15 slices and all 36 units of the last slice against the
    oracle, as above."""
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
                              theta=torch.as_tensor(theta, dtype=torch.float32, device=dev), map_z=0.0)
    s.synchronize()
    o = bufs["out"]
    counts = o["counts"].cpu().numpy()
    assert counts[3] == 0 and counts[1] == nt and counts[2] == nh
    unit = o["unit"][:nt].cpu().numpy()
    hit_begin = o["hit_begin"][:nt].cpu().numpy()
    n_hits_all = o["n_hits"][:nt].cpu().numpy()
    # one random unit of every slice, and every unit of the last slice
    rng = np.random.default_rng(1)
    per_slice = [int(rng.integers(36 * i, 36 * (i + 1))) for i in range(len(ncoll) - 1)]
    last = list(range(36 * (len(ncoll) - 1), 36 * len(ncoll)))
    for group in [[u] for u in per_slice] + [last]:
        u0, u1 = group[0], group[-1] + 1
        lo, hi = int(rb_h[u0 * G.N_ROWS]), int(rb_h[u1 * G.N_ROWS])
        print(f"units {u0}..{u1 - 1}: clusters {lo}..{hi}", flush=True)
        cu = SimpleNamespace(n_units=u1 - u0, row_begin=rb_h[u0 * G.N_ROWS:u1 * G.N_ROWS + 1] - lo,
                             y=y[lo:hi].cpu().numpy(), z=z[lo:hi].cpu().numpy(),
                             unit_sector=sectors[u0:u1])
        ref = oracle.track(cu, n_threads=16)
        k = oracle.kept_tracklets(ref)
        gi = np.nonzero((unit >= u0) & (unit < u1))[0]
        assert len(gi) == len(k["n"]) and len(gi) > 100
        np.testing.assert_array_equal(unit[gi] - u0, k["unit"])
        sel = torch.as_tensor(gi, device=dev)
        n_hits = n_hits_all[gi]
        np.testing.assert_array_equal(o["start"][sel].cpu().numpy() - lo, k["start"].astype(np.int32))
        np.testing.assert_array_equal(n_hits, k["n"])
        hb = hit_begin[gi]
        h0, h1 = int(hb[0]), int(hb[-1] + n_hits[-1])  # the units' tracklets are contiguous
        np.testing.assert_array_equal(o["hit_id"][h0:h1].cpu().numpy() - lo, k["hits"])
        np.testing.assert_array_equal(o["hit_row"][h0:h1].cpu().numpy(), k["rows"])
        param = o["param"][sel].cpu().numpy()
        cov = o["cov"][sel].cpu().numpy()
        chi2 = o["chi2"][sel].cpu().numpy()
        np.testing.assert_array_equal(param.astype(np.float64), k["param"])
        np.testing.assert_array_equal(cov.astype(np.float64), k["cov"])
        np.testing.assert_array_equal(chi2.astype(np.float64), k["chi2"])
        check_against_fp64_replay(cu, k, param, cov, chi2)
        tk = oracle.select_tracks(k, 20)
        want, ok_ref = oracle.refit(cu, tk, theta, unit_alpha=alpha_h[u0:u1], map_z=0.0)
        gsel = gi[n_hits >= 20]
        rchi2 = bufs["refit_chi2"][torch.as_tensor(gsel, device=dev)].cpu().numpy()
        rok = bufs["refit_ok"][torch.as_tensor(gsel, device=dev)].cpu().numpy().astype(bool)
        assert len(gsel) == len(want)
        np.testing.assert_array_equal(rok, ok_ref)
        rel = np.abs(rchi2[rok] - want[rok]) / np.maximum(want[rok], 1.0)
        print(f"refit: {rok.sum()} tracks, max rel {rel.max():.2e}", flush=True)
        assert not refit_chi2_bad(rchi2[rok].astype(np.float64), want[rok]).any(), rel.max()
        assert (rchi2[~rok] == 0).all()
