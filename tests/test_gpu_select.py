"""Ambiguity solving on the GPU (tpcx_select) against the oracle
(oracle.select), bit for bit: kept flags and the cluster assignment, on the
tracklets the GPU produced (themselves bit-exact against the oracle's), for
the single sector, the central event, ties between duplicated clusters, a
sampled time-frame unit, both shared fractions of the paper (10 %, 20 %) and
a degenerate one (0: no sharing)."""
import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import make_tracker

pytestmark = pytest.mark.gpu


def _gpu_select(cs, shared):
    import torch
    dev = torch.device("cuda")
    tr = make_tracker()
    rb = torch.as_tensor(cs.row_begin, dtype=torch.int64, device=dev)
    y = torch.as_tensor(cs.y, dtype=torch.float32, device=dev)
    z = torch.as_tensor(cs.z, dtype=torch.float32, device=dev)
    n = cs.n_clusters
    probe = tr.track(rb, y, z, cs.n_units)
    ns, nt, nh = probe["n_start"], len(probe["n_hits"]), len(probe["hit_id"])
    bufs = tr.allocate(cs.n_units, n, ns + 1, nt + 1, nh + 1)
    tr.track_into(rb, y, z, cs.n_units, bufs)
    out = []
    for sh in shared:
        sel = tr.allocate_select(cs.n_units, n, bufs["cap_tracks"])
        sel["keep"].fill_(7)
        sel["assign"].fill_(-7)
        tr.select_into(bufs, cs.n_units, n, sel, shared=sh)
        torch.cuda.synchronize()
        cnt = sel["counts"].cpu().numpy()
        out.append((sel["keep"][:bufs["cap_tracks"]].cpu().numpy(), sel["assign"][:n].cpu().numpy(), cnt))
    o = bufs["out"]
    g = {k: o[k][:nt].cpu().numpy() for k in ("unit", "n_hits", "hit_begin", "chi2", "ndf", "start")}
    g["hits"] = o["hit_id"][:nh].cpu().numpy()
    return g, nt, out


def _check(cs, shared=((1, 10), (1, 5), (0, 1))):
    g, nt, outs = _gpu_select(cs, shared)
    ref = oracle.kept_tracklets(oracle.track(cs, n_threads=16))
    np.testing.assert_array_equal(g["n_hits"], ref["n"])
    np.testing.assert_array_equal(g["hits"], ref["hits"])
    np.testing.assert_array_equal(g["chi2"].astype(np.float64), ref["chi2"])
    for sh, (keep, assign, cnt) in zip(shared, outs):
        want_keep, want_assign = oracle.select(ref, cs.n_clusters, shared=sh)
        print(f"shared {sh}: {want_keep.sum()} of {nt} tracklets kept", flush=True)
        np.testing.assert_array_equal(keep[:nt].astype(bool), want_keep)
        assert (keep[nt:] == 0).all()
        np.testing.assert_array_equal(assign, want_assign)
        assert cnt[0] == want_keep.sum() and cnt[1] == 0


def test_select_single_sector():
    print("case: single sector seed 1", flush=True)
    _check(synth.single_sector(seed=1))


def test_select_central_event():
    print("case: central event seed 2", flush=True)
    _check(synth.central_event(seed=2))


def test_select_duplicated_clusters():
    # every cluster twice: every tracklet has an exact twin built from the
    # other copies or the same ones; ranks tie on chi2/ndf and length
    from types import SimpleNamespace
    cs = synth.single_sector(seed=3, n_tracks=60)
    rb = cs.row_begin
    ys, zs, rbd = [], [], [0]
    for r in range(len(rb) - 1):
        y = cs.y[rb[r]:rb[r + 1]]
        z = cs.z[rb[r]:rb[r + 1]]
        ys += [y, y]
        zs += [z, z]
        rbd.append(rbd[-1] + 2 * len(y))
    d = SimpleNamespace(n_units=1, row_begin=np.array(rbd, np.int64), y=np.concatenate(ys),
                        z=np.concatenate(zs), n_clusters=int(rbd[-1]))
    print(f"case: duplicated clusters, {d.n_clusters}", flush=True)
    _check(d)


def test_select_timeframe_units():
    from types import SimpleNamespace
    cs = synth.timeframe_slice(seed=3001, n_collisions=24, device="cuda", truth=False)
    R = 152
    u0, u1 = 5, 8
    lo, hi = int(cs.row_begin[u0 * R]), int(cs.row_begin[u1 * R])
    cu = SimpleNamespace(n_units=u1 - u0, row_begin=cs.row_begin[u0 * R:u1 * R + 1] - lo,
                         y=np.asarray(cs.y[lo:hi]), z=np.asarray(cs.z[lo:hi]), n_clusters=hi - lo)
    print(f"case: time-frame slice seed 3001, units {u0}..{u1 - 1}, {cu.n_clusters} clusters", flush=True)
    _check(cu)
