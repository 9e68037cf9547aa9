"""Phase II rebuild on the GPU (tpcx_rebuild) against the oracle
(oracle.rebuild), bit for bit: the cluster kept at every row, ok flags, kept
counts, parameters, covariances and chi2.  Inputs are the oracle's own
selected tracklets (no value of the HIP path feeds the oracle): the single
sector, the central event, tracks with clusters left out of their input
lists, and time-frame units; with Phase III's extrapolation beyond the
tracks' ends: the central event, tracks cut to their middle rows and
time-frame units."""
import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import make_tracker

pytestmark = pytest.mark.gpu


def _selected(cs):
    k = oracle.kept_tracklets(oracle.track(cs, n_threads=16))
    keep, _ = oracle.select(k, cs.n_clusters)
    idx = np.nonzero(keep)[0]
    hb = k["hit_begin"]
    tk = {key: k[key][idx] for key in ("unit", "n", "param", "xref", "chi2", "ndf")}
    tk["hit_begin"] = np.concatenate([[0], np.cumsum(k["n"][idx].astype(np.int64))])
    tk["hits"] = np.concatenate([k["hits"][hb[i]:hb[i + 1]] for i in idx])
    tk["rows"] = np.concatenate([k["rows"][hb[i]:hb[i + 1]] for i in idx])
    return tk


def _check(cs, tk, name, **kw):
    import torch
    print(f"case: {name}, {len(tk['n'])} tracks {kw}", flush=True)
    dev = torch.device("cuda")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    tr = make_tracker()
    g = tr.rebuild(T(cs.row_begin, torch.int64), T(cs.y, torch.float32), T(cs.z, torch.float32), cs.n_units,
                   T(tk["unit"], torch.int32), T(tk["hit_begin"], torch.int64), T(tk["hits"], torch.int32),
                   T(tk["rows"], torch.uint8), T(np.asarray(tk["param"], np.float32), torch.float32),
                   T(np.asarray(tk["xref"], np.float32), torch.float32),
                   T(np.asarray(tk["chi2"], np.float32), torch.float32), T(tk["ndf"], torch.int32), **kw)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items() if k != "_ws"}
    r = oracle.rebuild(cs, tk, **kw)
    np.testing.assert_array_equal(g["ok"].astype(bool), r["ok"])
    np.testing.assert_array_equal(g["assigned"], r["assigned"])
    np.testing.assert_array_equal(g["n_kept"], r["n_kept"])
    for k in ("param", "cov", "chi2", "x_out"):
        np.testing.assert_array_equal(g[k].astype(np.float64), r[k], err_msg=k)
    print(f"  ok {r['ok'].sum()}, clusters kept {r['n_kept'].sum()} (input {tk['n'].sum()})", flush=True)


def test_rebuild_single_sector_and_central_event():
    cs = synth.single_sector(seed=1)
    _check(cs, _selected(cs), "single sector")
    cs = synth.central_event(seed=2)
    _check(cs, _selected(cs), "central event")


def test_rebuild_recovers_left_out_clusters():
    cs = synth.central_event(seed=8, n_primaries=2000)
    tk = _selected(cs)
    # every fourth cluster of every second track left out of the input
    keep = np.ones(len(tk["hits"]), bool)
    for t in range(0, len(tk["n"]), 2):
        b, e = tk["hit_begin"][t], tk["hit_begin"][t + 1]
        keep[b + 2:e - 2:4] = False
    n = np.array([keep[tk["hit_begin"][t]:tk["hit_begin"][t + 1]].sum() for t in range(len(tk["n"]))])
    sub = dict(tk)
    sub["hits"], sub["rows"] = tk["hits"][keep], tk["rows"][keep]
    sub["n"] = n
    sub["hit_begin"] = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    _check(cs, sub, "central event, clusters left out")


def test_rebuild_timeframe_units():
    from types import SimpleNamespace
    cs = synth.timeframe_slice(seed=3003, n_collisions=24, device="cuda", truth=False)
    R = 152
    u0, u1 = 20, 23
    lo, hi = int(cs.row_begin[u0 * R]), int(cs.row_begin[u1 * R])
    cu = SimpleNamespace(n_units=u1 - u0, row_begin=cs.row_begin[u0 * R:u1 * R + 1] - lo,
                         y=np.asarray(cs.y[lo:hi]), z=np.asarray(cs.z[lo:hi]), n_clusters=hi - lo)
    _check(cu, _selected(cu), "time-frame slice seed 3003, units 20..22")


def test_rebuild_with_phase3_extrapolation():
    from test_rebuild_oracle import _case, _cut
    cs, tk = _case(95)
    mid = _cut(tk, lambda r: (r >= 50) & (r <= 110))
    _check(cs, mid, "exact tracks cut to rows 50..110", extrapolate=True)
    cs = synth.central_event(seed=2)
    tk = _selected(cs)
    _check(cs, tk, "central event", extrapolate=True)
    _check(cs, _cut(tk, lambda r: r >= 20), "central event, inner 20 rows cut", extrapolate=True, chi2_extrap=16.0)


def test_rebuild_phase3_timeframe_units():
    from types import SimpleNamespace
    cs = synth.timeframe_slice(seed=3005, n_collisions=24, device="cuda", truth=False)
    R = 152
    u0, u1 = 7, 10
    lo, hi = int(cs.row_begin[u0 * R]), int(cs.row_begin[u1 * R])
    cu = SimpleNamespace(n_units=u1 - u0, row_begin=cs.row_begin[u0 * R:u1 * R + 1] - lo,
                         y=np.asarray(cs.y[lo:hi]), z=np.asarray(cs.z[lo:hi]), n_clusters=hi - lo)
    _check(cu, _selected(cu), "time-frame slice seed 3005, units 7..9", extrapolate=True)
