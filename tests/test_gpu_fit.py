"""Three-iteration fit with interpolation-based rejection on the GPU
(tpcx_fit) against the oracle (oracle.fit): rejection flags, kept counts, ok
flags, parameters, covariances and chi2 bit for bit against the float
oracle, and within tolerance of the FP64 replay of the same decisions.
Inputs are the oracle's own tracklets (no value of the HIP path feeds the
oracle): the single sector, the central event, time-frame units, tracks with
planted outliers, and degenerate track lengths (2, 3 clusters)."""
import numpy as np
import pytest

import oracle
import synth

from gpu_helpers import make_tracker

pytestmark = pytest.mark.gpu

UNIT = np.array([10.0, 10.0, 1.0, 1.0, 1.0])


def _gpu_fit(cs, tk):
    import torch
    dev = torch.device("cuda")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    tr = make_tracker()
    r = tr.fit(T(tk["hit_begin"], torch.int64), T(tk["hits"], torch.int32), T(tk["rows"], torch.uint8),
               T(np.asarray(tk["param"], np.float32), torch.float32),
               T(np.asarray(tk["xref"], np.float32), torch.float32), T(cs.y, torch.float32),
               T(cs.z, torch.float32))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items() if k != "_ws"}


def _check(cs, tk, name):
    print(f"case: {name}, {len(tk['hit_begin']) - 1} tracks", flush=True)
    g = _gpu_fit(cs, tk)
    f = oracle.fit(cs, tk)
    np.testing.assert_array_equal(g["reject"], f["reject"])
    np.testing.assert_array_equal(g["ok"].astype(bool), f["ok"])
    np.testing.assert_array_equal(g["n_kept"], f["n_kept"])
    for k in ("param", "cov", "chi2", "x_out"):
        np.testing.assert_array_equal(g[k].astype(np.float64), f[k], err_msg=k)
    r = oracle.fit(cs, tk, precision=64, reject=f["reject"])
    ok = f["ok"]
    assert r["ok"][ok].all()  # (a failed fit keeps no rejection flags to replay)
    rel = np.abs(f["param"][ok] - r["param"][ok]) / np.maximum(np.abs(r["param"][ok]), UNIT)
    mx = rel.max() if ok.any() else 0.0
    print(f"  ok {ok.sum()}, rejected {f['reject'].sum()} of {len(f['reject'])}, max rel vs FP64 {mx:.2e}",
          flush=True)
    assert mx < 1e-4
    assert (np.abs(f["chi2"][ok] - r["chi2"][ok]) <= 1e-3 * np.maximum(r["chi2"][ok], 1.0)).all()
    return f


def _tracklets(cs, min_hits=10):
    k = oracle.kept_tracklets(oracle.track(cs, n_threads=16))
    tk = oracle.select_tracks(k, min_hits)
    tk["xref"] = k["xref"][tk["index"]]
    return tk


def test_fit_single_sector_and_central_event():
    cs = synth.single_sector(seed=1)
    _check(cs, _tracklets(cs), "single sector")
    cs = synth.central_event(seed=2)
    _check(cs, _tracklets(cs), "central event")


def test_fit_timeframe_units():
    from types import SimpleNamespace
    cs = synth.timeframe_slice(seed=3002, n_collisions=24, device="cuda", truth=False)
    R = 152
    u0, u1 = 10, 13
    lo, hi = int(cs.row_begin[u0 * R]), int(cs.row_begin[u1 * R])
    cu = SimpleNamespace(n_units=u1 - u0, row_begin=cs.row_begin[u0 * R:u1 * R + 1] - lo,
                         y=np.asarray(cs.y[lo:hi]), z=np.asarray(cs.z[lo:hi]))
    f = _check(cu, _tracklets(cu, 20), "time-frame slice seed 3002, units 10..12")
    assert f["reject"].any()


def test_fit_planted_outliers_and_short_tracks():
    cs = synth.central_event(seed=6, n_primaries=2000)
    tk = _tracklets(cs, 20)
    y = cs.y.copy()
    rng = np.random.default_rng(5)
    for t in range(0, len(tk["n"]), 3):
        b, e = tk["hit_begin"][t], tk["hit_begin"][t + 1]
        y[tk["hits"][rng.integers(b, e)]] += np.float32(1.5)
    cs.y = y
    f = _check(cs, tk, "central event with planted outliers")
    assert f["reject"].sum() > len(tk["n"]) // 4
    # tracks of 2 and 3 clusters (the first fails, the second may succeed)
    sub = {k: v for k, v in tk.items()}
    hb = tk["hit_begin"]
    keep_n = np.where(np.arange(len(tk["n"])) % 2 == 0, 2, 3)
    sel = [np.arange(hb[t], hb[t] + keep_n[t]) for t in range(len(tk["n"]))]
    idx = np.concatenate(sel)
    sub["hits"], sub["rows"] = tk["hits"][idx], tk["rows"][idx]
    sub["hit_begin"] = np.concatenate([[0], np.cumsum(keep_n)]).astype(np.int64)
    sub["n"] = keep_n
    f = _check(cs, sub, "tracks cut to 2 and 3 clusters")
    assert not f["ok"][::2].any()
