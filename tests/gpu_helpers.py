"""Helpers shared by the GPU tests: run the HIP path and the oracle on one input."""
import numpy as np

import oracle
from synth import geometry as G
from tolerances import NEAR_GUARD, chi2_bad, cov_bad, param_bad


def make_tracker(tuning=None, params=None, row_x=None):
    import paper_2601_20569_amd as px
    return px.SectorTracker(G.row_x() if row_x is None else row_x, G.tan_half_opening(),
                            G.BZ_TESLA, params=params, tuning=tuning)


def run_gpu(cs, tracker=None, debug=True, **kw):
    import torch
    tr = tracker or make_tracker()
    dev = torch.device("cuda")
    rb = torch.as_tensor(cs.row_begin, dtype=torch.int64, device=dev)
    y = torch.as_tensor(cs.y, dtype=torch.float32, device=dev)
    z = torch.as_tensor(cs.z, dtype=torch.float32, device=dev)
    res = tr.track(rb, y, z, cs.n_units, debug=debug, **kw)
    torch.cuda.synchronize()
    out = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items()}
    hb = np.zeros(len(out["n_hits"]) + 1, np.int64)
    hb[:-1] = out["hit_begin"]
    hb[-1] = len(out["hit_id"])
    out["hit_begin_full"] = hb
    return out


def compare_decisions(gpu, ref, units=None, cs=None):
    """Bit-exact comparison of links, start hits and tracklet hit lists.

    With ``units=(lo, hi)`` only the clusters and tracklets of those units are
    compared (the oracle ran on that subset)."""
    if units is None:
        sel = slice(None)
        g_keep = np.ones(len(gpu["n_hits"]), bool)
    else:
        lo, hi = units
        b = cs.row_begin[lo * G.N_ROWS]
        e = cs.row_begin[hi * G.N_ROWS]
        sel = slice(b, e)
        g_keep = (gpu["unit"] >= lo) & (gpu["unit"] < hi)
    for k in ("link_up", "link_down", "clean_up", "clean_down"):
        np.testing.assert_array_equal(gpu[k][sel], ref[k][sel], err_msg=k)
    if units is None:
        np.testing.assert_array_equal(gpu["starts"], ref["starts"].astype(np.int32))
    k = oracle.kept_tracklets(ref)
    gi = np.nonzero(g_keep)[0]
    np.testing.assert_array_equal(gpu["start"][gi], k["start"].astype(np.int32))
    np.testing.assert_array_equal(gpu["n_hits"][gi], k["n"])
    np.testing.assert_array_equal(gpu["unit"][gi], k["unit"])
    ghb = gpu["hit_begin_full"]
    g_hits = np.concatenate([gpu["hit_id"][ghb[i]:ghb[i + 1]] for i in gi]) if len(gi) else np.zeros(0)
    g_rows = np.concatenate([gpu["hit_row"][ghb[i]:ghb[i + 1]] for i in gi]) if len(gi) else np.zeros(0)
    np.testing.assert_array_equal(g_hits, k["hits"])
    np.testing.assert_array_equal(g_rows, k["rows"])
    return k, gi


def compare_numbers(gpu, gi, k, rp):
    """Parameters, covariances and chi2 against the FP64 replay."""
    assert rp["ok"].all()
    p = gpu["param"][gi].astype(np.float64)
    np.testing.assert_array_equal(gpu["x_ref"][gi].astype(np.float64), rp["xref"])
    bad = param_bad(p, rp["param"], rp["smax"])
    assert not bad.any(), (np.argwhere(bad)[:5], p[bad][:5], rp["param"][bad][:5])
    assert not chi2_bad(gpu["chi2"][gi].astype(np.float64), rp["chi2"]).any()
    assert not cov_bad(gpu["cov"][gi].astype(np.float64), rp["cov"], rp["smax"]).any()
    if len(gi) >= 1000:  # the near-guard class stays a minority of a real event's tracklets
        assert (rp["smax"] >= NEAR_GUARD).mean() < 0.2
    np.testing.assert_array_equal(gpu["ndf"][gi], 2 * k["n"] - 5)
