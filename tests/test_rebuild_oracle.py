"""Pins of the Phase II rebuild oracle (oracle.rebuild): iteration 2 queries
every cluster of each row compatible with the interpolation, a second
ambiguity solving hands candidates to tracks by rank (a track that loses its
best candidate takes its next), iteration 3 fits with a plain chi2 cut
(paper, Section 3, Phase II).

* noise-free isolated helices: every track keeps exactly its own clusters,
  chi2 ~ 0 and the truth parameters (FP64);
* late attachment: clusters left out of a track's input list are picked up;
* a wrong cluster in the input (the true one moved 3 cm away and a
  misplaced copy attached instead) is replaced by the true one;
* clones: two identical input tracks; the better-ranked one gets the
  clusters, the other one gets none and fails;
* FP32 against FP64: the same assignments on a central event (all but a
  handful of near-tie rows) and parameters within 1e-4 where they agree.
"""
import numpy as np

import oracle
import synth
from synth import geometry as G

from test_refit_oracle import truth_tracklets


def _case(seed, smear=0.0, n_tracks=12):
    tr = synth.exact_tracks(seed, n_tracks=n_tracks, pt_range=(1.0, 10.0), eta_range=(0.05, 0.7)).tracks
    cs = synth.build_clusters(tr, [0], seed + 1, smear_sigma=smear, noise_frac=0.0)
    tk = truth_tracklets(cs)
    n = len(tk["n"])
    tk["unit"] = np.zeros(n, np.int32)
    tk["xref"] = G.row_x()[tk["rows"][tk["hit_begin"][:-1]]].astype(np.float64)
    tk["chi2"] = np.ones(n)
    tk["ndf"] = 2 * tk["n"] - 5
    return cs, tk


def _hits(tk, t):
    return tk["hits"][tk["hit_begin"][t]:tk["hit_begin"][t + 1]]


def _subset(tk, t, keep_mask):
    """Track t's hit list reduced to keep_mask (other tracks unchanged)."""
    hb = tk["hit_begin"]
    hits, rows, n = [], [], []
    for u in range(len(tk["n"])):
        h, r = tk["hits"][hb[u]:hb[u + 1]], tk["rows"][hb[u]:hb[u + 1]]
        if u == t:
            h, r = h[keep_mask], r[keep_mask]
        hits.append(h)
        rows.append(r)
        n.append(len(h))
    out = dict(tk)
    out["hits"], out["rows"] = np.concatenate(hits), np.concatenate(rows)
    out["n"] = np.array(n)
    out["hit_begin"] = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    return out


def test_isolated_exact_tracks_keep_their_own_clusters():
    cs, tk = _case(91)
    r = oracle.rebuild(cs, tk, precision=64)
    assert r["ok"].all()
    truth = truth_tracklets(cs)["param"]
    for t in range(len(tk["n"])):
        got = r["assigned"][t]
        np.testing.assert_array_equal(np.sort(got[got >= 0]), np.sort(_hits(tk, t)))
    np.testing.assert_allclose(r["param"], truth, rtol=1e-6, atol=1e-6)
    assert (r["chi2"] < 1e-6).all()


def test_clusters_missing_from_the_input_are_attached():
    cs, tk = _case(92, smear=0.1)
    t = 3
    h = _hits(tk, t)
    mask = np.ones(len(h), bool)
    mask[5:len(h) - 5:3] = False  # every third inner cluster left out
    sub = _subset(tk, t, mask)
    r = oracle.rebuild(cs, sub)
    assert r["ok"][t]
    got = r["assigned"][t]
    assert set(h[~mask]) <= set(got[got >= 0]), "left-out clusters not picked up"
    np.testing.assert_array_equal(np.sort(got[got >= 0]), np.sort(h))


def test_a_wrong_cluster_is_replaced_by_the_true_one():
    from types import SimpleNamespace
    cs, tk = _case(93, smear=0.1)
    t = 5
    h = _hits(tk, t)
    q = h[len(h) // 2]
    # a stray cluster 3 cm off the track in the same row, attached in the input instead of q
    y = np.append(cs.y, np.float32(cs.y[q] + 3.0))
    z = np.append(cs.z, cs.z[q])
    stray = len(cs.y)
    row = int(cs.row_of()[q])
    order = np.concatenate([np.arange(cs.row_begin[row + 1]), [stray], np.arange(cs.row_begin[row + 1], len(cs.y))])
    inv = np.empty_like(order)
    inv[order] = np.arange(len(order))
    rb = cs.row_begin.copy()
    rb[row + 1:] += 1
    cs2 = SimpleNamespace(n_units=1, row_begin=rb, y=y[order], z=z[order])
    tk2 = dict(tk)
    hits = inv[tk["hits"]].astype(np.int32)
    hits[np.nonzero(tk["hits"] == q)[0]] = inv[stray]
    tk2["hits"] = hits
    r = oracle.rebuild(cs2, tk2)
    got = r["assigned"][t]
    assert inv[q] in got and inv[stray] not in got


def test_clones_the_better_ranked_track_gets_the_clusters():
    cs, tk = _case(94, smear=0.1, n_tracks=4)
    hb = tk["hit_begin"]
    n0 = tk["n"][0]
    dup = {k: v for k, v in tk.items()}
    dup["hits"] = np.concatenate([tk["hits"][:hb[1]], tk["hits"]])
    dup["rows"] = np.concatenate([tk["rows"][:hb[1]], tk["rows"]])
    dup["n"] = np.concatenate([[n0], tk["n"]])
    dup["hit_begin"] = np.concatenate([[0], np.cumsum(dup["n"])]).astype(np.int64)
    for k in ("param", "xref", "unit", "ndf"):
        dup[k] = np.concatenate([tk[k][:1], tk[k]])
    dup["chi2"] = np.concatenate([[2.0], tk["chi2"]])  # the copy ranks lower (larger chi2/ndf)
    r = oracle.rebuild(cs, dup)
    assert r["ok"][1] and not r["ok"][0]
    assert (r["assigned"][0] < 0).all()
    got = r["assigned"][1]
    np.testing.assert_array_equal(np.sort(got[got >= 0]), np.sort(_hits(tk, 0)))


def test_fp32_against_fp64_on_a_central_event():
    cs = synth.central_event(seed=2, n_primaries=3000)
    k = oracle.kept_tracklets(oracle.track(cs, n_threads=8))
    keep, _ = oracle.select(k, cs.n_clusters)
    idx = np.nonzero(keep)[0]
    hb = k["hit_begin"]
    tk = {key: k[key][idx] for key in ("unit", "n", "param", "xref", "chi2", "ndf")}
    tk["hit_begin"] = np.concatenate([[0], np.cumsum(k["n"][idx].astype(np.int64))])
    tk["hits"] = np.concatenate([k["hits"][hb[i]:hb[i + 1]] for i in idx])
    tk["rows"] = np.concatenate([k["rows"][hb[i]:hb[i + 1]] for i in idx])
    a = oracle.rebuild(cs, tk)
    b = oracle.rebuild(cs, tk, precision=64)
    both = a["ok"] & b["ok"]
    same = (a["assigned"] == b["assigned"]).all(1) & both
    assert (a["ok"] == b["ok"]).mean() > 0.999 and a["ok"].mean() > 0.99
    assert same.sum() > 0.999 * both.sum()
    unit = np.array([10.0, 10.0, 1.0, 1.0, 1.0])
    rel = np.abs(a["param"][same] - b["param"][same]) / np.maximum(np.abs(b["param"][same]), unit)
    assert rel.max() < 1e-4, rel.max()


def _cut(tk, keep_row):
    """tk with every track's clusters reduced to the rows keep_row accepts."""
    hb = tk["hit_begin"]
    hits, rows, n = [], [], []
    for u in range(len(tk["n"])):
        h, r = tk["hits"][hb[u]:hb[u + 1]], tk["rows"][hb[u]:hb[u + 1]]
        m = keep_row(r)
        hits.append(h[m])
        rows.append(r[m])
        n.append(int(m.sum()))
    out = dict(tk)
    out["hits"], out["rows"] = np.concatenate(hits), np.concatenate(rows)
    out["n"] = np.array(n)
    out["hit_begin"] = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    return out


def test_phase3_extrapolation_recovers_the_cut_off_ends():
    """Phase III (Section 3): exact helices given only their middle rows get
    their inner and outer clusters back from the extrapolation beyond the
    track's ends; without it the rebuild keeps to the given rows."""
    cs, tk = _case(95)
    full = {t: set(_hits(tk, t)) for t in range(len(tk["n"]))}
    rows_of = {t: tk["rows"][tk["hit_begin"][t]:tk["hit_begin"][t + 1]] for t in range(len(tk["n"]))}
    mid = _cut(tk, lambda r: (r >= 50) & (r <= 110))
    on = oracle.rebuild(cs, mid, precision=64, extrapolate=True)
    off = oracle.rebuild(cs, mid, precision=64, extrapolate=False)
    assert on["ok"].all() and off["ok"].all()
    recovered = 0
    for t in range(len(tk["n"])):
        got_on = set(on["assigned"][t][on["assigned"][t] >= 0])
        got_off = set(off["assigned"][t][off["assigned"][t] >= 0])
        assert got_on == full[t], t
        r = rows_of[t]
        assert got_off == set(_hits(tk, t)[(r >= 50) & (r <= 110)])
        assert (np.nonzero(off["assigned"][t] >= 0)[0] >= 50).all() and (np.nonzero(off["assigned"][t] >= 0)[0] <= 110).all()
        recovered += len(got_on) - len(got_off)
    assert recovered > 100
    truth = truth_tracklets(cs)["param"]
    np.testing.assert_allclose(on["param"], truth, rtol=1e-6, atol=1e-6)


def test_phase3_extrapolated_candidates_go_to_the_better_ranked_track():
    cs, tk = _case(96, smear=0.1, n_tracks=3)
    mid = _cut(tk, lambda r: r >= 40)
    hb = mid["hit_begin"]
    dup = {k: v for k, v in mid.items()}
    n0 = mid["n"][0]
    dup["hits"] = np.concatenate([mid["hits"][:hb[1]], mid["hits"]])
    dup["rows"] = np.concatenate([mid["rows"][:hb[1]], mid["rows"]])
    dup["n"] = np.concatenate([[n0], mid["n"]])
    dup["hit_begin"] = np.concatenate([[0], np.cumsum(dup["n"])]).astype(np.int64)
    for k in ("param", "xref", "unit", "ndf"):
        dup[k] = np.concatenate([mid[k][:1], mid[k]])
    dup["chi2"] = np.concatenate([[2.0], mid["chi2"]])  # the copy ranks lower
    r = oracle.rebuild(cs, dup, extrapolate=True)
    assert r["ok"][1] and not r["ok"][0]
    inner = set(_hits(tk, 0)[tk["rows"][tk["hit_begin"][0]:tk["hit_begin"][1]] < 40])
    got = set(r["assigned"][1][r["assigned"][1] >= 0])
    assert len(inner) > 10 and len(inner & got) > 0.9 * len(inner)
