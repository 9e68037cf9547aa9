"""Pins of the three-iteration fit oracle (oracle.fit): inwards, outwards with
the interpolation chi2 cut, inwards over the kept clusters (paper, Section 2
track fit; Section 3, Phase I).

* noise-free exact helices: no cluster is rejected and the result equals the
  truth at the innermost cluster, chi2 ~ 0 (FP64);
* smeared tracks: chi2/ndf = 1 and pulls of the final parameters against the
  truth have mean 0 and width 1;
* planted outliers (one cluster per track moved by 1.5 cm, 15 sigma): the
  moved cluster is rejected and almost no other one;
* FP32 within 1e-4 of the FP64 replay of its own decisions, and the FP32
  replay reproduces the FP32 fit bit for bit.
"""
import math

import numpy as np

import oracle
import synth
from synth import geometry as G

from test_refit_oracle import truth_tracklets


def _truth_case(seed, smear, n_tracks=20, pt=(1.0, 10.0)):
    tr = synth.exact_tracks(seed, n_tracks=n_tracks, pt_range=pt, eta_range=(0.05, 0.7)).tracks
    cs = synth.build_clusters(tr, [0], seed + 1, smear_sigma=smear, noise_frac=0.0)
    tk = truth_tracklets(cs)
    # the seed (the tracking result) sits at the innermost cluster
    tk["xref"] = G.row_x()[tk["rows"][tk["hit_begin"][:-1]]].astype(np.float64)
    return cs, tk


def test_exact_helices_keep_every_cluster_and_recover_the_truth():
    cs, tk = _truth_case(81, smear=0.0)
    # perturb the seed: the fit must not depend on it beyond linearisation
    tk["param"] = tk["param"] * np.array([1.0, 1.0, 1.0, 1.0, 1.02])
    f = oracle.fit(cs, tk, precision=64)
    assert f["ok"].all() and len(f["ok"]) >= 15
    assert not f["reject"].any()
    np.testing.assert_array_equal(f["n_kept"], tk["n"])
    truth = truth_tracklets(cs)["param"]
    np.testing.assert_allclose(f["param"], truth, rtol=1e-6, atol=1e-6)
    assert (f["chi2"] < 1e-6).all(), f["chi2"]


def test_smeared_tracks_chi2_and_pulls():
    ratios, pulls = [], []
    for seed in range(4):
        cs, tk = _truth_case(300 + seed, smear=0.1)
        truth = truth_tracklets(synth.build_clusters(
            synth.exact_tracks(300 + seed, n_tracks=20, pt_range=(1.0, 10.0), eta_range=(0.05, 0.7)).tracks,
            [0], 300 + seed + 1, smear_sigma=0.0, noise_frac=0.0))["param"]
        f = oracle.fit(cs, tk, precision=64)
        ok = f["ok"] & (f["n_kept"] == tk["n"])
        ratios += list(f["chi2"][ok] / (2 * f["n_kept"][ok] - 5))
        sig = np.sqrt(f["cov"][ok][:, [0, 2, 5, 9, 14]])
        # y, z at the innermost cluster carry the cluster's own smear; compare s, t, w
        pulls.append(((f["param"][ok] - truth[ok]) / sig)[:, 2:])
    p = np.concatenate(pulls)
    assert len(ratios) > 60
    assert abs(np.mean(ratios) - 1.0) < 0.06
    assert np.all(np.abs(p.mean(0)) < 0.15), p.mean(0)
    assert np.all(np.abs(p.std(0) - 1.0) < 0.2), p.std(0)


def test_planted_outliers_are_rejected():
    rng = np.random.default_rng(9)
    hit, miss, false = 0, 0, 0
    n_other = 0
    for seed in range(4):
        cs, tk = _truth_case(400 + seed, smear=0.1)
        y = cs.y.copy()
        moved = []
        for t in range(len(tk["n"])):
            b, e = tk["hit_begin"][t], tk["hit_begin"][t + 1]
            q = int(rng.integers(b + 3, e - 3))
            y[tk["hits"][q]] += np.float32(1.5 if rng.random() < 0.5 else -1.5)
            moved.append(q)
        cs.y = y
        f = oracle.fit(cs, tk)
        mask = np.zeros(len(tk["hits"]), bool)
        mask[moved] = True
        hit += int(f["reject"][mask].sum())
        miss += int((~f["reject"][mask].astype(bool)).sum())
        false += int(f["reject"][~mask].sum())
        n_other += int((~mask).sum())
    assert hit >= 0.95 * (hit + miss), (hit, miss)
    assert false <= 0.01 * n_other, (false, n_other)


def test_fp32_fit_within_tolerance_of_fp64_replay():
    cs = synth.central_event(seed=2, n_primaries=3000)
    k = oracle.kept_tracklets(oracle.track(cs, n_threads=8))
    tk = oracle.select_tracks(k, 20)
    tk["xref"] = k["xref"][tk["index"]]
    f = oracle.fit(cs, tk)
    r = oracle.fit(cs, tk, precision=64, reject=f["reject"])
    f32r = oracle.fit(cs, tk, precision=32, reject=f["reject"])
    # a failed float fit keeps no rejection flags, so its replay is not comparable
    assert r["ok"][f["ok"]].all() and f["ok"].mean() > 0.99
    ok = f["ok"]
    for key in ("param", "cov", "chi2", "n_kept"):
        np.testing.assert_array_equal(f32r[key][ok], f[key][ok], err_msg=key)
    unit = np.array([10.0, 10.0, 1.0, 1.0, 1.0])
    rel = np.abs(f["param"][ok] - r["param"][ok]) / np.maximum(np.abs(r["param"][ok]), unit)
    assert rel.max() < 1e-4, rel.max()
    assert (np.abs(f["chi2"][ok] - r["chi2"][ok]) <= 1e-3 * np.maximum(r["chi2"][ok], 1.0)).all()
