"""Pins of the track-merging oracle (oracle.merge, oracle.merge_views):
segments of one helix found separately inside a sector, in two adjacent
sectors or on the two sides of the central electrode are merged (paper,
Section 2, track merging).

* views: a track's state carried to the plane x_m in its own frame and in
  the two sector-boundary frames equals the closed-form helix state there
  (FP64, the helix from the generator's kinematics, independent of the
  oracle's circle step and rotation);
* exact helices cut into an inner and an outer segment inside a sector, and
  helices crossing from one sector into the next, merge into one chain each,
  and no link joins segments of different particles;
* a helix crossing the central electrode, cut at the electrode, merges;
* hand cases: the better-matching of two outer candidates wins, an exact tie
  goes to the smaller index, overlapping rows never link, a missing view
  (a track turning away) never links;
* random tiny inputs against a brute-force enumeration of the mutual-best
  rule on the oracle's own views.
"""
import math

import numpy as np

import oracle
import synth
from synth import geometry as G

KAP = G.C_LIGHT_GEV * G.BZ_TESLA


def helix_state(tr, t, frame_alpha, x):
    """Closed-form state (y, z, sin phi, dz/ds, q/pT) of particle t at the plane
    x of the frame whose x axis has azimuth frame_alpha (first crossing on the
    outgoing leg), or None."""
    q, pt, phi, tl = tr.q[t], tr.pt[t], tr.phi[t], tr.tanl[t]
    R = pt / KAP
    cx = tr.vx[t] + q * R * math.sin(phi)
    cy = tr.vy[t] - q * R * math.cos(phi)
    theta0 = math.atan2(tr.vy[t] - cy, tr.vx[t] - cx)
    ca, sa = math.cos(frame_alpha), math.sin(frame_alpha)
    cxl, cyl = cx * ca + cy * sa, -cx * sa + cy * ca
    d = x - cxl
    disc = R * R - d * d
    if disc < 0:
        return None
    best = None
    for br in (1.0, -1.0):
        Y = cyl + br * math.sqrt(disc)
        th = math.atan2(Y - cyl, d) + frame_alpha
        psi = (q * (theta0 - th)) % (2 * math.pi)
        if best is None or psi < best[0]:
            best = (psi, Y)
    psi, Y = best
    z = tr.vz[t] + tl * R * psi
    return np.array([Y, z, math.sin(phi - q * psi - frame_alpha), tl, q / pt])


def segments(cs, min_n=3, split=None):
    """One segment per (particle, unit) of a cluster set (split=(k, gap): the
    first k clusters, then the rest after leaving out `gap`), with the truth
    state at its innermost cluster."""
    rows = cs.row_of()
    units = cs.unit_of()
    tr = cs.tracks
    segs = []
    for t in np.unique(cs.truth_track[cs.truth_track >= 0]):
        for u in range(cs.n_units):
            idx = np.nonzero((cs.truth_track == t) & (units == u))[0]
            idx = idx[np.argsort(rows[idx])]
            parts = [idx] if split is None else [idx[:split[0]], idx[split[0] + split[1]:]]
            for part in parts:
                if len(part) < min_n:
                    continue
                j = part[0]
                a0 = float(G.sector_alpha(cs.unit_sector[u]))
                phi = tr.phi[t] - tr.q[t] * cs.truth_psi[j]
                segs.append(dict(particle=int(t), unit=u, r_in=int(rows[part[0]]), r_out=int(rows[part[-1]]),
                                 param=[cs.y[j], cs.z[j], math.sin(phi - a0), tr.tanl[t], tr.q[t] / tr.pt[t]],
                                 xref=float(G.row_x()[rows[j]])))
    segs.sort(key=lambda s: s["unit"])
    return segs


def as_tracks(segs):
    return dict(unit=np.array([s["unit"] for s in segs], np.int32),
                param=np.array([s["param"] for s in segs], np.float64),
                xref=np.array([s["xref"] for s in segs]),
                r_in=np.array([s["r_in"] for s in segs], np.int32),
                r_out=np.array([s["r_out"] for s in segs], np.int32))


def test_views_equal_the_closed_form_helix():
    cs = synth.exact_tracks(61, n_tracks=12, pt_range=(0.8, 8.0))
    segs = segments(cs)
    tk = as_tracks(segs)
    views, ok = oracle.merge_views(tk, precision=64)
    a0 = float(G.sector_alpha(0))
    h = G.HALF_OPENING_RAD
    x_m = oracle.MERGE_DEFAULTS["x_m"]
    checked = 0
    for i, s in enumerate(segs):
        for v, beta in ((0, a0), (1, a0 + h), (2, a0 - h)):
            want = helix_state(cs.tracks, s["particle"], beta, x_m)
            if want is None or not ok[i, v]:
                continue
            # float inputs (rounded state at the segment's first cluster):
            # ~1e-6 cm after the step, plus the float rotation constants
            np.testing.assert_allclose(views[i, v, :2], want[:2], atol=2e-4)
            np.testing.assert_allclose(views[i, v, 2], want[2], atol=2e-6)
            np.testing.assert_allclose(views[i, v, 3:], want[3:], rtol=1e-6)
            checked += 1
    assert checked >= 30


def _links(out):
    return {(int(a), int(b)) for a, b in enumerate(out["next"]) if b >= 0}


def test_segments_split_inside_a_sector_merge():
    cs = synth.exact_tracks(62, n_tracks=14, pt_range=(0.8, 8.0))
    segs = segments(cs, split=(40, 6))
    tk = as_tracks(segs)
    out = oracle.merge(tk, oracle.unit_neighbours([0]), 1)
    want = set()
    for i, a in enumerate(segs):
        for j, b in enumerate(segs):
            if a["particle"] == b["particle"] and a["r_out"] < b["r_in"]:
                want.add((i, j))
    assert len(want) >= 10
    assert _links(out) == want
    for i, j in want:
        assert out["prev"][j] == i and out["root"][j] == i and out["root"][i] == i


def test_helices_crossing_into_the_next_sector_merge():
    rng = np.random.default_rng(7)
    n = 60
    # aimed at the boundary between sectors 0 and 1 (20 degrees), both charges
    phi = rng.uniform(math.radians(8.0), math.radians(32.0), n)
    pt = np.exp(rng.uniform(math.log(0.3), math.log(1.0), n))
    tr = synth.events.Tracks(np.zeros(n), np.zeros(n), np.zeros(n), pt, phi, rng.uniform(0.05, 0.5, n),
                             rng.choice([-1.0, 1.0], n), np.zeros(n))
    cs = synth.build_clusters(tr, [0, 1], 5, smear_sigma=0.0, noise_frac=0.0)
    segs = segments(cs)
    tk = as_tracks(segs)
    out = oracle.merge(tk, oracle.unit_neighbours([0, 1]), 2)
    want = set()
    for i, a in enumerate(segs):
        for j, b in enumerate(segs):
            if a["particle"] == b["particle"] and a["unit"] != b["unit"] and a["r_out"] < b["r_in"]:
                want.add((i, j))
    assert len(want) >= 10
    got = _links(out)
    assert got == want, (sorted(got ^ want), len(want))


def test_a_helix_crossing_the_central_electrode_merges():
    # vertex at z = +12 cm, dz/ds < 0: z = 0 is reached at ~120 cm of path
    n = 6
    rng = np.random.default_rng(3)
    phi = rng.uniform(math.radians(3.0), math.radians(17.0), n)
    tr = synth.events.Tracks(np.zeros(n), np.zeros(n), np.full(n, 12.0), np.full(n, 5.0), phi,
                             np.full(n, -0.1), rng.choice([-1.0, 1.0], n), np.zeros(n))
    x = G.row_x()
    a0 = float(G.sector_alpha(0))
    segs = []
    for t in range(n):
        states = [helix_state(tr, t, a0, xr) for xr in x]
        zs = np.array([s[1] for s in states])
        k = int(np.argmax(zs < 0))  # first row on the C side
        assert 5 < k < len(x) - 5
        segs.append(dict(unit=0, r_in=0, r_out=k - 1, param=states[0], xref=float(x[0]), particle=t))
        segs.append(dict(unit=1, r_in=k, r_out=len(x) - 1, param=states[k], xref=float(x[k]), particle=t))
    segs.sort(key=lambda s: s["unit"])
    tk = as_tracks(segs)
    nbr = oracle.unit_neighbours([0, 18])
    assert nbr[0, 2] == 1 and nbr[1, 2] == 0
    out = oracle.merge(tk, nbr, 2)
    want = {(i, j) for i, a in enumerate(segs) for j, b in enumerate(segs)
            if a["particle"] == b["particle"] and a["unit"] == 0 and b["unit"] == 1}
    assert _links(out) == want
    # without the electrode step nothing merges
    out = oracle.merge(tk, nbr, 2, cross_electrode=False)
    assert (out["next"] < 0).all()


def _pair_case():
    cs = synth.exact_tracks(63, n_tracks=1, pt_range=(2.0, 2.0))
    segs = segments(cs, split=(40, 6))
    assert len(segs) == 2
    return segs


def test_the_better_of_two_outer_candidates_wins_and_ties_go_to_the_smaller_index():
    inner, outer = _pair_case()
    shifted = dict(outer, param=[outer["param"][0] + 0.5] + list(outer["param"][1:]))
    for order in ((inner, shifted, outer), (inner, outer, shifted)):
        tk = as_tracks(list(order))
        out = oracle.merge(tk, oracle.unit_neighbours([0]), 1)
        j = [k for k, s in enumerate(order) if s is outer][0]
        assert out["next"][0] == j and out["prev"][j] == 0
        assert (out["next"][1:] < 0).all() and out["prev"][3 - j] == -1
    tk = as_tracks([inner, outer, dict(outer)])  # exact tie: index 1 wins
    out = oracle.merge(tk, oracle.unit_neighbours([0]), 1)
    assert out["next"][0] == 1 and out["prev"][2] == -1


def test_overlapping_rows_and_missing_views_never_link():
    inner, outer = _pair_case()
    over = dict(outer, r_in=inner["r_out"])
    out = oracle.merge(as_tracks([inner, over]), oracle.unit_neighbours([0]), 1)
    assert (out["next"] < 0).all() and (out["prev"] < 0).all()
    # an inner segment that cannot reach x_m (|sin phi| guard) has no view
    turned = dict(inner, param=[inner["param"][0], inner["param"][1], 0.995] + list(inner["param"][3:]))
    views, ok = oracle.merge_views(as_tracks([turned]), precision=32)
    assert not ok[0].any()
    out = oracle.merge(as_tracks([turned, outer]), oracle.unit_neighbours([0]), 1)
    assert (out["next"] < 0).all()


def test_random_tiny_inputs_against_brute_force():
    rng = np.random.default_rng(11)
    tol = np.array(oracle.MERGE_DEFAULTS["tol"], np.float32)
    itol2 = (np.float32(1.0) / (tol * tol)).astype(np.float32)
    cut = np.float32(oracle.MERGE_DEFAULTS["chi2_cut"])
    for case in range(200):
        n_units = int(rng.integers(1, 4))
        sectors = rng.choice([0, 1, 2, 18, 19], n_units, replace=False)
        n = int(rng.integers(2, 14))
        unit = np.sort(rng.integers(0, n_units, n)).astype(np.int32)
        base = np.array([rng.uniform(-10, 10), rng.uniform(-50, 50), rng.uniform(-0.3, 0.3), 0.2, 0.5])
        param = base + rng.normal(0, 1, (n, 5)) * np.array([0.6, 0.6, 0.01, 0.01, 0.05])
        if case % 5 == 0:
            param[1::2] = param[0::2][:len(param[1::2])]  # exact ties
        r_in = rng.integers(0, 150, n).astype(np.int32)
        r_out = np.minimum(151, r_in + rng.integers(2, 60, n)).astype(np.int32)
        tk = dict(unit=unit, param=param, xref=G.row_x()[r_in].astype(np.float64), r_in=r_in, r_out=r_out)
        nbr = oracle.unit_neighbours(sectors)
        views, ok = oracle.merge_views(tk, precision=32)
        views = views.astype(np.float32)
        out = oracle.merge(tk, nbr, n_units)
        best_out, best_in = {}, {}
        for a in range(n):
            ua = unit[a]
            for ub, va, vb in ((ua, 0, 0), (nbr[ua, 2], 0, 0), (nbr[ua, 0], 1, 2), (nbr[ua, 1], 2, 1)):
                if ub < 0 or not ok[a, va]:
                    continue
                for b in np.nonzero(unit == ub)[0]:
                    if b == a or not ok[b, vb] or not r_out[a] < r_in[b]:
                        continue
                    c2 = np.float32(0.0)
                    for i in range(5):
                        d = np.float32(views[a, va, i] - views[b, vb, i])
                        c2 = np.float32(c2 + np.float32(d * d) * itol2[i])
                    if not c2 <= cut:
                        continue
                    if a not in best_out or (c2, b) < best_out[a]:
                        best_out[a] = (c2, b)
                    if b not in best_in or (c2, a) < best_in[b]:
                        best_in[b] = (c2, a)
        want_next = [best_out[a][1] if a in best_out and best_in[best_out[a][1]][1] == a else -1 for a in range(n)]
        np.testing.assert_array_equal(out["next"], want_next, err_msg=f"case {case}")
        for a in range(n):
            r = a
            while out["prev"][r] >= 0:
                r = out["prev"][r]
            assert out["root"][a] == r


def test_links_join_segments_of_one_particle_on_the_central_event():
    """On the selected tracklets of a central event, the links join segments
    of one particle (the majority particle of each tracklet's clusters)."""
    cs = synth.central_event(seed=2)
    k = oracle.kept_tracklets(oracle.track(cs, n_threads=16))
    keep, _ = oracle.select(k, cs.n_clusters)
    idx = np.nonzero(keep)[0]
    hb = k["hit_begin"]
    tk = dict(unit=k["unit"][idx].astype(np.int32), param=k["param"][idx], xref=k["xref"][idx],
              r_in=np.array([k["rows"][hb[i]] for i in idx], np.int32),
              r_out=np.array([k["rows"][hb[i + 1] - 1] for i in idx], np.int32))
    out = oracle.merge(tk, oracle.unit_neighbours(cs.unit_sector), cs.n_units)
    truth = np.array([np.bincount(np.maximum(cs.truth_track[k["hits"][hb[i]:hb[i + 1]]], 0)).argmax()
                      for i in idx])
    a = np.nonzero(out["next"] >= 0)[0]
    assert len(a) > 3000
    assert (truth[a] == truth[out["next"][a]]).mean() > 0.99
