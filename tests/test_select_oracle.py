"""Pins of the ambiguity-solving oracle (oracle.select), CPU only.

The paper (Section 2) states the step's purpose -- keep the best instance of
each track, give it the clusters, remove the clones, allow a fraction of
shared clusters -- and Section 3 (Phase I) the criteria: smaller global chi2
first, track length second, shared clusters counted from the outermost pad
row.  Pinned here without re-stating the oracle's code:
  * noise-free isolated tracks: clones collapse to exactly one tracklet per
    particle, holding every cluster of that particle in the sector;
  * hand-built tracklet lists: ranking ties, and the shared-fraction
    boundary for sharing at the inner and at the outer end;
  * brute force over every ordering on tiny random inputs: the oracle's
    selection equals the one obtained by enumerating, for each cluster, the
    tracklets that contain it, ranked by an explicit sort of tuples;
  * invariants on a tracked sector: every selected tracklet's overall shared
    fraction is within the limit and each assigned cluster belongs to a
    selected tracklet that contains it.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth


def _tracklets(spec):
    """spec: list of (unit, chi2, ndf, [cluster ids innermost first])."""
    n = np.array([len(h) for _, _, _, h in spec], np.int32)
    hb = np.zeros(len(spec) + 1, np.int64)
    np.cumsum(n, out=hb[1:])
    return dict(unit=np.array([u for u, *_ in spec], np.int32), n=n, hit_begin=hb,
                hits=np.array([c for *_, h in spec for c in h], np.int32),
                chi2=np.array([c for _, c, _, _ in spec], np.float64),
                ndf=np.array([d for _, _, d, _ in spec], np.int32))


def test_noise_free_clones_collapse_to_one_tracklet_per_particle():
    found = 0
    for seed in range(3):
        cs = synth.exact_tracks(seed=100 + seed, n_tracks=12)
        k = oracle.kept_tracklets(oracle.track(cs))
        keep, assign = oracle.select(k, cs.n_clusters)
        truth = cs.truth_track
        for t in np.nonzero(keep)[0]:
            hits = k["hits"][k["hit_begin"][t]:k["hit_begin"][t + 1]]
            p = np.unique(truth[hits])
            assert len(p) == 1 and p[0] >= 0
            # every cluster of that particle in the sector, and only those
            np.testing.assert_array_equal(np.sort(hits), np.nonzero(truth == p[0])[0])
            np.testing.assert_array_equal(assign[hits], t)
            found += 1
        owners = truth[k["hits"][np.concatenate([np.arange(k["hit_begin"][t], k["hit_begin"][t + 1])
                                                 for t in np.nonzero(keep)[0]])]]
        assert len(np.unique(owners)) == keep.sum()  # one tracklet per particle
        # clones existed and were removed
    assert found >= 20


def test_duplicated_tracklets_keep_the_better_ranked_one():
    a = list(range(0, 20))
    # equal chi2/ndf and length: the first in start order wins
    keep, assign = oracle.select(_tracklets([(0, 10.0, 35, a), (0, 10.0, 35, a)]), 40)
    assert keep.tolist() == [True, False]
    assert (assign[:20] == 0).all() and (assign[20:] == -1).all()
    # smaller chi2/ndf wins over start order
    keep, _ = oracle.select(_tracklets([(0, 10.0, 35, a), (0, 9.0, 35, a)]), 40)
    assert keep.tolist() == [False, True]
    # equal chi2/ndf: the longer one wins (6/15 == 10/25 exactly in float)
    b = list(range(0, 15))
    keep, _ = oracle.select(_tracklets([(0, 6.0, 15, b), (0, 10.0, 25, a)]), 40)
    assert keep.tolist() == [False, True]
    # a tie only breaks by order inside one unit: two units are independent
    keep, _ = oracle.select(_tracklets([(0, 10.0, 35, a), (1, 10.0, 35, list(range(20, 40)))]), 40)
    assert keep.tolist() == [True, True]


@pytest.mark.parametrize("frac,limit", [((1, 10), 2), ((1, 5), 4)])
def test_shared_fraction_boundary_inner_and_outer_end(frac, limit):
    a = list(range(100, 120))  # the better track, 20 clusters
    # the second track shares m clusters at its inner end (its first clusters)
    for m in range(limit + 2):
        b = a[:m] + list(range(200, 200 + 20 - m))
        keep, assign = oracle.select(_tracklets([(0, 1.0, 35, a), (0, 2.0, 35, b)]), 300, shared=frac)
        assert keep[0]
        assert keep[1] == (m <= limit), (m, keep)
    # one shared cluster at the outer end: counted first, over the limit at once
    b = list(range(200, 219)) + [a[-1]]
    keep, _ = oracle.select(_tracklets([(0, 1.0, 35, a), (0, 2.0, 35, b)]), 300, shared=frac)
    assert keep.tolist() == [True, False]


def test_against_brute_force_on_tiny_inputs():
    rng = np.random.default_rng(7)
    for _ in range(300):
        n_cl = int(rng.integers(5, 25))
        n_tr = int(rng.integers(1, 7))
        spec = []
        for t in range(n_tr):
            size = int(rng.integers(1, min(n_cl, 12) + 1))
            hits = sorted(rng.choice(n_cl, size, replace=False).tolist())
            chi2 = float(rng.choice([1.0, 2.0, 3.0, 4.5]))  # ties on purpose
            spec.append((int(rng.integers(0, 2)), chi2, int(rng.choice([5, 7, 9])), hits))
        spec.sort(key=lambda s: s[0])  # units contiguous
        frac = [(1, 10), (1, 5), (1, 3), (1, 2)][int(rng.integers(0, 4))]
        keep, assign = oracle.select(_tracklets(spec), n_cl, shared=frac)
        # brute force: rank by an explicit tuple sort, per cluster take the
        # best-ranked container, then test every outer prefix
        pos_in_unit = [sum(1 for s in spec[:i] if s[0] == spec[i][0]) for i in range(n_tr)]
        rank = sorted(range(n_tr), key=lambda i: (np.float32(spec[i][1]) / np.float32(spec[i][2]),
                                                  -len(spec[i][3]), pos_in_unit[i]))
        pos = {t: r for r, t in enumerate(rank)}
        owner = {}
        for t in range(n_tr):
            for c in spec[t][3]:
                if c not in owner or pos[t] < pos[owner[c]]:
                    owner[c] = t
        want = []
        for t in range(n_tr):
            hits = spec[t][3][::-1]
            ok = all(sum(owner[c] != t for c in hits[:k]) * frac[1] <= frac[0] * k
                     for k in range(1, len(hits) + 1))
            want.append(ok)
        assert keep.tolist() == want, (spec, frac)
        best = {}
        for t in rank:
            if want[t]:
                for c in spec[t][3]:
                    best.setdefault(c, t)
        np.testing.assert_array_equal(assign, [best.get(c, -1) for c in range(n_cl)])


def test_invariants_on_a_tracked_sector():
    cs = synth.single_sector(seed=1)
    k = oracle.kept_tracklets(oracle.track(cs))
    for frac in ((1, 10), (1, 5)):
        keep, assign = oracle.select(k, cs.n_clusters, shared=frac)
        assert 0 < keep.sum() < len(keep)
        for t in np.nonzero(keep)[0]:
            hits = k["hits"][k["hit_begin"][t]:k["hit_begin"][t + 1]]
            shared = (assign[hits] != t).sum()
            assert shared * frac[1] <= frac[0] * len(hits)
        sel = np.nonzero(assign >= 0)[0]
        for c in sel[::50]:
            t = assign[c]
            assert keep[t] and c in k["hits"][k["hit_begin"][t]:k["hit_begin"][t + 1]]
