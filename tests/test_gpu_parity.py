"""Parity of the HIP path with the oracle, through the C interface.

Decisions (links, cleaned links, start hits, tracklet cluster lists) must be
bit-identical to the float oracle; parameters, covariances and chi2 must lie
within tolerance of the FP64 replay of the same decisions (and, since both
sides evaluate the same float operations in the same order, they are expected
to equal the float oracle bit for bit as well).
"""
import numpy as np
import pytest

import oracle
import synth
from synth import geometry as G

from gpu_helpers import compare_decisions, compare_numbers, make_tracker, run_gpu

pytestmark = pytest.mark.gpu


def _full_parity(cs, tuning=None, bitwise=True):
    ref = oracle.track(cs)
    gpu = run_gpu(cs, make_tracker(tuning))
    assert gpu["status"] == 0
    assert gpu["n_start"] == len(ref["starts"])
    k, gi = compare_decisions(gpu, ref)
    rp = oracle.replay(cs, k)
    compare_numbers(gpu, gi, k, rp)
    if bitwise:
        np.testing.assert_array_equal(gpu["param"].astype(np.float64), k["param"])
        np.testing.assert_array_equal(gpu["chi2"].astype(np.float64), k["chi2"])
        np.testing.assert_array_equal(gpu["cov"].astype(np.float64), k["cov"])
    return gpu, ref


def test_single_sector_parity():
    print("case: single sector, seed 1", flush=True)
    gpu, ref = _full_parity(synth.single_sector(seed=1))
    assert len(gpu["n_hits"]) > 200


def test_central_event_parity():
    print("case: central event, seed 2 (36 sectors, ~2M clusters)", flush=True)
    gpu, ref = _full_parity(synth.central_event(seed=2))
    assert len(gpu["n_hits"]) > 30000


@pytest.mark.parametrize("nz,bin_y", [(1, 50.0), (7, 0.7), (300, 3.0)])
def test_results_do_not_depend_on_search_grid(nz, bin_y):
    import paper_2601_20569_amd as px
    print(f"case: grid nz={nz} bin_y={bin_y}", flush=True)
    t = px.default_tuning(1, 20000)
    t.n_zbins, t.bin_y = nz, bin_y
    t.construct_grid = 3
    _full_parity(synth.single_sector(seed=5), tuning=t)


def test_ragged_units_and_edge_cases():
    print("case: ragged units, empty rows, empty units", flush=True)
    cs = synth.central_event(seed=7, n_primaries=300, noise_frac=0.5)
    # drop every cluster of a few units and rows to make empty ranges
    row = cs.row_of()
    unit = cs.unit_of()
    keep = ~np.isin(unit, [0, 5, 35]) & ~((unit == 3) & (row % 7 == 0))
    cs2 = _subset(cs, keep)
    _full_parity(cs2)


def _subset(cs, keep):
    key = cs.unit_of().astype(np.int64) * G.N_ROWS + cs.row_of()
    key = key[keep]
    counts = np.bincount(key, minlength=cs.n_units * G.N_ROWS)
    rb = np.zeros(cs.n_units * G.N_ROWS + 1, np.int64)
    np.cumsum(counts, out=rb[1:])
    return synth.ClusterSet(cs.n_units, cs.unit_sector, rb, cs.y[keep], cs.z[keep],
                            cs.truth_track[keep], cs.truth_y[keep], cs.truth_z[keep],
                            cs.truth_psi[keep], cs.tracks, cs.meta)


def _doubled(cs):
    """Every cluster twice, at the same coordinates, in its own row."""
    key = cs.unit_of().astype(np.int64) * G.N_ROWS + cs.row_of()
    idx = np.concatenate([np.arange(cs.n_clusters), np.arange(cs.n_clusters)])
    idx = idx[np.argsort(np.concatenate([key, key]), kind="stable")]
    rb = cs.row_begin * 2
    return synth.ClusterSet(cs.n_units, cs.unit_sector, rb, cs.y[idx], cs.z[idx],
                            cs.truth_track[idx], cs.truth_y[idx], cs.truth_z[idx],
                            cs.truth_psi[idx], cs.tracks, cs.meta)


def _dense_row(cs, row, n_extra, seed):
    """cs with n_extra uniform noise clusters appended to (unit 0, row)."""
    rng = np.random.default_rng(seed)
    x = G.row_x()[row]
    ye = rng.uniform(-1.0, 1.0, n_extra) * x * G.tan_half_opening()
    ze = rng.uniform(-240.0, 240.0, n_extra)
    at = int(cs.row_begin[row + 1])  # after the row's own clusters
    ins = lambda a, v: np.concatenate([a[:at], v.astype(a.dtype), a[at:]])
    rb = cs.row_begin.copy()
    rb[row + 1:] += n_extra
    m = -np.ones(n_extra)
    return synth.ClusterSet(cs.n_units, cs.unit_sector, rb, ins(cs.y, ye), ins(cs.z, ze),
                            ins(cs.truth_track, m), ins(cs.truth_y, ye), ins(cs.truth_z, ze),
                            ins(cs.truth_psi, 0 * m), cs.tracks, cs.meta)


def test_row_longer_than_one_start_bitmap_segment():
    """A pad row of more than 65,536 clusters: the start-hit ordering takes
    its id range in several bitmap segments and the neighbour finder's lists
    overflow into the direct scan; results still equal the oracle's."""
    print("case: single sector seed 4, 140,000 extra clusters in row 30", flush=True)
    cs = _dense_row(synth.single_sector(seed=4), 30, 140_000, seed=4)
    assert np.diff(cs.row_begin)[30] > 2 * 65536
    gpu, ref = _full_parity(cs)
    assert len(gpu["n_hits"]) > 100
    row = cs.row_of()
    s30 = ref["starts"][row[ref["starts"]] == 30]
    # start hits in all three segments of the row's id range
    assert len(np.unique((s30 - cs.row_begin[30]) // 65536)) == 3


def test_exact_ties_between_duplicated_clusters():
    """Each cluster has a twin with the same coordinates, so every search of
    the constructor (and every neighbour choice) meets an exact tie, decided
    by the smaller caller id (Section 2.2 selection rule, ties by index)."""
    print("case: single sector seed 1, every cluster duplicated", flush=True)
    cs = _doubled(synth.single_sector(seed=1))
    gpu, ref = _full_parity(cs)
    assert len(gpu["n_hits"]) > 100
    # a row holds its clusters, then their twins: every attached cluster must
    # be from the first half of its row (the smaller id of each pair)
    k = oracle.kept_tracklets(ref)
    counts = np.diff(cs.row_begin)
    key = np.repeat(np.arange(len(counts)), counts)[k["hits"]]
    assert np.all(k["hits"] - cs.row_begin[key] < counts[key] // 2)


def test_empty_and_tiny_inputs():
    print("case: empty input", flush=True)
    cs = synth.single_sector(seed=3, n_tracks=0, noise_frac=0.0)
    assert cs.n_clusters == 0
    gpu = run_gpu(cs)
    assert gpu["n_start"] == 0 and len(gpu["n_hits"]) == 0
    print("case: one track, no noise", flush=True)
    _full_parity(synth.exact_tracks(4, n_tracks=1))
    print("case: noise only", flush=True)
    cs = synth.single_sector(seed=3, n_tracks=40, noise_frac=0.0)
    cs.y = np.random.default_rng(0).uniform(-10, 10, cs.n_clusters).astype(np.float32)
    _full_parity(cs)


def test_capacity_overflow_reports_required_sizes():
    import paper_2601_20569_amd as px
    import torch
    print("case: capacities of 1", flush=True)
    cs = synth.single_sector(seed=1)
    tr = make_tracker()
    dev = torch.device("cuda")
    rb = torch.as_tensor(cs.row_begin, device=dev)
    y = torch.as_tensor(cs.y, device=dev)
    z = torch.as_tensor(cs.z, device=dev)
    bufs = tr.allocate(cs.n_units, cs.n_clusters, cap_start=1, cap_tracks=1, cap_hits=1)
    tr.track_into(rb, y, z, cs.n_units, bufs)
    counts = bufs["out"]["counts"].cpu().numpy()
    ref = oracle.track(cs)
    k = oracle.kept_tracklets(ref)
    assert counts[3] & px.ST_START_OVERFLOW
    assert counts[0] == len(ref["starts"])
    # with one start slot only the first start hit is built
    assert counts[1] == (1 if k["start"][0] == ref["starts"][0] else 0)
    res = tr.track(rb, y, z, cs.n_units, cap_start=1, cap_tracks=1, cap_hits=1)
    assert res["status"] == 0 and len(res["n_hits"]) == len(k["n"])


def test_start_capacity_exactly_full():
    """With exactly as many start slots as start hits the constructor still
    takes its work in sorted-position order (the order list is written when
    all start hits fit); results equal the oracle's."""
    print("case: central event seed 7, start capacity = number of start hits", flush=True)
    cs = synth.central_event(seed=7, n_primaries=2000)
    ref = oracle.track(cs)
    n_start = len(ref["starts"])
    gpu = run_gpu(cs, make_tracker(), cap_start=n_start)
    assert gpu["status"] == 0 and gpu["n_start"] == n_start
    k, gi = compare_decisions(gpu, ref)
    compare_numbers(gpu, gi, k, oracle.replay(cs, k))


def test_run_twice_bitwise_identical():
    print("case: determinism", flush=True)
    cs = synth.central_event(seed=11, n_primaries=3000)
    tr = make_tracker()
    a = run_gpu(cs, tr)
    b = run_gpu(cs, tr)
    for key in ("link_up", "link_down", "starts", "hit_id", "param", "cov", "chi2"):
        np.testing.assert_array_equal(a[key], b[key])


def test_gpu_links_equal_double_oracle_on_margin_clean_input():
    """After the generator's margin step, the GPU's (float) neighbour-finder
    and cleaning decisions equal the double-precision oracle's."""
    from margins import margin_clean
    print("case: central event seed 2, margin-clean, against the double oracle", flush=True)
    cs, _, _ = margin_clean(synth.central_event(seed=2), seed=2)
    gpu = run_gpu(cs)
    ref = oracle.track(cs, precision=64, n_threads=16)
    for k in ("link_up", "link_down", "clean_up", "clean_down"):
        np.testing.assert_array_equal(gpu[k], ref[k], err_msg=k)
    np.testing.assert_array_equal(gpu["starts"], ref["starts"].astype(np.int32))


def test_non_finite_clusters_are_reported_and_join_nothing():
    """NaN and infinite coordinates: the status word carries the non-finite
    bit, and everything else equals the oracle bit for bit."""
    from types import SimpleNamespace
    cs = synth.single_sector(seed=1)
    rng = np.random.default_rng(4)
    y, z = cs.y.copy(), cs.z.copy()
    y[rng.choice(cs.n_clusters, 20, replace=False)] = np.nan
    z[rng.choice(cs.n_clusters, 20, replace=False)] = np.inf
    z[rng.choice(cs.n_clusters, 20, replace=False)] = np.nan
    bad = SimpleNamespace(n_units=1, row_begin=cs.row_begin, y=y, z=z, n_clusters=cs.n_clusters)
    print("case: single sector with 60 non-finite clusters", flush=True)
    ref = oracle.track(bad)
    gpu = run_gpu(bad, make_tracker())
    assert gpu["status"] == 8
    k, gi = compare_decisions(gpu, ref)
    np.testing.assert_array_equal(gpu["param"].astype(np.float64), k["param"])
    np.testing.assert_array_equal(gpu["chi2"].astype(np.float64), k["chi2"])
