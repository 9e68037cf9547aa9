"""Float against double decisions on margin-clean inputs (CPU, oracle).

The generator's margin-rejection step (tests/margins.py) re-draws every cluster
whose decision lies within 1e-5 of a threshold in double.  On the inputs it
leaves, the float and double instances of the oracle take the same
decisions: links, cleaned links, start hits and every tracklet's clusters agree
exactly (the step covers the neighbour finder's windows, D cut and gaps, the
constructor's chi2 cut and gaps, and the propagation guards on sin(phi) and
the chord).  Without the step the double and float links of the central event
differ (the control case below).
"""
import numpy as np

import oracle
import synth

from margins import margin_clean


def _compare(cs):
    a = oracle.track(cs, precision=32, n_threads=8)
    b = oracle.track(cs, precision=64, n_threads=8)
    return a, b


def test_margin_step_makes_float_and_double_decisions_agree_single_sector():
    cs, rounds, n = margin_clean(synth.single_sector(seed=1), seed=1)
    assert rounds <= 10 and not oracle.nf_margins(cs, constructor=True).any()
    a, b = _compare(cs)
    for k in ("link_up", "link_down", "clean_up", "clean_down", "starts"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    ka, kb = oracle.kept_tracklets(a), oracle.kept_tracklets(b)
    np.testing.assert_array_equal(ka["n"], kb["n"])
    np.testing.assert_array_equal(ka["hits"], kb["hits"])


def test_margin_step_on_central_event():
    raw = synth.central_event(seed=2)
    a, b = _compare(raw)
    raw_diff = sum(int((a[k] != b[k]).sum()) for k in ("link_up", "link_down"))
    assert raw_diff > 0  # control: without the step the decisions differ
    cs, rounds, n = margin_clean(synth.central_event(seed=2), seed=2)
    print(f"re-drawn {n} of {cs.n_clusters} clusters in {rounds} rounds")
    a, b = _compare(cs)
    for k in ("link_up", "link_down", "clean_up", "clean_down", "starts"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    ka, kb = oracle.kept_tracklets(a), oracle.kept_tracklets(b)
    np.testing.assert_array_equal(ka["start"], kb["start"])
    np.testing.assert_array_equal(ka["n"], kb["n"])
    np.testing.assert_array_equal(ka["hits"], kb["hits"])
    np.testing.assert_array_equal(ka["rows"], kb["rows"])
