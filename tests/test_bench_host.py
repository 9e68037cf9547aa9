"""Host logic of bench.py: the counted-traffic lookup in the profile summary
must be used only while the kernel sources are the ones that were profiled."""
import hashlib
import os

import bench


def _tree(tmp_path, src_text, sha=None):
    csrc = tmp_path / "paper_2601_20569_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "a.h").write_text(src_text)
    h = hashlib.sha256(src_text.encode()).hexdigest() if sha is None else sha
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "hbm_traffic_wl.md").write_text(
        "# summary\n\n```\n"
        f"source_sha256: {h}\nworkload: wl\n"
        "traffic_bytes_per_launch k_construct: 1234\n"
        "traffic_bytes_per_launch k_neighbours: 99\n```\n")


def test_traffic_read_when_sources_match(tmp_path, monkeypatch):
    _tree(tmp_path, "kernel v1")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("construct", "wl") == 1234
    assert bench.recorded_traffic("neighbours", "wl") == 99
    # a stage whose kernels are not in the summary has no traffic
    assert bench.recorded_traffic("refit", "wl") is None
    assert bench.recorded_traffic("construct", "other") is None


def test_traffic_dropped_when_sources_changed(tmp_path, monkeypatch):
    _tree(tmp_path, "kernel v1", sha=hashlib.sha256(b"kernel v0").hexdigest())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("construct", "wl") is None


def test_committed_summary_names_every_timed_kernel():
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                        "hbm_traffic_timeframe-slice-batch.md")
    text = open(path).read()
    for stage in ("grid", "neighbours", "construct", "refit"):
        for k in bench.STAGE_KERNELS[stage]:
            assert f"traffic_bytes_per_launch {k}:" in text
