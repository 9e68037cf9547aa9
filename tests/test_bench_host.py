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


def test_valu_figures_read_only_when_sources_match(tmp_path, monkeypatch):
    _tree(tmp_path, "kernel v1")
    h = hashlib.sha256(b"kernel v1").hexdigest()
    (tmp_path / "profiles" / "valu_wl.md").write_text(
        "# summary\n\n```\n"
        f"source_sha256: {h}\n"
        "valu k_construct: per_cu_cycle=0.8 lanes=0.75 waiting=0.6 l2_hit=0.26\n```\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_valu("construct", "wl") == {
        "k_construct": {"per_cu_cycle": 0.8, "lanes": 0.75, "waiting": 0.6, "l2_hit": 0.26}}
    assert bench.recorded_valu("refit", "wl") is None
    (tmp_path / "paper_2601_20569_amd" / "csrc" / "a.h").write_text("kernel v2")
    assert bench.recorded_valu("construct", "wl") is None


def test_committed_summary_names_every_timed_kernel():
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                        "hbm_traffic_timeframe-slice-batch.md")
    text = open(path).read()
    for stage in ("grid", "neighbours", "construct", "refit"):
        for k in bench.STAGE_KERNELS[stage]:
            assert f"traffic_bytes_per_launch {k}:" in text


def test_order_rows_by_z_sorts_within_rows_only():
    import numpy as np
    import torch
    rng = np.random.default_rng(0)
    counts = np.array([5, 0, 7, 1, 9])
    rb = torch.as_tensor(np.concatenate([[0], np.cumsum(counts)]))
    y = torch.as_tensor(rng.normal(size=counts.sum()).astype(np.float32))
    z = torch.as_tensor(rng.normal(size=counts.sum()).astype(np.float32))
    y2, z2 = bench.order_rows_by_z(rb, y, z)
    for b, e in zip(rb[:-1].tolist(), rb[1:].tolist()):
        # the same (y, z) pairs in each row, now in ascending z
        want = sorted(zip(z[b:e].tolist(), y[b:e].tolist()))
        assert list(zip(z2[b:e].tolist(), y2[b:e].tolist())) == want
