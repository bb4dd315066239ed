"""bench.py's use of the committed rocprofv3 summary (host logic): the HBM
traffic figure is taken only while the summary's kernel-source hash and its
views per launch match the run."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write(tmp_path, text):
    p = tmp_path / "summary.txt"
    p.write_text(text)
    return str(p)


def test_traffic_needs_matching_hash_and_views(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    good = f"kernel_source_hash: {h}\nviews_per_launch: 108\nhbm_bytes_per_launch raycast_batch: 123\n"
    monkeypatch.setattr(bench, "PROFILE", _write(tmp_path, good))
    assert bench.recorded_traffic(108) == 123.0
    assert bench.recorded_traffic(36) is None
    stale = good.replace(h, "0" * 16)
    monkeypatch.setattr(bench, "PROFILE", _write(tmp_path, stale))
    assert bench.recorded_traffic(108) is None
    no_views = f"kernel_source_hash: {h}\nhbm_bytes_per_launch raycast_batch: 123\n"
    monkeypatch.setattr(bench, "PROFILE", _write(tmp_path, no_views))
    assert bench.recorded_traffic(108) is None



def test_l2_figures_follow_the_same_rule(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    good = (f"kernel_source_hash: {h}\nviews_per_launch: 108\n"
            "hbm_bytes_per_launch raycast_batch: 123\n"
            "l2_read_bytes_per_launch raycast_batch: 4.5e10\nl2_hit_rate raycast_batch: 0.66\n")
    monkeypatch.setattr(bench, "PROFILE", _write(tmp_path, good))
    assert bench.recorded_l2(108) == (4.5e10, 0.66)
    assert bench.recorded_l2(36) == (None, None)
    monkeypatch.setattr(bench, "PROFILE", _write(tmp_path, good.replace(h, "f" * 16)))
    assert bench.recorded_l2(108) == (None, None)
    r = bench.roofline([50.0, 50.0], {op: __import__("numpy").array([[10, 4, 2, 1, 0, 0, 0, 0]])
                                       for op in bench.OPS}, 108)
    assert r["traffic"] is None and r["l2_gbs"] is None and r["hbm_gbs"] is None
    monkeypatch.setattr(bench, "PROFILE", _write(tmp_path, good))
    r = bench.roofline([50.0, 50.0], {op: __import__("numpy").array([[10, 4, 2, 1, 0, 0, 0, 0]])
                                       for op in bench.OPS}, 108)
    assert r["l2_gbs"] == round(4.5e10 / 0.05 / 1e9, 1) and r["l2_hit"] == 0.66
    assert r["hbm_gbs"] == round(123 / 0.05 / 1e9, 1)
