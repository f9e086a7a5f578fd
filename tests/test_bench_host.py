"""Host logic of bench.py: the batched workloads' base lists, and the rule that
counter-measured figures (profiles/counters_<workload>.txt) are used only while
the kernel sources they were taken on are unchanged."""
import os
import shutil
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_batched_workloads_use_their_base_lists():
    assert bench.base_workload("c2x64") == "c2"
    assert bench.base_workload("c4x8") == "c4"
    for w in ("c1", "c2", "c3", "c4", "c5", "f2", "f3"):
        assert bench.base_workload(w) == w


def _tree(tmp_path):
    """A copy of the kernel sources and an empty profiles folder."""
    root = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, "paper_2008_13490_amd", "csrc"), root / "paper_2008_13490_amd" / "csrc")
    (root / "profiles").mkdir()
    return root


def test_counters_are_used_only_on_their_sources(tmp_path, monkeypatch):
    root = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    h = bench.kernel_source_hash(bench.FAMILY_SOURCE["leaf"])
    (root / "profiles" / "counters_cx.txt").write_text(
        "# a summary\n"
        f"leaf_source_hash = {h}\n"
        "leaf_fp64_flop_per_launch = 1000\n"
        "leaf_fetch_bytes_per_launch = 300\n"
        "leaf_write_bytes_per_launch = 200\n")
    assert bench.read_counters("cx", "leaf") == {"fp64_flop": 1000.0, "fetch_bytes": 300.0, "write_bytes": 200.0}
    assert bench.read_counters("cx", "trunk_fwd") is None   # no entry for that family
    assert bench.read_counters("cy", "leaf") is None        # no summary for that workload
    # a header the family's kernels include changes: the summary no longer applies
    hdr = root / "paper_2008_13490_amd" / "csrc" / "gst_device.h"
    hdr.write_text(hdr.read_text() + "\n// changed\n")
    assert bench.kernel_source_hash(bench.FAMILY_SOURCE["leaf"]) != h
    assert bench.read_counters("cx", "leaf") is None


def test_source_hash_ignores_files_the_family_does_not_include(tmp_path, monkeypatch):
    root = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    h = bench.kernel_source_hash(bench.FAMILY_SOURCE["tiles_2q"])
    other = root / "paper_2008_13490_amd" / "csrc" / "gst_predict.hip"
    other.write_text(other.read_text() + "\n// changed\n")
    assert bench.kernel_source_hash(bench.FAMILY_SOURCE["tiles_2q"]) == h


def test_with_counters_adds_rates_and_traffic():
    roof = {"avg_launch_us": 10.0, "peak": 78.6, "algorithmic_flop_per_launch": 5e8}
    out = bench.with_counters(dict(roof), {"fp64_flop": 1e9, "fetch_bytes": 3e6, "write_bytes": 1e6})
    assert abs(out["counter_tflops"] - 100.0) < 1e-9
    assert abs(out["counter_frac"] - 100.0 / 78.6) < 1e-12
    assert abs(out["counter_to_algorithmic"] - 2.0) < 1e-12
    assert out["traffic"] == 4e6 and abs(out["hbm_gbs"] - 400.0) < 1e-9
    assert bench.with_counters(dict(roof), None)["counter_flop_per_launch"] is None
