"""Host-side figures of bench.py that its JSON line reports."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def test_issue_ceiling_of_the_pair_kernel():
    """The FP32 pair kernel's issue-bound ceiling: 256 CUs x 4 SIMDs x 16 lanes
    x 2.4 GHz non-packed lane-ops/s, 3 slots per ordered pair in the symmetric
    scheme at d = 1 (5 ordered), times 6 FLOP per pair."""
    import bench
    assert abs(bench.issue_ceiling_tflops(1, "symmetric") - 3.93216e13 / 3 * 6 / 1e12) < 1e-9
    assert abs(bench.issue_ceiling_tflops(1, "ordered") - 3.93216e13 / 5 * 6 / 1e12) < 1e-9
    assert abs(bench.issue_ceiling_tflops(3, "symmetric") - 3.93216e13 / 7 * 16 / 1e12) < 1e-9


def test_recorded_traffic_needs_matching_sources_and_key(tmp_path, monkeypatch):
    """traffic is reported only for the recorded tiling key and only while the
    kernel sources hash to the recorded value."""
    import json
    import bench
    rec = {"k": {"kernel_sources_sha256": bench.kernel_sources_sha256(), "hbm_bytes_per_launch": 123}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: rec["k"]["kernel_sources_sha256"])
    assert bench.recorded_traffic("k") == 123
    assert bench.recorded_traffic("other tiling") is None
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: "0" * 64)
    assert bench.recorded_traffic("k") is None


def test_cpu_baseline_line_shape():
    """The cpu_baseline object: the oracle timed on whole steps of the same
    system, with the fields the benchmark line carries."""
    import bench
    from paper_2105_09688_amd import workloads as W
    w = W.single_gpu_d1(N=512)
    out = bench.cpu_baseline(w, 0.0)
    assert out["kind"] == "oracle" and out["unit"] == "particle-steps/s"
    assert out["value"] > 0 and out["cores"] >= 1 and "1 full time steps" in out["sample"]


def test_training_snapshots_are_dense_early():
    """The surrogate's training states: every 2 ticks over the first 1/16 of
    the run, every 8 up to 1/4, every 32 after; strictly increasing, inside
    the run, 40 of them at the surrogate case's 512 ticks."""
    import bench
    s = bench.training_snapshots(512)
    assert s[:3] == [0, 2, 4] and s[15:18] == [30, 32, 40] and s[27:30] == [120, 128, 160]
    assert len(s) == 40 and s[-1] == 480
    assert all(a < b for a, b in zip(s, s[1:])) and all(0 <= t < 512 for t in s)
    assert bench.training_snapshots(16) == list(range(16))
