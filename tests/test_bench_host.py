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
