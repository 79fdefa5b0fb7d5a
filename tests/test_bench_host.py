"""Host-side checks of bench.py's command-line contract (no GPU)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_names_the_two_step_kernel():
    sys.path.insert(0, ROOT)
    import bench

    rec = bench.traffic_from_profiles("k_step_fused2", "rm_4096x1024")
    # either the record matches the current kernel sources (bytes per launch
    # of two steps: about the 256 B per node one step moves, plus the strips'
    # overlap) or it is null
    assert rec is None or 0.95 < rec / (256 * 4096 * 1024) < 1.25
    assert bench.traffic_from_profiles("k_step_window", "rm_4096x1024") is None
    assert bench.traffic_from_profiles("k_step_fused", "rm_4096x1024") is None
