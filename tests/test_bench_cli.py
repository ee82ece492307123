"""Host-side behaviour of bench.py that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counter_profile_names_the_kernel_it_was_taken_on():
    import json
    sys.path.insert(0, ROOT)
    import bench
    with open(os.path.join(ROOT, "profiles", "vgc_bfs_batched16_knn10m_counters.txt")) as f:
        pc = json.load(f)
    assert len(pc["kernel_hash"]) == len(bench.kernel_source_hash()) == 16
    assert pc["hbm_bytes_per_launch"] > 0 and pc["copy_calibration"]["fetch_scale"] > 0
