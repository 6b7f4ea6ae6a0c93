"""bench.py's command line on the host: it measures one GPU only and says so for more."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_counter_record_matches_the_kernel_sources():
    """The committed HBM-counter record is valid for the current propagator kernel sources, so the
    bench line reports roofline.traffic."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.counter_traffic("row_apply") is not None
    assert bench.counter_traffic("row_apply", "vector2048") is None   # taken on scalar1024 only
