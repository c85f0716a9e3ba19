"""bench.py's command line on a host without a GPU: the single-GPU contract
and the record fields that do not need a device."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_is_tied_to_the_kernel_source():
    sys.path.insert(0, ROOT)
    import bench

    t = bench.TRAFFIC
    assert set(t) == {"bytes_per_launch", "kernel_source_sha256"}
    assert t["bytes_per_launch"] is None or t["bytes_per_launch"] > 0
    # the lookup returns the stored bytes only for the source they were measured on
    got = bench.measured_traffic()
    assert got is None or got == t["bytes_per_launch"]
    json.dumps({"traffic": got})
