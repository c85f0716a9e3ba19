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
    assert set(t) == {"family", "bytes_per_launch", "kernel_source_sha256"}
    assert t["bytes_per_launch"] is None or t["bytes_per_launch"] > 0
    # the lookup returns the stored bytes only for the family and the source they were measured on
    fam = t["family"] or "pass1"
    got = bench.measured_traffic(fam)
    assert got is None or got == t["bytes_per_launch"]
    assert bench.measured_traffic("no such family") is None
    json.dumps({"traffic": got})


def test_roofline_picks_the_dominant_family():
    sys.path.insert(0, ROOT)
    import bench

    class FakeSolver:
        def time_kernel(self, k, j, reps):
            return 0.05, 1e8

        def launch_config(self, fam, j):
            return {"grid": 2048, "block": 256, "per_cu": 8, "basis_align": 4096}

    fam = {"spmv": {"ms_per_solve": 20.0, "launches": 600, "ms_active": 19.0, "active_launches": 585,
                    "alg_bytes": 585 * 1.4e8},
           "pass1": {"ms_per_solve": 30.0, "launches": 600, "ms_active": 29.5, "active_launches": 585,
                     "alg_bytes": 585 * 2.7e8},
           "reduce": {"ms_per_solve": 40.0, "launches": 2000, "ms_active": 39.0, "active_launches": 1800,
                      "alg_bytes": 0.0}}
    rf = bench.roofline_from_profile(FakeSolver(), fam, 50, 3)
    # the latency-bound reductions take longest but move no algorithmic bytes
    assert rf["family"] == "pass1"
    assert abs(rf["achieved"] - 585 * 2.7e8 / 29.5e-3 / 1e9) < 0.1
    assert abs(rf["frac"] - rf["achieved"] / 8000.0) < 1e-4
    assert abs(rf["avg_launch_ms"] - 29.5 / 585) < 1e-5
