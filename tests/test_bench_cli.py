"""bench.py's command line on a host without a GPU: the single-GPU contract
and the record fields that do not need a device."""
import hashlib
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
    assert all(b > 0 for b in t["bytes_per_launch"].values())
    # the lookup returns the stored bytes only for a kernel measured on this source
    with open(bench.KERNEL_SOURCE, "rb") as f:
        current = hashlib.sha256(f.read()).hexdigest() == t["kernel_source_sha256"]
    for k, b in t["bytes_per_launch"].items():
        assert bench.measured_traffic(k) == (b if current else None)
    assert bench.measured_traffic("no such kernel") is None
    json.dumps({"traffic": bench.measured_traffic("k_mdot<float, float, 64>")})


def test_tile_widths_follow_the_column():
    sys.path.insert(0, ROOT)
    import bench

    assert [bench.tile_width(j) for j in (0, 7, 8, 15, 16, 31, 32, 49, 63, 64, 200)] == \
        [8, 8, 16, 16, 32, 32, 64, 64, 64, 64, 64]
    units = bench.kernel_units("pass1", 50, "fp32", "cgsr")
    assert [u[0] for u in units] == [f"k_mdot<float, float, {L}>" for L in (8, 16, 32, 64)]
    assert sum(len(c) for _, c in units) == 50 and units[3][1] == list(range(32, 50))
    assert bench.kernel_units("pass2", 50, "fp64", "cgsr")[0][0].startswith("k_axpy_mdot64<double, double")
    assert bench.kernel_units("final", 40, "fp32", "mgs") == [("k_mgs_final<float, float>", list(range(40)))]
    sell = {"format": "sell", "block_nnz": 2048, "xcd_remap": True}
    assert bench.kernel_units("spmv", 50, "fp32", "cgsr", sell) == [("k_sell<float, float, float, 0, false>",
                                                                     list(range(50)))]
    sell16 = dict(sell, format="sell16")
    assert bench.kernel_units("spmv", 50, "fp32", "cgsr", sell16)[0][0] == "k_sell<float, float, float, 0, true>"
    # the finaliser merged into the product: the first two projections run their _ds kernels
    merged = dict(sell16, fin_merged=True)
    assert bench.kernel_units("pass1", 50, "fp32", "cgsr", merged)[3][0] == "k_mdot_ds<float, float, 64>"
    assert bench.kernel_units("pass2", 50, "fp64", "cgsr", merged)[0][0].startswith("k_axpy_mdot64_ds<double, double")
    assert bench.kernel_units("pass2", 50, "fp32", "cgsr", merged)[3][0] == "k_axpy_mdot_ds<float, float, 64>"
    assert bench.kernel_units("final", 50, "fp32", "cgsr", merged)[3][0] == "k_final_tile<float, float, 64>"
    csr = dict(sell, format="csr")
    assert bench.kernel_units("spmv", 50, "fp64", "cgsr", csr)[0][0] == "k_spmv<double, double, double, 0>"
    assert bench.kernel_units("spmv", 50, "limited", "cgsr", csr)[0][0] == "k_spmv<float, float, double, 0>"


def _fam_entry(ms, launches, act, byts, m=50, cols=None):
    cols = cols or range(m)
    by_col = [{"ms": 0.0, "launches": 0, "ms_active": 0.0, "active": 0, "bytes": 0.0} for _ in range(m)]
    for j in cols:
        by_col[j] = {"ms": ms / len(cols), "launches": launches // len(cols), "ms_active": 0.95 * ms / len(cols),
                     "active": act // len(cols), "bytes": byts / len(cols)}
    return {"ms_per_solve": ms, "launches": launches, "ms_active": 0.95 * ms, "active_launches": act,
            "alg_bytes": byts, "by_col": by_col}


def test_roofline_picks_the_dominant_kernel():
    sys.path.insert(0, ROOT)
    import bench

    class FakeSolver:
        def time_kernel(self, k, j, reps):
            return 0.05, 1e8

        def launch_config(self, fam, j):
            return {"grid": 1024, "block": 256, "per_cu": 4, "basis_align": 2 ** 21}

    fam = {"spmv": _fam_entry(20.0, 650, 600, 600 * 1.4e8),
           "pass1": _fam_entry(30.0, 650, 600, 600 * 2.7e8, cols=range(32, 50)),
           "reduce": {"ms_per_solve": 40.0, "launches": 2000, "ms_active": 39.0, "active_launches": 1800,
                      "alg_bytes": 0.0, "by_col": []}}
    harness = bench.harness_times(FakeSolver(), 50, 3, families=("spmv", "pass1"))
    rf = bench.roofline_from_profile(FakeSolver(), fam, 50, 3, harness=harness)
    # the latency-bound reductions take longest but move no algorithmic bytes
    assert rf["family"] == "pass1" and rf["kernel"] == "k_mdot<float, float, 64>"
    per = 600 // 18 * 18  # launches the fake table spreads over columns 32..49
    assert abs(rf["achieved"] - 600 * 2.7e8 / 28.5e-3 / 1e9) < 0.5 and rf["avg_launch_ms"] == round(28.5 / per, 5)
    assert abs(rf["frac"] - rf["achieved"] / 8000.0) < 1e-4
    assert "reduce" in rf["in_solve_families"] and rf["harness_back_to_back"]["j"] == 49
    original = bench.measured_traffic
    try:
        # no counter record for this kernel: no traffic, and no rate from it
        bench.measured_traffic = lambda k: None
        rf = bench.roofline_from_profile(FakeSolver(), fam, 50, 3, harness=harness)
        assert rf["traffic"] is None and rf["traffic_GBps"] is None and rf["traffic_frac"] is None
        # with one, the measured rate is the measured bytes over the same launch time
        bench.measured_traffic = lambda k: 2.0e8 if k == "k_mdot<float, float, 64>" else None
        rf = bench.roofline_from_profile(FakeSolver(), fam, 50, 3, harness=harness)
        assert rf["traffic"] == 2.0e8 and abs(rf["traffic_over_alg"] - 2.0e8 / (600 * 2.7e8 / per)) < 1e-3
        assert abs(rf["traffic_GBps"] - 2.0e8 / (rf["avg_launch_ms"] * 1e-3) / 1e9) < 0.1
        assert abs(rf["traffic_frac"] - rf["traffic_GBps"] / 8000.0) < 1e-4
    finally:
        bench.measured_traffic = original
