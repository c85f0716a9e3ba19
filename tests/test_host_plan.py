"""The engine's host planning tables under the address and undefined-behaviour
sanitizers (CPU only).

`paper_2011_01850_amd/csrc/host_plan.cpp` holds every table that setup builds
on the host from the CSR structure (the Arnoldi product's row blocks and
canonical lane widths, the persistent passes' tile split, the ILU(0)
dependency levels, the sliced ELL layout, the size and row-pointer checks).
It is compiled here with g++ alone, together with `host_plan_check.cpp`,
which compares each table with a brute-force recomputation on seeded random
structures (empty rows, long rows, empty systems, grids larger than the tile
count) and checks the refusals.  Any wrong table, heap or stack overrun,
signed overflow or out-of-range container index fails the run.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2011_01850_amd", "csrc")
HERE = os.path.dirname(os.path.abspath(__file__))

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _build_and_run(tmp_path, flags):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_plan_check")
    cmd = [gxx, "-std=c++17", "-g", "-Wall", "-Wextra", "-Werror", "-D_GLIBCXX_ASSERTIONS", *flags,
           "-I", CSRC, os.path.join(HERE, "host_plan_check.cpp"), os.path.join(CSRC, "host_plan.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host plan checks:" in r.stdout and "passed" in r.stdout
    return r.stdout


def test_host_plan_tables_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, ["-O1", *SAN])
    assert int(out.split(":")[1].split()[0]) > 10000


def test_host_plan_tables_optimised(tmp_path):
    # the same checks at -O3 without instrumentation (the library's optimisation level)
    _build_and_run(tmp_path, ["-O3"])
