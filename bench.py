#!/usr/bin/env python3
"""Time to a 1e-10 relative residual: mixed-precision vs float64 restarted GMRES on one GPU.

Workload: 3-D convection-diffusion on a 128^3 grid (n = 2,097,152 rows,
14,581,760 non-zeros, 7-point first-order upwind stencil, beta = (50, 20,
10)), b = A x_true with x_true ~ U[-1, 1], x0 = 0, GMRES(50) with CGSR (or
MGS), float32 Arnoldi with float64 residual and update.  One step = one
time-to-solution: gmres_create (matrix copies, float32 copy, SpMV row
blocks and autotuning, workspace) + gmres_solve to 1e-10, inputs already
resident in HBM.  The float64 solver is timed the same way for the speedup.

Also reported, on the same JSON line:
  roofline      achieved HBM bandwidth of the dominant kernel (the fused
                second CGS projection at its 64-column tile width, launches
                j = 31..49 of a cycle, timed with HIP events on the solver's
                stream) against the 8 TB/s peak;
  cpu_baseline  the CPU oracle on a bounded sample of the same system.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to 1e-10 rel. residual: mixed/learned vs FP64 GMRES; HBM GB/s"
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the roofline kernel, from two rocprofv3 counter runs
# of this script (FETCH_SIZE, then WRITE_SIZE, each scaled by what it reads
# for a plain 1 GiB device copy: x2.0 and x1.0), averaged over the roofline
# launches.  Valid only for the kernel source they were taken from.
TRAFFIC = {"bytes_per_launch": 346543305, "kernel_source_sha256": "9f604e3b53c3b7acc9c068a9543cba3f9690106ff4882a681d85516800440d31"}
KERNEL_SOURCE = os.path.join(ROOT, "paper_2011_01850_amd", "csrc", "gmres_kernels.hip")


def measured_traffic():
    if TRAFFIC["bytes_per_launch"] is None:
        return None
    with open(KERNEL_SOURCE, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != TRAFFIC["kernel_source_sha256"]:
            return None  # the kernels changed since the counters were taken
    return TRAFFIC["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="convdiff3d",
                    choices=["convdiff3d", "powerlaw", "batch", "learned", "restart", "variables"],
                    help="convdiff3d: the headline time-to-solution (default); powerlaw: the n = 1e6 "
                         "power-law system in every precision mode; batch: 512 uneven 2-D systems in one handle; "
                         "learned: train the sparse-approximate-inverse network on the GPU, then FGMRES on "
                         "held-out variable-coefficient systems; restart: restart strategies; variables: "
                         "the per-variable precision study (one correction variable in float32 at a time)")
    ap.add_argument("--train-instances", type=int, default=2000)
    ap.add_argument("--test-instances", type=int, default=200)
    ap.add_argument("--baseline-instances", type=int, default=20,
                    help="held-out instances also solved without preconditioner (float32 and float64)")
    ap.add_argument("--epochs", type=float, default=2.0)
    ap.add_argument("--learned-N", type=int, default=64)
    ap.add_argument("--steps", type=int, default=5, help="timed steps (5, with their median, min and max, as the paper times)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=128, help="grid side (128 is the benchmark workload)")
    ap.add_argument("--ortho", default="cgsr", choices=["cgsr", "mgs"])
    ap.add_argument("--precision", default=None, choices=["fp32", "bf16", "fp16"],
                    help="mixed mode timed as `value` (default fp32; bf16 for powerlaw)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 baseline")
    ap.add_argument("--modes", default="fp64,fp32,bf16,fp16",
                    help="powerlaw: comma-separated precision modes to run (fp64 is always run first)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--roofline-reps", type=int, default=10)
    ap.add_argument("--cpu-iters", type=int, default=20, help="oracle sample: inner iterations")
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with a plain 1 GiB device copy (reference kernel for HBM byte counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_to_solution(torch, Solver, A_dev, b_dev, n, m, ortho, precision, steps, warmup, stall_cycles=10,
                     a_storage="copy"):
    rp, ci, va = A_dev
    times, infos = [], []
    last = None
    for it in range(warmup + steps):
        if last is not None:  # the previous step's handle is released before this step starts
            last[0].close()
            last = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = Solver(rp, ci, va, m=m, ortho=ortho, precision=precision, tol=1e-10, max_iters=100_000,
                   stall_cycles=stall_cycles, a_storage=a_storage)
        x, info = s.solve(b_dev)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        info["setup_seconds"] = dt - info["seconds"]
        if it >= warmup:
            times.append(dt)
            infos.append(info)
        log(f"  {precision:5s} {'warm' if it < warmup else 'step'} {it}: {dt * 1e3:8.2f} ms "
            f"(solve {info['seconds'] * 1e3:.2f} ms) iters {info['iters']} restarts {info['restarts']} "
            f"relres {info['rel_residual']:.3e} {info['status']}")
        last = (s, x)
    return times, infos, last


def roofline(solver, m, reps):
    """Dominant kernel: fused CGS projection 2 at its 64-column tile (j = 31..m-1).

    For each column j the library launches the kernel once untimed, then
    `reps` times back to back between two HIP events on the solver's stream;
    the timed launches sit in a ROCTx range named "timed:k_axpy_mdot(cgs pass
    2)", which `rocprofv3 --marker-trace --kernel-rename` reports as one row.
    """
    js = list(range(min(31, m - 1), m))
    t_ms, byts = [], []
    for j in js:
        ms, by = solver.time_kernel(2, j, reps)
        t_ms.append(ms)
        byts.append(by)
    avg_ms = sum(t_ms) / len(t_ms)
    avg_bytes = sum(byts) / len(byts)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    # the rest of the step's kernels at the last column, for the report
    other = {}
    for k, name in [(0, "spmv_arnoldi"), (1, "cgs_pass1"), (3, "final_pass"), (5, "residual64"), (6, "update64"),
                    (7, "finalize_pass2")]:
        ms, by = solver.time_kernel(k, m - 1, reps)
        other[name] = {"ms": round(ms, 5), "GB/s": round(by / (ms * 1e-3) / 1e9, 1)}
    return {
        "bound": "hbm",
        "kernel": "k_axpy_mdot<float,float,64> (CGS projection 2, fused w -= V h1 and V^T w)",
        "achieved": round(achieved, 1),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4),
        "traffic": traffic,
        "traffic_over_alg": (round(traffic / avg_bytes, 4) if traffic else None),
        "avg_launch_ms": round(avg_ms, 5),
        "alg_bytes_per_launch": avg_bytes,
        "launches": f"j = {js[0]}..{js[-1]}, {reps} timed back-to-back launches each (after 1 untimed)",
        "other_kernels_at_j_last": other,
    }


def cpu_baseline(pr, m, ortho, iters_ref, sample_iters):
    import numpy as np  # noqa: F401

    from oracle import gmres as O

    try:
        from threadpoolctl import threadpool_info

        blas = [d.get("num_threads") for d in threadpool_info() if d.get("user_api") == "blas"]
        threads = max(blas) if blas else 1
    except Exception:  # pragma: no cover
        threads = 1
    A = O.Matrix.from_csr(pr.A)
    t0 = time.perf_counter()
    r = O.gmres(A, pr.b, m=m, tol=1e-10, max_iters=sample_iters, ortho=ortho)
    dt = time.perf_counter() - t0
    per_iter = dt / max(1, r.iters)
    return {
        "value": round(per_iter * iters_ref, 3),
        "unit": "s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"first {r.iters} inner iterations (+2 float64 residuals) of the float64 {ortho.upper()} "
                   f"oracle on the same system took {dt:.2f} s; value = that per-iteration cost x the "
                   f"{iters_ref} iterations the GPU float64 solve needed (a lower bound: later iterations "
                   f"of a cycle orthogonalise against more vectors)"),
        "host_cpus": len(os.sched_getaffinity(0)),
        "cpu_model": _cpu_model(),
        "threads_note": "the oracle is NumPy: single-threaded except the BLAS calls of the CGS projections",
    }


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_convdiff3d(args):
    import numpy as np
    import torch

    import problems as P
    from paper_2011_01850_amd import Solver

    args.precision = args.precision or "fp32"
    m = 50
    log(f"generating 3-D convection-diffusion N={args.N} ...")
    pr = P.c2_convdiff3d(args.N)
    A = pr.A
    A_dev = tuple(torch.as_tensor(v, device="cuda") for v in (A.row_ptr, A.col_idx, A.vals))
    b_dev = torch.as_tensor(pr.b, device="cuda")
    torch.cuda.synchronize()
    log(f"n = {A.n:,}, nnz = {A.nnz:,}; mixed {args.precision} {args.ortho}")
    t_mix, i_mix, (solver, x) = time_to_solution(torch, Solver, A_dev, b_dev, A.n, m, args.ortho, args.precision,
                                                 args.steps, args.warmup)
    xs = x.cpu().numpy()
    fwd = float(np.linalg.norm(xs - pr.x_true) / np.linalg.norm(pr.x_true))
    rf = roofline(solver, m, args.roofline_reps) if args.ortho == "cgsr" else None
    mem_mixed = solver.memory_bytes()
    solver.close()
    out_fp64 = None
    if not args.no_fp64:
        t64, i64, (s64, _) = time_to_solution(torch, Solver, A_dev, b_dev, A.n, m, args.ortho, "fp64",
                                              args.steps, max(0, min(args.warmup, 1)))
        out_fp64 = {"seconds": statistics.mean(t64), "median": statistics.median(t64), "iters": i64[-1]["iters"],
                    "restarts": i64[-1]["restarts"], "rel_residual": i64[-1]["rel_residual"],
                    "memory_bytes": s64.memory_bytes()}
        s64.close()
    # split storage of A (high and low words; the Arnoldi product reads the
    # high words): the same solve without the float32 copy of the matrix
    log("split storage of A ...")
    t_sp, i_sp, (s_sp, x_sp) = time_to_solution(torch, Solver, A_dev, b_dev, A.n, m, args.ortho, args.precision,
                                                args.steps, min(args.warmup, 1), a_storage="split")
    out_split = {"seconds_mean": statistics.mean(t_sp), "seconds_median": statistics.median(t_sp),
                 "solve_seconds": i_sp[-1]["seconds"], "iters": i_sp[-1]["iters"],
                 "restarts": i_sp[-1]["restarts"], "rel_residual": i_sp[-1]["rel_residual"],
                 "forward_error": float(np.linalg.norm(x_sp.cpu().numpy() - pr.x_true) / np.linalg.norm(pr.x_true)),
                 "memory_bytes": s_sp.memory_bytes()}
    s_sp.close()
    # the limited mixed solver of the convergence study: float32 storage of
    # the Arnoldi copy of A and of the basis only, w and its dots float64
    log("limited mixed precision ...")
    t_li, i_li, (s_li, x_li) = time_to_solution(torch, Solver, A_dev, b_dev, A.n, m, args.ortho, "limited",
                                                args.steps, min(args.warmup, 1))
    out_limited = {"seconds_mean": statistics.mean(t_li), "seconds_median": statistics.median(t_li),
                   "solve_seconds": i_li[-1]["seconds"], "iters": i_li[-1]["iters"],
                   "restarts": i_li[-1]["restarts"], "rel_residual": i_li[-1]["rel_residual"],
                   "forward_error": float(np.linalg.norm(x_li.cpu().numpy() - pr.x_true)
                                          / np.linalg.norm(pr.x_true)),
                   "memory_bytes": s_li.memory_bytes()}
    s_li.close()
    # the 2-byte basis (IEEE half plus a power-of-two scale per vector) on the same system
    out_half = None
    if args.precision == "fp32":
        log("half-precision basis ...")
        t_h, i_h, (s_h, x_h) = time_to_solution(torch, Solver, A_dev, b_dev, A.n, m, args.ortho, "fp16",
                                                  args.steps, min(args.warmup, 1))
        out_half = {"seconds_mean": statistics.mean(t_h), "seconds_median": statistics.median(t_h),
                    "solve_seconds": i_h[-1]["seconds"], "iters": i_h[-1]["iters"],
                    "restarts": i_h[-1]["restarts"], "rel_residual": i_h[-1]["rel_residual"],
                    "forward_error": float(np.linalg.norm(x_h.cpu().numpy() - pr.x_true)
                                           / np.linalg.norm(pr.x_true)),
                    "memory_bytes": s_h.memory_bytes()}
        s_h.close()
    value = statistics.mean(t_mix)
    rec = {
        "metric": METRIC,
        "value": round(value, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(value * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "fp32" else f"{args.precision}+f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"3-D convection-diffusion {args.N}^3 (n={A.n}, nnz={A.nnz}), beta=(50,20,10), "
                        f"GMRES({m}) {args.ortho.upper()}, {args.precision} Arnoldi + fp64 residual/update, "
                        f"tol 1e-10, time incl. setup",
            "n": A.n, "nnz": A.nnz, "m": m, "ortho": args.ortho, "precision": args.precision,
        },
        "mixed": {"seconds_mean": value, "seconds_median": statistics.median(t_mix),
                  "seconds_min": min(t_mix), "seconds_max": max(t_mix),
                  "solve_seconds": i_mix[-1]["seconds"], "setup_seconds": i_mix[-1]["setup_seconds"],
                  "iters": i_mix[-1]["iters"], "restarts": i_mix[-1]["restarts"],
                  "rel_residual": i_mix[-1]["rel_residual"], "forward_error": fwd,
                  "memory_bytes": mem_mixed},
        "fp64": out_fp64,
        "split_storage": out_split,
        "limited": out_limited,
        "half_basis": out_half,
        "speedup_vs_fp64": (round(out_fp64["seconds"] / value, 3) if out_fp64 else None),
        "paper_context": "paper (2x10-core Haswell, Kokkos/MKL, ILU(0), SuiteSparse): mixed vs FP64 "
                         "geo-mean speedup +19% (MGS), +24% (CGSR) when restarted at least once",
        "roofline": rf,
    }
    if not args.no_cpu:
        iters_ref = out_fp64["iters"] if out_fp64 else i_mix[-1]["iters"]
        log("CPU oracle sample ...")
        rec["cpu_baseline"] = cpu_baseline(pr, m, args.ortho, iters_ref, args.cpu_iters)
    else:
        rec["cpu_baseline"] = None
    return rec


def _mode_summary(times, infos, fwd, mem):
    return {"seconds_mean": statistics.mean(times), "seconds_median": statistics.median(times),
            "seconds_min": min(times), "seconds_max": max(times),
            "solve_seconds": infos[-1]["seconds"], "setup_seconds": infos[-1]["setup_seconds"],
            "iters": infos[-1]["iters"], "restarts": infos[-1]["restarts"], "status": infos[-1]["status"],
            "rel_residual": infos[-1]["rel_residual"], "forward_error": fwd, "memory_bytes": mem}


def bench_powerlaw(args):
    """n = 1e6 power-law system, GMRES(30) CGSR, every precision mode."""
    import numpy as np
    import torch

    import problems as P
    from paper_2011_01850_amd import Solver

    value_mode = args.precision or "fp16"
    m = 30
    log("generating the power-law system n = 1e6 ...")
    pr = P.c3_powerlaw()
    A = pr.A
    A_dev = tuple(torch.as_tensor(v, device="cuda") for v in (A.row_ptr, A.col_idx, A.vals))
    b_dev = torch.as_tensor(pr.b, device="cuda")
    torch.cuda.synchronize()
    log(f"n = {A.n:,}, nnz = {A.nnz:,}; CGSR GMRES({m})")
    modes, kern = {}, {}
    # the bfloat16 basis makes the per-cycle progress noisy on this matrix
    # (dozens of cycles can pass between new lowest residuals), so the
    # no-progress stop is set far out for every mode
    stall = 1000
    run_modes = ["fp64"] + [md for md in ["fp32", "bf16", "fp16"] if md in args.modes.split(",")]
    if value_mode not in run_modes:
        raise SystemExit(f"--precision {value_mode} is not among --modes {args.modes}")
    for mode in run_modes:
        t, inf, (s, x) = time_to_solution(torch, Solver, A_dev, b_dev, A.n, m, args.ortho, mode,
                                          args.steps, args.warmup, stall_cycles=stall)
        xs = x.cpu().numpy()
        fwd = float(np.linalg.norm(xs - pr.x_true) / np.linalg.norm(pr.x_true))
        modes[mode] = _mode_summary(t, inf, fwd, s.memory_bytes())
        ks = {}
        for k, name in [(0, "spmv_arnoldi"), (1, "cgs_pass1"), (2, "cgs_pass2"), (3, "final_pass")]:
            ms, by = s.time_kernel(k, m - 1, args.roofline_reps)
            ks[name] = {"ms": round(ms, 5), "alg_bytes": by, "GB/s": round(by / (ms * 1e-3) / 1e9, 1)}
        kern[mode] = ks
        s.close()
    for mode in modes:
        modes[mode]["speedup_vs_fp64"] = round(modes["fp64"]["seconds_mean"] / modes[mode]["seconds_mean"], 3)
    v = modes[value_mode]["seconds_mean"]
    sp = kern[value_mode]["spmv_arnoldi"]
    rec = {
        "metric": METRIC, "value": round(v, 6), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(v * 1e3, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": f"{value_mode}+f32+f64" if value_mode != "fp32" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"power-law random sparse n={A.n}, nnz={A.nnz} (row lengths alpha=2.1, mean 20, "
                               f"max 2000, a_ii = 1.2 sum|a_ij|), GMRES({m}) {args.ortho.upper()}, {value_mode} "
                               f"basis, fp32 arithmetic, fp64 residual/update, tol 1e-10, time incl. setup, "
                               f"stall stop after {stall} cycles without a new lowest residual",
                   "n": A.n, "nnz": A.nnz, "m": m, "ortho": args.ortho, "precision": value_mode},
        "modes": modes,
        "kernels_at_j_last": kern,
        "roofline": {"bound": "hbm", "kernel": f"k_spmv (Arnoldi SpMV, float32 A, {value_mode} x)",
                     "achieved": sp["GB/s"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(sp["GB/s"] / PEAK_HBM_GBS, 4), "traffic": None,
                     "avg_launch_ms": sp["ms"], "alg_bytes_per_launch": sp["alg_bytes"]},
    }
    if not args.no_cpu:
        log("CPU oracle sample ...")
        rec["cpu_baseline"] = cpu_baseline(pr, m, args.ortho, modes["fp64"]["iters"], args.cpu_iters)
    else:
        rec["cpu_baseline"] = None
    return rec


def bench_variables(args):
    """Per-variable precision study (section 4.1): a 2-D convection-diffusion
    system of the size of the paper's airfoil_2d matrix, GMRES(256) (the
    longest cycle the library takes; the paper restarts every 300), with the
    correction's variables in float32 one at a time, then together."""
    import numpy as np
    import torch

    import problems as P
    from paper_2011_01850_amd import Solver

    N, m = 119, 256
    A = P.convdiff(N, (100.0, 50.0))
    x_true, b = P.manufactured_rhs(A, 21, 0)
    A_dev = tuple(torch.as_tensor(v, device="cuda") for v in (A.row_ptr, A.col_idx, A.vals))
    b_dev = torch.as_tensor(b, device="cuda")
    torch.cuda.synchronize()
    cases = [("none", "fp64", "default"), ("A (Krylov product)", "fp64", "fp32"),
             ("basis V", "limited", "fp64"), ("A, M, V (limited solver)", "limited", "default"),
             ("every correction variable", "fp32", "default")]
    rows = {}
    rp, ci, va = A_dev
    for ortho in ("mgs", "cgsr"):
        for label, prec, arnoldi_a in cases:
            times, info, hist = [], None, None
            for it in range(args.warmup + args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s = Solver(rp, ci, va, m=m, ortho=ortho, precision=prec, tol=1e-10, max_iters=100_000,
                           arnoldi_a=arnoldi_a)
                x, info = s.solve(b_dev)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                hist = s.history()
                s.close()
                if it >= args.warmup:
                    times.append(dt)
            fwd = float(np.linalg.norm(x.cpu().numpy() - x_true) / np.linalg.norm(x_true))
            key = f"{ortho}:{label}"
            rows[key] = {"precision": prec, "arnoldi_a": arnoldi_a, "seconds_mean": statistics.mean(times),
                         "iters": info["iters"], "restarts": info["restarts"], "status": info["status"],
                         "first_stall": info["first_stall"], "rel_residual": info["rel_residual"],
                         "restart_residuals": [float(h) for h in hist], "forward_error": fwd}
            log(f"  {key:40s} {statistics.mean(times) * 1e3:8.2f} ms iters {info['iters']} restarts "
                f"{info['restarts']} first stall {info['first_stall']} residuals "
                + " ".join(f"{h:.1e}" for h in hist))
    v = rows["cgsr:A, M, V (limited solver)"]["seconds_mean"]
    return {
        "metric": METRIC, "value": round(v, 6), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(v * 1e3, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"2-D convection-diffusion {N}^2 (n={A.n}, nnz={A.nnz}), beta=(100,50), "
                               f"GMRES({m}) MGS and CGSR with one correction variable in float32 at a time "
                               f"(value: the limited solver, CGSR), tol 1e-10, time incl. setup",
                   "n": A.n, "nnz": A.nnz, "m": m},
        "cases": rows, "roofline": None, "cpu_baseline": None,
    }


def bench_restart(args):
    """Restart strategies on a well-conditioned 3-D convection-diffusion
    system (the C2 operator plus a diagonal shift), MGS GMRES(64): float64
    GMRES converges within one short cycle, float32 Arnoldi stalls long
    before j = m unless a trigger restarts it."""
    import numpy as np
    import torch

    import problems as P
    from paper_2011_01850_amd import Solver

    log(f"generating the shifted 3-D convection-diffusion system N={args.N} ...")
    pr = P.restart_study_3d(args.N)
    A = pr.A
    m = 64
    A_dev = tuple(torch.as_tensor(v, device="cuda") for v in (A.row_ptr, A.col_idx, A.vals))
    b_dev = torch.as_tensor(pr.b, device="cuda")
    torch.cuda.synchronize()
    strategies = [
        ("fp64", "fp64", {}),
        ("fp32", "fp32", {}),
        ("fp32_stall", "fp32", {"restart_on_stall": True}),
        ("fp32_two_stage", "fp32", {"restart_improve": 1e-6, "restart_repeat": True}),
        ("fp32_improve", "fp32", {"restart_improve": 1e-6}),
        ("fp32_orth_spectral", "fp32", {"orth_restart": 0.5, "orth_norm": "spectral"}),
        ("fp32_orth_frobenius", "fp32", {"orth_restart": 0.5, "orth_norm": "frobenius"}),
        # the limited mixed solver (float32 storage of A, M and the basis only)
        ("limited", "limited", {}),
        ("limited_stall", "limited", {"restart_on_stall": True}),
    ]
    modes = {}
    rp, ci, va = A_dev
    for name, prec, kw in strategies:
        times, info = [], None
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s = Solver(rp, ci, va, m=m, ortho="mgs", precision=prec, tol=1e-10, max_iters=100_000, **kw)
            x, info = s.solve(b_dev)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            s.close()
            if it >= args.warmup:
                times.append(dt)
            log(f"  {name:20s} {'warm' if it < args.warmup else 'step'} {it}: {dt * 1e3:8.2f} ms iters "
                f"{info['iters']} restarts {info['restarts']} relres {info['rel_residual']:.3e} {info['status']}")
        fwd = float(np.linalg.norm(x.cpu().numpy() - pr.x_true) / np.linalg.norm(pr.x_true))
        modes[name] = {"seconds_mean": statistics.mean(times), "seconds_min": min(times), "iters": info["iters"],
                       "restarts": info["restarts"], "status": info["status"],
                       "rel_residual": info["rel_residual"], "forward_error": fwd, "options": kw}
    value_mode = "fp32_two_stage"
    v = modes[value_mode]["seconds_mean"]
    for name in modes:
        modes[name]["speedup_vs_fp64"] = round(modes["fp64"]["seconds_mean"] / modes[name]["seconds_mean"], 3)
    return {
        "metric": METRIC, "value": round(v, 6), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(v * 1e3, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"3-D convection-diffusion {args.N}^3 + 6/h^2 on the diagonal (n={A.n}, "
                               f"nnz={A.nnz}), beta=(50,20,10), MGS GMRES({m}), fp32 Arnoldi + fp64 "
                               f"residual/update, tol 1e-10, two-stage restarts (improvement 1e-6, then the "
                               f"first cycle's length), time incl. setup",
                   "n": A.n, "nnz": A.nnz, "m": m, "ortho": "mgs", "precision": "fp32"},
        "modes": modes, "roofline": None, "cpu_baseline": None,
    }


def batch_alg_bytes(n, nnz, iters, restarts, m):
    """Bytes one system's MGS solve must move with w held on chip (float32 A,
    basis and w; float64 residual and update), given its iteration count."""
    total, left = 0.0, iters
    cycles = max(1, restarts)
    for c in range(cycles):
        k = min(m, left) if c < cycles - 1 else left
        left -= k
        total += 12.0 * nnz + 4.0 * (n + 1) + 20.0 * n            # float64 residual, v1
        for j in range(k):
            total += 8.0 * nnz + 4.0 * (n + 1) + 8.0 * n          # SpMV
            total += (j + 1) * 4.0 * n + 12.0 * n                 # MGS with w on chip, v_{j+1} written
        total += k * 4.0 * n + 16.0 * n                           # float64 update
    return total


def bench_batch(args):
    """512 uneven 2-D convection-diffusion systems, GMRES(40) MGS, one handle."""
    import numpy as np
    import torch

    import problems as P
    from paper_2011_01850_amd import BatchSolver

    m = 40
    mode = args.precision or "fp32"
    log("generating 512 2-D convection-diffusion systems ...")
    probs = P.c4_batch()
    systems = [tuple(torch.as_tensor(v, device="cuda") for v in (p.A.row_ptr, p.A.col_idx, p.A.vals))
               for p in probs]
    bs = [torch.as_tensor(p.b, device="cuda") for p in probs]
    ns = [p.A.n for p in probs]
    nnzs = [p.A.nnz for p in probs]
    torch.cuda.synchronize()
    log(f"{len(probs)} systems, sum n = {sum(ns):,}, sum nnz = {sum(nnzs):,}; MGS GMRES({m}) {mode}")

    def run(prec, steps, warmup):
        times, last = [], None
        for it in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bsol = BatchSolver(systems, m=m, tol=1e-10, ortho="mgs", precision=prec, max_iters=100_000)
            xs, infos = bsol.solve(bs)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            bsol.close()
            if it >= warmup:
                times.append(dt)
            iters = [i["iters"] for i in infos]
            log(f"  {prec} {'warm' if it < warmup else 'step'} {it}: {dt * 1e3:.1f} ms, iterations "
                f"min {min(iters)} median {int(np.median(iters))} max {max(iters)}, "
                f"converged {sum(i['status'] == 'CONVERGED' for i in infos)}/{len(infos)}")
            last = (xs, infos)
        return times, last

    t_mix, (xs, infos) = run(mode, args.steps, args.warmup)
    fwd = [float(np.linalg.norm(x.cpu().numpy() - p.x_true) / np.linalg.norm(p.x_true)) for x, p in zip(xs, probs)]
    alg = sum(batch_alg_bytes(n, z, i["iters"], i["restarts"], m) for n, z, i in zip(ns, nnzs, infos))
    v = statistics.mean(t_mix)
    out64 = None
    if not args.no_fp64:
        t64, (_, inf64) = run("fp64", 1, 0)
        out64 = {"seconds": t64[0], "iters_total": sum(i["iters"] for i in inf64),
                 "converged": sum(i["status"] == "CONVERGED" for i in inf64)}
    iters = [i["iters"] for i in infos]
    rec = {
        "metric": "batch throughput: systems solved to 1e-10 rel. residual per second", "value": round(len(probs) / v, 3),
        "unit": "systems/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(v * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if mode == "fp32" else f"{mode}+f32+f64", "data": "synthetic",
        "config": {"workload": f"{len(probs)} 2-D convection-diffusion systems, sides U{{32..256}}, beta ~ U[0,100]^2, "
                               f"sum n={sum(ns)}, sum nnz={sum(nnzs)}, GMRES({m}) MGS, {mode} Arnoldi + fp64 "
                               f"residual/update, tol 1e-10, one handle (create + solve timed)",
                   "systems": len(probs), "sum_n": sum(ns), "sum_nnz": sum(nnzs), "m": m, "precision": mode},
        "seconds": {"mean": v, "median": statistics.median(t_mix), "min": min(t_mix), "max": max(t_mix)},
        "iterations": {"min": min(iters), "median": float(np.median(iters)), "max": max(iters), "total": sum(iters)},
        "converged": sum(i["status"] == "CONVERGED" for i in infos),
        "max_rel_residual": max(i["rel_residual"] for i in infos),
        "max_forward_error": max(fwd),
        "effective_GBps": round(alg / v / 1e9, 1),
        "alg_bytes": alg,
        "fp64": out64,
        "roofline": {"bound": "hbm", "kernel": "whole batch solve (algorithmic bytes, MGS with w on chip)",
                     "achieved": round(alg / v / 1e9, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(alg / v / 1e9 / PEAK_HBM_GBS, 4), "traffic": None},
        "cpu_baseline": None,
    }
    return rec


def _gen_varcoef(job):
    """Values and right-hand side of one variable-coefficient instance (host worker)."""
    i, N = job
    import problems as P

    pr = P.c5_varcoef(i, N=N)
    return pr.A.vals, pr.b


def _varcoef_stream(ids, N, pool):
    """(A, b) in order of ids, generated by the worker pool; the pattern is shared."""
    from types import SimpleNamespace

    import problems as P

    pat = P.varcoef3d(N, 5, ids[0])
    for vals, b in pool.imap(_gen_varcoef, [(i, N) for i in ids], chunksize=4):
        yield SimpleNamespace(n=pat.n, nnz=pat.nnz, row_ptr=pat.row_ptr, col_idx=pat.col_idx, vals=vals), b


def bench_learned(args, pool):
    """Train the SPAI network on GPU-generated residual pairs, then time FGMRES(30) to 1e-10 on held-out
    instances: learned vs Jacobi (float32 Arnoldi), and plain float32 / float64 GMRES on a subset."""
    import numpy as np
    import torch

    from paper_2011_01850_amd import train as T

    N = args.learned_N
    m = 30
    train_ids = list(range(args.train_instances))
    test_ids = list(range(2000, 2000 + args.test_instances))
    log(f"training data: {len(train_ids)} instances of the 3-D variable-coefficient family, N = {N} ...")
    data = T.prepare(_varcoef_stream(train_ids, N, pool), K=4, m=m, log=log)
    log(f"  data ready in {data.seconds:.1f} s; training {args.epochs} epochs")
    res = T.train_on(data, epochs=args.epochs, lr=1e-3, batch=4, seed=0, log=log)
    del data
    torch.cuda.empty_cache()
    log(f"  loss {res['loss_first']:.4f} (Jacobi start) -> {res['loss_last']:.4f} in {res['seconds_train']:.1f} s")
    from paper_2011_01850_amd import spai as S

    rows = []
    nb = min(args.baseline_instances, len(test_ids))
    net, t_net = None, None
    for q, (A, b) in enumerate(_varcoef_stream(test_ids, N, pool)):
        dev = tuple(torch.as_tensor(v, device="cuda") for v in (A.row_ptr, A.col_idx, A.vals))
        bt = torch.as_tensor(b, device="cuda")
        if net is None:  # one network instance for the family's pattern, built once
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            net = S.SpaiNet(dev[0], dev[1], kmax=1)
            torch.cuda.synchronize()
            t_net = time.perf_counter() - t0
        kinds = ["jacobi", "ilu0", "learned"] + (["none", "fp64"] if q < nb else [])
        row = {"instance": test_ids[q]}
        for kind in kinds:
            _, row[kind] = T.solve_once(dev, bt, kind, params=res["params"], m=m, net=net)
        if q == 0:  # the one-off path: the solver builds its own network instance
            _, row["learned_own_instance"] = T.solve_once(dev, bt, "learned", params=res["params"], m=m)
        rows.append(row)
        if (q + 1) % 50 == 0:
            log(f"  evaluated {q + 1} held-out instances")
    net.close()

    def summary(kind, subset):
        rs = [r[kind] for r in subset if kind in r]
        return {"instances": len(rs), "seconds_mean": float(np.mean([r["seconds_total"] for r in rs])),
                "iters_mean": float(np.mean([r["iters"] for r in rs])),
                "iters_median": float(np.median([r["iters"] for r in rs])),
                "converged": sum(r["status"] == "CONVERGED" for r in rs),
                "fallback_used": sum(bool(r["fallback_used"]) for r in rs),
                "max_rel_residual": float(max(r["rel_residual"] for r in rs))}

    kinds_all = {k: summary(k, rows) for k in ("jacobi", "ilu0", "learned")}
    kinds_sub = {k: summary(k, rows[:nb]) for k in ("fp64", "none", "jacobi", "ilu0", "learned")}
    v = kinds_all["learned"]["seconds_mean"]
    n_a = N ** 3
    rec = {
        "metric": METRIC, "value": round(v, 6), "unit": "s", "n_gpus": 1, "steps": len(rows), "warmup": 0,
        "ms_per_step": round(v * 1e3, 3), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16-mfma-net+f32+f64", "data": "synthetic",
        "config": {"workload": f"3-D variable-coefficient diffusion-convection {N}^3 (n={n_a}), kappa = exp(1.5 GRF), "
                               f"beta=(30,0,0); learned SPAI (3-layer MPNN, width 32) trained on {len(train_ids)} "
                               f"instances, FGMRES({m}) CGSR float32 Arnoldi + fp64 residual/update, tol 1e-10, "
                               f"time per held-out instance incl. setup and inference (one network instance "
                               f"for the family's shared pattern)",
                   "N": N, "m": m, "train_instances": len(train_ids), "test_instances": len(test_ids)},
        "held_out_all": kinds_all,
        "held_out_baseline_subset": kinds_sub,
        "speedup_learned_vs_fp64": round(kinds_sub["fp64"]["seconds_mean"] / kinds_sub["learned"]["seconds_mean"], 3),
        "speedup_learned_vs_jacobi": round(kinds_all["jacobi"]["seconds_mean"] / v, 3),
        "speedup_learned_vs_ilu0": round(kinds_all["ilu0"]["seconds_mean"] / v, 3),
        "iteration_gain_vs_none": round(kinds_sub["none"]["iters_mean"] / kinds_sub["learned"]["iters_mean"], 3),
        "learned_one_off": {"network_instance_seconds": t_net,
                            "first_instance_seconds_own_instance": rows[0]["learned_own_instance"]["seconds_total"],
                            "first_instance_seconds_shared_instance": rows[0]["learned"]["seconds_total"]},
        "training": {k: res[k] for k in ("loss_first", "loss_last", "seconds_data", "seconds_train", "steps",
                                         "batch", "instances", "seconds_per_instance_step")},
        "roofline": None,
        "cpu_baseline": None,
    }
    return rec


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU row partitioning is described in the design notes only)", file=sys.stderr)
        sys.exit(2)
    pool = None
    if args.workload == "learned":
        # host workers for the instance generator, started before the GPU is touched
        import multiprocessing as mp

        workers = max(1, min(16, len(os.sched_getaffinity(0)) - 1))
        pool = mp.get_context("spawn").Pool(workers)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if pool is not None:
        with pool:
            rec = bench_learned(args, pool)
    else:
        rec = {"convdiff3d": bench_convdiff3d, "powerlaw": bench_powerlaw,
               "batch": bench_batch, "restart": bench_restart, "variables": bench_variables}[args.workload](args)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        rec["copy_probe_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4, "launches": 3}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
