#!/usr/bin/env python3
"""Time to a 1e-10 relative residual: mixed-precision vs float64 restarted GMRES on one GPU.

Workload: 3-D convection-diffusion on a 128^3 grid (n = 2,097,152 rows,
14,581,760 non-zeros, 7-point first-order upwind stencil, beta = (50, 20,
10)), b = A x_true with x_true ~ U[-1, 1], x0 = 0, GMRES(50) with CGSR (and
MGS), float32 Arnoldi with float64 residual and update.  One step = one
time-to-solution: gmres_create (matrix copies, float32 copy, SpMV row
blocks and autotuning, workspace) + gmres_solve to 1e-10, inputs already
resident in HBM.  The float64 solver is timed the same way for the speedup.

Also reported, on the same JSON line:
  roofline      achieved HBM bandwidth of the dominant kernel family (the
                one with the most kernel time inside a solve), measured
                inside one more solve of the same handle in which every
                launch sits between two HIP events on the solver's stream,
                against the 8 TB/s peak; the back-to-back harness time of
                its 64-column instantiation and its launch configuration are
                printed beside it;
  cpu_baseline  the CPU oracle on a bounded sample of the same system (two
                whole restart cycles, scaled to the float64 cycle count);
  mgs           the same system with MGS, mixed and float64, and the MGS
                step kernel's in-solve bandwidth;
  powerlaw, batch, learned
                compact results of the other workloads (--legs selects
                them; each has its own --workload for the full report).
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

# HBM bytes per launch of the kernels that can be the roofline kernel (the
# instantiations with the most in-solve time on the 128^3 workload; which one
# leads varies from run to run), from two rocprofv3 counter passes
# (FETCH_SIZE, WRITE_SIZE) over the launches that did work inside the
# profiled solve of `--legs none --mgs-steps 0 --no-cpu --no-fp64 --steps 1
# --warmup 0 --spmv-format sell16 --copy-probe`, each scaled by what the same
# counter reads for the 1 GiB copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0); void
# once the kernel source changes
TRAFFIC = {
    "kernel_source_sha256": "c039eb5a874701ebcbedb0f24359cafcf553969b59e9a064a9a445b68d6f29c5",
    "bytes_per_launch": {
        "k_axpy_mdot_ds<float, float, 64>": 364456778,
        "k_mdot_ds<float, float, 64>": 356072821,
        "k_final_tile<float, float, 64>": 364140105,
        "k_sell<float, float, float, 0, true>": 116114767,
    },
}
KERNEL_SOURCE = os.path.join(ROOT, "paper_2011_01850_amd", "csrc", "gmres_kernels.hip")


def measured_traffic(kernel):
    b = TRAFFIC["bytes_per_launch"].get(kernel)
    if b is None:
        return None
    with open(KERNEL_SOURCE, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != TRAFFIC["kernel_source_sha256"]:
            return None  # the kernels changed since the counters were taken
    return b


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
    ap.add_argument("--cpu-cycles", type=int, default=3,
                    help="oracle sample: whole restart cycles of the float64 oracle (default 3, about 11 s)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the whole float64 oracle solve instead of a sample (minutes)")
    ap.add_argument("--mgs-steps", type=int, default=3, help="timed steps of each MGS mode (default workload)")
    ap.add_argument("--legs", default="ilu,c3,c4,c5",
                    help="default workload: comma-separated extra legs to run after the headline system "
                         "(ilu = the paper's ILU(0) precision study on the same system, c3 = power-law, "
                         "c4 = batch, c5 = learned preconditioner), or 'none'")
    ap.add_argument("--c5-train", type=int, default=2000, help="c5 leg: training instances")
    ap.add_argument("--c5-test", type=int, default=200, help="c5 leg: held-out instances")
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with a plain 1 GiB device copy (reference kernel for HBM byte counters)")
    ap.add_argument("--spmv-format", default="auto", choices=["auto", "csr", "sell", "sell16"],
                    help="Arnoldi SpMV format of the time-to-solution handles (auto: the autotuner's choice; "
                         "a fixed format keeps counter passes on one kernel)")
    ap.add_argument("--trace-summary", metavar="DIR",
                    help="no GPU: summarise the rocprofv3 CSV output in DIR (kernel trace and/or counter "
                         "collection) for the last --last dispatches of --kernel, i.e. the launches of the "
                         "profiled solve of a run with --legs none --mgs-steps 0")
    ap.add_argument("--kernel", default="k_sell<float, float, float, 0, true>",
                    help="--trace-summary: the kernel (template instantiation, without 'void gm::')")
    ap.add_argument("--last", type=int, default=650, help="--trace-summary: dispatches of the profiled solve")
    ap.add_argument("--floor-us", type=float, default=10.0,
                    help="--trace-summary: dispatches shorter than this did no work (gated off)")
    return ap.parse_args()


def _csv_rows(d, suffix):
    import csv
    import glob

    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _short_kernel(name):
    name = name[5:] if name.startswith("void ") else name
    name = name[4:] if name.startswith("gm::") else name
    return name.split("(")[0]


def trace_summary(d, kernel, last, floor_us):
    """Per-dispatch figures of one kernel from rocprofv3 CSV files: durations
    from the kernel trace, and FETCH_SIZE / WRITE_SIZE (KiB) from the counter
    collection, over the last `last` dispatches of that kernel, split into the
    dispatches that did work and those the device gate switched off; with the
    copy kernel's counters when the run ended with --copy-probe."""
    out = {"kernel": kernel, "last": last}
    tr = [r for r in _csv_rows(d, "kernel_trace.csv") if _short_kernel(r["Kernel_Name"]) == kernel]
    if tr:
        tr.sort(key=lambda r: int(r["Dispatch_Id"]))
        sel = tr[-last:]
        us = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in sel]
        act = [u for u in us if u >= floor_us]
        out["trace"] = {"dispatches_of_kernel": len(tr), "selected": len(sel), "avg_us_all": sum(us) / len(us),
                        "worked": len(act), "avg_us_worked": (sum(act) / len(act)) if act else None,
                        "min_us_worked": min(act) if act else None, "max_us_worked": max(act) if act else None}
    cc = _csv_rows(d, "counter_collection.csv")
    if cc:
        per = {}
        for r in cc:
            k = _short_kernel(r["Kernel_Name"])
            per.setdefault(k, {}).setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
        mine = [per[kernel][i] for i in sorted(per.get(kernel, {}))][-last:]
        res = {}
        for cname in ("FETCH_SIZE", "WRITE_SIZE"):
            vals = [v[cname] for v in mine if cname in v]
            if not vals:
                continue
            top = max(vals)
            act = [v for v in vals if v > 0.05 * top]
            res[cname] = {"selected": len(vals), "worked": len(act), "avg_kib_worked": sum(act) / len(act)}
        # the --copy-probe copies: the last three copy dispatches of the run
        copy_ids = sorted(i for k, dd in per.items() if "copyBuffer" in k for i in dd)[-3:]
        copy = [dd[i] for k, dd in per.items() if "copyBuffer" in k for i in dd if i in copy_ids]
        for cname in ("FETCH_SIZE", "WRITE_SIZE"):
            vals = [v[cname] for v in copy if cname in v]
            if vals:
                res.setdefault("copy_probe", {})[cname] = vals
        out["counters"] = res
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


SPMV_FORMAT = "auto"  # --spmv-format: the Arnoldi SpMV format of every time-to-solution handle


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
                   stall_cycles=stall_cycles, a_storage=a_storage, spmv_format=SPMV_FORMAT)
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


# kernel families of the in-solve profile and the kernels each one launches
FAMILY_KERNELS = {
    "spmv": "k_spmv (Arnoldi SpMV w = A v_j, adaptive CSR row blocks)",
    "pass1": "k_mdot (CGS projection 1: V^T w; k_mdot_ds also scales w by v_j's decode scale)",
    "pass2": "k_axpy_mdot (CGS projection 2 fused: w -= V h1, then V^T w; the _ds variant as pass 1)",
    "final": "k_final_tile / k_mgs_final (last pass: w -= V h2 or the last MGS axpy, ||w||, v_{j+1})",
    "mgs": "k_mgs (MGS step: completes dot i-1, w -= h v_{i-1}, partial w . v_i)",
    "residual": "k_spmv RESID (float64 restart residual z = b - A x)",
    "update": "k_update (float64 update x += V y)",
    "precond": "preconditioner application z_j = M v_j",
}
HBM_FAMILIES = ("spmv", "pass1", "pass2", "final", "mgs", "residual", "update", "precond")
# gmres_time_kernel's numbering of the same kernels (the back-to-back harness)
HARNESS_KERNEL = {"spmv": 0, "pass1": 1, "pass2": 2, "final": 3, "mgs": 4, "residual": 5, "update": 6}
# template arguments (basis, w) of the basis kernels per precision mode
TYPES = {"fp32": "float, float", "fp64": "double, double", "fp16": "_Float16, float", "bf16": "gm::bf16_t, float",
         "limited": "float, double"}


def tile_width(j):
    """Columns of the register tile the CGS passes use at Arnoldi column j (8, 16, 32 or 64)."""
    L = 8
    while L < j + 1 and L < 64:
        L *= 2
    return L


def spmv_kernel(precision, spmv=None):
    """The Arnoldi SpMV's template instantiation for the handle's SpMV choice
    (Solver.spmv_config(): the sliced ELL kernel, with 32-bit columns or
    16-bit column offsets, or the CSR row blocks); the matrix values are
    float64 only in the float64 solver."""
    if not spmv:
        return FAMILY_KERNELS["spmv"]
    ta = "double" if precision == "fp64" else "float"
    ty = TYPES.get(precision, "?")
    if spmv["format"] in ("sell", "sell16"):
        return f"k_sell<{ta}, {ty}, 0, {'true' if spmv['format'] == 'sell16' else 'false'}>"
    return f"k_spmv<{ta}, {ty}, 0>"


def kernel_units(fam, m, precision, ortho, spmv=None):
    """The kernels (template instantiations) of one family: (name, columns)."""
    ty = TYPES.get(precision, "?")
    if fam == "spmv":
        return [(spmv_kernel(precision, spmv), list(range(m)))]
    if fam in ("pass1", "pass2") or (fam == "final" and ortho == "cgsr"):
        base = {"pass1": "k_mdot", "pass2": "k_axpy_mdot64" if precision in ("fp64", "limited") else "k_axpy_mdot",
                "final": "k_final_tile"}[fam]
        # with the finaliser merged into the product, the first two
        # projections apply the decode scale of v_j (the _ds kernels)
        if fam != "final" and spmv and spmv.get("fin_merged"):
            base += "_ds"
        units = {}
        for j in range(m):
            units.setdefault(tile_width(j), []).append(j)
        return [(f"{base}<{ty}, {L}>", cols) for L, cols in sorted(units.items())]
    if fam == "final":
        return [(f"k_mgs_final<{ty}>", list(range(m)))]
    if fam == "mgs":
        return [(f"k_mgs<{ty}>", list(range(m)))]
    return [(FAMILY_KERNELS.get(fam, fam), list(range(m)))]


def in_solve_profile(solver, b_dev):
    """One more solve on the same handle, every launch between two HIP events
    (gmres_solve_profiled): per kernel family, time per solve, launches, and
    the time, launches and algorithmic bytes of the launches that did work,
    with the per-column breakdown."""
    x, info, prof = solver.solve_profiled(b_dev)
    fam = {}
    for name, p in prof.items():
        if p["launches"] == 0:
            continue
        e = {"ms_per_solve": round(p["ms"], 4), "launches": p["launches"], "ms_active": round(p["ms_active"], 4),
             "active_launches": p["active"], "alg_bytes": p["bytes"], "by_col": p["by_col"]}
        if p["active"] and p["bytes"] > 0:
            e["avg_launch_ms"] = round(p["ms_active"] / p["active"], 5)
            e["GB/s"] = round(p["bytes"] / (p["ms_active"] * 1e-3) / 1e9, 1)
        fam[name] = e
    return x, info, fam


def harness_times(solver, m, reps, families=("spmv", "pass1", "pass2", "final", "mgs")):
    """gmres_time_kernel at the last column for each family (run before the
    profiled solve: back-to-back launches on the solver's stream), with the
    launch configuration."""
    out = {}
    for f in families:
        try:
            ms, by = solver.time_kernel(HARNESS_KERNEL[f], m - 1, reps)
            cfg = solver.launch_config(f, m - 1)
        except Exception:  # noqa: BLE001 - a family the handle does not run (MGS kernels on a CGSR handle)
            continue
        out[f] = {"j": m - 1, "reps": reps, "avg_launch_ms": round(ms, 5), "alg_bytes": by,
                  "GB/s": round(by / (ms * 1e-3) / 1e9, 1), "launch_config": cfg}
    return out


def roofline_from_profile(solver, fam, m, reps, precision="fp32", ortho="cgsr", families=HBM_FAMILIES,
                          harness=None):
    """The dominant kernel: the template instantiation with the most in-solve
    time among the HBM-bound families; achieved = its algorithmic bytes over
    its summed in-solve launch time (launches that did work).  Beside it: every
    instantiation and family, the back-to-back harness time of the same kernel
    at the last column, and its launch configuration."""
    try:
        spmv = solver.spmv_config()
    except Exception:  # noqa: BLE001 - a handle without the query (older library, test double)
        spmv = None
    units = []
    for f in families:
        if f not in fam or fam[f]["alg_bytes"] <= 0:
            continue
        for name, cols in kernel_units(f, m, precision, ortho, spmv):
            rows = [fam[f]["by_col"][j] for j in cols]
            ms_act = sum(r["ms_active"] for r in rows)
            act = sum(r["active"] for r in rows)
            if f in ("residual", "update"):  # launched at a cycle's start or end: no column
                ms_act, act = fam[f]["ms_active"], fam[f]["active_launches"]
                ms_all, launches, byts = fam[f]["ms_per_solve"], fam[f]["launches"], fam[f]["alg_bytes"]
            else:
                ms_all = sum(r["ms"] for r in rows)
                launches = sum(r["launches"] for r in rows)
                byts = sum(r["bytes"] for r in rows)
            if act == 0 or byts <= 0:
                continue
            units.append({"kernel": name, "family": f, "columns": f"{cols[0]}..{cols[-1]}", "ms_active": ms_act,
                          "active_launches": act, "ms_all": ms_all, "launches": launches, "alg_bytes": byts,
                          "avg_launch_ms": ms_act / act, "GB/s": byts / (ms_act * 1e-3) / 1e9})
    dom = max(units, key=lambda u: u["ms_active"])
    achieved = dom["GB/s"]
    per_launch = dom["alg_bytes"] / dom["active_launches"]
    traffic = measured_traffic(dom["kernel"])
    j_last = int(dom["columns"].split("..")[1])
    h = (harness or {}).get(dom["family"])
    if h is not None and h["j"] != j_last:
        h = None  # the harness timed another instantiation of the family
    cfg = h["launch_config"] if h else None
    fams = {k: {kk: vv for kk, vv in v.items() if kk != "by_col"} for k, v in fam.items()}
    return {
        "bound": "hbm",
        "kernel": dom["kernel"],
        "family": dom["family"],
        "family_role": FAMILY_KERNELS.get(dom["family"], dom["family"]),
        "achieved": round(achieved, 1),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4),
        "traffic": (round(traffic) if traffic else None),
        "traffic_over_alg": (round(traffic / per_launch, 4) if traffic else None),
        # the measured bytes over the same launch time (the physical rate; a
        # layout that moves fewer bytes than the algorithmic count shows here)
        "traffic_GBps": (round(traffic / (dom["avg_launch_ms"] * 1e-3) / 1e9, 1) if traffic else None),
        "traffic_frac": (round(traffic / (dom["avg_launch_ms"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4) if traffic else None),
        "avg_launch_ms": round(dom["avg_launch_ms"], 5),
        "alg_bytes_per_launch": round(per_launch),
        "launches": (f"{dom['active_launches']} launches that did work inside one solve, columns j = "
                     f"{dom['columns']} of every cycle (of {dom['launches']}; the rest are gated off after the "
                     f"last cycle converged), each between two HIP events on the solver's stream"),
        "avg_launch_ms_all_launches": round(dom["ms_all"] / dom["launches"], 5),
        "harness_back_to_back": ({k: v for k, v in h.items() if k != "launch_config"} if h else None),
        "launch_config_at_j_last": cfg,
        "spmv_config": spmv,
        "in_solve_kernels": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in u.items()} for u in units],
        "in_solve_families": fams,
    }


def cpu_baseline(pr, m, ortho, ref_iters, ref_cycles, cycles, full=False):
    """The float64 oracle on the host: `cycles` whole restart cycles (or the
    whole solve), scaled to the float64 GPU solve's cycle count."""
    from oracle import gmres as O

    try:
        from threadpoolctl import threadpool_info

        blas = [d.get("num_threads") for d in threadpool_info() if d.get("user_api") == "blas"]
        threads = max(blas) if blas else 1
    except Exception:  # pragma: no cover
        threads = 1
    A = O.Matrix.from_csr(pr.A)
    t0 = time.perf_counter()
    r = O.gmres(A, pr.b, m=m, tol=1e-10, max_iters=(10 ** 7 if full else cycles * m), ortho=ortho)
    dt = time.perf_counter() - t0
    if full:
        value = dt
        sample = (f"the whole float64 {ortho.upper()} oracle solve on the same system: {r.iters} iterations, "
                  f"{r.restarts} cycles, relres {r.rel_residual:.2e}, {dt:.1f} s")
    else:
        per_cycle = dt / max(1, r.restarts)
        value = per_cycle * ref_cycles
        sample = (f"{r.restarts} whole restart cycles ({r.iters} inner iterations and their float64 residuals) "
                  f"of the float64 {ortho.upper()} oracle on the same system took {dt:.2f} s; value = that time "
                  f"per cycle x the {ref_cycles} cycles ({ref_iters} iterations) the GPU float64 solve needed "
                  f"(its last cycle is shorter, so this slightly over-states the whole solve)")
    return {
        "value": round(value, 3),
        "unit": "s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": sample,
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


def _summary(times, infos, solver, x, pr, b_dev, np):
    """Time-to-solution statistics of one mode, with the errors of its last solution."""
    eta, rel = solver.backward_error(b_dev, x)
    xs = x.cpu().numpy()
    return {"seconds_mean": statistics.mean(times), "seconds_median": statistics.median(times),
            "seconds_min": min(times), "seconds_max": max(times),
            "solve_seconds": infos[-1]["seconds"], "setup_seconds": infos[-1]["setup_seconds"],
            "iters": infos[-1]["iters"], "restarts": infos[-1]["restarts"], "status": infos[-1]["status"],
            "rel_residual": infos[-1]["rel_residual"], "backward_error": eta,
            "forward_error": float(np.linalg.norm(xs - pr.x_true) / np.linalg.norm(pr.x_true)),
            "memory_bytes": solver.memory_bytes()}, xs


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

    def mode(ortho, precision, steps, warmup, **kw):
        t, inf, (s, x) = time_to_solution(torch, Solver, A_dev, b_dev, A.n, m, ortho, precision, steps, warmup,
                                          **kw)
        out, xs = _summary(t, inf, s, x, pr, b_dev, np)
        return out, xs, s

    mixed, x_mix, solver = mode(args.ortho, args.precision, args.steps, args.warmup)
    value = mixed["seconds_mean"]
    log("kernel harness (back-to-back launches at the last column) ...")
    harness = harness_times(solver, m, args.roofline_reps)
    log("in-solve kernel profile (one more solve, every launch between HIP events) ...")
    _, pinfo, fam = in_solve_profile(solver, b_dev)
    rf = roofline_from_profile(solver, fam, m, args.roofline_reps, args.precision, args.ortho, harness=harness)
    log(f"  dominant family {rf['family']}: {rf['avg_launch_ms'] * 1e3:.1f} us per launch, "
        f"{rf['achieved']:.0f} GB/s ({rf['frac']:.3f} of peak); harness "
        f"{(rf['harness_back_to_back'] or {}).get('avg_launch_ms', 0) * 1e3:.1f} us at j = {m - 1}")
    solver.close()
    out_fp64, x64 = None, None
    if not args.no_fp64:
        out_fp64, x64, s64 = mode(args.ortho, "fp64", args.steps, max(0, min(args.warmup, 1)))
        s64.close()
    # the error of each mode against the float64 solution, next to its iterations
    if x64 is not None:
        mixed["error_vs_fp64_solution"] = float(np.linalg.norm(x_mix - x64) / np.linalg.norm(x64))
    # split storage of A (high and low words; the Arnoldi product reads the
    # high words): the same solve without the float32 copy of the matrix
    log("split storage of A ...")
    out_split, xs_, s_ = mode(args.ortho, args.precision, args.steps, min(args.warmup, 1), a_storage="split")
    s_.close()
    # the limited mixed solver of the convergence study: float32 storage of
    # the Arnoldi copy of A and of the basis only, w and its dots float64
    log("limited mixed precision ...")
    out_limited, xl_, s_ = mode(args.ortho, "limited", args.steps, min(args.warmup, 1))
    s_.close()
    # the 2-byte basis (IEEE half plus a power-of-two scale per vector) on the same system
    out_half, xh_ = None, None
    if args.precision == "fp32":
        log("half-precision basis ...")
        out_half, xh_, s_ = mode(args.ortho, "fp16", args.steps, min(args.warmup, 1))
        s_.close()
    if x64 is not None:
        for o, xo in ((out_split, xs_), (out_limited, xl_), (out_half, xh_)):
            if o is not None:
                o["error_vs_fp64_solution"] = float(np.linalg.norm(xo - x64) / np.linalg.norm(x64))
    # MGS, the other orthogonalisation the configuration names: mixed and
    # float64, and the MGS step kernel's in-solve bandwidth
    out_mgs = None
    if args.ortho == "cgsr" and args.mgs_steps > 0:
        log("MGS ...")
        mg, xm, sm = mode("mgs", args.precision, args.mgs_steps, min(args.warmup, 1))
        hm = harness_times(sm, m, args.roofline_reps, families=("mgs",))
        _, _, fam_m = in_solve_profile(sm, b_dev)
        rf_m = roofline_from_profile(sm, fam_m, m, args.roofline_reps, args.precision, "mgs", families=("mgs",),
                                     harness=hm)
        sm.close()
        out_mgs = {"mixed": mg, "roofline_mgs_step": rf_m}
        if not args.no_fp64:
            m64, xm64, sm64 = mode("mgs", "fp64", args.mgs_steps, min(args.warmup, 1))
            sm64.close()
            out_mgs["fp64"] = m64
            out_mgs["speedup_vs_fp64"] = round(m64["seconds_mean"] / mg["seconds_mean"], 3)
            mg["error_vs_fp64_solution"] = float(np.linalg.norm(xm - xm64) / np.linalg.norm(xm64))
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
        "mixed": mixed,
        "fp64": out_fp64,
        "split_storage": out_split,
        "limited": out_limited,
        "half_basis": out_half,
        "mgs": out_mgs,
        "speedup_vs_fp64": (round(out_fp64["seconds_mean"] / value, 3) if out_fp64 else None),
        "paper_context": "paper (2x10-core Haswell, Kokkos/MKL, ILU(0), SuiteSparse): mixed vs FP64 "
                         "geo-mean speedup +19% (MGS), +24% (CGSR) when restarted at least once",
        "roofline": rf,
        "profiled_solve": {"iters": pinfo["iters"], "restarts": pinfo["restarts"], "status": pinfo["status"],
                           "seconds": pinfo["seconds"]},
    }
    if not args.no_cpu:
        ref = out_fp64 or mixed
        log("CPU oracle sample ...")
        rec["cpu_baseline"] = cpu_baseline(pr, m, args.ortho, ref["iters"], ref["restarts"], args.cpu_cycles,
                                           full=args.cpu_full)
    else:
        rec["cpu_baseline"] = None
    del A_dev, b_dev
    torch.cuda.empty_cache()
    legs = [] if args.legs in ("", "none") else args.legs.split(",")
    for leg in legs:
        log(f"leg {leg} ...")
        if leg == "c3":
            rec["powerlaw"] = leg_powerlaw(args)
        elif leg == "c4":
            rec["batch"] = leg_batch(args)
        elif leg == "c5":
            rec["learned"] = leg_learned(args)
        elif leg == "ilu":
            rec["ilu_precision_study"] = leg_ilu(args)
        else:
            raise SystemExit(f"unknown leg {leg}")
    return rec


def leg_ilu(args):
    """The precision study of the paper's experiments (Section 4.2) on the
    headline system: left ILU(0)-preconditioned GMRES(50) (4 Jacobi sweeps per
    triangle) with everything in float64, with only the preconditioner in
    float32 ("FP32 ILU only"), and the mixed solver (float32 Arnoldi and
    preconditioner); MGS and CGSR; time to 1e-10 including setup."""
    import numpy as np
    import torch

    import problems as P
    from paper_2011_01850_amd import Solver

    m = 50
    pr = P.c2_convdiff3d(args.N)
    A = pr.A
    A_dev = tuple(torch.as_tensor(v, device="cuda") for v in (A.row_ptr, A.col_idx, A.vals))
    b_dev = torch.as_tensor(pr.b, device="cuda")
    rp, ci, va = A_dev
    cases = [("fp64", "fp64", "native"), ("fp32_ilu_only", "fp64", "fp32"), ("mixed", "fp32", "native")]
    out = {"workload": f"3-D convection-diffusion {args.N}^3, left ILU(0) (4 sweeps per triangle), GMRES({m}), "
                       f"tol 1e-10, time incl. setup (ILU factorisation included, as the paper times it)"}
    for ortho in ("mgs", "cgsr"):
        rows = {}
        for name, prec, pcp in cases:
            times, info, x = [], None, None
            for it in range(1 + 3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s = Solver(rp, ci, va, m=m, ortho=ortho, precision=prec, tol=1e-10, precond="ilu0", ilu_sweeps=4,
                           precond_side="left", precond_precision=pcp)
                x, info = s.solve(b_dev)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if it:
                    times.append(dt)
                    eta = s.backward_error(b_dev, x)[0] if it == 3 else None
                s.close()
            fwd = float(np.linalg.norm(x.cpu().numpy() - pr.x_true) / np.linalg.norm(pr.x_true))
            rows[name] = {"seconds_mean": statistics.mean(times), "seconds_min": min(times), "iters": info["iters"],
                          "restarts": info["restarts"], "status": info["status"],
                          "rel_residual": info["rel_residual"], "backward_error": eta, "forward_error": fwd}
            log(f"  ILU(0) {ortho} {name}: {statistics.mean(times) * 1e3:.1f} ms, iters {info['iters']}, "
                f"{info['status']}")
        for name in rows:
            rows[name]["speedup_vs_fp64"] = round(rows["fp64"]["seconds_mean"] / rows[name]["seconds_mean"], 3)
        out[ortho] = rows
    out["paper_context"] = ("paper (2x10-core Haswell, SuiteSparse, left ILU(0)): mixed +19% (MGS) / +24% (CGSR), "
                            "FP32 ILU only +2% / +2% over FP64 GMRES")
    return out


def leg_powerlaw(args):
    """C3 in brief: one time-to-solution per basis format (after one untimed fp16 solve)."""
    import numpy as np
    import torch

    import problems as P
    from paper_2011_01850_amd import Solver

    m, stall = 30, 1000
    pr = P.c3_powerlaw()
    A = pr.A
    A_dev = tuple(torch.as_tensor(v, device="cuda") for v in (A.row_ptr, A.col_idx, A.vals))
    b_dev = torch.as_tensor(pr.b, device="cuda")
    out = {"workload": f"power-law random sparse n={A.n}, nnz={A.nnz}, GMRES({m}) CGSR, tol 1e-10, "
                       f"one time-to-solution per mode incl. setup", "modes": {}}
    for k, mode in enumerate(["fp64", "fp32", "fp16", "bf16"]):
        t, inf, (s, x) = time_to_solution(torch, Solver, A_dev, b_dev, A.n, m, "cgsr", mode, 1,
                                          1 if k == 0 else 0, stall_cycles=stall)
        o, _ = _summary(t, inf, s, x, pr, b_dev, np)
        if mode in ("fp32", "fp16"):
            _, _, fam = in_solve_profile(s, b_dev)
            o["spmv_in_solve"] = {k: v for k, v in fam["spmv"].items() if k != "by_col"}
        s.close()
        out["modes"][mode] = o
    for mode, o in out["modes"].items():
        o["speedup_vs_fp64"] = round(out["modes"]["fp64"]["seconds_mean"] / o["seconds_mean"], 3)
    return out


def leg_batch(args):
    """C4 in brief: the 512-system batch, one untimed and one timed solve (create + solve)."""
    import numpy as np
    import torch

    import problems as P
    from paper_2011_01850_amd import BatchSolver

    m = 40
    probs = P.c4_batch()
    systems = [tuple(torch.as_tensor(v, device="cuda") for v in (p.A.row_ptr, p.A.col_idx, p.A.vals))
               for p in probs]
    bs = [torch.as_tensor(p.b, device="cuda") for p in probs]
    ns = [p.A.n for p in probs]
    nnzs = [p.A.nnz for p in probs]
    times, infos, tune = [], None, None
    for it in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bsol = BatchSolver(systems, m=m, tol=1e-10, ortho="mgs", precision="fp32", max_iters=100_000)
        xs, infos = bsol.solve(bs)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tune = bsol.tuning() if hasattr(bsol, "tuning") else None
        bsol.close()
        if it > 0:
            times.append(dt)
    alg = sum(batch_alg_bytes(n, z, i["iters"], i["restarts"], m) for n, z, i in zip(ns, nnzs, infos))
    iters = [i["iters"] for i in infos]
    v = times[0]
    fwd = max(float(np.linalg.norm(x.cpu().numpy() - p.x_true) / np.linalg.norm(p.x_true))
              for x, p in zip(xs, probs))
    return {"workload": f"{len(probs)} 2-D convection-diffusion systems (sum n={sum(ns)}), GMRES({m}) MGS "
                        f"float32 Arnoldi, one persistent launch, create + solve timed",
            "systems_per_s": round(len(probs) / v, 2), "seconds": v,
            "iterations": {"min": min(iters), "median": float(np.median(iters)), "max": max(iters)},
            "converged": sum(i["status"] == "CONVERGED" for i in infos),
            "max_rel_residual": max(i["rel_residual"] for i in infos), "max_forward_error": fwd,
            "effective_GBps": round(alg / v / 1e9, 1), "frac_of_peak": round(alg / v / 1e9 / PEAK_HBM_GBS, 4),
            "tuning": tune}


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
        modes[mode]["backward_error"] = s.backward_error(b_dev, x)[0]
        hs = harness_times(s, m, args.roofline_reps, families=("spmv",))
        _, _, fam = in_solve_profile(s, b_dev)
        kern[mode] = {"spmv_roofline": roofline_from_profile(s, fam, m, args.roofline_reps, mode, args.ortho,
                                                             families=("spmv",), harness=hs)}
        s.close()
    for mode in modes:
        modes[mode]["speedup_vs_fp64"] = round(modes["fp64"]["seconds_mean"] / modes[mode]["seconds_mean"], 3)
    v = modes[value_mode]["seconds_mean"]
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
        "kernels_in_solve": kern,
        "roofline": kern[value_mode]["spmv_roofline"],
    }
    if not args.no_cpu:
        log("CPU oracle sample ...")
        rec["cpu_baseline"] = cpu_baseline(pr, m, args.ortho, modes["fp64"]["iters"], modes["fp64"]["restarts"],
                                           args.cpu_cycles, full=args.cpu_full)
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

    tuning = []

    def run(prec, steps, warmup):
        times, last = [], None
        for it in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bsol = BatchSolver(systems, m=m, tol=1e-10, ortho="mgs", precision=prec, max_iters=100_000)
            xs, infos = bsol.solve(bs)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if prec == mode and not tuning:
                tuning.append(bsol.tuning())
                log(f"  SpMV tuner: {tuning[0]['variant']} (probe us {tuning[0]['probe_us']})")
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
        "spmv_tuning": tuning[0] if tuning else None,
        "roofline": {"bound": "hbm", "kernel": "whole batch solve (algorithmic bytes, MGS with w on chip)",
                     "achieved": round(alg / v / 1e9, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(alg / v / 1e9 / PEAK_HBM_GBS, 4), "traffic": None},
        "cpu_baseline": None,
    }
    return rec


def _varcoef_stream(ids, N, workers=None, window=32):
    """(A, b) in order of ids, generated by host threads (the generator's NumPy
    work releases the GIL), at most `window` instances in flight; the pattern
    is shared."""
    from collections import deque
    from concurrent.futures import ThreadPoolExecutor
    from types import SimpleNamespace

    import problems as P

    workers = workers or max(1, min(8, len(os.sched_getaffinity(0)) - 1))
    pat = P.varcoef3d(N, 5, ids[0])

    def gen(i):
        pr = P.c5_varcoef(i, N=N)
        return pr.A.vals, pr.b

    with ThreadPoolExecutor(workers) as ex:
        pending = deque()
        it = iter(ids)
        for i in it:
            pending.append(ex.submit(gen, i))
            if len(pending) >= window:
                break
        while pending:
            vals, b = pending.popleft().result()
            nxt = next(it, None)
            if nxt is not None:
                pending.append(ex.submit(gen, nxt))
            yield SimpleNamespace(n=pat.n, nnz=pat.nnz, row_ptr=pat.row_ptr, col_idx=pat.col_idx, vals=vals), b


def leg_learned(args):
    """C5 in brief: train on the GPU, then FGMRES on held-out instances
    (learned, Jacobi, ILU(0)); none and float64 on the first few."""
    res = learned_run(args.c5_train, args.c5_test, 5, args.epochs, args.learned_N)
    keep = ("held_out_all", "held_out_baseline_subset", "speedup_learned_vs_fp64", "speedup_learned_vs_jacobi",
            "speedup_learned_vs_ilu0", "iteration_gain_vs_none", "iteration_gain_vs_jacobi", "training")
    out = {k: res[k] for k in keep}
    out["workload"] = res["config"]["workload"]
    return out


def bench_learned(args):
    """Train the SPAI network on GPU-generated residual pairs, then time FGMRES(30) to 1e-10 on held-out
    instances: learned vs Jacobi (float32 Arnoldi), and plain float32 / float64 GMRES on a subset."""
    return learned_run(args.train_instances, args.test_instances, args.baseline_instances, args.epochs,
                       args.learned_N)


def learned_run(n_train, n_test, n_baseline, epochs, N):
    import numpy as np
    import torch

    from paper_2011_01850_amd import train as T

    m = 30
    train_ids = list(range(n_train))
    test_ids = list(range(2000, 2000 + n_test))
    log(f"training data: {len(train_ids)} instances of the 3-D variable-coefficient family, N = {N} ...")
    data = T.prepare(_varcoef_stream(train_ids, N), K=4, m=m, log=log)
    log(f"  data ready in {data.seconds:.1f} s; training {epochs} epochs")
    res = T.train_on(data, epochs=epochs, lr=1e-3, batch=4, seed=0, log=log)
    del data
    torch.cuda.empty_cache()
    log(f"  loss {res['loss_first']:.4f} (Jacobi start) -> {res['loss_last']:.4f} in {res['seconds_train']:.1f} s")
    from paper_2011_01850_amd import spai as S

    rows = []
    nb = min(n_baseline, len(test_ids))
    net, t_net = None, None
    for q, (A, b) in enumerate(_varcoef_stream(test_ids, N)):
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
        "iteration_gain_vs_jacobi": round(kinds_all["jacobi"]["iters_mean"] / kinds_all["learned"]["iters_mean"], 3),
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
    if args.trace_summary:
        print(json.dumps(trace_summary(args.trace_summary, args.kernel, args.last, args.floor_us), indent=1))
        return
    global SPMV_FORMAT
    SPMV_FORMAT = args.spmv_format
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU row partitioning is described in the design notes only)", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    rec = {"convdiff3d": bench_convdiff3d, "powerlaw": bench_powerlaw, "learned": bench_learned,
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
