"""Python front end of libgmres: device memory via torch, every step in the HIP library.

The classes only move arguments across the C-ABI: they allocate torch
tensors on the GPU for inputs and outputs and pass their device pointers.
No part of the solve runs in Python, and there is no CPU fallback: without
a GPU or without the built library the constructors raise.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("libgmres needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _dev(t, dtype, torch):
    """A contiguous device tensor of the given dtype (copies numpy / host input)."""
    if isinstance(t, torch.Tensor):
        t = t.to(device="cuda", dtype=dtype)
    else:
        t = torch.as_tensor(np.ascontiguousarray(t), dtype=dtype, device="cuda")
    return t.contiguous()


def _options(m, tol, max_iters, ortho, precision, precond, restart_improve, stall_cycles, use_graph,
             autotune, schedule="auto", spmv_block_nnz=0, a_storage="copy", restart_repeat=False,
             restart_on_stall=False, orth_restart=0.0, orth_norm="spectral", ilu_sweeps=4,
             arnoldi_a="default", precond_precision="native", persistent_spmv="tuned",
             precond_side="right", spmv_format="auto") -> L.Options:
    o = L.default_options()
    o.m = int(m)
    o.tol = float(tol)
    o.max_iters = int(max_iters)
    o.ortho = L.ORTHOS[ortho] if isinstance(ortho, str) else int(ortho)
    o.precision = L.PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.precond = L.PRECONDS[precond] if isinstance(precond, str) else int(precond)
    o.restart_improve = float(restart_improve)
    o.stall_cycles = int(stall_cycles)
    o.use_graph = int(bool(use_graph))
    o.autotune = int(bool(autotune))
    o.batch_schedule = L.SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    o.spmv_block_nnz = int(spmv_block_nnz)
    o.a_storage = L.A_STORAGES[a_storage] if isinstance(a_storage, str) else int(a_storage)
    o.restart_repeat = int(bool(restart_repeat))
    o.restart_on_stall = int(bool(restart_on_stall))
    o.orth_restart = float(orth_restart)
    o.orth_norm = L.ORTH_NORMS[orth_norm] if isinstance(orth_norm, str) else int(orth_norm)
    o.ilu_sweeps = int(ilu_sweeps)
    o.arnoldi_a = L.ARNOLDI_AS[arnoldi_a] if isinstance(arnoldi_a, str) else int(arnoldi_a)
    o.precond_precision = (L.PRECOND_PRECISIONS[precond_precision] if isinstance(precond_precision, str)
                           else int(precond_precision))
    o.persistent_spmv = (L.PERSISTENT_SPMVS[persistent_spmv] if isinstance(persistent_spmv, str)
                         else int(persistent_spmv))
    o.precond_side = L.PRECOND_SIDES[precond_side] if isinstance(precond_side, str) else int(precond_side)
    o.spmv_format = L.SPMV_FORMATS[spmv_format] if isinstance(spmv_format, str) else int(spmv_format)
    return o


class Solver:
    """Restarted GMRES(m) for one sparse system A x = b on the current GPU."""

    def __init__(self, row_ptr, col_idx, vals, m=50, tol=1e-10, ortho="cgsr", precision="fp32",
                 precond="none", max_iters=100_000, restart_improve=0.0, stall_cycles=10,
                 use_graph=True, autotune=True, schedule="auto", spmv_block_nnz=0,
                 a_storage="copy", restart_repeat=False, restart_on_stall=False, orth_restart=0.0,
                 orth_norm="spectral", ilu_sweeps=4, arnoldi_a="default", precond_precision="native",
                 precond_side="right", spmv_format="auto"):
        torch = _torch()
        self._torch = torch
        self.lib = L.load()
        rp = _dev(row_ptr, torch.int32, torch)
        ci = _dev(col_idx, torch.int32, torch)
        va = _dev(vals, torch.float64, torch)
        self.n = int(rp.numel() - 1)
        self.nnz = int(ci.numel())
        self.m = int(m)
        self.opt = _options(m, tol, max_iters, ortho, precision, precond, restart_improve, stall_cycles,
                            use_graph, autotune, schedule, spmv_block_nnz, a_storage, restart_repeat,
                            restart_on_stall, orth_restart, orth_norm, ilu_sweeps, arnoldi_a, precond_precision,
                            precond_side=precond_side, spmv_format=spmv_format)
        self.precision = precision
        h = C.c_void_p()
        stream = torch.cuda.current_stream().cuda_stream
        torch.cuda.synchronize()
        rc = self.lib.gmres_create(C.byref(h), self.n, self.nnz, rp.data_ptr(), ci.data_ptr(), va.data_ptr(),
                                   C.byref(self.opt), C.c_void_p(stream))
        L.check(rc, "gmres_create")
        self.h = h

    # -- lifetime
    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.gmres_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- solve
    def solve(self, b, x0=None):
        """Returns (x, info): x a float64 device tensor, info a dict (status, iters, ...)."""
        torch = self._torch
        bt = _dev(b, torch.float64, torch)
        x = torch.zeros(self.n, dtype=torch.float64, device="cuda") if x0 is None else \
            _dev(x0, torch.float64, torch).clone()
        torch.cuda.synchronize()
        res = L.Result()
        L.check(self.lib.gmres_solve(self.h, bt.data_ptr(), x.data_ptr(), C.byref(res)), "gmres_solve")
        return x, res.as_dict()

    def solve_profiled(self, b, x0=None):
        """The same solve with every kernel launched directly between HIP events.

        Returns (x, info, profile): profile maps each kernel family to its
        summed milliseconds, launches, and the milliseconds, launches and
        algorithmic bytes of the launches that did work; profile[family]
        ["by_col"] lists the same per Arnoldi column j = 0..m-1."""
        torch = self._torch
        bt = _dev(b, torch.float64, torch)
        x = torch.zeros(self.n, dtype=torch.float64, device="cuda") if x0 is None else \
            _dev(x0, torch.float64, torch).clone()
        torch.cuda.synchronize()
        res = L.Result()
        nk = len(L.PROFILE_KINDS)
        prof = (L.KernelProfile * nk)()
        cols = (L.KernelProfile * (nk * self.m))()
        L.check(self.lib.gmres_solve_profiled(self.h, bt.data_ptr(), x.data_ptr(), C.byref(res), prof, cols),
                "gmres_solve_profiled")

        def row(p):
            return {"ms": p.ms, "launches": int(p.launches), "ms_active": p.ms_active, "active": int(p.active),
                    "bytes": p.bytes}

        out = {}
        for k, name in enumerate(L.PROFILE_KINDS):
            out[name] = row(prof[k])
            out[name]["by_col"] = [row(cols[k * self.m + j]) for j in range(self.m)]
        return x, res.as_dict(), out

    def set_preconditioner(self, spai_vals):
        torch = self._torch
        v = _dev(spai_vals, torch.float32, torch)
        torch.cuda.synchronize()
        L.check(self.lib.gmres_set_preconditioner(self.h, v.data_ptr()), "gmres_set_preconditioner")

    def spai_infer(self, params_bf16, net=None, return_m=True):
        """Run the learned network on this solver's matrix and install M.

        net: an optional SpaiNet created for the same sparsity pattern (reused
        across a family of matrices); without it the handle builds its own.
        Returns M (float32 tensor) or None."""
        torch = self._torch
        pb = _dev(params_bf16, torch.int16, torch)
        if pb.numel() != L.SPAI_NPARAMS:
            raise ValueError(f"expected {L.SPAI_NPARAMS} bfloat16 parameters")
        out = torch.empty(self.nnz, dtype=torch.float32, device="cuda") if return_m else None
        optr = out.data_ptr() if return_m else None
        torch.cuda.synchronize()
        if net is None:
            L.check(self.lib.gmres_spai_infer(self.h, pb.data_ptr(), pb.numel() * 2, optr), "gmres_spai_infer")
        else:
            L.check(self.lib.gmres_spai_infer_with(self.h, net.h, pb.data_ptr(), pb.numel() * 2, optr),
                    "gmres_spai_infer_with")
        return out

    def residual(self, b, x):
        """(r, ||r||) with r = b - A x in float64 on the GPU."""
        torch = self._torch
        bt = _dev(b, torch.float64, torch)
        xt = _dev(x, torch.float64, torch)
        r = torch.empty(self.n, dtype=torch.float64, device="cuda")
        nrm = C.c_double()
        torch.cuda.synchronize()
        L.check(self.lib.gmres_residual(self.h, bt.data_ptr(), xt.data_ptr(), r.data_ptr(), C.byref(nrm)),
                "gmres_residual")
        return r, nrm.value

    def backward_error(self, b, x):
        """(eta, relres): normwise backward error ||r|| / (||A||_F ||x|| + ||b||) and ||r|| / ||b||, float64."""
        torch = self._torch
        bt = _dev(b, torch.float64, torch)
        xt = _dev(x, torch.float64, torch)
        eta, rel = C.c_double(), C.c_double()
        torch.cuda.synchronize()
        L.check(self.lib.gmres_backward_error(self.h, bt.data_ptr(), xt.data_ptr(), C.byref(eta), C.byref(rel)),
                "gmres_backward_error")
        return eta.value, rel.value

    def residual_unit(self, b, x, out=None):
        """(float32 z / ||z||, ||z||) with z = b - A x in float64; `out` is an optional float32 device tensor."""
        torch = self._torch
        bt = _dev(b, torch.float64, torch)
        xt = _dev(x, torch.float64, torch)
        if out is None:
            out = torch.empty(self.n, dtype=torch.float32, device="cuda")
        elif out.dtype != torch.float32 or out.numel() != self.n or not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 CUDA tensor of n elements")
        nrm = C.c_double()
        torch.cuda.synchronize()
        L.check(self.lib.gmres_residual_unit(self.h, bt.data_ptr(), xt.data_ptr(), out.data_ptr(), C.byref(nrm)),
                "gmres_residual_unit")
        return out, nrm.value

    def precond_apply(self, v, f64=False):
        """z = M^-1 v with the handle's ILU(0) preconditioner: float32 tensors, or
        float64 ones (f64=True) for a float64 solver with a float64 preconditioner."""
        torch = self._torch
        vt = _dev(v, torch.float64 if f64 else torch.float32, torch)
        z = torch.empty_like(vt)
        torch.cuda.synchronize()
        fn, name = (self.lib.gmres_precond_apply_f64, "gmres_precond_apply_f64") if f64 else \
            (self.lib.gmres_precond_apply, "gmres_precond_apply")
        L.check(fn(self.h, vt.data_ptr(), z.data_ptr()), name)
        return z

    def spmv(self, x, precision="fp64"):
        torch = self._torch
        dt = torch.float64 if precision == "fp64" else torch.float32
        xt = _dev(x, dt, torch)
        y = torch.empty(self.n, dtype=torch.float32 if precision == "fp32" else torch.float64, device="cuda")
        torch.cuda.synchronize()
        L.check(self.lib.gmres_spmv(self.h, L.PRECISIONS[precision], xt.data_ptr(), y.data_ptr()), "gmres_spmv")
        return y

    def last_cycle(self, with_basis=True):
        """(k, Hbar [(m+1) x m numpy], V [n x (k+1)] device tensor or None)."""
        torch = self._torch
        k = C.c_int32()
        Hb = np.zeros((self.m, self.m + 1), dtype=np.float64)  # column-major storage
        L.check(self.lib.gmres_last_cycle(self.h, 0, C.byref(k), Hb.ctypes.data, None), "gmres_last_cycle")
        V = None
        if with_basis:
            V = torch.zeros((self.m + 1, self.n), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            L.check(self.lib.gmres_last_cycle(self.h, 0, None, None, V.data_ptr()), "gmres_last_cycle")
            V = V[: k.value + 1].T
        return k.value, Hb.T.copy(), V

    def history(self, cap=4096):
        out = np.zeros(cap, dtype=np.float64)
        cnt = C.c_int32()
        L.check(self.lib.gmres_history(self.h, 0, out.ctypes.data, cap, C.byref(cnt)), "gmres_history")
        return out[: min(cnt.value, cap)].copy()

    def memory_bytes(self):
        v = C.c_size_t()
        L.check(self.lib.gmres_memory_bytes(self.h, C.byref(v)), "gmres_memory_bytes")
        return int(v.value)

    def launch_config(self, family, j):
        """Launch configuration of a kernel family at column j: dict(grid, block, per_cu, basis_align)."""
        fam = L.PROFILE_KINDS.index(family) if isinstance(family, str) else int(family)
        g, b, o, al = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
        L.check(self.lib.gmres_launch_config(self.h, fam, int(j), C.byref(g), C.byref(b), C.byref(o), C.byref(al)),
                "gmres_launch_config")
        return {"grid": g.value, "block": b.value, "per_cu": o.value, "basis_align": al.value}

    def spmv_config(self):
        """The Arnoldi SpMV the handle runs: dict(format, block_nnz, xcd_remap,
        fin_merged) (fin_merged: each step's finaliser runs in the next
        product's launch and the projections apply v_j's decode scale)."""
        f, bn, xr, fm = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        L.check(self.lib.gmres_spmv_config(self.h, C.byref(f), C.byref(bn), C.byref(xr), C.byref(fm)),
                "gmres_spmv_config")
        fmt = {v: k for k, v in L.SPMV_FORMATS.items()}[f.value]
        return {"format": fmt, "block_nnz": bn.value, "xcd_remap": bool(xr.value), "fin_merged": bool(fm.value)}

    def time_kernel(self, kernel, j, reps=20):
        """(mean ms per launch, algorithmic bytes per launch) of one hot-path kernel."""
        ms = C.c_double()
        by = C.c_double()
        L.check(self.lib.gmres_time_kernel(self.h, int(kernel), int(j), int(reps), C.byref(ms), C.byref(by)),
                "gmres_time_kernel")
        return ms.value, by.value


class BatchSolver:
    """Many independent systems advanced together by every kernel launch."""

    def __init__(self, systems, m=40, tol=1e-10, ortho="mgs", precision="fp32", precond="none",
                 max_iters=100_000, restart_improve=0.0, stall_cycles=10, use_graph=True, autotune=True,
                 schedule="auto", spmv_block_nnz=0, a_storage="copy", restart_repeat=False,
                 restart_on_stall=False, orth_restart=0.0, orth_norm="spectral", ilu_sweeps=4,
                 arnoldi_a="default", persistent_spmv="tuned"):
        torch = _torch()
        self._torch = torch
        self.lib = L.load()
        self._keep = []
        ns, nnzs, rps, cis, vas = [], [], [], [], []
        for (rp, ci, va) in systems:
            rp = _dev(rp, torch.int32, torch)
            ci = _dev(ci, torch.int32, torch)
            va = _dev(va, torch.float64, torch)
            self._keep += [rp, ci, va]
            ns.append(rp.numel() - 1)
            nnzs.append(ci.numel())
            rps.append(rp.data_ptr())
            cis.append(ci.data_ptr())
            vas.append(va.data_ptr())
        S = len(ns)
        self.S = S
        self.ns = ns
        self.m = int(m)
        self.opt = _options(m, tol, max_iters, ortho, precision, precond, restart_improve, stall_cycles,
                            use_graph, autotune, schedule, spmv_block_nnz, a_storage, restart_repeat,
                            restart_on_stall, orth_restart, orth_norm, ilu_sweeps, arnoldi_a,
                            persistent_spmv=persistent_spmv)
        arr64 = C.c_int64 * S
        arrp = C.c_void_p * S
        h = C.c_void_p()
        torch.cuda.synchronize()
        rc = self.lib.gmres_batch_create(C.byref(h), S, arr64(*ns), arr64(*nnzs), arrp(*rps), arrp(*cis),
                                         arrp(*vas), C.byref(self.opt), None)
        self._keep = []
        L.check(rc, "gmres_batch_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.gmres_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, bs, x0s=None):
        """Returns (list of x device tensors, list of info dicts)."""
        torch = self._torch
        bt = [_dev(b, torch.float64, torch) for b in bs]
        xs = [torch.zeros(n, dtype=torch.float64, device="cuda") for n in self.ns] if x0s is None else \
            [_dev(x, torch.float64, torch).clone() for x in x0s]
        arrp = C.c_void_p * self.S
        res = (L.Result * self.S)()
        torch.cuda.synchronize()
        L.check(self.lib.gmres_batch_solve(self.h, arrp(*[t.data_ptr() for t in bt]),
                                           arrp(*[t.data_ptr() for t in xs]), res), "gmres_batch_solve")
        return xs, [r.as_dict() for r in res]

    def history(self, sys, cap=4096):
        out = np.zeros(cap, dtype=np.float64)
        cnt = C.c_int32()
        L.check(self.lib.gmres_history(self.h, int(sys), out.ctypes.data, cap, C.byref(cnt)), "gmres_history")
        return out[: min(cnt.value, cap)].copy()

    def tuning(self):
        """The persistent schedule's SpMV tuner: dict(variant, probe_us, classes), or None."""
        cnt = C.c_int32()
        var = C.c_int32()
        probe = (C.c_double * 3)()
        out = (L.TuneClass * 16)()
        rc = self.lib.gmres_batch_tuning(self.h, C.byref(var), probe, out, 16, C.byref(cnt))
        if rc == L.ESTATE:
            return None
        L.check(rc, "gmres_batch_tuning")
        return {"variant": L.PERSISTENT_SPMV_NAMES[var.value],
                "probe_us": {L.PERSISTENT_SPMV_NAMES[v]: round(probe[v], 2) for v in range(3) if probe[v] >= 0},
                "classes": [{"rows_per_thread": c.rows_per_thread, "systems": c.systems, "largest_n": c.largest_n,
                             "probe_system": c.probe_system} for c in out[: min(cnt.value, 16)]]}


def release_cached_memory():
    """Free the device blocks destroyed handles left for reuse; returns the bytes freed."""
    n = C.c_size_t()
    L.check(L.load().gmres_release_cached_memory(C.byref(n)), "gmres_release_cached_memory")
    return n.value


def encode(w, inv_h, fmt="fp16", out=None, noalloc=False):
    """2-byte basis storage of v = w * inv_h exactly as the solver does it: (uint16 tensor, scale).

    noalloc=True calls gmres_encode_noalloc (no device allocation inside the
    library; `out` may be given so that the binding allocates nothing either)."""
    torch = _torch()
    lib = L.load()
    wt = _dev(w, torch.float32, torch)
    if out is None:
        out = torch.empty(wt.numel(), dtype=torch.int16, device="cuda")
    elif out.numel() < wt.numel() or out.element_size() != 2 or not out.is_cuda:
        raise ValueError("out must be a 2-byte CUDA tensor of at least len(w) elements")
    sc = C.c_double()
    torch.cuda.synchronize()
    fn, name = (lib.gmres_encode_noalloc, "gmres_encode_noalloc") if noalloc else (lib.gmres_encode, "gmres_encode")
    L.check(fn(L.PRECISIONS[fmt], wt.numel(), wt.data_ptr(), float(inv_h), out.data_ptr(),
               C.byref(sc), C.c_void_p(torch.cuda.current_stream().cuda_stream)), name)
    return out, sc.value
