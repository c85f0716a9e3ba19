"""ctypes declarations of libgmres (include/gmres.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmres.so")

MGS, CGSR = 0, 1
FP64, MIXED_FP32, MIXED_BF16, MIXED_FP16, MIXED_LIMITED = 0, 1, 2, 3, 4
PRECOND_NONE, PRECOND_JACOBI, PRECOND_SPAI, PRECOND_ILU0 = 0, 1, 2, 3
RUNNING, CONVERGED, MAXITER, STALLED = 0, 1, 2, 3
OK, EINVAL, EHIP, ENOMEM, EHANDLE, ESTATE = 0, -1, -2, -3, -4, -5

STATUS_NAMES = {RUNNING: "RUNNING", CONVERGED: "CONVERGED", MAXITER: "MAXITER", STALLED: "STALLED"}
PRECISIONS = {"fp64": FP64, "fp32": MIXED_FP32, "bf16": MIXED_BF16, "fp16": MIXED_FP16,
              "limited": MIXED_LIMITED}
ORTHOS = {"mgs": MGS, "cgsr": CGSR}
PRECONDS = {"none": PRECOND_NONE, "jacobi": PRECOND_JACOBI, "spai": PRECOND_SPAI, "ilu0": PRECOND_ILU0}
SCHEDULE_AUTO, SCHEDULE_DEVICE_WIDE, SCHEDULE_PERSISTENT = 0, 1, 2
SCHEDULES = {"auto": SCHEDULE_AUTO, "device_wide": SCHEDULE_DEVICE_WIDE, "persistent": SCHEDULE_PERSISTENT}
A_COPY, A_SPLIT = 0, 1
A_STORAGES = {"copy": A_COPY, "split": A_SPLIT}
ORTH_SPECTRAL, ORTH_FROBENIUS = 0, 1
ORTH_NORMS = {"spectral": ORTH_SPECTRAL, "frobenius": ORTH_FROBENIUS}
ARNOLDI_A_DEFAULT, ARNOLDI_A_FP64, ARNOLDI_A_FP32 = 0, 1, 2
ARNOLDI_AS = {"default": ARNOLDI_A_DEFAULT, "fp64": ARNOLDI_A_FP64, "fp32": ARNOLDI_A_FP32}
PRECOND_NATIVE, PRECOND_FP32 = 0, 1
PRECOND_PRECISIONS = {"native": PRECOND_NATIVE, "fp32": PRECOND_FP32}
SPMV_AUTO, SPMV_CSR, SPMV_SELL, SPMV_SELL16 = 0, 1, 2, 3
SPMV_FORMATS = {"auto": SPMV_AUTO, "csr": SPMV_CSR, "sell": SPMV_SELL, "sell16": SPMV_SELL16}
PRECOND_RIGHT, PRECOND_LEFT = 0, 1
PRECOND_SIDES = {"right": PRECOND_RIGHT, "left": PRECOND_LEFT}
PSPMV_CSR8, PSPMV_CSR4, PSPMV_ELL16 = 0, 1, 2
PERSISTENT_SPMV_NAMES = {PSPMV_CSR8: "csr8", PSPMV_CSR4: "csr4", PSPMV_ELL16: "ell16"}
PERSISTENT_SPMVS = {"tuned": 0, "csr8": 1 + PSPMV_CSR8, "csr4": 1 + PSPMV_CSR4, "ell16": 1 + PSPMV_ELL16}


class Options(C.Structure):
    _fields_ = [
        ("m", C.c_int32),
        ("tol", C.c_double),
        ("max_iters", C.c_int64),
        ("ortho", C.c_int32),
        ("precision", C.c_int32),
        ("precond", C.c_int32),
        ("restart_improve", C.c_double),
        ("stall_cycles", C.c_int32),
        ("use_graph", C.c_int32),
        ("autotune", C.c_int32),
        ("batch_schedule", C.c_int32),
        ("spmv_block_nnz", C.c_int32),
        ("a_storage", C.c_int32),
        ("restart_repeat", C.c_int32),
        ("restart_on_stall", C.c_int32),
        ("orth_restart", C.c_double),
        ("orth_norm", C.c_int32),
        ("ilu_sweeps", C.c_int32),
        ("arnoldi_a", C.c_int32),
        ("precond_precision", C.c_int32),
        ("persistent_spmv", C.c_int32),
        ("precond_side", C.c_int32),
        ("spmv_format", C.c_int32),
    ]


class Result(C.Structure):
    _fields_ = [
        ("status", C.c_int32),
        ("iters", C.c_int64),
        ("restarts", C.c_int64),
        ("rel_residual", C.c_double),
        ("seconds", C.c_double),
        ("fallback_used", C.c_int32),
        ("first_stall", C.c_int32),
    ]

    def as_dict(self):
        return {
            "status": STATUS_NAMES.get(self.status, str(self.status)),
            "iters": int(self.iters),
            "restarts": int(self.restarts),
            "rel_residual": float(self.rel_residual),
            "seconds": float(self.seconds),
            "fallback_used": bool(self.fallback_used),
            "first_stall": int(self.first_stall),
        }


class KernelProfile(C.Structure):
    _fields_ = [
        ("ms", C.c_double),
        ("ms_active", C.c_double),
        ("bytes", C.c_double),
        ("launches", C.c_int64),
        ("active", C.c_int64),
    ]


class TuneClass(C.Structure):
    _fields_ = [
        ("rows_per_thread", C.c_int32),
        ("systems", C.c_int32),
        ("largest_n", C.c_int32),
        ("probe_system", C.c_int32),
    ]


# kernel families of gmres_solve_profiled (GMRES_PK_* in gmres.h)
PROFILE_KINDS = ["spmv", "pass1", "pass2", "final", "mgs", "residual", "update", "reduce", "precond", "encode"]

_vp = C.c_void_p
_SIGS = {
    "gmres_default_options": (None, [C.POINTER(Options)]),
    "gmres_strerror": (C.c_char_p, [C.c_int]),
    "gmres_create": (C.c_int, [C.POINTER(_vp), C.c_int64, C.c_int64, _vp, _vp, _vp, C.POINTER(Options), _vp]),
    "gmres_batch_create": (C.c_int, [C.POINTER(_vp), C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp), C.POINTER(Options), _vp]),
    "gmres_set_preconditioner": (C.c_int, [_vp, _vp]),
    "gmres_solve": (C.c_int, [_vp, _vp, _vp, C.POINTER(Result)]),
    "gmres_batch_solve": (C.c_int, [_vp, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(Result)]),
    "gmres_destroy": (C.c_int, [_vp]),
    "gmres_release_cached_memory": (C.c_int, [C.POINTER(C.c_size_t)]),
    "gmres_residual": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double)]),
    "gmres_backward_error": (C.c_int, [_vp, _vp, _vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "gmres_residual_unit": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double)]),
    "gmres_spmv": (C.c_int, [_vp, C.c_int32, _vp, _vp]),
    "gmres_precond_apply": (C.c_int, [_vp, _vp, _vp]),
    "gmres_precond_apply_f64": (C.c_int, [_vp, _vp, _vp]),
    "gmres_encode": (C.c_int, [C.c_int32, C.c_int64, _vp, C.c_double, _vp, C.POINTER(C.c_double), _vp]),
    "gmres_encode_noalloc": (C.c_int, [C.c_int32, C.c_int64, _vp, C.c_double, _vp, C.POINTER(C.c_double), _vp]),
    "gmres_last_cycle": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int32), _vp, _vp]),
    "gmres_history": (C.c_int, [_vp, C.c_int32, _vp, C.c_int32, C.POINTER(C.c_int32)]),
    "gmres_memory_bytes": (C.c_int, [_vp, C.POINTER(C.c_size_t)]),
    "gmres_batch_tuning": (C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(TuneClass),
                                     C.c_int32, C.POINTER(C.c_int32)]),
    "gmres_time_kernel": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]),
    "gmres_solve_profiled": (C.c_int, [_vp, _vp, _vp, C.POINTER(Result), C.POINTER(KernelProfile),
                                       C.POINTER(KernelProfile)]),
    "gmres_launch_config": (C.c_int, [_vp, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "gmres_spmv_config": (C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]),
    "gmres_spai_infer": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
    "spai_create": (C.c_int, [C.POINTER(_vp), C.c_int64, C.c_int64, _vp, _vp, C.c_int32, _vp]),
    "spai_set_values": (C.c_int, [_vp, _vp]),
    "spai_forward": (C.c_int, [_vp, _vp, _vp]),
    "spai_loss": (C.c_int, [_vp, _vp, _vp, C.c_int32, C.POINTER(C.c_double), _vp]),
    "spai_backward": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int32]),
    "spai_destroy": (C.c_int, [_vp]),
    "spai_same_pattern": (C.c_int, [_vp, C.c_int64, C.c_int64, _vp, _vp, C.POINTER(C.c_int32)]),
    "gmres_spai_infer_with": (C.c_int, [_vp, _vp, _vp, C.c_size_t, _vp]),
    "spai_adam_step": (C.c_int, [C.c_int64, _vp, _vp, _vp, C.c_float, _vp, _vp, C.c_float, C.c_float, C.c_float,
                                 C.c_float, C.c_int32, _vp]),
}

SPAI_NPARAMS, SPAI_HIDDEN = 9665, 32

_LIB = None


class GmresError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


def load(path: str | None = None):
    """Load the built library (fails loudly when it has not been built)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libgmres.so is not built ({p}); run `python -m paper_2011_01850_amd.build`")
    lib = C.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _LIB = lib
    return lib


def strerror(code: int) -> str:
    return load().gmres_strerror(int(code)).decode()


def check(code: int, what: str):
    if code != OK:
        raise GmresError(code, what)


def default_options() -> Options:
    o = Options()
    load().gmres_default_options(C.byref(o))
    return o
