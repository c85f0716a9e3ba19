"""Host-side checks of the C-ABI library: it loads, exports what the header declares,
and rejects bad arguments before touching the GPU (no compute calls here)."""
import ctypes as C
import os
import re

import pytest

from paper_2011_01850_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("gmres.h", "spai.h")]


def _declared():
    names = set()
    for hdr in HEADERS:
        src = open(hdr).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b((?:gmres|spai)_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 22
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares every one of them
    assert set(names) == set(L._SIGS), set(names) ^ set(L._SIGS)


def test_default_options(lib):
    o = L.default_options()
    assert (o.m, o.tol, o.max_iters) == (50, 1e-10, 100000)
    assert o.ortho == L.CGSR and o.precision == L.MIXED_FP32 and o.precond == L.PRECOND_NONE
    assert o.restart_improve == 0.0 and o.stall_cycles == 10 and o.use_graph == 1 and o.autotune == 1
    assert o.batch_schedule == L.SCHEDULE_AUTO and o.spmv_block_nnz == 0 and o.a_storage == L.A_COPY
    assert o.restart_repeat == 0 and o.restart_on_stall == 0 and o.orth_restart == 0.0 and o.orth_norm == 0
    assert o.ilu_sweeps == 4 and o.arnoldi_a == L.ARNOLDI_A_DEFAULT


def test_strerror(lib):
    assert L.strerror(0) == "ok"
    assert "invalid" in L.strerror(L.EINVAL)
    assert "handle" in L.strerror(L.EHANDLE)
    assert L.strerror(-99) == "unknown error"


def test_invalid_arguments_rejected_before_device_work(lib):
    o = L.default_options()
    h = C.c_void_p()
    assert lib.gmres_create(C.byref(h), 0, 0, None, None, None, C.byref(o), None) == L.EINVAL
    assert lib.gmres_create(C.byref(h), 10, 5, None, None, None, C.byref(o), None) == L.EINVAL
    assert lib.gmres_create(None, 10, 5, 1, 1, 1, C.byref(o), None) == L.EINVAL
    for field, bad in [("m", 0), ("m", 257), ("tol", -1.0), ("ortho", 7), ("precision", 9), ("precision", 5), ("precision", -1),
                       ("precond", 5), ("stall_cycles", 0), ("restart_improve", -0.5), ("batch_schedule", 3),
                       ("batch_schedule", -1), ("spmv_block_nnz", 32), ("spmv_block_nnz", 100),
                       ("spmv_block_nnz", 8256), ("a_storage", 2), ("a_storage", -1), ("restart_repeat", 2),
                       ("restart_on_stall", -1), ("orth_restart", -1.0), ("orth_restart", float("inf")),
                       ("orth_norm", 2), ("ilu_sweeps", -1), ("ilu_sweeps", 4097),
                       ("arnoldi_a", 3), ("arnoldi_a", -1), ("persistent_spmv", -1), ("persistent_spmv", 4), ("precond_side", 2),
                       ("precond_side", -1), ("spmv_format", 4), ("spmv_format", -1)]:
        ob = L.default_options()
        setattr(ob, field, bad)
        assert lib.gmres_create(C.byref(h), 10, 5, 1, 1, 1, C.byref(ob), None) == L.EINVAL, field
    # the loss-of-orthogonality monitor keeps U and S in LDS: m <= 64
    ob = L.default_options()
    ob.orth_restart = 0.5
    ob.m = 65
    assert lib.gmres_create(C.byref(h), 10, 5, 1, 1, 1, C.byref(ob), None) == L.EINVAL
    # the preconditioner's precision: the solver's own, or float32
    for bad in (2, -1):
        ob = L.default_options()
        ob.precision = L.FP64
        ob.precond = L.PRECOND_JACOBI
        ob.precond_precision = bad
        assert lib.gmres_create(C.byref(h), 10, 5, 1, 1, 1, C.byref(ob), None) == L.EINVAL
    assert lib.gmres_encode(L.FP64, 10, 1, 1.0, 1, None, None) == L.EINVAL
    assert lib.gmres_encode(L.MIXED_FP16, 10, 1, 0.0, 1, None, None) == L.EINVAL
    # the no-allocation variant: the same checks, and no more than 2^24 elements
    assert lib.gmres_encode_noalloc(L.FP64, 10, 1, 1.0, 1, None, None) == L.EINVAL
    assert lib.gmres_encode_noalloc(L.MIXED_FP16, 10, 1, 0.0, 1, None, None) == L.EINVAL
    assert lib.gmres_encode_noalloc(L.MIXED_BF16, 10, None, 1.0, 1, None, None) == L.EINVAL
    assert lib.gmres_encode_noalloc(L.MIXED_BF16, 2 ** 24 + 1, 1, 1.0, 1, None, None) == L.EINVAL


def test_unaddressable_sizes_rejected_before_device_work(lib):
    # the basis is read through 32-bit buffer offsets: (m + 1) padded columns
    # must stay below 4 GiB; row pointers and column indices are int32.  The
    # pointers below are never dereferenced: the sizes are refused first.
    h = C.c_void_p()
    n128 = 128 ** 3  # 2,097,152 rows, a multiple of the 256-row tile
    # (accepted sizes are not tried here: the call would go on to read the fake pointers)
    for prec, m in [(L.FP64, 255), (L.FP64, 256)]:  # 256 x 2^21 x 8 = 2^32 bytes
        o = L.default_options()
        o.precision, o.m = prec, m
        assert lib.gmres_create(C.byref(h), n128, 7 * n128, 16, 16, 16, C.byref(o), None) == L.EINVAL, m
    # float32 / half bases of the same system fit: 257 x 2^21 x 4 < 2^32
    assert 257 * n128 * 4 < 2 ** 32
    # float32 basis of 4 GiB: 2^23 + 256 rows pad to 2^23 + 256, (m + 1) = 128 columns
    o = L.default_options()
    o.precision, o.m = L.MIXED_FP32, 127
    assert lib.gmres_create(C.byref(h), 2 ** 23 + 1, 10, 16, 16, 16, C.byref(o), None) == L.EINVAL
    # rows and non-zeros beyond int32
    o = L.default_options()
    o.m = 1
    assert lib.gmres_create(C.byref(h), 2 ** 31, 10, 16, 16, 16, C.byref(o), None) == L.EINVAL
    assert lib.gmres_create(C.byref(h), 1000, 2 ** 31 - 1028, 16, 16, 16, C.byref(o), None) == L.EINVAL
    # a batch whose padded rows add up past int32
    ns = (C.c_int64 * 2)(2 ** 30, 2 ** 30)
    zs = (C.c_int64 * 2)(10, 10)
    ptrs = (C.c_void_p * 2)(16, 16)
    assert lib.gmres_batch_create(C.byref(h), 2, ns, zs, ptrs, ptrs, ptrs, C.byref(o), None) == L.EINVAL


def test_handle_checks(lib):
    assert lib.gmres_destroy(None) == L.OK
    r = L.Result()
    assert lib.gmres_solve(None, 1, 1, C.byref(r)) == L.EHANDLE
    v = C.c_size_t()
    assert lib.gmres_memory_bytes(None, C.byref(v)) == L.EHANDLE
    assert lib.gmres_precond_apply(None, None, None) == L.EHANDLE
    assert lib.gmres_precond_apply_f64(None, 1, 1) == L.EHANDLE
    prof = (L.KernelProfile * len(L.PROFILE_KINDS))()
    assert lib.gmres_solve_profiled(None, 1, 1, None, prof, None) == L.EHANDLE
    # a pointer to something that is not a handle
    junk = (C.c_uint32 * 64)()
    assert lib.gmres_memory_bytes(C.cast(junk, C.c_void_p), C.byref(v)) == L.EHANDLE


def test_struct_layouts_match_header():
    # offsets that C gives the two structs on x86-64
    assert C.sizeof(L.Options) == 120
    assert L.Options.tol.offset == 8 and L.Options.max_iters.offset == 16
    assert L.Options.restart_improve.offset == 40 and L.Options.autotune.offset == 56
    assert L.Options.batch_schedule.offset == 60 and L.Options.spmv_block_nnz.offset == 64
    assert L.Options.a_storage.offset == 68 and L.Options.restart_repeat.offset == 72
    assert L.Options.restart_on_stall.offset == 76 and L.Options.orth_restart.offset == 80
    assert L.Options.orth_norm.offset == 88 and L.Options.ilu_sweeps.offset == 92
    assert L.Options.arnoldi_a.offset == 96 and L.Options.precond_precision.offset == 100
    assert L.Options.persistent_spmv.offset == 104 and L.Options.precond_side.offset == 108
    assert L.Options.spmv_format.offset == 112
    assert C.sizeof(L.Result) == 48
    assert L.Result.iters.offset == 8 and L.Result.first_stall.offset == 44


def test_spai_arguments_rejected_before_device_work(lib):
    h = C.c_void_p()
    assert lib.spai_create(None, 10, 5, 1, 1, 4, None) == L.EINVAL
    assert lib.spai_create(C.byref(h), 0, 5, 1, 1, 4, None) == L.EINVAL
    assert lib.spai_create(C.byref(h), 10, 0, 1, 1, 4, None) == L.EINVAL
    assert lib.spai_create(C.byref(h), 10, 5, None, 1, 4, None) == L.EINVAL
    assert lib.spai_create(C.byref(h), 10, 5, 1, 1, 0, None) == L.EINVAL
    assert lib.spai_create(C.byref(h), 10, 5, 1, 1, 65, None) == L.EINVAL
    assert lib.spai_destroy(None) == L.OK
    assert lib.spai_adam_step(0, 1, 1, 1, 1.0, 1, 1, 1e-3, 0.9, 0.999, 1e-8, 1, None) == L.EINVAL
    assert lib.spai_adam_step(10, 1, 1, 1, 1.0, 1, 1, 1e-3, 1.0, 0.999, 1e-8, 1, None) == L.EINVAL
    assert lib.spai_adam_step(10, 1, 1, 1, 1.0, 1, 1, 1e-3, 0.9, 0.999, 1e-8, 0, None) == L.EINVAL
    assert lib.gmres_spai_infer(None, 1, 2 * L.SPAI_NPARAMS, None) == L.EHANDLE


def test_spai_layout_matches_oracle():
    from oracle import mpnn as N
    from paper_2011_01850_amd import spai as S
    assert S.NPARAMS == N.NPARAMS == L.SPAI_NPARAMS
    assert S.offsets() == N.OFFSETS


def test_struct_layouts_match_compiled_header(tmp_path):
    # the ctypes mirrors against what a C compiler makes of include/gmres.h
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "gmres.h"', "int main(void) {"]
    structs = (("gmres_options", L.Options), ("gmres_result", L.Result), ("gmres_kernel_profile", L.KernelProfile),
               ("gmres_tune_class", L.TuneClass))
    for cname, ct in structs:
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in ct._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append('  printf("GMRES_PK_COUNT value %d\\n", (int)GMRES_PK_COUNT);')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, ct in structs:
        assert got[(cname, "sizeof")] == C.sizeof(ct), cname
        for fname, _ in ct._fields_:
            assert got[(cname, fname)] == getattr(ct, fname).offset, (cname, fname)
    assert got[("GMRES_PK_COUNT", "value")] == len(L.PROFILE_KINDS)


def test_binding_forwards_every_solver_option(lib):
    # every keyword of the Python front end reaches a field of gmres_options
    import inspect

    from paper_2011_01850_amd import solver as S

    params = inspect.signature(S._options).parameters
    for cls in (S.Solver, S.BatchSolver):
        for name in inspect.signature(cls.__init__).parameters:
            if name in ("self", "row_ptr", "col_idx", "vals", "systems"):
                continue
            assert name in params, (cls.__name__, name)
    o = S._options(30, 1e-9, 500, "mgs", "fp64", "ilu0", 1e-6, 7, False, False, "persistent", 1024, "split",
                   True, True, 0.5, "frobenius", 0, "fp32", "fp32", "ell16", "left", "sell")
    assert (o.m, o.max_iters, o.ortho, o.precision, o.precond) == (30, 500, L.MGS, L.FP64, L.PRECOND_ILU0)
    assert (o.stall_cycles, o.use_graph, o.autotune, o.batch_schedule) == (7, 0, 0, L.SCHEDULE_PERSISTENT)
    assert (o.spmv_block_nnz, o.a_storage, o.restart_repeat, o.restart_on_stall) == (1024, L.A_SPLIT, 1, 1)
    assert (o.orth_norm, o.ilu_sweeps, o.arnoldi_a) == (L.ORTH_FROBENIUS, 0, L.ARNOLDI_A_FP32)
    assert (o.precond_precision, o.persistent_spmv) == (L.PRECOND_FP32, 1 + L.PSPMV_ELL16)
    assert o.precond_side == L.PRECOND_LEFT and o.spmv_format == L.SPMV_SELL
    assert o.tol == 1e-9 and o.restart_improve == 1e-6 and o.orth_restart == 0.5
