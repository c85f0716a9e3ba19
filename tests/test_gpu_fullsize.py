"""The benchmark workload at full size (128^3 convection-diffusion, n = 2,097,152)
in the launch configuration bench.py times, checked by properties that hold at
any size and by outputs the oracle computes one by one."""
import math
import time

import numpy as np
import pytest

import problems as P
from oracle import gmres as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2011_01850_amd.solver import Solver  # noqa: E402


@pytest.fixture(scope="module")
def c2():
    return P.c2_convdiff3d(128)


def test_fullsize_spmv_rows_sampled(c2):
    A = c2.A
    s = Solver(A.row_ptr, A.col_idx, A.vals, m=50, ortho="cgsr", precision="fp32")
    g = np.random.default_rng(7)
    x = g.standard_normal(A.n)
    y64 = s.spmv(x, "fp64").cpu().numpy()
    y32 = s.spmv(x.astype(np.float32), "fp32").cpu().numpy()
    s.close()
    rows = np.concatenate([g.integers(0, A.n, 2000), [0, 1, A.n - 2, A.n - 1, 128 * 128 - 1]])
    for r in rows:
        lo, hi = A.row_ptr[r], A.row_ptr[r + 1]
        ref = float(np.dot(A.vals[lo:hi], x[A.col_idx[lo:hi]]))
        ref32 = float(np.dot(A.vals[lo:hi].astype(np.float32).astype(np.float64),
                             x.astype(np.float32)[A.col_idx[lo:hi]].astype(np.float64)))
        scale = float(np.abs(A.vals[lo:hi]).dot(np.abs(x[A.col_idx[lo:hi]])))
        assert abs(y64[r] - ref) <= 8 * O.U64 * scale
        assert abs(y32[r] - ref32) <= 8 * O.U32 * scale


@pytest.mark.parametrize("ortho", ["cgsr", "mgs"])
def test_fullsize_mixed_solve_reaches_1e10(c2, ortho):
    A = c2.A
    s = Solver(A.row_ptr, A.col_idx, A.vals, m=50, ortho=ortho, precision="fp32", tol=1e-10)
    x, info = s.solve(c2.b)
    hist = s.history()
    s.close()
    x = x.cpu().numpy()
    rr = O.relative_residual(O.Matrix.from_csr(A), c2.b, x)
    fwd = np.linalg.norm(x - c2.x_true) / np.linalg.norm(c2.x_true)
    print(f"128^3 {ortho} fp32: {info['status']} iters {info['iters']} restarts {info['restarts']} "
          f"relres {rr:.3e} forward error {fwd:.2e}", flush=True)
    assert info["status"] == "CONVERGED"
    assert rr <= 1e-10 * 1.001
    assert info["rel_residual"] == pytest.approx(rr, rel=1e-6)
    # restart residuals never increase (the convergence argument of the numerics section)
    assert np.all(np.diff(hist) <= 0)


@pytest.fixture(scope="module")
def c2_oracle(c2):
    # the float64 oracle (CGSR) at full size to 1e-13: the solution every
    # mode is compared with (several minutes on the host's cores)
    # Run cycle by cycle (each call: the residual of the current x, then one
    # GMRES(50) cycle from it), which is restarted GMRES itself, so that every
    # cycle reports its progress
    t0 = time.perf_counter()
    A = O.Matrix.from_csr(c2.A)
    m, x, iters, restarts = 50, None, 0, 0
    while True:
        r = O.gmres(A, c2.b, x0=x, m=m, tol=1e-13, ortho="cgsr", max_iters=m)
        iters += r.iters
        restarts += r.restarts
        x = r.x
        print(f"  oracle cycle {restarts}: relres {r.history[-1]:.2e} after {iters} iterations "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
        if r.status != O.MAXITER:
            break
    print(f"128^3 float64 oracle: {r.status_name} iters {iters} restarts {restarts} relres "
          f"{r.rel_residual:.2e} in {time.perf_counter() - t0:.1f} s", flush=True)
    assert r.status == O.CONVERGED
    r.iters, r.restarts = iters, restarts
    return r


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("ortho,precision", [("cgsr", "fp32"), ("mgs", "fp32"), ("cgsr", "fp64"),
                                             ("mgs", "fp64"), ("cgsr", "fp16"), ("cgsr", "limited")])
def test_fullsize_solution_matches_oracle(c2, c2_oracle, ortho, precision):
    # the benchmark system at full size, each mode to 1e-13 (the launch
    # configuration the benchmark times, autotuned): the solution agrees
    # element by element with the float64 oracle's to 1e-8 relative
    A = c2.A
    s = Solver(A.row_ptr, A.col_idx, A.vals, m=50, ortho=ortho, precision=precision, tol=1e-13)
    x, info = s.solve(c2.b)
    s.close()
    x = x.cpu().numpy()
    rr = O.relative_residual(O.Matrix.from_csr(A), c2.b, x)
    err = float(np.linalg.norm(x - c2_oracle.x) / np.linalg.norm(c2_oracle.x))
    fwd = float(np.linalg.norm(x - c2.x_true) / np.linalg.norm(c2.x_true))
    print(f"128^3 {ortho} {precision}: {info['status']} iters {info['iters']} restarts {info['restarts']} "
          f"relres {rr:.2e} | vs oracle x {err:.2e} (oracle iters {c2_oracle.iters}) | vs x_true {fwd:.2e}",
          flush=True)
    assert info["status"] == "CONVERGED" and rr <= 1.01e-13
    assert err <= 1e-8
    # mixed and float64 need about the same number of cycles (the paper finds
    # equal iteration counts on most of its matrices)
    assert abs(info["restarts"] - c2_oracle.restarts) <= 2


def test_fullsize_first_cycle_basis(c2):
    # one full cycle of the benchmark solver at 128^3: CGS2 keeps the float32
    # basis orthogonal to working accuracy, and A V_k = V_{k+1} Hbar_k holds
    # (A applied by the float64 product, checked above row by row)
    A = c2.A
    m = 50
    s = Solver(A.row_ptr, A.col_idx, A.vals, m=m, ortho="cgsr", precision="fp32", tol=0.0, max_iters=m)
    s.solve(c2.b)
    k, Hb, V = s.last_cycle()
    assert k == m
    G = V.T @ V
    orth = torch.linalg.matrix_norm(torch.eye(k + 1, dtype=torch.float64, device="cuda") - G, ord=2).item()
    AV = torch.stack([s.spmv(V[:, j], "fp64") for j in range(k)], dim=1)
    R = AV - V @ torch.as_tensor(Hb[: k + 1, :k], device="cuda")
    rel = (torch.linalg.norm(R) / np.linalg.norm(A.vals)).item()
    s.close()
    print(f"128^3 first cycle: ||I - V^T V||_2 = {orth:.2e}, ||A V - V Hbar||_F / ||A||_F = {rel:.2e}", flush=True)
    assert orth <= 10 * (k + 1) * O.U32 * 10
    assert rel <= 10 * k * O.U32 * 50


@pytest.fixture(scope="module")
def c3():
    return P.c3_powerlaw()


def test_fullsize_powerlaw_rows_sampled(c3):
    # the power-law workload at its full size: rows up to 2000 entries go
    # through the chunked long-row path; sampled rows against dot products
    A = c3.A
    s = Solver(A.row_ptr, A.col_idx, A.vals, m=30, ortho="cgsr", precision="fp16")
    g = np.random.default_rng(9)
    x = g.standard_normal(A.n)
    y64 = s.spmv(x, "fp64").cpu().numpy()
    s.close()
    lens = np.diff(A.row_ptr)
    rows = np.concatenate([g.integers(0, A.n, 1000), np.argsort(lens)[-20:]])
    assert lens[rows].max() >= 1000
    for r in rows:
        lo, hi = A.row_ptr[r], A.row_ptr[r + 1]
        ref = float(np.dot(A.vals[lo:hi], x[A.col_idx[lo:hi]]))
        scale = float(np.abs(A.vals[lo:hi]).dot(np.abs(x[A.col_idx[lo:hi]])))
        assert abs(y64[r] - ref) <= 16 * O.U64 * scale


def test_fullsize_powerlaw_half_basis_reaches_1e10(c3):
    A = c3.A
    s = Solver(A.row_ptr, A.col_idx, A.vals, m=30, ortho="cgsr", precision="fp16", tol=1e-10, stall_cycles=1000)
    x, info = s.solve(c3.b)
    s.close()
    rr = O.relative_residual(O.Matrix.from_csr(A), c3.b, x.cpu().numpy())
    print(f"power-law 1e6 fp16: {info['status']} iters {info['iters']} relres {rr:.3e}", flush=True)
    assert info["status"] == "CONVERGED" and rr <= 1e-10 * 1.001


def test_fullsize_batch_persistent():
    # the 512-system batch exactly as the batch benchmark solves it (one
    # persistent launch): every system reaches 1e-10 by its own float64
    # residual, and sampled systems are bitwise their single-system solves
    from paper_2011_01850_amd import BatchSolver

    probs = P.c4_batch()
    bs = BatchSolver([(p.A.row_ptr, p.A.col_idx, p.A.vals) for p in probs], m=40, ortho="mgs",
                     precision="fp32", tol=1e-10, schedule="persistent")
    xs, infos = bs.solve([p.b for p in probs])
    bs.close()
    assert all(i["status"] == "CONVERGED" for i in infos)
    worst = 0.0
    for p, x in zip(probs, xs):
        rr = O.relative_residual(O.Matrix.from_csr(p.A), p.b, x.cpu().numpy())
        worst = max(worst, rr)
    its = [i["iters"] for i in infos]
    print(f"batch of 512: iterations {min(its)} / {int(np.median(its))} / {max(its)}, worst relres {worst:.3e}",
          flush=True)
    assert worst <= 1e-10 * 1.001
    g = np.random.default_rng(4)
    for k in list(g.choice(512, 3, replace=False)) + [int(np.argmax(its))]:
        p = probs[k]
        s = Solver(p.A.row_ptr, p.A.col_idx, p.A.vals, m=40, ortho="mgs", precision="fp32", tol=1e-10,
                   schedule="persistent")
        x1, i1 = s.solve(p.b)
        s.close()
        assert i1["iters"] == infos[k]["iters"]
        assert torch.equal(x1, xs[k]), k


def _spai_theta(seed):
    from oracle import mpnn as N

    g = np.random.default_rng(seed)
    th = N.init_params(seed)
    o, _ = N.OFFSETS["wo"]
    th[o:o + N.U] = g.normal(0, 0.05, N.U)
    th[N.OFFSETS["bo"][0]] = 0.01
    for name in ("bn", "be", "b1", "b2", "b3"):
        o, shape = N.OFFSETS[name]
        th[o:o + shape[0]] = g.normal(0, 0.1, shape[0])
    return th


def test_fullsize_spai_forward():
    # the learned preconditioner's inference on a held-out 64^3
    # variable-coefficient instance against the float64 network oracle on the
    # same bfloat16-rounded parameters (the learned part of M: M minus its
    # Jacobi start)
    from oracle import mpnn as N
    from paper_2011_01850_amd import spai

    A = P.c5_varcoef(2000).A
    G = N.graph(A.n, A.row_ptr, A.col_idx, A.vals)
    th = _spai_theta(1)
    M_or = N.forward(torch.as_tensor(N.round_bf16(th)), G).numpy()
    net = spai.SpaiNet(A.row_ptr, A.col_idx, kmax=4)
    net.set_values(A.vals)
    M_gpu = net.forward(torch.as_tensor(spai.params_to_bf16(th)).cuda()).cpu().numpy().astype(np.float64)
    net.close()
    diag = (G.rows == G.cols).numpy()
    J = np.where(diag, G.sigma.numpy()[G.rows.numpy()] / np.sqrt(G.d.numpy()[G.rows.numpy()] ** 2), 0.0)
    a, b = M_gpu - J, M_or - J
    cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
    rel = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    print(f"64^3 inference: learned part cos {cos:.7f} rel {rel:.2e}", flush=True)
    assert np.all(np.isfinite(M_gpu))
    assert cos >= 0.99999 and rel <= 1e-3


@pytest.fixture(scope="module")
def c5():
    return P.c5_varcoef(2000)  # the first held-out instance of the learned-preconditioner workload


@pytest.mark.timeout(900)
@pytest.mark.parametrize("kind", ["jacobi", "learned"])
def test_fullsize_varcoef_fgmres_matches_oracle(c5, kind):
    # FGMRES(30) on a held-out 64^3 variable-coefficient instance, to 1e-13:
    # Jacobi, and the network's M (GPU inference on bfloat16 weights; the
    # oracle applies the float64 network's M to the same weights), against the
    # float64 FGMRES oracle element by element
    from oracle import mpnn as N
    from paper_2011_01850_amd import spai

    A = c5.A
    M = O.Matrix.from_csr(A)
    if kind == "jacobi":
        d = M.diagonal()
        d32 = (1.0 / d).astype(np.float32)
        pc = lambda v: v / d  # noqa: E731
        # the mixed solver stores M = D^-1 in float32; this slowly converging
        # system is sensitive to that rounding (about 25% more cycles), so the
        # float32 emulation applies the same float32 D^-1
        pc32 = lambda v: (np.asarray(v, dtype=np.float32) * d32).astype(np.float32)  # noqa: E731
    else:
        # seeded weights with the decoder's output scaled so that the learned
        # part of M is a few percent of its Jacobi start (a usable preconditioner)
        th = _spai_theta(1)
        o, _ = N.OFFSETS["wo"]
        th[o:o + N.U] *= 0.03
        th[N.OFFSETS["bo"][0]] *= 0.03
        G = N.graph(A.n, A.row_ptr, A.col_idx, A.vals)
        Mo = O.Matrix(A.row_ptr, A.col_idx, N.forward(torch.as_tensor(N.round_bf16(th)), G).numpy(), A.n)
        pc = pc32 = Mo.matvec
    t0 = time.perf_counter()
    ref = O.gmres(M, c5.b, m=30, tol=1e-13, ortho="cgsr", precond=pc, fallback=False, max_iters=20000)
    t_or = time.perf_counter() - t0
    print(f"  float64 oracle: {ref.status_name} iters {ref.iters} ({t_or:.1f} s)", flush=True)
    # the GPU's float32 Arnoldi needs more steps near 1e-13 than float64: its
    # iteration count is compared with the oracle's float32 emulation
    emu = O.gmres(M, c5.b, m=30, tol=1e-13, ortho="cgsr", precond=pc32, fallback=False, max_iters=20000,
                  precision="fp32")
    s = Solver(A.row_ptr, A.col_idx, A.vals, m=30, ortho="cgsr", precision="fp32",
               precond="jacobi" if kind == "jacobi" else "spai", tol=1e-13)
    if kind == "learned":
        s.spai_infer(torch.as_tensor(spai.params_to_bf16(th)).cuda(), return_m=False)
    x, info = s.solve(c5.b)
    hist = s.history()
    s.close()
    x = x.cpu().numpy()
    rr = O.relative_residual(M, c5.b, x)
    err = float(np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x))

    def cycles_to(h, level):
        return next(k for k, v in enumerate(h) if v <= level)
    print(f"64^3 FGMRES {kind}: gpu {info['status']} iters {info['iters']} relres {rr:.2e} fallback "
          f"{info['fallback_used']} | oracle {ref.status_name} iters {ref.iters} ({t_or:.1f} s), float32 "
          f"emulation {emu.status_name} iters {emu.iters} | cycles to 1e-10: gpu {cycles_to(hist, 1e-10)}, "
          f"emulation {cycles_to(emu.history, 1e-10)} | vs oracle x {err:.2e}", flush=True)
    assert ref.status == O.CONVERGED and emu.status == O.CONVERGED
    assert info["status"] == "CONVERGED" and not info["fallback_used"] and rr <= 1.01e-13
    assert err <= 1e-8
    # this FGMRES converges slowly and its float32 trajectory is sensitive to
    # rounding: on the host alone, rounding D^-1 to float32 moves the count to
    # 1e-10 by 5 of 21 cycles, and the GPU's sums run in another order; the
    # counts are reported and held to within a third of the emulation's
    ce = cycles_to(emu.history, 1e-10)
    assert abs(cycles_to(hist, 1e-10) - ce) <= max(2, math.ceil(0.35 * ce))
