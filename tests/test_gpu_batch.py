"""The persistent batch schedule (one workgroup per system, one launch per
solve) against the CPU oracle, and its invariants.

Parity bar (as for the single-system path): both sides run to tol 1e-13,
and ||x_gpu - x_oracle|| / ||x_oracle|| <= 1e-8, with the float64 relative
residual of the GPU iterate <= 1e-13.  A system's result must not depend
on the rest of the batch: a batch and the same system solved alone under the
same schedule agree bitwise.
"""
import numpy as np
import pytest
import torch

import problems as P
from oracle import gmres as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_01850_amd import GmresError
    from paper_2011_01850_amd.solver import BatchSolver, Solver
    return BatchSolver, Solver, GmresError


# sides chosen for every row-count path: n = 400 (1 row per thread), 1089
# (2, ragged), 4096 (4), 10000 (10 -> 16), 16900 (17 -> 32), 40000 (40 -> 64)
SIDES = [(20, (10.0, 3.0)), (33, (0.0, 0.0)), (64, (80.0, 40.0)), (100, (5.0, 50.0)), (130, (30.0, 0.0)),
         (200, (60.0, 60.0))]


def _systems():
    systems = [P.convdiff(N, beta) for N, beta in SIDES]
    rhs = [P.manufactured_rhs(A, 96, i)[1] for i, A in enumerate(systems)]
    return systems, rhs


def test_persistent_batch_matches_oracle(mods):
    BatchSolver, Solver, _ = mods
    systems, rhs = _systems()
    bs = BatchSolver([(A.row_ptr, A.col_idx, A.vals) for A in systems], m=40, ortho="mgs", precision="fp32",
                     tol=1e-13, schedule="persistent")
    xs, infos = bs.solve(rhs)
    bs.close()
    for A, b, x, info in zip(systems, rhs, xs, infos):
        ref = O.gmres(O.Matrix.from_csr(A), b, m=40, tol=1e-13, ortho="mgs")
        xg = x.cpu().numpy()
        err = np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x)
        rr = O.relative_residual(O.Matrix.from_csr(A), b, xg)
        print(f"n={A.n}: iters gpu {info['iters']} oracle {ref.iters}, err {err:.2e}, relres {rr:.2e}")
        assert info["status"] == "CONVERGED"
        assert rr <= 1e-13 * 1.01 and abs(info["rel_residual"] - rr) <= 1e-3 * rr + 1e-16
        assert err <= 1e-8


def test_batch_equals_persistent_single_bitwise(mods):
    BatchSolver, Solver, _ = mods
    systems, rhs = _systems()
    bs = BatchSolver([(A.row_ptr, A.col_idx, A.vals) for A in systems], m=40, ortho="mgs", precision="fp32")
    xb, ib = bs.solve(rhs)
    xb2, ib2 = bs.solve(rhs)  # a replay of the same graph gives the same bits
    bs.close()
    for k, (A, b) in enumerate(zip(systems, rhs)):
        assert np.array_equal(xb[k].cpu().numpy(), xb2[k].cpu().numpy())
        s = Solver(A.row_ptr, A.col_idx, A.vals, m=40, ortho="mgs", precision="fp32", schedule="persistent")
        x1, i1 = s.solve(b)
        s.close()
        assert ib[k]["iters"] == i1["iters"] and ib[k]["restarts"] == i1["restarts"]
        assert np.array_equal(xb[k].cpu().numpy(), x1.cpu().numpy())


def test_spmv_variants_are_bitwise_equal_and_tuned(mods):
    # the persistent kernel's SpMV variants (CSR in groups of 8 or 4, the ELL
    # copy with 16-bit columns) add each row's products in storage order: the
    # whole solve is the same bit for bit whichever the tuner picks
    BatchSolver, Solver, _ = mods
    systems, rhs = _systems()
    csr = [(A.row_ptr, A.col_idx, A.vals) for A in systems]
    out = {}
    for var in ("csr8", "csr4", "ell16", "tuned"):
        bs = BatchSolver(csr, m=40, ortho="mgs", precision="fp32", persistent_spmv=var)
        xs, infos = bs.solve(rhs)
        tune = bs.tuning()
        bs.close()
        out[var] = ([x.cpu().numpy() for x in xs], [i["iters"] for i in infos])
        print(var, out[var][1], tune, flush=True)
        assert len(tune["classes"]) == 6  # one size class per row-count tier of SIDES
        assert sum(c["systems"] for c in tune["classes"]) == len(systems)
        if var != "tuned":
            assert tune["variant"] == var and tune["probe_us"] == {}
        else:
            assert set(tune["probe_us"]) == {"csr8", "csr4", "ell16"}
            assert tune["variant"] == min(tune["probe_us"], key=tune["probe_us"].get)
    for var in ("csr4", "ell16", "tuned"):
        assert out[var][1] == out["csr8"][1]
        for a, b in zip(out[var][0], out["csr8"][0]):
            assert np.array_equal(a, b), var


def test_graph_and_stream_agree(mods):
    BatchSolver, _, _ = mods
    systems, rhs = _systems()
    out = []
    for g in (True, False):
        bs = BatchSolver([(A.row_ptr, A.col_idx, A.vals) for A in systems[:4]], m=30, ortho="mgs",
                         precision="fp32", use_graph=g)
        xs, infos = bs.solve(rhs[:4])
        out.append([x.cpu().numpy() for x in xs])
        bs.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_edge_cases(mods):
    """A zero right-hand side, a 1x1 system, n = 1024 exactly, the largest
    size (65,536 rows), and a system that runs out of iterations."""
    BatchSolver, _, _ = mods
    A0 = P.convdiff(32, (5.0, 5.0))                  # n = 1024
    A1 = P.dense_to_csr(np.array([[4.0]]))           # 1 x 1
    A2 = P.convdiff(256, (20.0, 20.0))               # n = 65536
    A3 = P.convdiff(48, (0.0, 0.0))                  # budget-limited
    systems = [A0, A1, A2, A3]
    rhs = [np.zeros(A0.n), np.array([2.0]), P.manufactured_rhs(A2, 97, 0)[1], P.manufactured_rhs(A3, 97, 1)[1]]
    bs = BatchSolver([(A.row_ptr, A.col_idx, A.vals) for A in systems], m=40, ortho="mgs", precision="fp32",
                     max_iters=2000)
    xs, infos = bs.solve(rhs)
    bs.close()
    assert infos[0]["status"] == "CONVERGED" and infos[0]["iters"] == 0 and not xs[0].abs().max().item()
    assert infos[1]["status"] == "CONVERGED" and abs(xs[1].item() - 0.5) <= 1e-15
    assert infos[2]["status"] == "CONVERGED"
    assert O.relative_residual(O.Matrix.from_csr(A2), rhs[2], xs[2].cpu().numpy()) <= 1e-10 * 1.01
    # max_iters = 2000 is enough for the small Poisson system; a tight budget gives MAXITER
    bs = BatchSolver([(A3.row_ptr, A3.col_idx, A3.vals)] * 2, m=20, ortho="mgs", precision="fp32", max_iters=30)
    xs, infos = bs.solve([rhs[3], rhs[3]])
    bs.close()
    assert all(i["status"] == "MAXITER" and i["iters"] == 30 for i in infos)


def test_arnoldi_relation_of_last_cycle(mods):
    """A V_k = V_{k+1} Hbar_k to float32 working accuracy in the persistent kernel."""
    BatchSolver, _, _ = mods
    import ctypes as C
    A = P.convdiff(40, (30.0, 10.0))
    b = P.manufactured_rhs(A, 98, 0)[1]
    bs = BatchSolver([(A.row_ptr, A.col_idx, A.vals)] * 2, m=25, ortho="mgs", precision="fp32", max_iters=25,
                     tol=0.0)
    bs.solve([b, b])
    k = C.c_int32()
    Hb = np.zeros((26, 25), order="F")
    V = torch.zeros((26, A.n), dtype=torch.float64, device="cuda")
    assert bs.lib.gmres_last_cycle(bs.h, 1, C.byref(k), Hb.ctypes.data, V.data_ptr()) == 0
    bs.close()
    kk = k.value
    assert kk == 25
    Vn = V.cpu().numpy()[: kk + 1].T
    Ad = O.Matrix.from_csr(A).dense()
    lhs = Ad @ Vn[:, :kk]
    rhs_ = Vn @ Hb[: kk + 1, :kk]
    rel = np.linalg.norm(lhs - rhs_) / np.linalg.norm(Ad)
    orth = np.linalg.norm(Vn.T @ Vn - np.eye(kk + 1), 2)
    print(f"relation {rel:.2e}, loss of orthogonality {orth:.2e}")
    # the normalised basis is rounded to float32 after the division by h_{j+1,j}
    assert rel <= 10 * kk * 2.0 ** -24 * 8
    assert np.allclose(np.linalg.norm(Vn, axis=0), 1.0, atol=1e-5)


def test_persistent_requires_its_conditions(mods):
    BatchSolver, Solver, GmresError = mods
    A = P.convdiff(20, (1.0, 1.0))
    for kw in (dict(precision="fp64"), dict(ortho="cgsr"), dict(precond="jacobi"), dict(m=65),
               dict(a_storage="split"), dict(orth_restart=0.5), dict(precision="limited"),
               dict(arnoldi_a="fp64")):
        opts = dict(m=20, ortho="mgs", precision="fp32", schedule="persistent")
        opts.update(kw)
        with pytest.raises(GmresError):
            BatchSolver([(A.row_ptr, A.col_idx, A.vals)] * 2, **opts)
    big = P.convdiff(257, (1.0, 1.0))  # n = 66,049 > 65,536
    with pytest.raises(GmresError):
        Solver(big.row_ptr, big.col_idx, big.vals, m=20, ortho="mgs", precision="fp32", schedule="persistent")


def test_row_pointer_checks_and_large_batch_offsets(mods):
    # the host checks of the row pointer run in parallel chunks on inputs of
    # a million rows and more: every kind of broken row pointer is refused,
    # and the shifted, padded global row pointer of a batch of large systems
    # gives each system its single-system result (up to the float32 rounding
    # order of the device-wide passes, whose partial sums are cut per batch)
    BatchSolver, Solver, GmresError = mods
    A = P.convdiff(102, (5.0, 2.0, 1.0))  # n = 1,061,208
    n = A.n
    for i, bad in [(0, 1), (n, A.nnz - 1), (500_000, int(A.row_ptr[500_001]) + 1)]:
        rp = A.row_ptr.copy()
        rp[i] = bad
        with pytest.raises(GmresError):
            Solver(rp, A.col_idx, A.vals, m=10, precision="fp32")
    ci = A.col_idx.copy()
    ci[777_777] = n  # a column past the matrix
    with pytest.raises(GmresError):
        Solver(A.row_ptr, ci, A.vals, m=10, precision="fp32")
    systems = [P.convdiff(760, (1.0 + k, 0.5)) for k in range(3)]  # 577,600 rows each
    bs = [P.manufactured_rhs(S, 5, k)[1] for k, S in enumerate(systems)]
    kw = dict(m=20, ortho="cgsr", precision="fp32", tol=1e-12, max_iters=40, autotune=False)
    batch = BatchSolver([(S.row_ptr, S.col_idx, S.vals) for S in systems], schedule="device_wide", **kw)
    xs, infos = batch.solve(bs)
    batch.close()
    for k, S in enumerate(systems):
        s = Solver(S.row_ptr, S.col_idx, S.vals, **kw)
        x, info = s.solve(bs[k])
        s.close()
        assert info["iters"] == infos[k]["iters"] == 40
        assert infos[k]["rel_residual"] == pytest.approx(info["rel_residual"], rel=1e-3)
        assert (torch.linalg.norm(x - xs[k]) / torch.linalg.norm(x)).item() <= 1e-4, k
