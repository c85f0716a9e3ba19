"""Pins for the CPU oracle: facts fixed by the paper and by the mathematics.

None of these tests re-types the oracle's own formulas: each compares it with
a hand-worked example, a closed form, a textbook invariant, a library routine
or brute force, chosen so that a dropped term, a wrong sign, a wrong index or
a transposed operand in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import problems as P
from oracle import gmres as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mat(A):
    return O.Matrix.from_csr(A)


def _load_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            out[k] = float(v)
    return out


# --------------------------------------------------------------------------
# hand-worked example (Algorithm 1 on a 2x2 system)

@pytest.mark.parametrize("ortho", ["mgs", "cgsr"])
def test_golden_2x2_worked_example(ortho):
    g = _load_golden("gmres_2x2_worked.txt")
    A = _mat(P.dense_to_csr(np.array([[2.0, 1.0], [0.0, 3.0]])))
    r = O.gmres(A, np.array([0.0, 1.0]), m=2, tol=1e-15, ortho=ortho, record=True)
    assert r.iters == int(g["iters"]) and r.restarts == 1
    c = r.cycles[0]
    Hb = c["Hbar"]
    assert Hb[0, 0] == g["hbar_11"] and Hb[1, 0] == g["hbar_21"]
    assert abs(Hb[0, 1] - g["hbar_12"]) < 1e-15 and abs(Hb[1, 1] - g["hbar_22"]) < 1e-15
    assert abs(Hb[2, 1] - g["hbar_32"]) < 1e-15
    assert math.isclose(c["cs"][0], g["alpha_1"], rel_tol=1e-15)
    assert math.isclose(c["sn"][0], g["beta_1"], rel_tol=1e-15)
    assert c["cs"][1] == g["alpha_2"] and c["sn"][1] == g["beta_2"]
    assert math.isclose(r.arnoldi[0][0], g["s_after_1"], rel_tol=1e-15)
    assert abs(r.arnoldi[0][1] - g["s_after_2"]) < 1e-15
    assert np.allclose(c["y"], [g["y_1"], g["y_2"]], rtol=1e-15, atol=1e-16)
    assert np.allclose(r.x, [g["x_1"], g["x_2"]], rtol=1e-15, atol=1e-16)


# --------------------------------------------------------------------------
# building blocks against library routines / brute force

def test_csr_matvec_integer_exact_vs_dense():
    g = np.random.default_rng(1)
    D = g.integers(-5, 6, size=(37, 37)).astype(float)
    D[g.random((37, 37)) < 0.6] = 0.0
    D[5, :] = 0.0  # an empty row
    A = _mat(P.dense_to_csr(D))
    x = g.integers(-7, 8, size=37).astype(float)
    assert np.array_equal(A.matvec(x), D @ x)
    assert np.array_equal(A.matvec32(x.astype(np.float32)), (D @ x).astype(np.float32))


def test_givens_zeroes_subdiagonal():
    g = np.random.default_rng(2)
    for a, b in list(g.standard_normal((50, 2))) + [(0.0, 1.0), (3.0, 0.0), (-2.0, 0.0), (0.0, 0.0)]:
        b = abs(b)
        c, s = O.givens(a, b)
        assert abs(c * c + s * s - 1.0) < 1e-15
        top = c * a + s * b
        bot = -s * a + c * b
        assert abs(bot) <= 1e-15 * max(1.0, abs(a), b)
        if b != 0.0:
            assert math.isclose(top, math.hypot(a, b), rel_tol=1e-15)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(3)
    x = (g.standard_normal(20000) * 10.0 ** g.integers(-8, 8, 20000)).astype(np.float32)
    # exact ties: low 16 bits = 0x8000, both parities of the kept lsb
    ties = (np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x40490000 | 0x8000], dtype=np.uint32)
            .view(np.float32))
    x = np.concatenate([x, ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(O.round_bf16(x), ref)
    # ties go to even: 1 + 2^-8 (halfway between 1 and 1 + 2^-7) rounds to 1
    assert O.round_bf16(np.float32(1.0 + 2.0 ** -8)) == np.float32(1.0)
    assert O.round_bf16(np.float32(1.0 + 3 * 2.0 ** -8)) == np.float32(1.0 + 2.0 ** -6)


def test_fp16_rounding_ties_to_even():
    assert O.round_fp16(np.float32(1.0 + 2.0 ** -11)) == np.float32(1.0)
    assert O.round_fp16(np.float32(1.0 + 3 * 2.0 ** -11)) == np.float32(1.0 + 2.0 ** -9)
    assert O.round_fp16(np.float32(32768.0 * (1 + 2.0 ** -20))) == np.float32(32768.0)


@pytest.mark.parametrize("fmt", ["fp16", "bf16"])
def test_encode_scale_range_and_exact_decode(fmt):
    g = np.random.default_rng(4)
    T = 2.0 ** O.FMT_TARGET_LOG2[fmt]
    for mag in [1e-30, 1e-6, 0.3, 1.0, 7.0, 2.0 ** 10, 1e20]:
        w = (g.standard_normal(1000) * mag).astype(np.float32)
        h = float(np.linalg.norm(w.astype(np.float64)))
        st, sc = O.encode(w, 1.0 / h, fmt)
        mx = float(np.max(np.abs(st)))
        assert T / 2 * (1 - 2 ** -10) < mx <= T
        # decode is a power-of-two scaling: exact
        dec = st.astype(np.float64) * sc
        assert np.array_equal(dec, (st * np.float32(sc)).astype(np.float64))
        rel = np.linalg.norm(dec - w / h) / np.linalg.norm(w / h)
        assert rel < (2 ** -8 if fmt == "bf16" else 2 ** -11)
    # power of two exactly at the boundary
    assert O.scale_exponent(1.0, fmt) == O.FMT_TARGET_LOG2[fmt]
    assert O.scale_exponent(0.75, fmt) == O.FMT_TARGET_LOG2[fmt]


def test_stall_point_definition():
    # 5% of m = 40 is 2 inner steps: steady 10x gains, then flat after 7 steps
    seq = [10.0 ** -j for j in range(8)] + [1e-7 * (1 - 1e-5 * i) for i in range(1, 6)]
    assert O.stall_window(40) == 2
    assert O.stall_point(seq, 40) == 7
    assert O.stall_point([1.0, 0.5, 0.25, 0.1], 40) is None
    assert O.stall_window(10) == 1


# --------------------------------------------------------------------------
# Arnoldi process: relation, orthogonality, least-squares residual

def _one_cycle(A, b, m, ortho):
    return O.gmres(A, b, m=m, tol=0.0, max_iters=m, ortho=ortho, record=True).cycles[0]


@pytest.mark.parametrize("ortho", ["mgs", "cgsr"])
def test_arnoldi_relation(ortho):
    Ac = P.random_dense_nonsym(80, 1, shift=2.0)
    A = _mat(Ac)
    D = A.dense()
    b = np.random.default_rng(5).standard_normal(80)
    c = _one_cycle(A, b, 30, ortho)
    k = c["k"]
    V = np.stack(c["V"], 1)
    lhs = D @ V[:, :k] - V[:, : k + 1] @ c["Hbar"]
    assert np.linalg.norm(lhs) <= 10 * k * O.U64 * np.linalg.norm(D)


def test_cgs2_orthogonality_and_mgs_loss():
    # a convection-diffusion Krylov basis is ill-conditioned: one classical pass
    # loses orthogonality to about 1e-11 here, the re-orthogonalised pair keeps it at u
    A = _mat(P.convdiff(32, (20.0, 10.0)))
    b = np.random.default_rng(6).standard_normal(A.n)
    out = {}
    for ortho in ("cgsr", "mgs"):
        c = _one_cycle(A, b, 60, ortho)
        V = np.stack(c["V"], 1)
        out[ortho] = np.linalg.norm(np.eye(V.shape[1]) - V.T @ V, 2)
    assert out["cgsr"] <= 10 * 60 * O.U64
    # MGS loses orthogonality in proportion to the conditioning of the basis
    assert out["cgsr"] < out["mgs"] < 1e-8


@pytest.mark.parametrize("ortho", ["mgs", "cgsr"])
def test_arnoldi_residual_is_least_squares_minimum(ortho):
    Ac = P.random_dense_nonsym(60, 3, shift=1.0)
    A = _mat(Ac)
    b = np.random.default_rng(7).standard_normal(60)
    m = 25
    r = O.gmres(A, b, m=m, tol=0.0, max_iters=m, ortho=ortho, record=True)
    c = r.cycles[0]
    beta = c["beta"]
    bn = np.linalg.norm(b)
    for j in range(1, c["k"] + 1):
        Hj = c["Hbar"][: j + 1, :j]
        rhs = np.zeros(j + 1)
        rhs[0] = beta
        y, *_ = np.linalg.lstsq(Hj, rhs, rcond=None)
        ls = np.linalg.norm(rhs - Hj @ y)
        assert abs(r.arnoldi[0][j - 1] * bn - ls) <= 1e-12 * beta
    # closed form after the first step: |s_2| = beta h21 / hypot(h11, h21)
    h11, h21 = c["Hbar"][0, 0], c["Hbar"][1, 0]
    assert math.isclose(r.arnoldi[0][0] * bn, beta * h21 / math.hypot(h11, h21), rel_tol=1e-13)
    # monotone non-increasing inside the cycle
    seq = [beta / bn] + r.arnoldi[0]
    assert all(seq[i + 1] <= seq[i] * (1 + 1e-14) for i in range(len(seq) - 1))
    # the Arnoldi residual predicts the true residual of the cycle's x (exact arithmetic up to u)
    assert math.isclose(np.linalg.norm(b - A.matvec(r.x)) / bn, r.arnoldi[0][-1], rel_tol=1e-6)


# --------------------------------------------------------------------------
# whole solver

def test_finite_termination_distinct_eigenvalues():
    n, kdist = 48, 6
    g = np.random.default_rng(8)
    Q = np.eye(n) + 0.3 * g.standard_normal((n, n)) / np.sqrt(n)
    lam = np.repeat(np.arange(1.0, kdist + 1.0), n // kdist)
    D = Q @ np.diag(lam) @ np.linalg.inv(Q)
    A = _mat(P.dense_to_csr(D))
    b = g.standard_normal(n)
    for ortho in ("mgs", "cgsr"):
        r = O.gmres(A, b, m=20, tol=1e-11, ortho=ortho)
        assert r.status == O.CONVERGED
        assert r.iters == kdist
        assert np.allclose(D @ r.x, b, atol=1e-9)


def test_random_small_systems_converge_within_n_steps():
    for seed in range(4):
        n = 16 + 4 * seed
        Ac = P.random_dense_nonsym(n, 10 + seed, shift=0.0)
        A = _mat(Ac)
        b = np.random.default_rng(seed).standard_normal(n)
        r = O.gmres(A, b, m=n, tol=1e-11, ortho="cgsr")
        assert r.status == O.CONVERGED and r.iters <= n


def test_identity_and_scaled_identity():
    n = 50
    b = np.random.default_rng(9).standard_normal(n)
    I = _mat(P.dense_to_csr(np.eye(n)))
    r = O.gmres(I, b, m=10, tol=1e-14)
    assert r.iters == 1 and np.allclose(r.x, b, rtol=8 * O.U64, atol=0)
    S = _mat(P.dense_to_csr(3.0 * np.eye(n)))
    r = O.gmres(S, b, m=10, tol=1e-14)
    assert r.iters == 1 and np.allclose(r.x, b / 3.0, rtol=8 * O.U64, atol=0)


def test_zero_rhs_returns_zero_without_iterating():
    A = _mat(P.convdiff(8, (1.0, 1.0)))
    r = O.gmres(A, np.zeros(64), x0=np.ones(64), m=10, tol=1e-10)
    assert r.iters == 0 and r.status == O.CONVERGED and not r.x.any()


def test_singular_matrix_stops_without_nan():
    D = np.diag([1.0, 2.0, 3.0, 0.0, 5.0])
    A = _mat(P.dense_to_csr(D))
    b = np.ones(5)
    r = O.gmres(A, b, m=5, tol=1e-12, max_iters=200)
    assert r.status in (O.MAXITER, O.STALLED)
    assert np.all(np.isfinite(r.x))
    # no correction can remove the component of b along the null space
    assert min(r.history) >= (1.0 - 1e-9) / math.sqrt(5.0)
    # the first cycle reaches that floor: the Krylov space is invariant after 5 steps
    assert math.isclose(r.history[1], 1.0 / math.sqrt(5.0), rel_tol=1e-6)


def test_dense_lu_agrees_on_c1():
    pr = P.c1_convdiff2d()
    A = _mat(pr.A)
    D = A.dense()
    x_lu = np.linalg.solve(D, pr.b)
    r = O.gmres(A, pr.b, m=pr.m, tol=1e-12, ortho="mgs")
    assert r.status == O.CONVERGED
    kappa = np.linalg.cond(D, 1)
    err = np.linalg.norm(r.x - x_lu) / np.linalg.norm(x_lu)
    assert err <= kappa * 1e-12
    assert np.linalg.norm(x_lu - pr.x_true) / np.linalg.norm(pr.x_true) <= kappa * 1e-15


@pytest.mark.parametrize("ortho", ["mgs", "cgsr"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_power_of_two_scaling_is_bitwise_invariant(ortho, precision):
    pr = P.c1_convdiff2d(24)
    A = _mat(pr.A)
    r0 = O.gmres(A, pr.b, m=20, tol=1e-10, ortho=ortho, precision=precision)
    As = _mat(pr.A.scaled(2.0 ** 7))
    r1 = O.gmres(As, pr.b * 2.0 ** 7, m=20, tol=1e-10, ortho=ortho, precision=precision)
    assert r0.iters == r1.iters and r0.restarts == r1.restarts
    assert np.array_equal(r0.x, r1.x)


def test_restart_residuals_never_increase():
    pr = P.c1_convdiff2d(32)
    A = _mat(pr.A)
    r = O.gmres(A, pr.b, m=8, tol=1e-10, ortho="mgs")
    assert r.status == O.CONVERGED and r.restarts > 5
    h = r.history
    assert all(h[i + 1] <= h[i] for i in range(len(h) - 1))


# --------------------------------------------------------------------------
# mixed precision: the claims of the numerics section and section 4.1

@pytest.mark.parametrize("ortho", ["mgs", "cgsr"])
def test_mixed_reaches_double_accuracy_after_restarts(ortho):
    pr = P.c1_convdiff2d(32)
    A = _mat(pr.A)
    r64 = O.gmres(A, pr.b, m=30, tol=1e-10, ortho=ortho)
    r32 = O.gmres(A, pr.b, m=30, tol=1e-10, ortho=ortho, precision="fp32")
    assert r32.status == O.CONVERGED and r32.rel_residual <= 1e-10
    assert r32.restarts >= 2
    # with restarts forced well before the FP32 stall, counts match FP64 closely
    assert abs(r32.iters - r64.iters) <= 30


@pytest.mark.parametrize("flag", ["residual_fp32", "update_fp32"])
def test_negative_control_reduced_precision_residual_or_update_stalls(flag):
    pr = P.c1_convdiff2d(32)
    A = _mat(pr.A)
    r = O.gmres(A, pr.b, m=30, tol=1e-10, ortho="mgs", max_iters=1500, **{flag: True})
    assert r.status != O.CONVERGED
    assert min(r.history) > 1e-9


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_two_byte_basis_still_reaches_double_accuracy(fmt):
    pr = P.c1_convdiff2d(24)
    A = _mat(pr.A)
    r = O.gmres(A, pr.b, m=20, tol=1e-10, ortho="cgsr", precision=fmt, max_iters=4000)
    assert r.status == O.CONVERGED


# (precision, arnoldi_a) -> (basis stored in float32, values of A the Arnoldi product reads)
_VARIABLE_CASES = {
    ("limited", "default"): (True, 32),  # the limited solver: A, M and V in float32
    ("limited", "fp64"): (True, 64),  # the basis alone in float32
    ("fp64", "fp32"): (False, 32),  # A for the next Krylov vector alone in float32
    ("fp64", "default"): (False, 64),  # nothing in float32
}


@pytest.mark.parametrize("ortho", ["mgs", "cgsr"])
def test_per_variable_precision_storage_split(ortho):
    # the limited solver and the single-variable runs of section 4.1 store
    # only their chosen variables in float32 and keep w in float64: a stored
    # basis vector is float32-representable exactly when the basis is a
    # float32 variable, and w'' = A v_j - V_j h_j holds to float64 rounding
    # with the values of A the product is meant to read, but only to about u32
    # with the other ones; in the fully float32 mode (w in float32) it holds
    # only to about u32 with either
    A0 = P.convdiff(12, (20.0, 10.0))
    g = np.random.default_rng(9)
    A = O.Matrix(A0.row_ptr, A0.col_idx, A0.vals * (1.0 + g.uniform(0.0, 1e-3, A0.nnz)), A0.n)
    D = {64: A.dense()}
    D[32] = D[64].astype(np.float32).astype(np.float64)
    b = np.random.default_rng(3).standard_normal(A.n)
    m = 30

    def relation(prec, arnoldi_a):
        c = O.gmres(A, b, m=m, tol=0.0, max_iters=m, ortho=ortho, precision=prec, record=True,
                    arnoldi_a=arnoldi_a).cycles[0]
        k, V, Hb, W = c["k"], np.stack(c["V"], 1), c["Hbar"], c["W"]
        assert k == m
        rel = {}
        for bits in (32, 64):
            r = []
            for j in range(k):
                scale = np.linalg.norm(D[32], 2) * np.linalg.norm(V[:, j]) + np.abs(Hb[: j + 1, j]).sum()
                r.append(np.linalg.norm(D[bits] @ V[:, j] - V[:, : j + 1] @ Hb[: j + 1, j] - W[j]) / scale)
            rel[bits] = (max(r), min(r))
        return np.array_equal(V, V.astype(np.float32).astype(np.float64)), rel

    for (prec, arnoldi_a), (basis32, bits) in _VARIABLE_CASES.items():
        stored32, rel = relation(prec, arnoldi_a)
        assert stored32 == basis32, (prec, arnoldi_a)
        assert rel[bits][0] <= 10 * m * O.U64, (prec, arnoldi_a)  # float64 w over these values
        assert rel[96 - bits][1] >= 1e-3 * O.U32, (prec, arnoldi_a)  # ... and not over the others
    for arnoldi_a in ("default", "fp64"):
        stored32, rel = relation("fp32", arnoldi_a)
        assert stored32 and rel[32][0] >= 1e-2 * O.U32 and rel[64][0] >= 1e-2 * O.U32


@pytest.mark.parametrize("ortho", ["mgs", "cgsr"])
def test_limited_mode_reaches_double_accuracy(ortho):
    # section 4.1: after restarting, both mixed solvers regain float64 accuracy
    pr = P.c1_convdiff2d(32)
    A = _mat(pr.A)
    r64 = O.gmres(A, pr.b, m=30, tol=1e-10, ortho=ortho)
    rl = O.gmres(A, pr.b, m=30, tol=1e-10, ortho=ortho, precision="limited")
    assert rl.status == O.CONVERGED and rl.rel_residual <= 1e-10 and rl.restarts >= 2
    assert abs(rl.iters - r64.iters) <= 30


# --------------------------------------------------------------------------
# restart strategies of the restart study (section 3)

def _stall_case():
    A0 = P.convdiff(24, (5.0, 5.0))
    xt, b = P.manufactured_rhs(A0, 7, 24)
    return O.Matrix.from_csr(A0), b


def test_restart_on_stall_ends_each_cycle_at_its_stall_point():
    # float32 MGS with a long restart length: the Arnoldi residual stops
    # improving long before j = m; the trigger ends the cycle there
    A, b = _stall_case()
    m = 200
    base = O.gmres(A, b, m=m, tol=1e-10, ortho="mgs", precision="fp32", record=True)
    st = O.gmres(A, b, m=m, tol=1e-10, ortho="mgs", precision="fp32", record=True, restart_on_stall=True)
    assert base.status == O.CONVERGED and st.status == O.CONVERGED
    assert len(base.arnoldi[0]) == m  # without the trigger the first cycle runs to m
    w = O.stall_window(m)
    for c, arn in enumerate(st.arnoldi[:-1]):  # every cycle but the converging one
        res = [st.history[c]] + list(arn)  # |s_1| .. |s_{k+1}|, relative to ||b||
        J = O.stall_point(res, m)
        assert J is not None and len(arn) == J + w
    assert st.iters < 0.6 * base.iters
    # where nothing stalls (float64) the trigger changes nothing
    r64 = O.gmres(A, b, m=m, tol=1e-10, ortho="mgs")
    s64 = O.gmres(A, b, m=m, tol=1e-10, ortho="mgs", restart_on_stall=True)
    assert np.array_equal(r64.x, s64.x) and r64.iters == s64.iters


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_two_stage_restart_repeats_the_first_cycle_length(precision):
    A, b = _stall_case()
    delta = 1e-5
    r = O.gmres(A, b, m=200, tol=1e-10, ortho="cgsr", precision=precision, record=True,
                restart_improve=delta, restart_repeat=True)
    assert r.status == O.CONVERGED and r.restarts >= 2
    lens = [len(a) for a in r.arnoldi]
    # the first cycle ends at the first step with |s_{j+1}| <= delta beta
    first = r.arnoldi[0]
    k1 = next(j + 1 for j, v in enumerate(first) if v <= delta * r.history[0])
    assert lens[0] == k1
    # every later cycle but the last has the same length (the threshold no
    # longer applies: those cycles improve by less or more than delta)
    assert all(L == k1 for L in lens[1:-1]) and lens[-1] <= k1
    # without a threshold the first cycle runs to m: plain GMRES(m), bit for bit
    p = O.gmres(A, b, m=60, tol=1e-10, ortho="cgsr", precision=precision)
    q = O.gmres(A, b, m=60, tol=1e-10, ortho="cgsr", precision=precision, restart_repeat=True)
    assert np.array_equal(p.x, q.x) and p.iters == q.iters


def _s_from_basis(V):
    k = V.shape[1]
    OU = np.zeros((k, k))
    OS = np.zeros((k, k))
    for c in range(1, k):
        O.orth_s_append(OU, OS, c, V[:, :c].T @ V[:, c])
    return OU, OS


def test_orth_s_matrix_properties():
    g = np.random.default_rng(11)
    # orthonormal basis: U = 0, so S = 0
    Q, _ = np.linalg.qr(g.standard_normal((50, 8)))
    _, S = _s_from_basis(Q)
    assert np.max(np.abs(S)) < 1e-14
    # two unit vectors with cosine c: S = U = [[0, c], [0, 0]], ||S||_2 = |c|
    v1 = np.array([1.0, 0.0, 0.0])
    v2 = np.array([0.6, 0.8, 0.0])
    _, S = _s_from_basis(np.stack([v1, v2], 1))
    assert np.allclose(S, [[0.0, 0.6], [0.0, 0.0]], atol=1e-15)
    # unit columns that are linearly dependent: ||S||_2 = 1 (the criterion)
    v3 = (Q[:, 0] + Q[:, 1]) / np.sqrt(2.0)
    V = np.concatenate([Q[:, :3], v3[:, None], Q[:, 3:5]], axis=1)
    _, S = _s_from_basis(V)
    assert abs(np.linalg.norm(S, 2) - 1.0) < 1e-12
    # ... and independent but non-orthogonal unit columns: below 1, and the
    # leading blocks (earlier steps) never have a larger norm
    W = g.standard_normal((40, 7))
    W /= np.linalg.norm(W, axis=0)
    _, S = _s_from_basis(W)
    norms = [np.linalg.norm(S[:c, :c], 2) for c in range(1, 8)]
    assert norms[-1] < 1.0 and all(a <= b + 1e-15 for a, b in zip(norms, norms[1:]))
    # the appended columns reproduce the definition (I + U)^-1 U
    U = np.triu(W.T @ W, 1)
    assert np.allclose(S, np.linalg.solve(np.eye(7) + U, U), atol=1e-13)


def test_power_norm_estimate():
    g = np.random.default_rng(12)
    S = np.triu(g.standard_normal((9, 9)), 1)
    est = O.power_norm(S)
    true = np.linalg.norm(S, 2)
    assert est <= true * (1 + 1e-12)  # a Rayleigh-quotient estimate never exceeds the norm
    assert est >= 0.9 * true
    assert O.power_norm(np.zeros((4, 4))) == 0.0
    assert O.power_norm(S, iters=200) == pytest.approx(true, rel=1e-9)


@pytest.mark.parametrize("norm,tau", [("spectral", 0.5), ("frobenius", 0.5)])
def test_orth_restart_ends_cycles_when_the_basis_loses_orthogonality(norm, tau):
    A, b = (lambda A0: (O.Matrix.from_csr(A0), P.manufactured_rhs(A0, 7, 12)[1]))(P.convdiff(12, (5.0, 5.0)))
    base = O.gmres(A, b, m=64, tol=1e-10, ortho="mgs", precision="fp32", record=True)
    r = O.gmres(A, b, m=64, tol=1e-10, ortho="mgs", precision="fp32", record=True, orth_restart=tau,
                orth_norm=norm)
    assert r.status == O.CONVERGED and r.iters < base.iters
    assert len(r.arnoldi[0]) < 64 == len(base.arnoldi[0])
    # float64 CGSR keeps the basis orthogonal to working accuracy: never fires
    p = O.gmres(A, b, m=64, tol=1e-10, ortho="cgsr")
    q = O.gmres(A, b, m=64, tol=1e-10, ortho="cgsr", orth_restart=tau, orth_norm=norm)
    assert np.array_equal(p.x, q.x) and p.iters == q.iters


# --------------------------------------------------------------------------
# ILU(0)

def _lu_dense(A, lu, diag):
    n = A.n
    L = np.eye(n)
    U = np.zeros((n, n))
    for i in range(n):
        for p in range(A.row_ptr[i], A.row_ptr[i + 1]):
            j = A.col_idx[p]
            if j < i:
                L[i, j] = lu[p]
            else:
                U[i, j] = lu[p]
    return L, U


def test_ilu0_reproduces_a_on_its_pattern():
    # the defining property of ILU(0): (L U)_ij = a_ij wherever A stores an entry
    A = O.Matrix.from_csr(P.convdiff(7, (20.0, 5.0)))
    lu, diag = O.ilu0(A)
    L, U = _lu_dense(A, lu, diag)
    LU = L @ U
    D = A.dense()
    on = np.zeros_like(D, dtype=bool)
    on[A.rows, A.col_idx] = True
    assert np.allclose(LU[on], D[on], rtol=1e-13, atol=1e-12 * np.abs(D).max())
    assert np.max(np.abs(LU[~on] - D[~on])) > 1e-3  # and it is incomplete: fill is dropped


def test_ilu0_of_a_tridiagonal_matrix_is_exact_lu():
    n = 30
    g = np.random.default_rng(5)
    D = np.diag(4.0 + g.random(n)) + np.diag(g.random(n - 1) - 0.5, 1) + np.diag(g.random(n - 1) - 0.5, -1)
    A = O.Matrix.from_csr(P.dense_to_csr(D))
    lu, diag = O.ilu0(A)
    L, U = _lu_dense(A, lu, diag)
    assert np.allclose(L @ U, D, rtol=0, atol=1e-14)
    v = g.standard_normal(n)
    assert np.allclose(D @ O.ilu_apply(A, lu, diag, v), v, atol=1e-12)


def test_ilu_sweeps_reach_the_substitution_at_the_triangle_depth():
    A = O.Matrix.from_csr(P.convdiff(6, (10.0, 3.0)))
    lu, diag = O.ilu0(A)
    dl, du = O.triangle_depths(A, diag)
    assert dl == 2 * 6 - 1 and du == 2 * 6 - 1  # 5-point stencil, natural order
    v = np.random.default_rng(6).standard_normal(A.n)
    exact = O.ilu_apply(A, lu, diag, v)
    deep = O.ilu_apply(A, lu, diag, v, sweeps=max(dl, du))
    shallow = O.ilu_apply(A, lu, diag, v, sweeps=3)
    assert np.allclose(deep, exact, rtol=1e-13, atol=1e-13)
    assert np.linalg.norm(shallow - exact) > 1e-6 * np.linalg.norm(exact)


def test_ilu_preconditioned_gmres_beats_jacobi():
    A0 = P.varcoef3d(8, family=94, index=0)
    A = O.Matrix.from_csr(A0)
    b = P.manufactured_rhs(A0, 94, 0)[1]
    lu, diag = O.ilu0(A)
    d = A.diagonal()
    rj = O.gmres(A, b, m=30, tol=1e-10, ortho="cgsr", precond=lambda v: v / d)
    ri = O.gmres(A, b, m=30, tol=1e-10, ortho="cgsr", precond=lambda v: O.ilu_apply(A, lu, diag, v))
    assert ri.status == O.CONVERGED and rj.status == O.CONVERGED
    assert ri.iters < 0.8 * rj.iters


# --------------------------------------------------------------------------
# split storage of A (high and low 32-bit words of each float64 value)

def test_high_word_value_hand_cases():
    # the high word holds sign, exponent and the first 20 significand bits
    vals = np.array([1.0 + 2.0 ** -20, 1.0 + 2.0 ** -21, -(1.0 + 2.0 ** -21), 3.0, 0.0, -0.0,
                     2.0 ** -1000 * (1.0 + 2.0 ** -30), 1.5 * 2.0 ** 300])
    want = np.array([1.0 + 2.0 ** -20, 1.0, -1.0, 3.0, 0.0, -0.0, 2.0 ** -1000, 1.5 * 2.0 ** 300])
    got = O.high_word_value(vals)
    assert np.array_equal(got, want) and np.array_equal(np.signbit(got), np.signbit(want))


def test_high_word_value_is_a_truncation_exact_in_float32():
    g = np.random.default_rng(7)
    v = g.standard_normal(20000) * np.exp(g.uniform(-30, 30, 20000))
    h = O.high_word_value(v)
    # never larger in magnitude, same sign, relative error below 2^-20
    assert np.all(np.abs(h) <= np.abs(v)) and np.all(np.sign(h) == np.sign(v))
    assert np.all(np.abs(v - h) < 2.0 ** -20 * np.abs(v))
    # 20 significand bits fit float32's 23: the conversion is exact in range
    assert np.array_equal(h.astype(np.float32).astype(np.float64), h)
    # the low word is what was dropped: high word + low word = the value
    lo = (v.view(np.uint64) & np.uint64(0xFFFFFFFF)).astype(np.uint64)
    assert np.array_equal((h.view(np.uint64) | lo).view(np.float64), v)


@pytest.mark.parametrize("ortho", ["mgs", "cgsr"])
def test_split_storage_mixed_reaches_double_accuracy(ortho):
    # the Arnoldi copy of A is perturbed by up to 2^-20 relative; the float64
    # residual (both words) still drives the solve to 1e-10
    pr = P.c1_convdiff2d(32)
    A = _mat(pr.A)
    r32 = O.gmres(A, pr.b, m=30, tol=1e-10, ortho=ortho, precision="fp32")
    rs = O.gmres(A, pr.b, m=30, tol=1e-10, ortho=ortho, precision="fp32", a_storage="split")
    assert rs.status == O.CONVERGED and O.relative_residual(A, pr.b, rs.x) <= 1e-10
    assert abs(rs.iters - r32.iters) <= 30
    # float64 mode reads both words: identical to the copy storage
    r64 = O.gmres(A, pr.b, m=30, tol=1e-10, ortho=ortho)
    r64s = O.gmres(A, pr.b, m=30, tol=1e-10, ortho=ortho, a_storage="split")
    assert np.array_equal(r64.x, r64s.x) and r64.iters == r64s.iters


# --------------------------------------------------------------------------
# flexible (right-preconditioned) form

def test_fgmres_with_identity_is_plain_gmres_bitwise():
    pr = P.c1_convdiff2d(20)
    A = _mat(pr.A)
    r0 = O.gmres(A, pr.b, m=15, tol=1e-10)
    r1 = O.gmres(A, pr.b, m=15, tol=1e-10, precond=lambda v: v.copy())
    assert r0.iters == r1.iters and np.array_equal(r0.x, r1.x)


def test_fgmres_with_jacobi_equals_right_preconditioned_gmres():
    A0 = P.varcoef3d(10, family=90, index=1)
    A = _mat(A0)
    d = A.diagonal()
    xt = np.random.default_rng(11).uniform(-1, 1, A.n)
    b = A.matvec(xt)
    r1 = O.gmres(A, b, m=20, tol=1e-11, precond=lambda v: v / d, fallback=False)
    # explicit right preconditioning: solve (A D^-1) u = b, then x = D^-1 u
    AD = O.Matrix(A0.row_ptr, A0.col_idx, A0.vals / d[A0.col_idx], A.n)
    r2 = O.gmres(AD, b, m=20, tol=1e-11)
    assert r1.iters == r2.iters and r1.restarts == r2.restarts
    assert np.linalg.norm(r1.x - r2.x / d) <= 1e-9 * np.linalg.norm(r1.x)


# --------------------------------------------------------------------------
# left preconditioning (the form of the paper's experiments): r = M^-1 (b - A x),
# w = M^-1 A v_j, x += V y

def test_left_preconditioning_with_identity_is_plain_gmres_bitwise():
    pr = P.c1_convdiff2d(20)
    A = _mat(pr.A)
    for ortho in ("mgs", "cgsr"):
        r0 = O.gmres(A, pr.b, m=15, tol=1e-10, ortho=ortho)
        r1 = O.gmres(A, pr.b, m=15, tol=1e-10, ortho=ortho, precond=lambda v: v.copy(), side="left")
        assert r0.iters == r1.iters and np.array_equal(r0.x, r1.x) and r0.history == r1.history


def test_left_preconditioning_with_the_exact_inverse_takes_one_step():
    # M^-1 = A^-1: M^-1 A = I, so the first Arnoldi step spans the solution
    D = np.array([[4.0, 1.0, 0.0], [2.0, 5.0, 1.0], [0.0, 3.0, 6.0]])
    A = O.Matrix.from_csr(P.dense_to_csr(D))
    Ainv = np.linalg.inv(D)
    b = np.array([1.0, -2.0, 0.5])
    r = O.gmres(A, b, m=3, tol=1e-13, precond=lambda v: Ainv @ v, side="left", fallback=False, record=True)
    assert r.status == O.CONVERGED and r.iters == 1
    assert np.allclose(r.x, np.linalg.solve(D, b), rtol=1e-14, atol=1e-15)


def test_left_preconditioning_is_gmres_on_the_preconditioned_system():
    # one cycle of left-preconditioned GMRES with M^-1 = D^-1 is GMRES on
    # (D^-1 A) x = D^-1 b: the same iterate up to rounding, and its Arnoldi
    # residual |s_{k+1}| is the preconditioned residual ||D^-1 (b - A x)||,
    # the quantity it minimises
    A0 = P.varcoef3d(8, family=90, index=2)
    A = _mat(A0)
    d = A.diagonal()
    xt = np.random.default_rng(12).uniform(-1, 1, A.n)
    b = A.matvec(xt)
    m = 20
    rl = O.gmres(A, b, m=m, tol=0.0, max_iters=m, precond=lambda v: v / d, side="left", fallback=False,
                 record=True)
    rows = np.repeat(np.arange(A.n), np.diff(A0.row_ptr))
    DA = O.Matrix(A0.row_ptr, A0.col_idx, A0.vals / d[rows], A.n)
    re = O.gmres(DA, b / d, m=m, tol=0.0, max_iters=m)
    assert rl.iters == re.iters == m
    assert np.linalg.norm(rl.x - re.x) <= 1e-12 * np.linalg.norm(re.x)
    s_last = abs(rl.cycles[0]["s"][m])
    pres = np.linalg.norm((b - A.matvec(rl.x)) / d)
    assert s_last == pytest.approx(pres, rel=1e-8)


def test_left_preconditioned_mixed_and_ilu_reach_double_accuracy():
    # the restart residual b - A x judges convergence whatever the side
    A0 = P.varcoef3d(10, family=90, index=3)
    A = _mat(A0)
    xt = np.random.default_rng(13).uniform(-1, 1, A.n)
    b = A.matvec(xt)
    lu, diag = O.ilu0(A)
    for precision, dt in (("fp64", np.float64), ("fp32", np.float32)):
        r = O.gmres(A, b, m=20, tol=1e-11, precision=precision, side="left",
                    precond=lambda v: O.ilu_apply(A, lu, diag, v, sweeps=0, dtype=dt))
        assert r.status == O.CONVERGED and O.relative_residual(A, b, r.x) <= 1e-11
        plain = O.gmres(A, b, m=20, tol=1e-11, precision=precision)
        assert r.iters < plain.iters


# --------------------------------------------------------------------------
# normwise backward error (the stopping metric the paper's experiments use)

def test_backward_error_closed_form_2x2():
    # A = [[2, 1], [0, 3]], x = [1, 1], b = [3, 2]: r = [0, -1], ||A||_F = sqrt(14)
    A = O.Matrix(np.array([0, 2, 3]), np.array([0, 1, 1]), np.array([2.0, 1.0, 3.0]))
    eta = O.backward_error(A, np.array([3.0, 2.0]), np.array([1.0, 1.0]))
    assert eta == pytest.approx(1.0 / (math.sqrt(14.0) * math.sqrt(2.0) + math.sqrt(13.0)), rel=1e-15)


def test_backward_error_is_the_size_of_an_exact_perturbation():
    # Rigal-Gaches: with dA = t ||A|| r x^T / ||x||^2 and db = -(1 - t) r,
    # t = ||A|| ||x|| / (||A|| ||x|| + ||b||), (A + dA) x = b + db holds exactly
    # and ||dA||_F / ||A||_F = ||db|| / ||b|| = eta (a rank-one dA has equal
    # Frobenius and 2-norms); eta never exceeds the relative residual, is
    # zero at the solution and does not change when A and b are scaled together
    g = np.random.default_rng(5)
    D = g.standard_normal((7, 7)) + 4 * np.eye(7)
    A = O.Matrix.from_csr(P.dense_to_csr(D))
    b = g.standard_normal(7)
    x = np.linalg.solve(D, b) + 1e-3 * g.standard_normal(7)
    eta = O.backward_error(A, b, x)
    r = b - D @ x
    nA, nx, nb = np.linalg.norm(D), np.linalg.norm(x), np.linalg.norm(b)
    t = nA * nx / (nA * nx + nb)
    dA = (t / nx ** 2) * np.outer(r, x)
    db = -(1.0 - t) * r
    assert np.allclose((D + dA) @ x, b + db, rtol=0, atol=1e-13)
    assert np.linalg.norm(dA) / nA == pytest.approx(eta, rel=1e-12)
    assert np.linalg.norm(db) / nb == pytest.approx(eta, rel=1e-12)
    assert eta <= O.relative_residual(A, b, x)
    xs = np.linalg.solve(D, b)
    assert O.backward_error(A, b, xs) <= 1e-15
    A3 = O.Matrix.from_csr(P.dense_to_csr(3.0 * D))
    assert O.backward_error(A3, 3.0 * b, x) == pytest.approx(eta, rel=1e-12)


# --------------------------------------------------------------------------
# ILU(0) sweeps in float32: every operation rounded, checked against exact
# rational arithmetic with an explicit round-to-nearest-even to float32

def _rne32(q):
    """The float32 nearest to the rational q (ties to even), as a Fraction."""
    from fractions import Fraction

    if q == 0:
        return Fraction(0)
    sign = -1 if q < 0 else 1
    q = abs(q)
    e = 0  # q * 2^-e in [2^23, 2^24): 24 significand bits
    while q / Fraction(2) ** e >= 2 ** 24:
        e += 1
    while q / Fraction(2) ** e < 2 ** 23:
        e -= 1
    e = max(e, -149)  # subnormals: fixed quantum 2^-149
    m = q / Fraction(2) ** e
    f = m.numerator // m.denominator
    rem = m - f
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and f % 2 == 1):
        f += 1
    return sign * Fraction(f) * Fraction(2) ** e


def test_ilu_float32_sweeps_round_every_operation():
    from fractions import Fraction

    # a 4x4 matrix with full lower and upper triangles and values that are
    # not float32-exact, so every product, difference and quotient rounds
    D = np.array([[3.0, 0.1, 0.0, 0.7],
                  [0.3, 2.5, 0.2, 0.0],
                  [0.0, 0.9, 4.1, 0.6],
                  [0.2, 0.0, 0.4, 1.9]])
    A = O.Matrix.from_csr(P.dense_to_csr(D))
    lu, diag = O.ilu0(A)
    v = np.array([1.0, -2.0 / 3.0, 0.1, 5.0 / 7.0], dtype=np.float32)
    n, rp, ci = A.n, A.row_ptr, A.col_idx
    lu32 = [Fraction(float(np.float32(t))) for t in lu]
    vq = [Fraction(float(t)) for t in v]
    dinv = [_rne32(1 / lu32[diag[i]]) for i in range(n)]
    for sweeps in (1, 2, 3, 4):
        y = [Fraction(0)] * n
        for _ in range(sweeps):  # y <- v - L' y, the row sum in storage order
            new = []
            for i in range(n):
                acc = Fraction(0)
                for p in range(rp[i], rp[i + 1]):
                    if ci[p] < i:
                        acc = _rne32(acc + _rne32(lu32[p] * y[ci[p]]))
                new.append(_rne32(vq[i] - acc))
            y = new
        x = [Fraction(0)] * n
        for _ in range(sweeps):  # x <- D^-1 (y - U' x)
            new = []
            for i in range(n):
                acc = Fraction(0)
                for p in range(rp[i], rp[i + 1]):
                    if ci[p] > i:
                        acc = _rne32(acc + _rne32(lu32[p] * x[ci[p]]))
                new.append(_rne32(_rne32(y[i] - acc) * dinv[i]))
            x = new
        got = O.ilu_apply(A, lu, diag, v, sweeps=sweeps, dtype=np.float32)
        assert got.dtype == np.float32
        assert [Fraction(float(t)) for t in got] == x, sweeps
    # the float32 result differs from the float64 one (rounding is really emulated)
    z64 = O.ilu_apply(A, lu, diag, v.astype(np.float64), sweeps=4)
    assert not np.array_equal(got.astype(np.float64), z64)
    assert np.allclose(got, z64, rtol=1e-6)
