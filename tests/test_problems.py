"""Checks of the seeded synthetic inputs (shapes, counts, structure, statistics)."""
import numpy as np
import pytest

import problems as P


def _csr_ok(A):
    rp, ci = A.row_ptr, A.col_idx
    assert rp.dtype == np.int32 and ci.dtype == np.int32 and A.vals.dtype == np.float64
    assert rp[0] == 0 and rp[-1] == ci.size == A.vals.size
    assert np.all(np.diff(rp) >= 0)
    assert ci.min() >= 0 and ci.max() < A.n
    rows = np.repeat(np.arange(A.n), np.diff(rp))
    key = rows.astype(np.int64) * A.n + ci
    assert np.all(np.diff(key) > 0), "columns sorted and unique within each row"


@pytest.mark.parametrize("N,beta,nnz", [(64, (20.0, 10.0), 5 * 64 ** 2 - 4 * 64),
                                        (16, (50.0, 20.0, 10.0), 7 * 16 ** 3 - 6 * 16 ** 2),
                                        (9, (-3.0, 4.0), 5 * 81 - 36)])
def test_convdiff_counts_and_values(N, beta, nnz):
    A = P.convdiff(N, beta)
    _csr_ok(A)
    assert A.nnz == nnz
    d = len(beta)
    h = 1.0 / (N + 1)
    S = A.to_scipy()
    diag = S.diagonal()
    assert np.allclose(diag, 2 * d / h ** 2 + sum(abs(b) for b in beta) / h)
    # an interior row: lower/upper neighbours in x carry the upwind term on the upstream side
    i = sum((N // 2) * N ** k for k in range(d))
    assert np.isclose(S[i, i - 1], -1 / h ** 2 - max(beta[0], 0) / h)
    assert np.isclose(S[i, i + 1], -1 / h ** 2 - max(-beta[0], 0) / h)
    # row sums of an interior row vanish (consistency of both operators on constants)
    assert abs(S[i].sum()) < 1e-9 * diag[i]


def test_c2_full_size_nnz():
    # 7 N^3 - 6 N^2 with the boundary eliminated (the workload's "about 14.7M" is 7 N^3)
    assert 7 * 128 ** 3 - 6 * 128 ** 2 == 14_581_760


def test_powerlaw_structure_and_statistics():
    A = P.powerlaw(50_000)
    _csr_ok(A)
    L = np.diff(A.row_ptr)
    assert L.min() >= 1 and L.max() <= 2000
    assert 18.0 < L.mean() < 23.0
    S = A.to_scipy()
    d = S.diagonal()
    off = np.asarray(abs(S).sum(axis=1)).ravel() - np.abs(d)
    assert np.allclose(d, 1.2 * off)
    assert np.all(d > 0)
    # determinism
    B = P.powerlaw(50_000)
    assert np.array_equal(A.col_idx, B.col_idx) and np.array_equal(A.vals, B.vals)


def test_grf_statistics_and_varcoef_matrix():
    g = P.gaussian_random_field(32, 4.0, P.rng(99, P.GRF, 0))
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1) < 1e-12
    # correlation at one correlation length along x is about exp(-1/2)
    c1 = np.mean(g * np.roll(g, 4, axis=2))
    assert 0.4 < c1 < 0.8
    A = P.varcoef3d(16, family=99, index=0)
    _csr_ok(A)
    assert A.nnz == 7 * 16 ** 3 - 6 * 16 ** 2
    S = A.to_scipy()
    d = S.diagonal()
    off = np.asarray(abs(S).sum(axis=1)).ravel() - np.abs(d)
    assert np.all(d >= off - 1e-9 * d)  # weakly diagonally dominant (M-matrix)


def test_rhs_and_batch_specs_are_seeded():
    A = P.convdiff(8, (1.0, 2.0))
    x1, b1 = P.manufactured_rhs(A, 1, 0)
    x2, b2 = P.manufactured_rhs(A, 1, 0)
    assert np.array_equal(x1, x2) and np.array_equal(b1, b2)
    assert np.all(np.abs(x1) <= 1)
    specs = P.c4_batch_specs(64)
    assert specs == P.c4_batch_specs(64)
    Ns = [s[0] for s in specs]
    assert min(Ns) >= 32 and max(Ns) <= 256
    assert all(0 <= b <= 100 for s in specs for b in s[1])


def test_restart_study_system_is_c2_plus_a_diagonal_shift():
    a = P.convdiff(12, (50.0, 20.0, 10.0))
    pr = P.restart_study_3d(12, shift=1.0)
    assert np.array_equal(pr.A.row_ptr, a.row_ptr) and np.array_equal(pr.A.col_idx, a.col_idx)
    rows = np.repeat(np.arange(a.n), np.diff(a.row_ptr))
    d = rows == a.col_idx
    h = 1.0 / 13
    assert np.allclose(pr.A.vals[d] - a.vals[d], 6.0 / h ** 2, rtol=1e-14)
    assert np.array_equal(pr.A.vals[~d], a.vals[~d])
