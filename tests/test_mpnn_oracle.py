"""Pins of the learned-preconditioner oracle (oracle/mpnn.py), CPU only."""
import math

import numpy as np
import pytest
import torch

from oracle import mpnn as N
import problems as P


def small_matrix(n=40, seed=3):
    """Random sparse non-symmetric matrix with a dominant positive diagonal
    and a few one-sided entries (so some transposed entries are missing)."""
    g = np.random.default_rng(seed)
    D = np.zeros((n, n))
    for i in range(n):
        for j in g.choice(n, size=4, replace=False):
            if j != i:
                D[i, j] = g.normal()
        D[i, i] = 1.5 * np.abs(D[i]).sum() + 0.5
    csr = P.dense_to_csr(D)
    return csr, D


def random_theta(seed):
    g = np.random.default_rng(seed)
    th = N.init_params(seed)
    o, shape = N.OFFSETS["wo"]
    th[o:o + N.U] = g.normal(0, 0.05, N.U)
    th[N.OFFSETS["bo"][0]] = 0.02
    for name in ("bn", "be", "b1", "b2", "b3"):
        o, shape = N.OFFSETS[name]
        th[o:o + shape[0]] = g.normal(0, 0.1, shape[0])
    return th


def test_layout_size():
    assert N.NPARAMS == 3 * 32 + 32 + 3 * 32 + 32 + 3 * (32 * 96 + 32) + 96 + 1
    assert N.OFFSETS["W1"][0] % 8 == 0 and N.OFFSETS["W2"][0] % 8 == 0 and N.OFFSETS["W3"][0] % 8 == 0


def test_zero_decoder_is_jacobi():
    csr, D = small_matrix()
    G = N.graph(csr.n, csr.row_ptr, csr.col_idx, csr.vals)
    th = N.init_params(0)
    M = N.forward(torch.as_tensor(th), G).numpy()
    rows = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
    diag = rows == csr.col_idx
    np.testing.assert_allclose(M[diag], 1.0 / np.diag(D)[rows[diag]], rtol=1e-15)
    assert np.all(M[~diag] == 0.0)


def test_negative_diagonal_jacobi_sign():
    D = np.array([[-2.0, 1.0], [0.5, 4.0]])
    csr = P.dense_to_csr(D)
    G = N.graph(2, csr.row_ptr, csr.col_idx, csr.vals)
    M = N.forward(torch.as_tensor(N.init_params(1)), G).numpy()
    np.testing.assert_allclose(M[[0, 3]], [-0.5, 0.25], rtol=1e-15)


def test_hand_worked_message_pass():
    """A = [[2, -1], [0.5, 4]]; weights chosen so each stage can be followed
    by hand: h = 1 after the encoder, e_ij = relu(ahat_ij), layer 1 copies e
    into m, so h_i = 1 + mean_j relu(ahat_ij); layers 2 and 3 are zero; the
    decoder returns h_i."""
    A = np.array([[2.0, -1.0], [0.5, 4.0]])
    csr = P.dense_to_csr(A)
    G = N.graph(2, csr.row_ptr, csr.col_idx, csr.vals)
    th = np.zeros(N.NPARAMS)
    Pm = N.unpack(th)  # views into th
    Pm["bn"][:] = 1.0
    Pm["We"][:, 0] = 1.0
    Pm["W1"][:, 64:96] = 1.0 / 32
    Pm["wo"][:32] = 1.0 / 32
    M = N.forward(torch.as_tensor(th), G).numpy()
    r8 = math.sqrt(8.0)
    h0 = 1.0 + 0.5 * (1.0 + 0.0)            # relu(ahat_00) = 1, relu(-1/sqrt 8) = 0
    h1 = 1.0 + 0.5 * (0.5 / r8 + 1.0)
    expect = [(1.0 + h0) / 2.0, h0 / r8, h1 / r8, (1.0 + h1) / 4.0]
    np.testing.assert_allclose(M, expect, rtol=1e-14)


def test_decoder_closed_form():
    """Constant states: every s_ij = wo . u + bo = 1.06 for the weights below."""
    A = np.array([[2.0, -1.0], [0.5, 4.0]])
    csr = P.dense_to_csr(A)
    G = N.graph(2, csr.row_ptr, csr.col_idx, csr.vals)
    th = np.zeros(N.NPARAMS)
    Pm = N.unpack(th)
    Pm["bn"][:] = 1.0
    Pm["wo"][:32] = 0.01
    Pm["wo"][32:64] = 0.02
    Pm["wo"][64:] = 0.5
    Pm["bo"][0] = 0.1
    M = N.forward(torch.as_tensor(th), G).numpy()
    s = 0.32 + 0.64 + 0.1
    np.testing.assert_allclose(M, [(1 + s) / 2, s / math.sqrt(8), s / math.sqrt(8), (1 + s) / 4], rtol=1e-14)


def test_inputs_by_hand():
    A = np.array([[2.0, -1.0, 0.0], [0.5, 4.0, 3.0], [0.0, 0.0, 1.0]])
    csr = P.dense_to_csr(A)
    G = N.graph(3, csr.row_ptr, csr.col_idx, csr.vals)
    # entries in CSR order: (0,0) (0,1) (1,0) (1,1) (1,2) (2,2)
    ah = [1.0, -1 / math.sqrt(8), 0.5 / math.sqrt(8), 1.0, 3.0 / 2.0, 1.0]
    np.testing.assert_allclose(G.ahat.numpy(), ah, rtol=1e-15)
    np.testing.assert_array_equal(G.tpos.numpy(), [0, 2, 1, 3, -1, 5])
    np.testing.assert_allclose(G.f.numpy()[:, 1], [1.0, ah[2], ah[1], 1.0, 0.0, 1.0], rtol=1e-15)
    np.testing.assert_allclose(G.x.numpy(), [[ah[1], abs(ah[1]), ah[2]],
                                             [ah[2] + ah[4], ah[2] + ah[4], ah[1]],
                                             [0.0, 0.0, ah[4]]], rtol=1e-15)
    np.testing.assert_array_equal(G.deg.numpy(), [2, 3, 1])


def test_loss_matches_dense_definition():
    csr, D = small_matrix()
    G = N.graph(csr.n, csr.row_ptr, csr.col_idx, csr.vals)
    th = random_theta(5)
    Mv = N.forward(torch.as_tensor(th), G).numpy()
    Md = np.zeros_like(D)
    rows = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
    Md[rows, csr.col_idx] = Mv
    Z = np.random.default_rng(9).normal(size=(csr.n, 3))
    ref = np.mean([np.sum((D @ Md @ Z[:, k] - Z[:, k]) ** 2) / np.sum(Z[:, k] ** 2) for k in range(3)])
    got = float(N.loss(torch.as_tensor(Mv), G, torch.as_tensor(csr.vals), torch.as_tensor(Z)))
    assert got == pytest.approx(ref, rel=1e-12)


def test_grad_M_closed_form_against_finite_differences():
    csr, D = small_matrix(n=30, seed=7)
    G = N.graph(csr.n, csr.row_ptr, csr.col_idx, csr.vals)
    Mv = torch.as_tensor(N.forward(torch.as_tensor(random_theta(2)), G).numpy())
    av = torch.as_tensor(csr.vals)
    Z = torch.as_tensor(np.random.default_rng(1).normal(size=(csr.n, 2)))
    g = N.loss_grad_M(Mv, G, av, Z).numpy()
    h = 1e-6
    for e in np.random.default_rng(4).choice(Mv.numel(), 25, replace=False):
        Mp, Mm = Mv.clone(), Mv.clone()
        Mp[e] += h
        Mm[e] -= h
        fd = (float(N.loss(Mp, G, av, Z)) - float(N.loss(Mm, G, av, Z))) / (2 * h)
        assert fd == pytest.approx(g[e], rel=1e-6, abs=1e-9 * np.abs(g).max())


def test_network_gradient_against_finite_differences():
    """Central differences (step 1e-6) on coordinates from every parameter block."""
    csr, D = small_matrix(n=50, seed=11)
    G = N.graph(csr.n, csr.row_ptr, csr.col_idx, csr.vals)
    th = random_theta(3)
    Z = np.random.default_rng(2).normal(size=(csr.n, 2))
    L0, grad, _ = N.value_and_grad(th, G, csr.vals, Z)
    g = np.random.default_rng(6)
    idx = []
    for name, (o, shape) in N.OFFSETS.items():
        size = int(np.prod(shape))
        idx += list(o + g.choice(size, min(size, 5), replace=False))
    h = 1e-6
    scale = np.abs(grad).max()
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (N.value_and_grad(tp, G, csr.vals, Z)[0] - N.value_and_grad(tm, G, csr.vals, Z)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(abs(grad[i]), 1e-3 * scale), (i, fd, grad[i])


def test_chain_rule_split_matches_autograd():
    """Gradient through M (closed form) then through the network equals the
    end-to-end gradient: the split the GPU path uses."""
    csr, D = small_matrix(n=40, seed=12)
    G = N.graph(csr.n, csr.row_ptr, csr.col_idx, csr.vals)
    th = random_theta(8)
    Z = np.random.default_rng(3).normal(size=(csr.n, 3))
    L, grad, Mv = N.value_and_grad(th, G, csr.vals, Z)
    dM = N.loss_grad_M(torch.as_tensor(Mv), G, torch.as_tensor(csr.vals), torch.as_tensor(Z)).numpy()
    np.testing.assert_allclose(N.backprop_from_M(th, G, dM), grad, rtol=1e-10, atol=1e-12 * np.abs(grad).max())


def test_permutation_equivariance():
    csr, D = small_matrix(n=25, seed=13)
    perm = np.random.default_rng(0).permutation(25)
    Dp = D[np.ix_(perm, perm)]
    th = torch.as_tensor(random_theta(4))
    c1, c2 = P.dense_to_csr(D), P.dense_to_csr(Dp)
    M1 = N.forward(th, N.graph(25, c1.row_ptr, c1.col_idx, c1.vals)).numpy()
    M2 = N.forward(th, N.graph(25, c2.row_ptr, c2.col_idx, c2.vals)).numpy()
    A1 = np.zeros((25, 25))
    A2 = np.zeros((25, 25))
    A1[np.repeat(np.arange(25), np.diff(c1.row_ptr)), c1.col_idx] = M1
    A2[np.repeat(np.arange(25), np.diff(c2.row_ptr)), c2.col_idx] = M2
    np.testing.assert_allclose(A2, A1[np.ix_(perm, perm)], rtol=1e-13, atol=1e-15)


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -3.140625, 1e-3])
    r = N.round_bf16(x)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(r, ref)
