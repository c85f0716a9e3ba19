"""CPU oracle for the learned sparse approximate inverse: test infrastructure only.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module; the GPU library never does, and this
module never imports the GPU library.

The paper's solver takes a preconditioner M^-1 ~ A^-1 as an input of
Algorithm 1 and its experiments use ILU(0).  The learned preconditioner is
this project's extension: a small message-passing network over the
stored entries (edges) of A emits the values of M on A's own sparsity
pattern, and M is applied on the right in flexible GMRES.  The paper
prescribes no network, so everything below is this project's definition,
written out plainly in float64 with PyTorch CPU tensors; the gradient is
taken by PyTorch's autograd, which the tests pin against central finite
differences.

Definition (n rows, edges e = (i, j) = the stored entries of A in CSR order):

* d_i = |a_ii| (1 if a_ii = 0), sigma_i = sign(a_ii) (1 if a_ii = 0),
  deg_i = stored entries of row i, ahat_ij = a_ij / sqrt(d_i d_j).
* edge input f_ij = [ahat_ij, ahat_ji (0 if (j, i) is not stored), [i == j]].
* node input x_i = [sum_{j != i} ahat_ij, sum_{j != i} |ahat_ij|,
  sum_{j != i} ahat_ji] (sums over the stored entries of row i, and of
  column i for the last one).
* encoders: h_i = relu(Wn x_i + bn), e_ij = relu(We f_ij + be), width 32.
* three message layers l = 1, 2, 3, with u_ij = [h_i, h_j, e_ij] (96 wide):
  m_ij = relu(W_l u_ij + b_l); then h_i <- h_i + (1/deg_i) sum_j m_ij and
  e_ij <- m_ij (u is taken before the update).
* decoder: s_ij = wo . [h_i, h_j, e_ij] + bo, and
  M_ij = (sigma_i [i == j] + s_ij) / sqrt(d_i d_j), so wo = 0, bo = 0 gives
  Jacobi, M = diag(1 / a_ii).

Training loss over pairs (z_k, k = 1..K) that the solver produces (its
restart residuals):  L = (1/K) sum_k ||A M z_k - z_k||^2 / ||z_k||^2, whose
gradient on the pattern is dL/dM_ij = (2/K) sum_k (A^T r_k)_i z_kj / ||z_k||^2
with r_k = A M z_k - z_k.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

H = 32          # hidden width
NIN = 3         # node / edge input features
U = 3 * H       # message input width

# flat parameter layout: (name, shape); matrices row-major (out x in)
LAYOUT = [("Wn", (H, NIN)), ("bn", (H,)), ("We", (H, NIN)), ("be", (H,)),
          ("W1", (H, U)), ("b1", (H,)), ("W2", (H, U)), ("b2", (H,)),
          ("W3", (H, U)), ("b3", (H,)), ("wo", (U,)), ("bo", (1,))]


def offsets():
    off, out = 0, {}
    for name, shape in LAYOUT:
        size = int(np.prod(shape))
        out[name] = (off, shape)
        off += size
    return out, off


OFFSETS, NPARAMS = offsets()


def unpack(theta):
    """Flat parameter vector -> dict of tensors (views)."""
    return {name: theta[o:o + int(np.prod(shape))].reshape(shape) for name, (o, shape) in OFFSETS.items()}


def init_params(seed: int) -> np.ndarray:
    """He-style random hidden weights, zero biases, zero decoder (M = Jacobi)."""
    g = np.random.default_rng(seed)
    theta = np.zeros(NPARAMS)
    for name, (o, shape) in OFFSETS.items():
        if name.startswith("W"):
            fan_in = shape[1]
            theta[o:o + int(np.prod(shape))] = g.normal(0.0, np.sqrt(2.0 / fan_in), int(np.prod(shape)))
    return theta


@dataclass
class Graph:
    n: int
    rows: torch.Tensor    # [nnz] row of each edge
    cols: torch.Tensor    # [nnz] column of each edge
    deg: torch.Tensor     # [n]
    tpos: torch.Tensor    # [nnz] position of the transposed entry, -1 if not stored
    d: torch.Tensor       # [n]
    sigma: torch.Tensor   # [n]
    ahat: torch.Tensor    # [nnz]
    x: torch.Tensor       # [n, 3] node inputs
    f: torch.Tensor       # [nnz, 3] edge inputs


def graph(n, row_ptr, col_idx, vals) -> Graph:
    """Inputs of the network for one matrix (float64)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    where = {(int(r), int(c)): e for e, (r, c) in enumerate(zip(rows, col_idx))}
    tpos = np.array([where.get((int(c), int(r)), -1) for r, c in zip(rows, col_idx)], dtype=np.int64)
    a_ii = np.zeros(n)
    on = rows == col_idx
    a_ii[rows[on]] = vals[on]
    d = np.where(a_ii != 0.0, np.abs(a_ii), 1.0)
    sigma = np.where(a_ii < 0.0, -1.0, 1.0)
    ahat = vals / np.sqrt(d[rows] * d[col_idx])
    ahat_t = np.where(tpos >= 0, ahat[np.maximum(tpos, 0)], 0.0)
    diag = (rows == col_idx).astype(np.float64)
    off = 1.0 - diag
    x = np.zeros((n, 3))
    np.add.at(x[:, 0], rows, ahat * off)
    np.add.at(x[:, 1], rows, np.abs(ahat) * off)
    np.add.at(x[:, 2], col_idx, ahat * off)   # sum over column i of ahat_ji = sum_j ahat_ji
    f = np.stack([ahat, ahat_t, diag], axis=1)
    t = lambda a, dt=torch.float64: torch.as_tensor(a, dtype=dt)  # noqa: E731
    return Graph(n=n, rows=t(rows, torch.int64), cols=t(col_idx, torch.int64),
                 deg=t(np.diff(row_ptr).astype(np.float64)), tpos=t(tpos, torch.int64), d=t(d), sigma=t(sigma),
                 ahat=t(ahat), x=t(x), f=t(f))


def forward(theta: torch.Tensor, G: Graph, return_states=False):
    """Values of M on A's pattern (float64 tensor [nnz])."""
    P = unpack(theta)
    relu = torch.relu
    h = relu(G.x @ P["Wn"].T + P["bn"])
    e = relu(G.f @ P["We"].T + P["be"])
    states = [(h, e)]
    for l in (1, 2, 3):
        u = torch.cat([h[G.rows], h[G.cols], e], dim=1)
        m = relu(u @ P[f"W{l}"].T + P[f"b{l}"])
        agg = torch.zeros_like(h).index_add(0, G.rows, m)
        h = h + agg / torch.clamp(G.deg, min=1.0)[:, None]  # a row without entries gets no message
        e = m
        states.append((h, e))
    u = torch.cat([h[G.rows], h[G.cols], e], dim=1)
    s = u @ P["wo"] + P["bo"]
    diag = (G.rows == G.cols).to(torch.float64)
    M = (G.sigma[G.rows] * diag + s) / torch.sqrt(G.d[G.rows] * G.d[G.cols])
    return (M, s, states) if return_states else M


def spmv(n, rows, cols, vals, x):
    """y = A x with A given by its stored entries (rows, cols, vals)."""
    return torch.zeros(n, dtype=x.dtype).index_add(0, rows, vals * x[cols])


def loss(Mv: torch.Tensor, G: Graph, avals: torch.Tensor, Z: torch.Tensor):
    """L = (1/K) sum_k ||A M z_k - z_k||^2 / ||z_k||^2 for the K columns of Z ([n, K])."""
    K = Z.shape[1]
    total = torch.zeros((), dtype=torch.float64)
    for k in range(K):
        z = Z[:, k]
        r = spmv(G.n, G.rows, G.cols, avals, spmv(G.n, G.rows, G.cols, Mv, z)) - z
        total = total + (r @ r) / (z @ z)
    return total / K


def loss_grad_M(Mv, G: Graph, avals, Z):
    """dL/dM on the pattern by the closed form 2/K sum_k (A^T r_k)_i z_kj / ||z_k||^2."""
    K = Z.shape[1]
    g = torch.zeros_like(Mv)
    for k in range(K):
        z = Z[:, k]
        r = spmv(G.n, G.rows, G.cols, avals, spmv(G.n, G.rows, G.cols, Mv, z)) - z
        atr = spmv(G.n, G.cols, G.rows, avals, r)  # A^T r: swap the roles of rows and columns
        g = g + 2.0 * atr[G.rows] * z[G.cols] / (z @ z)
    return g / K


def value_and_grad(theta_np, G: Graph, avals_np, Z_np):
    """(L, dL/dtheta, M) in float64; the gradient through the network by autograd."""
    theta = torch.tensor(np.asarray(theta_np, dtype=np.float64), requires_grad=True)
    avals = torch.as_tensor(np.asarray(avals_np, dtype=np.float64))
    Z = torch.as_tensor(np.asarray(Z_np, dtype=np.float64))
    Mv = forward(theta, G)
    L = loss(Mv, G, avals, Z)
    L.backward()
    return float(L.detach()), theta.grad.detach().numpy().copy(), Mv.detach().numpy().copy()


def backprop_from_M(theta_np, G: Graph, dM_np):
    """dtheta = (dM/dtheta)^T dM for a given upstream gradient on the M values."""
    theta = torch.tensor(np.asarray(theta_np, dtype=np.float64), requires_grad=True)
    Mv = forward(theta, G)
    Mv.backward(torch.as_tensor(np.asarray(dM_np, dtype=np.float64)))
    return theta.grad.detach().numpy().copy()


def round_bf16(theta):
    """Parameters rounded to bfloat16 (nearest, ties to even), as float64."""
    x = np.asarray(theta, dtype=np.float32).view(np.uint32).astype(np.uint64)
    x = (x + 0x7FFF + ((x >> 16) & 1)) >> 16 << 16
    return x.astype(np.uint32).view(np.float32).astype(np.float64)
