"""Seeded synthetic linear systems for the restarted-GMRES solver and its oracle.

This module only builds inputs: sparse matrices in CSR form, exact solutions
and right-hand sides.  It holds none of the solver's arithmetic, so both the
GPU library and the CPU oracle can be fed from it without sharing code.

The paper measures on SuiteSparse matrices (experimental setup, section 4),
which are not available here; the families below stand in for them:

* constant-coefficient convection-diffusion, 2-D five-point and 3-D
  seven-point first-order upwind stencils on the unit square / cube with a
  zero Dirichlet boundary eliminated (grid interior only, h = 1/(N+1));
* a random non-symmetric matrix with power-law row lengths and a strictly
  dominant diagonal;
* a 3-D variable-coefficient diffusion-convection operator whose diffusivity
  is a log-normal Gaussian random field (cell-centred, h = 1/N).

Every random draw comes from ``numpy.random.default_rng`` seeded with
``SeedSequence([family, purpose, index])`` so that each purpose (matrix,
exact solution, ...) has an independent, reproducible stream.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

# purpose codes for the seed sequences
MATRIX = 0
XTRUE = 1
ROWLEN = 2
COLS = 3
VALS = 4
GRF = 5
BATCH = 6


def rng(family: int, purpose: int, index: int = 0) -> np.random.Generator:
    """Independent PCG64 stream for (family, purpose, index)."""
    return np.random.default_rng(np.random.SeedSequence([int(family), int(purpose), int(index)]))


@dataclass
class CSR:
    """CSR matrix with int32 indices and float64 values (column indices sorted per row)."""

    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    vals: np.ndarray  # float64 [nnz]
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.vals, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    def scaled(self, alpha: float) -> "CSR":
        return CSR(self.n, self.row_ptr.copy(), self.col_idx.copy(), self.vals * alpha, dict(self.meta))


def _from_stencil(cols: np.ndarray, vals: np.ndarray, mask: np.ndarray, meta: dict) -> CSR:
    """Pack an (n, k) table of candidate entries, already in column order, into CSR."""
    n = cols.shape[0]
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[mask].astype(np.int32)
    v = vals[mask].astype(np.float64)
    return CSR(n, row_ptr.astype(np.int32), col_idx, v, meta)


def convdiff(N: int, beta) -> CSR:
    """-Laplace(u) + beta . grad(u) on the unit square (len(beta)=2) or cube (3).

    Grid interior only (N points per side, h = 1/(N+1)), zero Dirichlet
    boundary eliminated, rows in lexicographic order with x fastest.  The
    Laplacian is the standard (2d+1)-point stencil / h^2; the convection term
    is first-order upwind: a backward difference for beta_k > 0 and a forward
    difference for beta_k < 0.  Diagonal: 2d/h^2 + sum_k |beta_k|/h.
    """
    beta = [float(b) for b in beta]
    d = len(beta)
    if d not in (2, 3):
        raise ValueError("beta must have 2 or 3 components")
    n = N ** d
    h = 1.0 / (N + 1)
    idx = np.arange(n, dtype=np.int64)
    coord = [(idx // N ** k) % N for k in range(d)]
    cols, vals, mask = [], [], []
    # columns in increasing order: -N^(d-1) ... -1, 0, +1 ... +N^(d-1)
    for k in reversed(range(d)):
        cols.append(idx - N ** k)
        vals.append(np.full(n, -1.0 / h ** 2 - max(beta[k], 0.0) / h))
        mask.append(coord[k] > 0)
    cols.append(idx)
    vals.append(np.full(n, 2.0 * d / h ** 2 + sum(abs(b) for b in beta) / h))
    mask.append(np.ones(n, dtype=bool))
    for k in range(d):
        cols.append(idx + N ** k)
        vals.append(np.full(n, -1.0 / h ** 2 - max(-beta[k], 0.0) / h))
        mask.append(coord[k] < N - 1)
    return _from_stencil(np.stack(cols, 1), np.stack(vals, 1), np.stack(mask, 1),
                         {"family": "convdiff", "N": N, "dim": d, "beta": beta})


def powerlaw(n: int, family: int = 3, index: int = 0, alpha: float = 2.1,
             lmin: float = 3.917, lmax: int = 2000, dominance: float = 1.2) -> CSR:
    """Random non-symmetric matrix with power-law row lengths.

    Row length L_i (diagonal included) is a continuous power law with density
    proportional to l^-alpha on [lmin, lmax + 0.5], rounded and clipped to
    [2, lmax]; lmin = 3.917 gives a mean of about 20.  L_i - 1 off-diagonal
    columns are uniform over {0..n-1} minus {i}; duplicates are summed.
    Off-diagonal values are N(0, 1); the diagonal is dominance * sum |a_ij|.
    """
    a1 = 1.0 - alpha
    u = rng(family, ROWLEN, index).random(n)
    L = (lmin ** a1 + u * ((lmax + 0.5) ** a1 - lmin ** a1)) ** (1.0 / a1)
    L = np.clip(np.rint(L), 2, lmax).astype(np.int64)
    noff = L - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), noff)
    cols = rng(family, COLS, index).integers(0, n - 1, size=rows.size, dtype=np.int64)
    cols += cols >= rows  # uniform over {0..n-1} \ {i}
    vals = rng(family, VALS, index).standard_normal(rows.size)
    key = rows * n + cols
    ukey, inv = np.unique(key, return_inverse=True)
    uval = np.bincount(inv, weights=vals, minlength=ukey.size)
    urow = ukey // n
    diag = dominance * np.bincount(urow, weights=np.abs(uval), minlength=n)
    allkey = np.concatenate([ukey, np.arange(n, dtype=np.int64) * (n + 1)])
    allval = np.concatenate([uval, diag])
    order = np.argsort(allkey, kind="stable")
    allkey = allkey[order]
    allval = allval[order]
    r = allkey // n
    c = allkey % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=row_ptr[1:])
    return CSR(n, row_ptr.astype(np.int32), c.astype(np.int32), allval.astype(np.float64),
               {"family": "powerlaw", "alpha": alpha, "lmin": lmin, "lmax": lmax})


def gaussian_random_field(N: int, ell: float, g: np.random.Generator) -> np.ndarray:
    """Periodic Gaussian random field on an N^3 grid, mean 0 and std 1.

    White noise filtered by a periodic Gaussian kernel of std ell/sqrt(2)
    cells, so the covariance decays like exp(-r^2 / (2 ell^2)).
    Returned with shape (N, N, N) indexed [z, y, x].
    """
    noise = g.standard_normal((N, N, N))
    f = np.fft.fftfreq(N)
    s = ell / np.sqrt(2.0)
    fz, fy, fx = np.meshgrid(f, f, f, indexing="ij")
    K = np.exp(-2.0 * np.pi ** 2 * s ** 2 * (fx ** 2 + fy ** 2 + fz ** 2))
    field_ = np.fft.ifftn(np.fft.fftn(noise) * K).real
    field_ -= field_.mean()
    field_ /= field_.std()
    return field_


def varcoef3d(N: int, family: int = 5, index: int = 0, ell: float = 8.0, sigma: float = 1.5,
              beta=(30.0, 0.0, 0.0)) -> CSR:
    """-div(kappa grad u) + beta . grad(u), cell-centred on the unit cube.

    kappa = exp(sigma * g) with g a Gaussian random field (correlation length
    ell cells).  h = 1/N; interior faces use the harmonic mean of the two cell
    diffusivities, boundary faces the cell value over a half-cell distance
    (zero Dirichlet data).  Convection is first-order upwind.
    """
    g = gaussian_random_field(N, ell, rng(family, GRF, index))
    kap = np.exp(sigma * g).reshape(-1)  # [z,y,x] flattened: x fastest
    n = N ** 3
    h = 1.0 / N
    idx = np.arange(n, dtype=np.int64)
    coord = [(idx // N ** k) % N for k in range(3)]
    diag = np.zeros(n)
    cols, vals, mask = [], [], []
    lower, upper = {}, {}
    for k in range(3):
        st = N ** k
        has_lo = coord[k] > 0
        has_hi = coord[k] < N - 1
        nb_lo = np.where(has_lo, idx - st, idx)
        nb_hi = np.where(has_hi, idx + st, idx)
        k_lo = np.where(has_lo, 2.0 * kap * kap[nb_lo] / (kap + kap[nb_lo]), 2.0 * kap)
        k_hi = np.where(has_hi, 2.0 * kap * kap[nb_hi] / (kap + kap[nb_hi]), 2.0 * kap)
        diag += (k_lo + k_hi) / h ** 2 + abs(beta[k]) / h
        lower[k] = (idx - st, -k_lo / h ** 2 - max(beta[k], 0.0) / h, has_lo)
        upper[k] = (idx + st, -k_hi / h ** 2 - max(-beta[k], 0.0) / h, has_hi)
    for k in reversed(range(3)):
        c, v, msk = lower[k]
        cols.append(c), vals.append(v), mask.append(msk)
    cols.append(idx), vals.append(diag), mask.append(np.ones(n, dtype=bool))
    for k in range(3):
        c, v, msk = upper[k]
        cols.append(c), vals.append(v), mask.append(msk)
    return _from_stencil(np.stack(cols, 1), np.stack(vals, 1), np.stack(mask, 1),
                         {"family": "varcoef3d", "N": N, "ell": ell, "sigma": sigma,
                          "beta": list(beta), "index": index})


def manufactured_rhs(A: CSR, family: int, index: int = 0):
    """x_true ~ U[-1, 1] (seeded) and b = A x_true in float64."""
    x_true = rng(family, XTRUE, index).uniform(-1.0, 1.0, A.n)
    b = A.to_scipy() @ x_true
    return x_true, b


@dataclass
class Problem:
    """One linear system A x = b with its manufactured solution and solver settings."""

    name: str
    A: CSR
    b: np.ndarray
    x_true: np.ndarray
    m: int
    tol: float
    ortho: str
    extra: dict = field(default_factory=dict)


# ---------------------------------------------------------------------------
# The five workloads.  Family ids are 1-based (C1..C5).

def c1_convdiff2d(N: int = 64) -> Problem:
    """2-D convection-diffusion, beta = (20, 10), GMRES(50) with MGS, FP64."""
    A = convdiff(N, (20.0, 10.0))
    xt, b = manufactured_rhs(A, 1, 0)
    return Problem(f"convdiff2d_N{N}", A, b, xt, 50, 1e-10, "mgs")


def c2_convdiff3d(N: int = 128) -> Problem:
    """3-D convection-diffusion, beta = (50, 20, 10), GMRES(50) with MGS or CGSR."""
    A = convdiff(N, (50.0, 20.0, 10.0))
    xt, b = manufactured_rhs(A, 2, 0)
    return Problem(f"convdiff3d_N{N}", A, b, xt, 50, 1e-10, "cgsr")


def restart_study_3d(N: int = 128, shift: float = 1.0) -> Problem:
    """The 3-D convection-diffusion operator of C2 plus shift * 6/h^2 on the
    diagonal: well conditioned, so float64 GMRES converges within one short
    cycle and a float32 Arnoldi process stalls well before a long restart
    length (the regime of the restart-strategy study)."""
    A = convdiff(N, (50.0, 20.0, 10.0))
    h = 1.0 / (N + 1)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    vals = A.vals.copy()
    vals[rows == A.col_idx] += shift * 6.0 / h ** 2
    A = CSR(A.n, A.row_ptr, A.col_idx, vals, {"family": "convdiff_shifted", "N": N, "shift": shift})
    xt, b = manufactured_rhs(A, 8, N)
    return Problem(f"convdiff3d_shifted_N{N}", A, b, xt, 64, 1e-10, "mgs")


def c3_powerlaw(n: int = 1_000_000) -> Problem:
    """Power-law random sparse system, GMRES(30) with CGSR and a 2-byte basis."""
    A = powerlaw(n, 3, 0)
    xt, b = manufactured_rhs(A, 3, 0)
    return Problem(f"powerlaw_n{n}", A, b, xt, 30, 1e-10, "cgsr")


def c4_batch_specs(count: int = 512, side_lo: int = 32, side_hi: int = 256):
    """(N_i, beta_i) for the batch: N_i uniform on {side_lo..side_hi}, beta_i ~ U[0,100]^2."""
    specs = []
    for i in range(count):
        g = rng(4, BATCH, i)
        N = int(g.integers(side_lo, side_hi + 1))
        beta = tuple(float(v) for v in g.uniform(0.0, 100.0, 2))
        specs.append((N, beta))
    return specs


def c4_batch(count: int = 512, side_lo: int = 32, side_hi: int = 256):
    """The batch of independent 2-D systems, GMRES(40) with MGS."""
    out = []
    for i, (N, beta) in enumerate(c4_batch_specs(count, side_lo, side_hi)):
        A = convdiff(N, beta)
        xt, b = manufactured_rhs(A, 4, i)
        out.append(Problem(f"batch{i}_N{N}", A, b, xt, 40, 1e-10, "mgs", {"beta": beta}))
    return out


def c5_varcoef(index: int, N: int = 64) -> Problem:
    """3-D variable-coefficient instance `index` (train: 0..1999, test: 2000..2199)."""
    A = varcoef3d(N, 5, index)
    xt, b = manufactured_rhs(A, 5, index)
    return Problem(f"varcoef3d_N{N}_i{index}", A, b, xt, 30, 1e-10, "mgs", {"index": index})


def random_dense_nonsym(n: int, seed: int, shift: float = 0.0) -> CSR:
    """Small dense non-symmetric matrix in CSR form (for tests)."""
    g = rng(90, MATRIX, seed)
    M = g.standard_normal((n, n)) / np.sqrt(n) + shift * np.eye(n)
    return dense_to_csr(M)


def dense_to_csr(M: np.ndarray) -> CSR:
    S = sp.csr_matrix(M)
    S.sort_indices()
    return CSR(S.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32),
               S.data.astype(np.float64), {"family": "dense"})
