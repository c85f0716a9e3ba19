"""CPU oracle for restarted GMRES: test infrastructure, not part of the product.

A plain, slow and deliberately unoptimised NumPy implementation of the
method of Lindquist, Luszczek and Dongarra, "Improving the Performance of
the GMRES Method using Mixed-Precision Techniques" (arXiv 2011.01850).
Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the GPU library never does, and this module never
imports the GPU library.

Everything follows Algorithm 1 (restarted GMRES) of the paper, in its order
and notation, with the orthogonalisation procedures MGS and CGSR given with
it.  Floating point is float64 unless an emulated precision is requested.

Readings taken where the paper is silent or garbled (each one is also
listed in the design notes of the repository):

* CGSR shows one projection only; its name and the orthogonality property it
  is used for are those of re-orthogonalised classical Gram-Schmidt, so the
  oracle always performs two full projections (CGS2) and sums them.
* ``s_0 <- beta`` is read as s_1 = beta (1-based), consistent with the
  update of (s_j, s_{j+1}) in the Givens step.
* ``rotation_matrix`` is not defined; with the paper's matrix
  [[alpha, beta], [-beta, alpha]] the rotation that zeroes h_{j+1,j} is
  alpha = a / rho, beta = b / rho with rho = hypot(a, b), and (1, 0) when
  b = 0.
* The restart condition is not specified: the inner loop ends when j = m,
  when the Arnoldi residual |s_{j+1}| / ||b|| <= tol, on an exact breakdown
  (h_{j+1,j} = 0), when the iteration budget is spent, or, optionally, when
  |s_{j+1}| <= delta * beta (the improvement trigger of the restart study).
* "Small enough" is the relative residual ||b - A x||_2 / ||b||_2 <= tol,
  computed in float64 at every restart.
* The residual is z = b - A x (the numerics section writes A x - b; the norm
  is the same).
* A singular least-squares factor is truncated to its largest leading block
  with pivots |H_ii| > 16 k u max|H| (u of the Arnoldi arithmetic).

Emulated precisions (for predicting iteration counts, never for bitwise
parity): ``fp32`` keeps the Krylov basis, w and the Arnoldi copy of A in
float32 while the residual, the update, H, the rotations and the
back-solve stay float64 (the precision split of the numerics section);
``bf16`` / ``fp16`` additionally store each basis vector rounded to nearest
even in the 2-byte format after multiplying by a per-vector power-of-two
scale; ``limited`` is the second, limited mixed solver of the convergence
study (section 4.1): only the Arnoldi copy of A, the preconditioner's output
and the basis are stored in float32, while w, the dot products and the sums
of the Arnoldi product are float64.  Two debug switches reproduce the
negative control of the per-variable study (section 4.1): ``residual_fp32``
computes the restart residual in float32 and ``update_fp32`` keeps x in
float32.

Parity pins for this module live in tests/test_oracle.py.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

RUNNING, CONVERGED, MAXITER, STALLED = 0, 1, 2, 3
STATUS_NAMES = {RUNNING: "RUNNING", CONVERGED: "CONVERGED", MAXITER: "MAXITER", STALLED: "STALLED"}

U64 = 2.0 ** -53
U32 = 2.0 ** -24


class Matrix:
    """CSR matrix with a plain product: y_i = sum over the stored entries of row i of a_ik x_k."""

    def __init__(self, row_ptr, col_idx, vals, n=None):
        self.row_ptr = np.asarray(row_ptr, dtype=np.int64)
        self.col_idx = np.asarray(col_idx, dtype=np.int64)
        self.vals = np.asarray(vals, dtype=np.float64)
        self.n = int(n if n is not None else self.row_ptr.size - 1)
        self.rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        self.vals32 = self.vals.astype(np.float32)

    @classmethod
    def from_csr(cls, A):
        return cls(A.row_ptr, A.col_idx, A.vals, A.n)

    def matvec(self, x):
        """Float64 product (sums taken by bincount, in storage order)."""
        x = np.asarray(x, dtype=np.float64)
        return np.bincount(self.rows, weights=self.vals * x[self.col_idx], minlength=self.n)

    def matvec32(self, x32, vals32=None):
        """Emulated single-precision product: float32 products, result rounded to float32.

        ``vals32`` replaces the float32 copy of the values (the split-storage
        form passes the high-word values)."""
        v = self.vals32 if vals32 is None else vals32
        prod = (v * np.asarray(x32, dtype=np.float32)[self.col_idx]).astype(np.float64)
        return np.bincount(self.rows, weights=prod, minlength=self.n).astype(np.float32)

    def matvec_wide(self, x32, vals32=None):
        """The limited mode's product: float32-stored values and x, widened to
        float64 (each product is then exact) and summed in float64."""
        v = self.vals32 if vals32 is None else vals32
        return self.matvec_values(v, np.asarray(x32, dtype=np.float32))

    def matvec_values(self, vals, x):
        """Product with the given values (any precision, widened to float64)
        and x widened to float64, summed in float64."""
        prod = np.asarray(vals).astype(np.float64) * np.asarray(x).astype(np.float64)[self.col_idx]
        return np.bincount(self.rows, weights=prod, minlength=self.n)

    def diagonal(self):
        d = np.zeros(self.n)
        on = self.rows == self.col_idx
        d[self.rows[on]] = self.vals[on]
        return d

    def dense(self):
        D = np.zeros((self.n, self.n))
        np.add.at(D, (self.rows, self.col_idx), self.vals)
        return D


# ---------------------------------------------------------------------------
# ILU(0), the preconditioner of the paper's experiments: incomplete LU with
# the sparsity pattern of A (no fill).  L is unit lower triangular and U upper
# triangular, both stored in A's pattern.

def ilu0(A: Matrix):
    """Factor values on A's pattern (float64): entries below the diagonal hold
    L, the rest U.  Row by row (the IKJ order): for each stored a_ik, k < i,
    ascending, l_ik = a_ik / u_kk and every stored a_ij with j > k that row k
    also stores loses l_ik u_kj."""
    rp, ci = A.row_ptr, A.col_idx
    lu = A.vals.copy()
    diag = np.full(A.n, -1, dtype=np.int64)
    for i in range(A.n):
        for p in range(rp[i], rp[i + 1]):
            if ci[p] == i:
                diag[i] = p
    if np.any(diag < 0):
        raise ValueError("ILU(0) needs every diagonal entry stored")
    for i in range(A.n):
        for p in range(rp[i], diag[i]):
            k = ci[p]
            lik = lu[p] / lu[diag[k]]
            lu[p] = lik
            q, q_end = diag[k] + 1, rp[k + 1]
            p2, p2_end = p + 1, rp[i + 1]
            while q < q_end and p2 < p2_end:
                if ci[q] == ci[p2]:
                    lu[p2] -= lik * lu[q]
                    q += 1
                    p2 += 1
                elif ci[q] < ci[p2]:
                    q += 1
                else:
                    p2 += 1
    return lu, diag


def ilu_apply(A: Matrix, lu, diag, v, sweeps=0, dtype=np.float64):
    """z = U^-1 L^-1 v.  sweeps = 0: exact substitutions.  sweeps = s > 0:
    s Jacobi sweeps per triangle from a zero start (y <- v - L' y, then
    x <- D^-1 (y - U' x)), which equal the substitutions once s reaches the
    triangle's depth; arithmetic in `dtype`."""
    rp, ci = A.row_ptr, A.col_idx
    n = A.n
    lu_t = lu.astype(dtype)
    v = np.asarray(v, dtype=dtype)
    if sweeps == 0:
        y = np.zeros(n, dtype=dtype)
        for i in range(n):
            acc = v[i]
            for p in range(rp[i], diag[i]):
                acc = dtype(acc - lu_t[p] * y[ci[p]])
            y[i] = acc
        x = np.zeros(n, dtype=dtype)
        for i in range(n - 1, -1, -1):
            acc = y[i]
            for p in range(diag[i] + 1, rp[i + 1]):
                acc = dtype(acc - lu_t[p] * x[ci[p]])
            x[i] = dtype(acc / lu_t[diag[i]])
        return x
    rows = np.repeat(np.arange(n), np.diff(rp))
    lower = ci < rows
    upper = ci > rows
    dinv = (dtype(1.0) / lu_t[diag]).astype(dtype)

    def part_product(mask, src):
        if dtype == np.float64:  # float64: the row sums in storage order
            return np.bincount(rows[mask], weights=lu_t[mask] * src[ci[mask]], minlength=n)
        out = np.zeros(n, dtype=dtype)  # reduced precision: every partial sum rounded
        for i in range(n):
            acc = dtype(0.0)
            for p in range(rp[i], rp[i + 1]):
                if mask[p]:
                    acc = dtype(acc + lu_t[p] * src[ci[p]])
            out[i] = acc
        return out

    y = np.zeros(n, dtype=dtype)
    for _ in range(sweeps):
        y = (v - part_product(lower, y)).astype(dtype)
    x = np.zeros(n, dtype=dtype)
    for _ in range(sweeps):
        x = ((y - part_product(upper, x)) * dinv).astype(dtype)
    return x


def triangle_depths(A: Matrix, diag):
    """Number of levels of the lower and of the upper triangle's dependency graph."""
    rp, ci = A.row_ptr, A.col_idx
    lv = np.zeros(A.n, dtype=np.int64)
    for i in range(A.n):
        lo = ci[rp[i]:diag[i]]
        lv[i] = 1 + (lv[lo].max() if lo.size else 0)
    uv = np.zeros(A.n, dtype=np.int64)
    for i in range(A.n - 1, -1, -1):
        up = ci[diag[i] + 1:rp[i + 1]]
        uv[i] = 1 + (uv[up].max() if up.size else 0)
    return int(lv.max()), int(uv.max())


# ---------------------------------------------------------------------------
# Split storage of the float64 matrix values (the alternative organisation
# the paper suggests for the matrix it otherwise stores twice): the high and
# low 32-bit words of each value in two arrays.  Reading the high words only
# gives each value with its significand cut after 20 bits (towards zero).

def high_word_value(vals):
    """float64 values keeping only their high 32-bit word (sign, exponent and
    the first 20 significand bits; the low word set to zero)."""
    bits = np.ascontiguousarray(vals, dtype=np.float64).view(np.uint64)
    return (bits & np.uint64(0xFFFFFFFF00000000)).view(np.float64)


# ---------------------------------------------------------------------------
# 2-byte storage of a basis vector (the half-precision direction of the
# conclusion's future work; the paper prints no format, so the scale rule is
# this project's reading: a power of two that puts max|v| in (T/2, T]).

FMT_TARGET_LOG2 = {"fp16": 15, "bf16": 0}


def round_bf16(x32):
    """Round float32 values to bfloat16 (nearest, ties to even); returns float32."""
    b = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def round_fp16(x32):
    """Round float32 values to IEEE half (nearest, ties to even); returns float32."""
    return np.asarray(x32, dtype=np.float32).astype(np.float16).astype(np.float32)


def scale_exponent(vmax: float, fmt: str) -> int:
    """e such that vmax * 2**e lies in (T/2, T], T = 2**FMT_TARGET_LOG2[fmt]."""
    if not (vmax > 0.0) or not math.isfinite(vmax):
        return 0
    f, p = math.frexp(vmax)  # vmax = f * 2**p, f in [0.5, 1)
    return FMT_TARGET_LOG2[fmt] - p + (1 if f == 0.5 else 0)


def encode(w32, inv_h: float, fmt: str):
    """Store v = w / h in a 2-byte format with a power-of-two scale.

    vmax = max|w| / h; e = scale_exponent(vmax); f = float32(2**e / h);
    stored = round(float32(w * f)); the decoded vector is stored * 2**-e.
    Returns (stored values as float32, decode scale 2**-e).
    """
    w32 = np.asarray(w32, dtype=np.float32)
    vmax = float(np.max(np.abs(w32))) * inv_h if w32.size else 0.0
    e = scale_exponent(vmax, fmt)
    f = np.float32(math.ldexp(1.0, e) * inv_h)
    t = (w32 * f).astype(np.float32)
    stored = round_fp16(t) if fmt == "fp16" else round_bf16(t)
    return stored, math.ldexp(1.0, -e)


# ---------------------------------------------------------------------------

def givens(a: float, b: float):
    """(alpha, beta) of the rotation [[alpha, beta], [-beta, alpha]] taking (a, b) to (rho, 0)."""
    if b == 0.0:
        return 1.0, 0.0
    rho = math.hypot(a, b)
    return a / rho, b / rho


def back_solve(H, s, k, u):
    """y = H[:k,:k]^-1 s[:k] for upper-triangular H, truncated where H is singular.

    The leading block kept is the longest one whose pivots all exceed
    16 k u max|H|, u being the unit roundoff of the Arnoldi arithmetic.
    """
    if k == 0:
        return np.zeros(0), 0
    Hk = H[:k, :k]
    hn = np.max(np.abs(Hk))
    thr = 16 * k * u * hn
    kk = 0
    while kk < k and abs(Hk[kk, kk]) > thr:
        kk += 1
    y = np.zeros(kk)
    for i in range(kk - 1, -1, -1):
        y[i] = (s[i] - np.dot(Hk[i, i + 1:kk], y[i + 1:kk])) / Hk[i, i]
    return y, kk


def stall_window(m: int) -> int:
    """5% of the inner iterations per restart, at least one (the stall definition of Table 1)."""
    return max(1, math.ceil(0.05 * m))


def stall_point(arnoldi_res, m: int):
    """Number of inner iterations before the Arnoldi residual stalls (Table 1's definition).

    ``arnoldi_res[j]`` is the Arnoldi residual |s_{j+1}| after j inner steps
    of one cycle (``arnoldi_res[0]`` = beta).  The improvement has stalled
    after j steps when the next window of w = max(1, ceil(0.05 m)) steps
    improves it by less than a factor 1.001.  Returns the first such j, or
    None when no stall is seen in the recorded steps.
    """
    w = stall_window(m)
    seq = list(arnoldi_res)
    for j in range(len(seq) - w):
        if seq[j + w] > seq[j] / 1.001:
            return j
    return None


@dataclass
class Result:
    x: np.ndarray
    status: int
    iters: int
    restarts: int
    rel_residual: float
    history: list = field(default_factory=list)  # relative restart residuals
    arnoldi: list = field(default_factory=list)  # per cycle: list of |s_{j+1}| / ||b||
    cycles: list = field(default_factory=list)  # per cycle (record=True): dict(V, Hbar, H, s, k, beta)
    fallback_used: bool = False

    @property
    def status_name(self):
        return STATUS_NAMES[self.status]


# ---------------------------------------------------------------------------
# Loss of orthogonality of the basis (the last restart strategy of section 3):
# S_k = (I + U_k)^-1 U_k with U_k the strictly upper part of V_k^T V_k; the
# basis is linearly dependent exactly when ||S_k||_2 = 1.

def orth_s_append(OU, OS, c, u):
    """Column c of U and S from u = V_{0..c-1}^T v_c.

    Because S_{c+1} = [[S_c, (I + U_c)^-1 u], [0, 0]], only the new column
    needs computing: the unit upper triangular system (I + U_c) s = u, solved
    from the last row up.  OU and OS are square arrays updated in place;
    returns s."""
    OU[:c, c] = u
    sv = np.array(u, dtype=np.float64)
    for r in range(c - 1, -1, -1):
        for l in range(r + 1, c):
            sv[r] -= OU[r, l] * sv[l]
    OS[:c, c] = sv
    return sv


def power_norm(S, iters=10):
    """||S||_2 estimated by `iters` power iterations on S^T S from the
    all-ones vector (normalised), then ||S x||."""
    k = S.shape[0]
    x = np.full(k, 1.0 / math.sqrt(k))
    for _ in range(iters):
        z = S.T @ (S @ x)
        nz = float(np.linalg.norm(z))
        if not nz > 0.0:
            return 0.0
        x = z / nz
    return float(np.linalg.norm(S @ x))


def _cast(v, precision):
    return np.asarray(v, dtype=np.float64 if precision == "fp64" else np.float32)


# ---------------------------------------------------------------------------
# The steps of one restart cycle of Algorithm 1, each on its own.  Precision
# modes: "fp64"; "fp32" (basis, w and A's Arnoldi copy in float32); "bf16" /
# "fp16" (the float32 mode with each basis vector stored in a 2-byte format);
# "limited" (basis, A's Arnoldi copy and M in float32, w and its sums in
# float64).

class _Basis:
    """The stored Krylov basis of one cycle: v_i as stored (float64, float32
    or 2-byte values) with a decode scale each."""

    def __init__(self, m, n, precision):
        self.precision = precision
        self.two_byte = precision in ("bf16", "fp16")
        self.lowp = precision != "fp64"
        self.limited = precision == "limited"
        self.V = [None] * (m + 1)
        self.scale = np.zeros(m + 1)
        self.n, self.m = n, m
        self.Vmat = None  # [v_1 .. v_j] as one matrix for CGSR, filled column by column

    def store(self, i, vec, h):
        """v_i = vec / h in the mode's storage.  For the float32 modes vec is
        already what the mode holds (float32 w, or the float64 w of the
        limited mode) and is multiplied by float32(1/h)."""
        if self.two_byte:
            self.V[i], self.scale[i] = encode(np.asarray(vec).astype(np.float32), 1.0 / h, self.precision)
        elif self.lowp:
            self.V[i], self.scale[i] = (vec * np.float32(1.0 / h)).astype(np.float32), 1.0
        else:
            self.V[i], self.scale[i] = vec / h, 1.0

    def vec(self, i):
        """v_i decoded (float32 in the reduced modes)."""
        if self.two_byte:
            return (self.V[i] * np.float32(self.scale[i])).astype(np.float32)
        return self.V[i]

    def operand(self, i):
        """v_i as the orthogonalisation reads it (widened in the limited mode)."""
        return self.V[i].astype(np.float64) if self.limited else self.vec(i)

    def matrix(self, j):
        """[v_1 .. v_{j+1}] for the CGSR projections (column j added now)."""
        col = self.operand(j)
        if self.Vmat is None:
            self.Vmat = np.empty((self.n, self.m + 1), dtype=col.dtype)
        self.Vmat[:, j] = col
        return self.Vmat[:, : j + 1]


def _arnoldi_product(A: Matrix, src, a32, a64_values, wide_w):
    """w = A src: float64 values summed in float64 (rounded once to float32
    unless w is float64); float32 values widened and summed in float64 (w
    float64); or the float32 product."""
    if a64_values:
        w = A.matvec(np.asarray(src).astype(np.float64))
        return w if wide_w else w.astype(np.float32)
    if wide_w:
        return A.matvec_values(a32, src)
    return A.matvec32(src, a32)


def _mgs(w, basis: _Basis, j):
    """Modified Gram-Schmidt: for i = 1..j, h_ij = w . v_i, w -= h_ij v_i
    (h_ij rounded to float32 where w is float32)."""
    hcol = np.zeros(j + 1)
    single = basis.lowp and not basis.limited
    for i in range(j + 1):
        vi = basis.operand(i)
        hij = float(np.dot(w, vi))
        hcol[i] = hij
        w = (w - (np.float32(hij) if single else hij) * vi).astype(w.dtype)
    return w, hcol


def _cgsr(w, basis: _Basis, j):
    """CGSR: classical Gram-Schmidt, then its re-orthogonalisation pass, each
    one matrix-vector product with the stored basis; h = h1 + h2."""
    hcol = np.zeros(j + 1)
    Vj = basis.matrix(j)
    for _ in range(2):
        hp = Vj.T @ w
        w = (w - Vj @ hp.astype(w.dtype)).astype(w.dtype)
        hcol += hp.astype(np.float64)
    return w, hcol


def _givens_step(H, cs, sn, s, j):
    """Column j of H: apply the earlier rotations, form rotation j, update
    (s_j, s_{j+1}) and zero h_{j+1,j}."""
    for i in range(j):
        a, c = H[i, j], H[i + 1, j]
        H[i, j] = cs[i] * a + sn[i] * c
        H[i + 1, j] = -sn[i] * a + cs[i] * c
    cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
    s[j + 1] = -sn[j] * s[j]
    s[j] = cs[j] * s[j]
    H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
    H[j + 1, j] = 0.0


class _OrthMonitor:
    """Loss of orthogonality of the cycle's basis: ||S_k|| after each new vector."""

    def __init__(self, m, norm):
        self.OU = np.zeros((m + 1, m + 1))
        self.OS = np.zeros((m + 1, m + 1))
        self.fro2 = 0.0
        self.norm = norm

    def add(self, basis: _Basis, c):
        vn = basis.vec(c).astype(np.float64)
        u = np.array([float(np.dot(basis.vec(i).astype(np.float64), vn)) for i in range(c)])
        sv = orth_s_append(self.OU, self.OS, c, u)
        self.fro2 += float(sv @ sv)
        return math.sqrt(self.fro2) if self.norm == "frobenius" else power_norm(self.OS[: c + 1, : c + 1])


def gmres(A: Matrix, b, x0=None, m=50, tol=1e-10, max_iters=10 ** 7, ortho="mgs",
          precision="fp64", precond=None, restart_improve=0.0, stall_cycles=10,
          fallback=True, record=False, residual_fp32=False, update_fp32=False, a_storage="copy",
          restart_repeat=False, restart_on_stall=False, orth_restart=0.0, orth_norm="spectral",
          arnoldi_a="default", side="right"):
    """Restarted GMRES(m) following Algorithm 1, optionally preconditioned.

    ``precond`` is None (plain GMRES, M^-1 = I) or a callable v -> M^-1 v.
    ``side="right"``: flexible GMRES, z_j = M^-1 v_j, w = A z_j, and the
    correction is Z y (the form the learned preconditioner uses).
    ``side="left"`` (the paper's form): r = M^-1 (b - A x) starts the cycle
    (beta = ||r||), w = M^-1 A v_j, the correction is V y, and the inner
    loop's estimate |s_{j+1}| is compared with tol ||M^-1 b|| (it estimates
    the preconditioned residual); the restart residual b - A x stays the
    judge.  The preconditioner's input and output have w's precision.
    ``a_storage="split"`` emulates the split storage of A: the float32
    Arnoldi product uses the high-word values (the float64 residual is
    unchanged, as both words together are the float64 value).

    Restart strategies of the restart study (section 3), on top of j = m and
    the improvement threshold ``restart_improve``: ``restart_repeat`` is the
    two-stage strategy (the first cycle ends as usual; every later one after
    as many inner iterations as the first took; the improvement threshold
    only applies to the first cycle); ``restart_on_stall`` ends a cycle once
    the Arnoldi residual has stalled over the window of ``stall_window``;
    ``orth_restart`` > 0 ends a cycle once ||S_k|| (``orth_norm``: the
    10-step power estimate of the 2-norm, or the Frobenius norm) of the basis
    built so far reaches it.

    ``arnoldi_a`` picks the values of A the Arnoldi product reads, for the
    per-variable study of section 4.1: "default" (float64 in the fp64 mode,
    the float32 copy otherwise), "fp64" or "fp32" in any mode.  The sums are
    float64 whenever w or the values are float64.
    """
    if ortho not in ("mgs", "cgsr"):
        raise ValueError(ortho)
    if precision not in ("fp64", "fp32", "bf16", "fp16", "limited"):
        raise ValueError(precision)
    if a_storage not in ("copy", "split"):
        raise ValueError(a_storage)
    if arnoldi_a not in ("default", "fp64", "fp32"):
        raise ValueError(arnoldi_a)
    if side not in ("right", "left"):
        raise ValueError(side)
    # the Arnoldi product's copy of A in the reduced-precision modes: float32
    # rounding of the values, or (split storage) the high-word values
    a32 = A.vals32 if a_storage == "copy" else high_word_value(A.vals).astype(np.float32)
    b = np.asarray(b, dtype=np.float64)
    n = A.n
    bn = float(np.linalg.norm(b))
    if bn == 0.0:
        return Result(np.zeros(n), CONVERGED, 0, 0, 0.0, [0.0])
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    if update_fp32:
        x = x.astype(np.float32).astype(np.float64)
    lowp = precision != "fp64"
    wide_w = precision in ("fp64", "limited")  # w, its dots and the product's sums in float64
    a64_arnoldi = arnoldi_a == "fp64" or (arnoldi_a == "default" and precision == "fp64")
    orthogonalize = _mgs if ortho == "mgs" else _cgsr
    left = side == "left"

    def wprec(v):  # a vector in w's precision
        return np.asarray(v, dtype=np.float64 if wide_w else np.float32)

    # left preconditioning: the inner loop's estimate is measured against ||M^-1 b||
    bnp = float(np.linalg.norm(wprec(precond(wprec(b))).astype(np.float64))) if left and precond else bn
    total = 0
    restarts = 0
    hist, arn, cyc = [], [], []
    status = RUNNING
    fallback_used = False
    best_beta = math.inf
    no_progress = 0
    prev_beta = math.inf
    use_pc = precond is not None
    klimit = 0  # two-stage strategy: length of the first cycle once it has ended
    win = stall_window(m)
    while True:
        # Alg. 1: residual, in full precision unless the negative control asks otherwise
        if residual_fp32:
            Ax = A.matvec32(x.astype(np.float32)).astype(np.float64)
            z = (b.astype(np.float32) - Ax.astype(np.float32)).astype(np.float64)
        else:
            z = b - A.matvec(x)
        beta = float(np.linalg.norm(z))
        rel = beta / bn
        hist.append(rel)
        if rel <= tol:
            status = CONVERGED
            break
        if not math.isfinite(beta):
            status = STALLED
            break
        if total >= max_iters:
            status = MAXITER
            break
        # outer stall: a cycle that does not lower beta at all, several times running
        if beta >= best_beta:
            no_progress += 1
        else:
            no_progress = 0
        best_beta = min(best_beta, beta)
        if no_progress >= stall_cycles:
            status = STALLED
            break
        # fallback of the flexible solver: a cycle gaining less than 1.001x
        if use_pc and fallback and beta > prev_beta / 1.001:
            use_pc = False
            fallback_used = True
        prev_beta = beta

        basis = _Basis(m, n, precision)
        Z = [None] * m
        H = np.zeros((m + 1, m))
        Hbar = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        s = np.zeros(m + 1)
        left_pc = left and use_pc
        if left_pc:  # the cycle starts from the preconditioned residual
            r = wprec(precond(wprec(z)))
            beta_c = float(np.linalg.norm(r.astype(np.float64)))
            est_norm = bnp
            if not (beta_c > 0.0) or not math.isfinite(beta_c):
                # M^-1 z vanished or is not finite: the preconditioner is
                # switched off and the next cycle runs plain GMRES
                use_pc = False
                fallback_used = True
                continue
        else:
            r, beta_c, est_norm = z, beta, bn
        s[0] = beta_c  # s_1 = beta
        basis.store(0, r.astype(np.float32) if lowp else r, beta_c)
        monitor = _OrthMonitor(m, orth_norm) if orth_restart > 0.0 else None
        k = 0
        W = []  # (record) w after orthogonalisation, before normalisation, per step
        cycle_arn = []
        ares = [beta_c]  # |s_1| .. |s_{j+1}| of this cycle
        for j in range(m):
            # w <- A v_j (flexible form: z_j = M v_j, w <- A z_j)
            vj = basis.vec(j)
            right_pc = use_pc and not left
            if right_pc:
                Z[j] = _cast(precond(vj), precision)
            w = _arnoldi_product(A, Z[j] if right_pc else vj, a32, a64_arnoldi, wide_w)
            if left_pc:  # w <- M^-1 A v_j
                w = wprec(precond(w))
            w, hcol = orthogonalize(w, basis, j)
            hnext = float(np.linalg.norm(w.astype(np.float64)))
            if record:
                W.append(w.astype(np.float64))
            H[: j + 1, j] = hcol
            H[j + 1, j] = hnext
            Hbar[: j + 2, j] = H[: j + 2, j]
            total += 1
            k = j + 1
            _givens_step(H, cs, sn, s, j)
            cycle_arn.append(abs(s[j + 1]) / est_norm)
            ares.append(abs(s[j + 1]))
            if hnext == 0.0 or not math.isfinite(hnext):
                if not math.isfinite(hnext):
                    k = j  # drop the non-finite column
                break
            basis.store(j + 1, w, hnext)
            # restart conditions: the estimate, the budget, the triggers
            if abs(s[j + 1]) / est_norm <= tol or total >= max_iters:
                break
            first_stage = not restart_repeat or klimit == 0
            if restart_improve > 0.0 and first_stage and abs(s[j + 1]) <= restart_improve * beta_c:
                break
            if not first_stage and j + 1 >= klimit:
                break
            if restart_on_stall and j + 1 - win >= 0 and ares[j + 1] > ares[j + 1 - win] / 1.001:
                break
            if monitor is not None and monitor.add(basis, j + 1) >= orth_restart:
                break
        if restart_repeat and klimit == 0 and k > 0:
            klimit = k
        # correction u = V_j H^-1 s (Z y in the flexible form), applied in full precision
        y, kk = back_solve(H, s, k, U32 if lowp else U64)
        u = np.zeros(n)
        for i in range(kk):
            src = Z[i] if use_pc and not left else basis.vec(i)
            u += y[i] * src.astype(np.float64)
        if update_fp32:
            x = (x.astype(np.float32) + u.astype(np.float32)).astype(np.float64)
        else:
            x = x + u
        restarts += 1
        arn.append(cycle_arn)
        if record:
            cyc.append({"V": [basis.vec(i).astype(np.float64) for i in range(k + 1) if basis.V[i] is not None],
                        "Hbar": Hbar[: k + 1, :k].copy(), "H": H[:k, :k].copy(), "s": s[: k + 1].copy(),
                        "k": k, "beta": beta_c, "y": y, "cs": cs[:k].copy(), "sn": sn[:k].copy(), "W": W})
    return Result(x, status, total, restarts, hist[-1], hist, arn, cyc, fallback_used)


def relative_residual(A: Matrix, b, x) -> float:
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(b - A.matvec(x)) / np.linalg.norm(b))


def backward_error(A: Matrix, b, x) -> float:
    """||r|| / (||A||_F ||x|| + ||b||): normwise backward error with ||A||_F for ||A||_2."""
    r = np.asarray(b) - A.matvec(x)
    return float(np.linalg.norm(r) / (np.linalg.norm(A.vals) * np.linalg.norm(x) + np.linalg.norm(b)))
