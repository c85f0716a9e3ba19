"""Training and evaluation of the learned sparse approximate inverse.

The training data are residuals that the solver itself produces: for each
training matrix, the restart residuals z_k = b - A x_k of a few cycles of
unpreconditioned mixed-precision GMRES(m) (x_0 = 0, so z_0 = b).  The loss
is L = mean_k ||A M z_k - z_k||^2 / ||z_k||^2 (spai.h); forward, loss,
backward and the Adam update all run in the HIP library.  The network
starts as Jacobi (zero decoder).
"""
from __future__ import annotations

import time

import numpy as np

from . import spai as S
from .solver import Solver, _torch


def collect_pairs(A, b, K=4, m=30):
    """K restart residuals (float32, K x n, on the GPU) of plain GMRES(m) on A x = b."""
    torch = _torch()
    s = Solver(A.row_ptr, A.col_idx, A.vals, m=m, tol=0.0, ortho="cgsr", precision="fp32", max_iters=m,
               autotune=False, use_graph=False)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    Z = torch.empty((K, A.n), dtype=torch.float32, device="cuda")
    for k in range(K):
        r, nrm = s.residual(b, x)
        if not nrm > 0.0:
            raise ValueError("zero residual: the system is already solved")
        Z[k] = (r / nrm).to(torch.float32)
        if k + 1 < K:
            x, _ = s.solve(b, x0=x)
    s.close()
    return Z


def make_instances(ids, N, generator=None):
    """(A, b) for each instance index of the variable-coefficient family."""
    import problems as P

    out = []
    for i in ids:
        pr = P.c5_varcoef(i, N=N)
        out.append((pr.A, pr.b))
    return out


def train(train_ids, N=64, steps=100, lr=3e-3, seed=0, pairs_per_instance=4, batch=1, log=None,
          instances=None):
    """Adam on the residual loss over the training instances (cycled in order)."""
    torch = _torch()
    t0 = time.perf_counter()
    inst = instances if instances is not None else make_instances(train_ids, N)
    A0 = inst[0][0]
    net = S.SpaiNet(A0.row_ptr, A0.col_idx, kmax=pairs_per_instance)
    vals, pairs = [], []
    for A, b in inst:
        if A.nnz != A0.nnz or not np.array_equal(A.col_idx, A0.col_idx):
            raise ValueError("training instances must share one sparsity pattern")
        vals.append(torch.as_tensor(A.vals, device="cuda"))
        pairs.append(collect_pairs(A, b, K=pairs_per_instance))
    t_data = time.perf_counter() - t0
    opt = S.Adam(S.init_params(seed), lr=lr)
    grad = torch.zeros(S.NPARAMS, dtype=torch.float32, device="cuda")
    hist = []
    t1 = time.perf_counter()
    for step in range(steps):
        Ls = []
        for q in range(batch):
            k = (step * batch + q) % len(inst)
            net.set_values(vals[k])
            M = net.forward(opt.params)
            L, dm = net.loss(M, pairs[k])
            net.backward(opt.params, dm, grad=grad, accumulate=q > 0)
            Ls.append(L)
        opt.step(grad, scale=1.0 / batch)
        hist.append(float(np.mean(Ls)))
        if log and (step % max(1, steps // 10) == 0 or step == steps - 1):
            log(f"  step {step:5d} loss {hist[-1]:.5f}")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    # loss of the final parameters over all instances, and of the Jacobi start
    def mean_loss(params):
        out = []
        for k in range(len(inst)):
            net.set_values(vals[k])
            out.append(net.loss(net.forward(params), pairs[k], grad=False)[0])
        return float(np.mean(out))

    jac = torch.as_tensor(S.params_to_bf16(S.init_params(seed)), device="cuda")
    res = {"params": opt.params.clone(), "theta": opt.theta.clone(), "history": hist,
           "loss_first": mean_loss(jac), "loss_last": mean_loss(opt.params),
           "seconds_data": t_data, "seconds_train": t_train, "steps": steps, "batch": batch,
           "instances": len(inst)}
    net.close()
    return res


def evaluate(params, test_ids, N=64, m=30, tol=1e-10, ortho="cgsr", instances=None, max_iters=100_000):
    """Iterations and time to tol for none / Jacobi / learned right preconditioning."""
    torch = _torch()
    inst = instances if instances is not None else make_instances(test_ids, N)
    out = []
    for idx, (A, b) in zip(test_ids, inst):
        row = {"instance": idx}
        for kind in ("none", "jacobi", "learned"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s = Solver(A.row_ptr, A.col_idx, A.vals, m=m, tol=tol, ortho=ortho, precision="fp32",
                       precond="spai" if kind == "learned" else kind, max_iters=max_iters)
            if kind == "learned":
                s.spai_infer(params)
            x, info = s.solve(b)
            torch.cuda.synchronize()
            info["seconds_total"] = time.perf_counter() - t0
            s.close()
            row[kind] = info
        out.append(row)
    return out
