"""Training and evaluation of the learned sparse approximate inverse.

The training data are residuals that the solver itself produces: for each
training matrix, the restart residuals z_k = b - A x_k of a few cycles of
unpreconditioned mixed-precision GMRES(m) (x_0 = 0, so z_0 = b).  The loss
is L = mean_k ||A M z_k - z_k||^2 / ||z_k||^2 (spai.h); forward, loss,
backward and the Adam update all run in the HIP library.  The network
starts as Jacobi (zero decoder).  Matrices of one family share a sparsity
pattern, so one network instance serves them all and only the values
change between steps.
"""
from __future__ import annotations

import os
import time
from dataclasses import dataclass, field

import numpy as np

from . import spai as S
from .solver import Solver, _torch


def collect_pairs(row_ptr, col_idx, vals, b, K=4, m=30):
    """K restart residuals (float32, K x n, unit norm, on the GPU) of plain GMRES(m)."""
    torch = _torch()
    s = Solver(row_ptr, col_idx, vals, m=m, tol=0.0, ortho="cgsr", precision="fp32", max_iters=m,
               autotune=False, use_graph=False)
    x = torch.zeros(s.n, dtype=torch.float64, device="cuda")
    Z = torch.empty((K, s.n), dtype=torch.float32, device="cuda")
    for k in range(K):
        try:
            s.residual_unit(b, x, out=Z[k])
        except Exception as e:
            raise ValueError("zero or non-finite residual: the system is already solved or broken") from e
        if k + 1 < K:
            x, _ = s.solve(b, x0=x)
    s.close()
    return Z


@dataclass
class TrainingData:
    row_ptr: object = None      # device int32
    col_idx: object = None      # device int32
    vals: list = field(default_factory=list)   # device float64 per instance
    pairs: list = field(default_factory=list)  # device float32 K x n per instance
    seconds: float = 0.0


def prepare(instances, K=4, m=30, log=None):
    """GPU-resident training data from an iterable of (A, b) sharing one pattern."""
    torch = _torch()
    t0 = time.perf_counter()
    d = TrainingData()
    ci_host = None
    for q, (A, b) in enumerate(instances):
        if d.row_ptr is None:
            d.row_ptr = torch.as_tensor(A.row_ptr, dtype=torch.int32, device="cuda")
            d.col_idx = torch.as_tensor(A.col_idx, dtype=torch.int32, device="cuda")
            ci_host = np.asarray(A.col_idx)
        elif A.nnz != ci_host.size or not np.array_equal(A.col_idx, ci_host):
            raise ValueError("training instances must share one sparsity pattern")
        v = torch.as_tensor(A.vals, dtype=torch.float64, device="cuda")
        bt = torch.as_tensor(b, dtype=torch.float64, device="cuda")
        d.vals.append(v)
        d.pairs.append(collect_pairs(d.row_ptr, d.col_idx, v, bt, K=K, m=m))
        if log and (q + 1) % 200 == 0:
            log(f"  prepared {q + 1} instances ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    d.seconds = time.perf_counter() - t0
    return d


def save_checkpoint(path, opt, step, hist, seed, ninst, batch):
    """The training state after `step` steps (NumPy .npz, arrays only)."""
    st = opt.state_dict()
    tmp = path + ".tmp.npz"
    np.savez(tmp, theta=st["theta"], m1=st["m1"], m2=st["m2"],
             scalars=np.array([st["t"], st["lr"], st["beta1"], st["beta2"], st["eps"]], dtype=np.float64),
             step=np.array(step, dtype=np.int64), seed=np.array(seed, dtype=np.int64),
             ninst=np.array(ninst, dtype=np.int64), batch=np.array(batch, dtype=np.int64),
             history=np.asarray(hist, dtype=np.float64))
    os.replace(tmp, path)


def load_checkpoint(path):
    with np.load(path, allow_pickle=False) as z:
        sc = z["scalars"]
        return {"opt": {"theta": z["theta"], "m1": z["m1"], "m2": z["m2"], "t": int(sc[0]), "lr": float(sc[1]),
                        "beta1": float(sc[2]), "beta2": float(sc[3]), "eps": float(sc[4])},
                "step": int(z["step"]), "seed": int(z["seed"]), "ninst": int(z["ninst"]), "batch": int(z["batch"]),
                "history": [float(v) for v in z["history"]]}


def train_on(data: TrainingData, epochs=1.0, lr=1e-3, batch=4, seed=0, log=None, checkpoint=None,
             checkpoint_every=0, stop_after=None):
    """Adam on the residual loss, instances cycled in a seeded shuffled order.

    checkpoint: a file path.  When it exists, training resumes from it (the
    same data, seed and batch are required); every `checkpoint_every` steps
    and at the end the state is written to it.  stop_after: end after that
    many steps in total (an interrupted run, for resuming later)."""
    torch = _torch()
    ninst = len(data.vals)
    K = int(data.pairs[0].shape[0])
    net = S.SpaiNet(data.row_ptr, data.col_idx, kmax=K)
    opt = S.Adam(S.init_params(seed), lr=lr)
    grad = torch.zeros(S.NPARAMS, dtype=torch.float32, device="cuda")
    order = np.random.default_rng(seed).permutation(ninst)
    steps = max(1, int(round(epochs * ninst / batch)))
    hist = []
    first = 0
    if checkpoint and os.path.exists(checkpoint):
        ck = load_checkpoint(checkpoint)
        if (ck["seed"], ck["ninst"], ck["batch"]) != (seed, ninst, batch):
            raise ValueError("checkpoint was written for another seed, instance count or batch")
        opt.load_state_dict(ck["opt"])
        first, hist = ck["step"], ck["history"]
        if log:
            log(f"  resumed at step {first} from {checkpoint}")
    last = steps if stop_after is None else min(steps, int(stop_after))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for step in range(first, last):
        Ls = []
        for q in range(batch):
            k = int(order[(step * batch + q) % ninst])
            net.set_values(data.vals[k])
            M = net.forward(opt.params)
            L, dm = net.loss(M, data.pairs[k])
            net.backward(opt.params, dm, grad=grad, accumulate=q > 0)
            Ls.append(L)
        opt.step(grad, scale=1.0 / batch)
        hist.append(float(np.mean(Ls)))
        if log and (step % max(1, steps // 10) == 0 or step == steps - 1):
            log(f"  step {step:5d} loss {hist[-1]:.5f}")
        if checkpoint and checkpoint_every and (step + 1) % checkpoint_every == 0:
            save_checkpoint(checkpoint, opt, step + 1, hist, seed, ninst, batch)
    if checkpoint:
        save_checkpoint(checkpoint, opt, last, hist, seed, ninst, batch)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1

    def mean_loss(params):
        out = []
        for k in range(ninst):
            net.set_values(data.vals[k])
            out.append(net.loss(net.forward(params), data.pairs[k], grad=False)[0])
        return float(np.mean(out))

    jac = torch.as_tensor(S.params_to_bf16(S.init_params(seed)), device="cuda")
    res = {"params": opt.params.clone(), "theta": opt.theta.clone(), "history": hist,
           "loss_first": mean_loss(jac), "loss_last": mean_loss(opt.params),
           "seconds_data": data.seconds, "seconds_train": t_train, "steps": steps, "batch": batch,
           "instances": ninst, "seconds_per_instance_step": t_train / (max(1, last - first) * batch),
           "steps_done": last}
    net.close()
    return res


def make_instances(ids, N):
    """(A, b) for each instance index of the variable-coefficient family."""
    import problems as P

    for i in ids:
        pr = P.c5_varcoef(i, N=N)
        yield pr.A, pr.b


def train(train_ids, N=64, steps=100, lr=3e-3, seed=0, pairs_per_instance=4, batch=1, log=None):
    """Convenience wrapper: generate, prepare and train for a number of steps."""
    data = prepare(make_instances(train_ids, N), K=pairs_per_instance, log=log)
    return train_on(data, epochs=steps * batch / len(train_ids), lr=lr, batch=batch, seed=seed, log=log)


def solve_once(A, b, kind, params=None, m=30, tol=1e-10, ortho="cgsr", max_iters=100_000, net=None):
    """Time to tol including setup for one preconditioning kind:
    fp64 (no preconditioner), none, jacobi, ilu0 (4 sweeps), learned (float32 Arnoldi).
    For `learned`, `net` is an optional network instance shared by the
    family's sparsity pattern (else the solver builds its own)."""
    torch = _torch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prec = "fp64" if kind == "fp64" else "fp32"
    pc = {"fp64": "none", "none": "none", "jacobi": "jacobi", "learned": "spai", "ilu0": "ilu0"}[kind]
    s = Solver(A[0], A[1], A[2], m=m, tol=tol, ortho=ortho, precision=prec, precond=pc, max_iters=max_iters)
    if kind == "learned":
        s.spai_infer(params, net=net, return_m=False)
    x, info = s.solve(b)
    torch.cuda.synchronize()
    info["seconds_total"] = time.perf_counter() - t0
    s.close()
    return x, info


def evaluate(params, test_ids, N=64, m=30, tol=1e-10, ortho="cgsr", kinds=("none", "jacobi", "learned")):
    """Iterations and time to tol per instance and preconditioning kind."""
    torch = _torch()
    out = []
    net = None
    for idx, (A, b) in zip(test_ids, make_instances(test_ids, N)):
        dev = tuple(torch.as_tensor(v, device="cuda") for v in (A.row_ptr, A.col_idx, A.vals))
        bt = torch.as_tensor(b, device="cuda")
        if net is None:
            net = S.SpaiNet(dev[0], dev[1], kmax=1)
        row = {"instance": idx}
        for kind in kinds:
            _, row[kind] = solve_once(dev, bt, kind, params=params, m=m, tol=tol, ortho=ortho, net=net)
        out.append(row)
    if net is not None:
        net.close()
    return out
