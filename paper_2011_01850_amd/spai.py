"""Python front end of the learned sparse approximate inverse (include/spai.h).

Argument marshalling only: tensors live on the GPU (torch allocates them),
and every step (features, forward, loss, backward, optimiser) runs in the
HIP library.  Without a GPU or without the built library the constructors
raise; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L
from .solver import _dev, _torch

NPARAMS = L.SPAI_NPARAMS

# flat parameter layout (matrices row-major, output x input)
LAYOUT = [("Wn", (32, 3)), ("bn", (32,)), ("We", (32, 3)), ("be", (32,)),
          ("W1", (32, 96)), ("b1", (32,)), ("W2", (32, 96)), ("b2", (32,)),
          ("W3", (32, 96)), ("b3", (32,)), ("wo", (96,)), ("bo", (1,))]


def offsets():
    off, out = 0, {}
    for name, shape in LAYOUT:
        out[name] = (off, shape)
        off += int(np.prod(shape))
    assert off == NPARAMS
    return out


def init_params(seed: int) -> np.ndarray:
    """He-normal hidden weights, zero biases and a zero decoder, so the
    initial network is exactly Jacobi (float32 master weights)."""
    g = np.random.default_rng(seed)
    theta = np.zeros(NPARAMS, dtype=np.float32)
    for name, (o, shape) in offsets().items():
        if name.startswith("W"):
            size = int(np.prod(shape))
            theta[o:o + size] = g.normal(0.0, np.sqrt(2.0 / shape[1]), size)
    return theta


class SpaiNet:
    """Network instance for one sparsity pattern (CSR, no duplicate entries)."""

    def __init__(self, row_ptr, col_idx, kmax=8):
        torch = _torch()
        self._torch = torch
        self.lib = L.load()
        rp = _dev(row_ptr, torch.int32, torch)
        ci = _dev(col_idx, torch.int32, torch)
        self.n = int(rp.numel() - 1)
        self.nnz = int(ci.numel())
        self.kmax = int(kmax)
        h = C.c_void_p()
        torch.cuda.synchronize()
        L.check(self.lib.spai_create(C.byref(h), self.n, self.nnz, rp.data_ptr(), ci.data_ptr(), self.kmax, None),
                "spai_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.spai_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_values(self, vals):
        v = _dev(vals, self._torch.float64, self._torch)
        self._torch.cuda.synchronize()
        L.check(self.lib.spai_set_values(self.h, v.data_ptr()), "spai_set_values")

    def forward(self, params_bf16, out=None):
        torch = self._torch
        pb = _dev(params_bf16, torch.int16, torch)
        m = out if out is not None else torch.empty(self.nnz, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        L.check(self.lib.spai_forward(self.h, pb.data_ptr(), m.data_ptr()), "spai_forward")
        return m

    def loss(self, m_vals, Z, grad=True):
        """(L, dL/dM or None); Z: K x n float32 (one residual per row)."""
        torch = self._torch
        mv = _dev(m_vals, torch.float32, torch)
        Zt = _dev(Z, torch.float32, torch)
        K = int(Zt.shape[0]) if Zt.dim() == 2 else 1
        dm = torch.empty(self.nnz, dtype=torch.float32, device="cuda") if grad else None
        Lv = C.c_double()
        torch.cuda.synchronize()
        L.check(self.lib.spai_loss(self.h, mv.data_ptr(), Zt.data_ptr(), K, C.byref(Lv),
                                   dm.data_ptr() if grad else None), "spai_loss")
        return Lv.value, dm

    def backward(self, params_bf16, dm, grad=None, accumulate=False):
        torch = self._torch
        pb = _dev(params_bf16, torch.int16, torch)
        d = _dev(dm, torch.float32, torch)
        g = grad if grad is not None else torch.zeros(NPARAMS, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        L.check(self.lib.spai_backward(self.h, pb.data_ptr(), d.data_ptr(), g.data_ptr(), int(bool(accumulate))),
                "spai_backward")
        return g


class Adam:
    """Adam on float32 master weights with a bfloat16 copy for the network."""

    def __init__(self, theta0, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        torch = _torch()
        self._torch = torch
        self.lib = L.load()
        self.theta = _dev(theta0, torch.float32, torch).clone()
        self.m1 = torch.zeros_like(self.theta)
        self.m2 = torch.zeros_like(self.theta)
        self.params = torch.empty(NPARAMS, dtype=torch.int16, device="cuda")
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps
        self.t = 0
        # bfloat16 copy of the initial weights: a zero-gradient step with lr = 0
        zero = torch.zeros_like(self.theta)
        torch.cuda.synchronize()
        L.check(self.lib.spai_adam_step(NPARAMS, self.theta.data_ptr(), self.params.data_ptr(), zero.data_ptr(),
                                        1.0, zero.data_ptr(), zero.clone().data_ptr(), 0.0, beta1, beta2, eps, 1,
                                        None), "spai_adam_step")

    def state_dict(self):
        """Host copies of the optimiser state: float32 master weights, both
        moment estimates, the step count and the hyper-parameters."""
        return {"theta": self.theta.cpu().numpy(), "m1": self.m1.cpu().numpy(), "m2": self.m2.cpu().numpy(),
                "t": self.t, "lr": self.lr, "beta1": self.beta1, "beta2": self.beta2, "eps": self.eps}

    def load_state_dict(self, d):
        """Restore a state_dict (the bfloat16 copy is made again from the master weights)."""
        torch = self._torch
        for name in ("theta", "m1", "m2"):
            src = np.asarray(d[name], dtype=np.float32)
            if src.size != NPARAMS:
                raise ValueError(f"{name}: expected {NPARAMS} values")
            getattr(self, name).copy_(torch.as_tensor(src))
        self.t = int(d["t"])
        self.lr, self.beta1, self.beta2, self.eps = (float(d["lr"]), float(d["beta1"]), float(d["beta2"]),
                                                     float(d["eps"]))
        zero = torch.zeros_like(self.theta)
        torch.cuda.synchronize()
        L.check(self.lib.spai_adam_step(NPARAMS, self.theta.data_ptr(), self.params.data_ptr(), zero.data_ptr(),
                                        1.0, zero.data_ptr(), zero.clone().data_ptr(), 0.0, self.beta1, self.beta2,
                                        self.eps, 1, None), "spai_adam_step")

    def step(self, grad, scale=1.0, lr=None):
        self.t += 1
        self._torch.cuda.synchronize()
        L.check(self.lib.spai_adam_step(NPARAMS, self.theta.data_ptr(), self.params.data_ptr(), grad.data_ptr(),
                                        float(scale), self.m1.data_ptr(), self.m2.data_ptr(),
                                        float(self.lr if lr is None else lr), self.beta1, self.beta2, self.eps,
                                        self.t, None), "spai_adam_step")


def params_to_bf16(theta) -> np.ndarray:
    """float32 parameters -> bfloat16 bit patterns (round to nearest even), host side."""
    x = np.asarray(theta, dtype=np.float32).view(np.uint32).astype(np.uint64)
    x = (x + 0x7FFF + ((x >> 16) & 1)) >> 16
    return x.astype(np.uint16).view(np.int16)
