"""Learned correction of the block-Jacobi preconditioner (thin layer over the C ABI).

The network maps the 99 features of a tile (bem_precond_features) to U, V (64 x 8) with
M_b^{-1} = D_b^{-1} + s_b U V^T.  It is trained on the device by the library's kernels
(bem_mlp_loss_grad, bem_mlp_adam) on targets the solver generates itself
(bem_precond_targets: block least-squares approximate inverses from the near field), and installed with a fallback to plain
block-Jacobi decided by the true operator's GMRES residual (bem_precond_select).
"""
from __future__ import annotations

import numpy as np
import torch

from . import _bem as C

FEATURES = 99


def _stream():
    return torch.cuda.current_stream().cuda_stream


class CorrectionNet:
    def __init__(self, cplx: bool, hidden: int = 256, seed: int = 1906, precision: int = 1):
        self.cplx = bool(cplx)
        self.hidden = hidden
        self.out = (4 if cplx else 2) * 64 * 8
        self.precision = precision
        self.nparams, _ = C.bem_mlp_sizes(FEATURES, hidden, self.out, 1)
        dev = torch.device("cuda", torch.cuda.current_device())
        self.params = torch.empty(self.nparams, dtype=torch.float32, device=dev)
        C.bem_mlp_init(FEATURES, hidden, self.out, seed, self.params.data_ptr(), _stream())
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss_dev = torch.zeros(1, dtype=torch.float32, device=dev)
        self.step = 0
        self._ws = {}

    def _workspace(self, batch: int):
        if batch not in self._ws:
            _, nbytes = C.bem_mlp_sizes(FEATURES, self.hidden, self.out, batch)
            self._ws[batch] = (torch.empty(nbytes, dtype=torch.uint8, device=self.params.device), nbytes)
        return self._ws[batch]

    def forward(self, X: torch.Tensor, precision: int | None = None) -> torch.Tensor:
        X = X.contiguous()
        Y = torch.empty((X.shape[0], self.out), dtype=torch.float32, device=X.device)
        ws, nb = self._workspace(X.shape[0])
        C.bem_mlp_forward(FEATURES, self.hidden, self.out, X.shape[0], self.params.data_ptr(), X.data_ptr(),
                          Y.data_ptr(), self.precision if precision is None else precision, ws.data_ptr(), nb,
                          _stream())
        return Y

    def loss_grad(self, X: torch.Tensor, T: torch.Tensor, precision: int | None = None):
        X, T = X.contiguous(), T.contiguous()
        ws, nb = self._workspace(X.shape[0])
        C.bem_mlp_loss_grad(FEATURES, self.hidden, self.out, X.shape[0], int(self.cplx), self.params.data_ptr(),
                            X.data_ptr(), T.data_ptr(), self.grad.data_ptr(), self.loss_dev.data_ptr(),
                            self.precision if precision is None else precision, ws.data_ptr(), nb, _stream())
        return float(self.loss_dev.item()), self.grad

    def adam_step(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        C.bem_mlp_adam(self.nparams, self.params.data_ptr(), self.grad.data_ptr(), self.m.data_ptr(),
                       self.v.data_ptr(), self.step, lr, beta1, beta2, eps, _stream())

    def train(self, X: torch.Tensor, T: torch.Tensor, steps: int, batch: int = 128, lr: float = 1e-3,
              seed: int = 0) -> list[float]:
        """Adam on minibatches drawn (seeded) from (X, T); returns the loss of every step."""
        g = np.random.default_rng([1906, 90, seed])
        n = X.shape[0]
        batch = min(batch, n)
        losses = []
        for _ in range(steps):
            idx = torch.from_numpy(g.choice(n, batch, replace=False)).to(X.device)
            loss, _ = self.loss_grad(X[idx], T[idx])
            self.adam_step(lr)
            losses.append(loss)
        return losses


def training_data(op, ring: int = 2):
    """Features and targets of every tile of an operator (its preconditioner built)."""
    return op.precond_features(), op.precond_targets(ring=ring)


def install(op, net: CorrectionNet, b: torch.Tensor, restart: int = 30):
    """Predict the correction of every tile of `op`, keep it only if one GMRES(restart)
    cycle on b does better than plain block-Jacobi.  Returns (kept, (relres plain, learned))."""
    uv = net.forward(op.precond_features())
    nbytes = C.bem_solve_plan(op.h, 1, restart, restart, 1e-8) + op.ndof * 16 + 1024
    ws = torch.empty(nbytes, dtype=torch.uint8, device=uv.device)
    bb = b.reshape(-1).contiguous()
    return C.bem_precond_select(op.h, uv.data_ptr(), bb.data_ptr(), restart, ws.data_ptr(), nbytes, _stream())
