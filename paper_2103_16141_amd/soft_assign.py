"""SoftAssignLoss: the soft spherical assignment loss as a torch.autograd.Function.

loss = -sum_i log sum_j exp(S_ij / tau), S = X C^T (X sparse CSR, C dense k x d).
Forward and backward both run in libsivf.so (sivf_soft_assign_fwd / _bwd).
The forward keeps only lse[N]; the backward recomputes S, so nothing of size
N x k is stored between the passes.  Gradients: dC dense (k x d), dX only on
X's nonzeros (a value tensor aligned with the CSR's col array).
"""
from __future__ import annotations

import torch

from .api import Context, DeviceCsr

_contexts = {}


def _context(device: torch.device) -> Context:
    key = (device.index if device.index is not None else 0, torch.cuda.current_stream(device).cuda_stream)
    ctx = _contexts.get(key)
    if ctx is None:
        ctx = Context(device)
        _contexts[key] = ctx
    return ctx


class SoftAssignLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, row_ptr, col, xval, C, tau, n_cols):
        if xval.dtype != torch.float32 or C.dtype != torch.float32:
            raise TypeError("SoftAssignLoss takes float32 values and centroids")
        lib = _context(C.device)
        X = DeviceCsr(row_ptr, col, xval.detach().contiguous(), int(n_cols))
        Cc = C.detach().contiguous()
        lse, loss = lib.soft_assign_fwd(X, Cc, float(tau))
        ctx.save_for_backward(row_ptr, col, X.val, Cc, lse)
        ctx.tau = float(tau)
        ctx.n_cols = int(n_cols)
        return torch.tensor(loss, dtype=torch.float32, device=C.device)

    @staticmethod
    def backward(ctx, grad_out):
        row_ptr, col, xval, C, lse = ctx.saved_tensors
        lib = _context(C.device)
        X = DeviceCsr(row_ptr, col, xval, ctx.n_cols)
        dC, dX = lib.soft_assign_bwd(X, C, ctx.tau, lse, float(grad_out),
                                     want_dc=ctx.needs_input_grad[3], want_dx=ctx.needs_input_grad[2])
        return None, None, dX, dC, None, None


def soft_assign_loss(X: DeviceCsr, C: torch.Tensor, tau: float = 0.05) -> torch.Tensor:
    return SoftAssignLoss.apply(X.row_ptr, X.col, X.val, C, tau, X.n_cols)
