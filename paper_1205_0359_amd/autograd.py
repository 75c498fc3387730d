"""Differentiation form: a torch.autograd.Function around dsbcg_solve.

X_j = (sigma_j I + A)^{-1} B with A = D[U]^H D[U].  For a real loss L with
upstream gradients G_j = dL/dRe X_j + i dL/dIm X_j (PyTorch's convention for
complex tensors), the backward pass runs

  * one shifted block solve for the adjoints Lambda_j = (sigma_j + A)^{-1} G_j
    (dsbcg_solve_multi; sigma_j + A is hermitian, so the adjoint system is
    the forward system with new right-hand sides), and
  * the backward kernels of dsbcg_grad:
      dL/dB       = sum_j Lambda_j
      dL/dsigma_j = -Re <Lambda_j, X_j>
      dL/dU       = link-derivative stencil of -sum_j 2 Re <D Lambda_j, dD X_j>.

X_j is stored from the forward pass, or recomputed in the backward pass when
recompute=True (for when HBM is short).  All arithmetic runs in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from ._lib import DSBCG_FP64, Handle, dsbcg_grad, dsbcg_solve, dsbcg_solve_multi


class DSBCGSolve(torch.autograd.Function):
    """X = DSBCGSolve.apply(U, B, sigma, handle, kappa, tol, precision, recompute)."""

    @staticmethod
    def forward(ctx, U, B, sigma, handle: Handle, kappa: float, tol: float,
                precision: int = DSBCG_FP64, recompute: bool = False):
        sig = sigma.detach().to("cpu", torch.float64).numpy()
        X, _ = dsbcg_solve(handle, U.detach().contiguous(), kappa, B.detach().contiguous(), sig, tol,
                           precision=precision)
        ctx.handle, ctx.kappa, ctx.tol = handle, kappa, tol
        ctx.precision, ctx.recompute, ctx.sig = precision, recompute, sig
        if recompute:
            ctx.save_for_backward(U, B, sigma)
        else:
            ctx.save_for_backward(U, B, sigma, X)
        return X

    @staticmethod
    def backward(ctx, GX):
        if ctx.recompute:
            U, B, sigma = ctx.saved_tensors
            X, _ = dsbcg_solve(ctx.handle, U.detach().contiguous(), ctx.kappa, B.detach().contiguous(),
                               ctx.sig, ctx.tol, precision=ctx.precision)
        else:
            U, B, sigma, X = ctx.saved_tensors
        G = GX.contiguous()
        Lam, _ = dsbcg_solve_multi(ctx.handle, U.detach().contiguous(), ctx.kappa, G, ctx.sig, ctx.tol,
                                   precision=ctx.precision)
        need_U, need_B, need_sigma = ctx.needs_input_grad[:3]
        dU, dB, ds = dsbcg_grad(ctx.handle, U.detach().contiguous(), ctx.kappa, ctx.sig, X, Lam,
                                want_U=need_U, want_B=need_B, want_sigma=need_sigma)
        dsig = torch.from_numpy(np.asarray(ds)).to(sigma.dtype) if need_sigma else None
        return dU, dB, dsig, None, None, None, None, None


def solve(U, B, sigma, handle: Handle, kappa: float, tol: float = 1e-10,
          precision: int = DSBCG_FP64, recompute: bool = False):
    """Differentiable solve of (sigma_j I + D^H D) X_j = B; returns X (s, V, 4, 3, m)."""
    return DSBCGSolve.apply(U, B, sigma, handle, kappa, tol, precision, recompute)
