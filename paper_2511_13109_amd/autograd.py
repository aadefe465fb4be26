"""Differentiable AGCA solve: u = A(nu)^-1 b with the gradient taken by the adjoint.

The extension of the method to inverse problems: with A(nu) symmetric and each
element matrix linear in its own coefficient, the gradient of any scalar J(u)
with respect to log nu per finest element is

    dJ / dlog nu_e = -w_e^T A_e u_e,   A w = dJ/du,

so one extra solve with the same AGCA hierarchy (the adjoint solve) and one
per-element kernel (agca_grad_log_nu) give the whole gradient; dJ/db = w.
Every step runs in the library: the forward and adjoint solves, the
exponentiation of log nu, and the gradient kernel.
"""

from __future__ import annotations

from typing import Optional, Sequence

import torch

from .agca import Hierarchy


class AGCASolve(torch.autograd.Function):
    """u = AGCASolve.apply(log_nu, b, H, nu_coarse, tol, max_iter, solver).

    log_nu: (6 n_L^3,) float64 device tensor, log of the finest coefficient by element id;
    b: FP64 level vector of the finest level; H: a Hierarchy whose coefficient is
    replaced by exp(log_nu) (nu_coarse: the DCA coefficients of levels 0..L-1).
    Backward returns dJ/dlog nu and dJ/db = w.
    """

    @staticmethod
    def forward(ctx, log_nu, b, H: Hierarchy, nu_coarse: Sequence[torch.Tensor], tol: float = 1e-10,
                max_iter: int = 4000, solver: Optional[str] = None):
        H.set_log_nu(log_nu.detach().contiguous(), nu_coarse)
        slv = solver or ("pcg" if H.mg_dtype == 0 else "fcg")
        u, stats = H.solve(b.detach().contiguous(), solver=slv, tol=tol, max_iter=max_iter,
                           record_history=False, raise_on_noconv=True)
        ctx.H, ctx.nu_coarse, ctx.tol, ctx.max_iter, ctx.solver = H, list(nu_coarse), tol, max_iter, slv
        ctx.version = H.version
        ctx.stats = stats
        ctx.save_for_backward(log_nu.detach(), u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        log_nu, u = ctx.saved_tensors
        H = ctx.H
        if H.version != ctx.version:       # the hierarchy was rebuilt since the forward solve
            H.set_log_nu(log_nu.contiguous(), ctx.nu_coarse)
            ctx.version = H.version
        w, _ = H.solve(grad_u.contiguous(), solver=ctx.solver, tol=ctx.tol, max_iter=ctx.max_iter,
                       record_history=False, raise_on_noconv=True)
        g = H.grad_log_nu(u, w) if ctx.needs_input_grad[0] else None
        gb = w if ctx.needs_input_grad[1] else None
        return g, gb, None, None, None, None, None


def solve(log_nu: torch.Tensor, b: torch.Tensor, H: Hierarchy, nu_coarse: Sequence[torch.Tensor],
          tol: float = 1e-10, max_iter: int = 4000, solver: Optional[str] = None) -> torch.Tensor:
    """Differentiable solve (see AGCASolve)."""
    return AGCASolve.apply(log_nu, b, H, nu_coarse, tol, max_iter, solver)
