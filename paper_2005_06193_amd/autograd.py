"""Differentiable EGFEM solve: u* = S(f, kappa) with the implicit adjoint.

forward runs the Newton solve of F(u; d = M f, a0 = kappa) = 0 and keeps only
the converged u* (the checkpoint; no per-iteration trajectory).  backward
solves DF(u*)^T lambda = dJ/du on the GPU (egfem_adjoint) and returns
dJ/df = M lambda and dJ/dkappa = -(T ._2 u*)^T lambda.
"""
from __future__ import annotations

from typing import Optional

import torch

from .binding import NewtonOptions, Problem, Tensor, EgfemError


class EGFEMSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f: torch.Tensor, kappa: Optional[torch.Tensor], T: Tensor,
                template: Problem, opts: Optional[NewtonOptions] = None):
        opts = opts or NewtonOptions(tol=1e-13, krylov_rtol=1e-13)
        load = T.matvec(f.detach().contiguous(), "M")
        k = kappa.detach().contiguous() if kappa is not None else None
        p = Problem(T.n, load, template.dirichlet, k, template.a0_const, template.add_stiffness)
        u = torch.zeros_like(load)
        st = T.newton(p, u, opts)
        if st.status not in (0, 4):
            raise EgfemError(st.status, f"forward Newton solve ended with {st.status_name}")
        ctx.save_for_backward(u, k if k is not None else torch.empty(0, device=u.device))
        ctx.T = T
        ctx.template = template
        ctx.opts = opts
        ctx.has_kappa = kappa is not None
        ctx.forward_stats = st
        return u

    @staticmethod
    def backward(ctx, ubar: torch.Tensor):
        u, k = ctx.saved_tensors
        T, tpl = ctx.T, ctx.template
        p = Problem(T.n, None, tpl.dirichlet, k if ctx.has_kappa else None, tpl.a0_const,
                    tpl.add_stiffness)
        lam, ga, rc, its, rr = T.adjoint(p, u, ubar.contiguous(), ctx.opts,
                                         grad_a0=ctx.has_kappa and ctx.needs_input_grad[1])
        if rc != 0:
            raise EgfemError(rc, f"adjoint solve ended with status {rc} after {its} iterations")
        grad_f = T.matvec(lam, "M") if ctx.needs_input_grad[0] else None
        return grad_f, ga, None, None, None


def solve(f: torch.Tensor, kappa: Optional[torch.Tensor], T: Tensor, template: Problem,
          opts: Optional[NewtonOptions] = None) -> torch.Tensor:
    """u* = S(f, kappa); differentiable in f and kappa."""
    return EGFEMSolve.apply(f, kappa, T, template, opts)
