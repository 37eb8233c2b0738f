"""Differentiable Helmholtz solve: u(h1) = A(h1)^-1 b behind torch.autograd.

Forward: the Jacobi-PCG solve of libsem.  Backward (adjoint method, from the
h1-linearity of Eq. 9 of arXiv 2107.01243): with g_u = dL/du_L the incoming
local-layout gradient,
    lambda solves  mask QQ^T A_L lambda = mask QQ^T g_u     (A is symmetric)
    dL/dh1_p = -(D lambda)_p^T G_p (D u)_p                  (sem_ax_helm_adjoint)
Both solves and the contraction run in the HIP library.
"""
from __future__ import annotations

import torch

from . import sem


class HelmholtzSolve(torch.autograd.Function):
    """u = HelmholtzSolve.apply(h1, b, problem, h2, rtol) with h1 an FP64 local field."""

    @staticmethod
    def forward(ctx, h1, b, problem: "sem.BoxProblem", h2=0.0, rtol=1e-12):
        problem.coef.set_helmholtz(h1.detach().contiguous(), h2)
        u, info = problem.solve(b.detach().contiguous(), rtol=rtol)
        ctx.problem, ctx.h2, ctx.rtol = problem, h2, rtol
        ctx.info = info
        ctx.save_for_backward(h1.detach(), u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        h1, u = ctx.saved_tensors
        P = ctx.problem
        P.coef.set_helmholtz(h1.contiguous(), ctx.h2)
        rhs = P.assemble(grad_u.contiguous().to(torch.float64))
        lam, _ = P.solve(rhs, rtol=ctx.rtol)
        grad_h1 = P.adjoint(u, lam).neg_()
        return grad_h1, None, None, None, None
