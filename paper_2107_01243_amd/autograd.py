"""Differentiable Helmholtz solve: u(h1, b) = A(h1)^-1 b behind torch.autograd.

Forward: the Jacobi-PCG solve of libsem.  Backward (adjoint method, from the
h1-linearity of Eq. 9 of arXiv 2107.01243): with g_u = dL/du_L the incoming
local-layout gradient,
    lambda solves  mask QQ^T A_L lambda = mask QQ^T g_u     (A is symmetric)
    dL/dh1_p = -(D lambda)_p^T G_p (D u)_p                  (sem_ax_helm_adjoint)
    dL/db    = lambda / mult
Both solves and the contraction run in the HIP library.

b is an assembled load (equal copies on every shared point).  The solve reads its
unique-node value as the average of the copies, so the gradient with respect to the
local array b is lambda divided by the multiplicity; a load assembled as
b = mask QQ^T f then receives dL/df = mask QQ^T (lambda / mult) = lambda.

The Helmholtz coefficients live in the problem's coef handle (the paper's
ax_compute(w, u, coef, msh, Xh) interface keeps them there).  Forward and backward
set this call's h1 and h2 for their solves and restore what the handle held
before, so several live solves on one problem, and later solves that use the
handle's own coefficients, do not see each other's values.
"""
from __future__ import annotations

import contextlib

import torch

from . import sem


@contextlib.contextmanager
def _coefficients(coef: "sem.Coef", h1, h2):
    saved = coef.helmholtz()
    coef.set_helmholtz(h1, h2)
    try:
        yield
    finally:
        coef.set_helmholtz(*saved)


class HelmholtzSolve(torch.autograd.Function):
    """u = HelmholtzSolve.apply(h1, b, problem, h2, rtol) with h1 an FP64 local field
    and b an assembled, masked FP64 load; gradients flow to h1 and to b."""

    @staticmethod
    def forward(ctx, h1, b, problem: "sem.BoxProblem", h2=0.0, rtol=1e-12):
        h1d = h1.detach().contiguous()
        with _coefficients(problem.coef, h1d, h2):
            u, info = problem.solve(b.detach().contiguous(), rtol=rtol)
        ctx.problem, ctx.h2, ctx.rtol = problem, h2, rtol
        ctx.info = info
        ctx.save_for_backward(h1d, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        h1, u = ctx.saved_tensors
        P = ctx.problem
        with _coefficients(P.coef, h1, ctx.h2):
            rhs = P.assemble(grad_u.contiguous().to(torch.float64))
            lam, _ = P.solve(rhs, rtol=ctx.rtol)
            grad_h1 = P.adjoint(u, lam).neg_() if ctx.needs_input_grad[0] else None
        grad_b = lam / P.mult if ctx.needs_input_grad[1] else None
        return grad_h1, grad_b, None, None, None
