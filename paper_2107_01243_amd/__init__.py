"""MI355X (gfx950) spectral-element Helmholtz hot path (arXiv 2107.01243, Neko).

Python surface over libsem.so: the operator ax_helm (Eq. 9), gather-scatter
gs_op (Eq. 10 / Algorithm 1), Jacobi-PCG with FP64 or FP32/FP64 mixed precision
(Section 4, Section 10), flexible GMRES with point-Jacobi or two-level additive
Schwarz preconditioning (the pressure solver of Section 4),
projection onto previous solutions (Section 4, Table 2), and the h1-adjoint behind
torch.autograd.
"""
from .sem import (RTOL_MARGIN, BoxProblem, Coef, GS, GmresParams, Mesh, PcgInfo, PcgParams, Projection, SemError,
                  Space,
                  ax_helm, ax_helm_adjoint, box_mesh, gmres_solve, jacobi_inverse, lib, mask, pcg_solve,
                  schwarz_apply, stream_triad)
from .autograd import HelmholtzSolve

__all__ = ["RTOL_MARGIN", "BoxProblem", "Coef", "GS", "GmresParams", "Mesh", "PcgInfo", "PcgParams", "Projection", "SemError",
           "Space", "ax_helm", "ax_helm_adjoint", "box_mesh", "gmres_solve", "jacobi_inverse", "lib", "mask",
           "pcg_solve", "schwarz_apply", "stream_triad", "HelmholtzSolve"]
