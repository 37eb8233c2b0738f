"""MI355X (gfx950) spectral-element Helmholtz hot path (arXiv 2107.01243, Neko).

Python surface over libsem.so: the operator ax_helm (Eq. 9), gather-scatter
gs_op (Eq. 10 / Algorithm 1), Jacobi-PCG and FP32/FP64 mixed flexible CG
(Section 4, Section 10), and the h1-adjoint behind torch.autograd.
"""
from .sem import (BoxProblem, Coef, GS, Mesh, PcgInfo, PcgParams, SemError, Space, ax_helm,
                  ax_helm_adjoint, box_mesh, jacobi_inverse, lib, mask, pcg_solve)
from .autograd import HelmholtzSolve

__all__ = ["BoxProblem", "Coef", "GS", "Mesh", "PcgInfo", "PcgParams", "SemError", "Space",
           "ax_helm", "ax_helm_adjoint", "box_mesh", "jacobi_inverse", "lib", "mask", "pcg_solve",
           "HelmholtzSolve"]
