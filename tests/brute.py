"""Dense brute-force spectral-element matrices for tiny meshes (numpy only).

An independent derivation used to pin the oracle: it shares nothing with
``oracle/`` or with the HIP path.

* GLL points from numpy's Legendre-series roots of L_N'; weights from the
  moment equations sum_i w_i P_k(x_i) = int P_k (exact for k <= N).
* The derivative matrix from a Legendre-Vandermonde solve, D = V' V^-1.
* The element stiffness from the chain rule at every quadrature point,
  grad_x phi = J^-T grad_xi phi with numpy's 3x3 inverse, instead of the
  factored geometric tensor G.
* Assembly by a dense scatter on global ids; Dirichlet rows/columns dropped.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gll(lx):
    N = lx - 1
    cN = np.zeros(N + 1)
    cN[N] = 1.0
    inner = np.sort(npleg.legroots(npleg.legder(cN))) if N > 1 else np.array([])
    x = np.concatenate([[-1.0], np.real(inner), [1.0]])
    V = np.stack([npleg.legval(x, np.eye(N + 1)[k]) for k in range(N + 1)])  # V[k, i] = P_k(x_i)
    rhs = np.zeros(N + 1)
    rhs[0] = 2.0
    w = np.linalg.solve(V, rhs)
    return x, w


def dmat(x):
    n = len(x)
    V = np.stack([npleg.legval(x, np.eye(n)[k]) for k in range(n)], axis=1)        # V[i, k]
    Vd = np.stack([npleg.legval(x, npleg.legder(np.eye(n)[k])) for k in range(n)], axis=1)
    return Vd @ np.linalg.inv(V)


def box(nx, lx, eps):
    """Box mesh: element coordinates (nelv, lx^3, 3) and global ids (nelv, lx^3).

    Written with numpy broadcasting (point index q = i + lx*(j + lx*k))."""
    x, _ = gll(lx)
    N = lx - 1
    M = nx * N + 1
    E = nx ** 3
    ii, jj, kk = np.meshgrid(np.arange(lx), np.arange(lx), np.arange(lx), indexing="ij")
    ii, jj, kk = (a.transpose(2, 1, 0).reshape(-1) for a in (ii, jj, kk))  # i fastest
    xyz = np.zeros((E, lx ** 3, 3))
    gid = np.zeros((E, lx ** 3), np.int64)
    dirichlet = np.zeros((E, lx ** 3), bool)
    for e in range(E):
        ex, ey, ez = e % nx, (e // nx) % nx, e // (nx * nx)
        X = (ex + (x[ii] + 1) / 2) / nx
        Y = (ey + (x[jj] + 1) / 2) / nx
        Z = (ez + (x[kk] + 1) / 2) / nx
        s = lambda a: np.sin(2 * np.pi * a)
        xyz[e, :, 0] = X + eps * s(Y) * s(Z)
        xyz[e, :, 1] = Y + eps * s(Z) * s(X)
        xyz[e, :, 2] = Z + eps * s(X) * s(Y)
        gx, gy, gz = ex * N + ii, ey * N + jj, ez * N + kk
        gid[e] = gx + M * (gy + M * gz)
        dirichlet[e] = (gx == 0) | (gx == M - 1) | (gy == 0) | (gy == M - 1) | (gz == 0) | (gz == M - 1)
    return xyz, gid, dirichlet


def ref_ops(lx):
    x, w = gll(lx)
    D = dmat(x)
    I = np.eye(lx)
    Dr = np.kron(I, np.kron(I, D))    # acts on i (fastest)
    Ds = np.kron(I, np.kron(D, I))
    Dt = np.kron(D, np.kron(I, I))
    rho = np.kron(w, np.kron(w, w))
    return Dr, Ds, Dt, rho


def element_matrix(xyz_e, lx, h1=None, h2=None):
    """Dense A^e = sum_q rho_q |J_q| h1_q grad phi_m . grad phi_n + diag(h2 rho |J|)."""
    Dr, Ds, Dt, rho = ref_ops(lx)
    n = lx ** 3
    h1 = np.ones(n) if h1 is None else np.broadcast_to(h1, (n,))
    h2 = np.zeros(n) if h2 is None else np.broadcast_to(h2, (n,))
    # Jac[q, c, d] = d x_c / d r_d
    Jac = np.stack([np.stack([Dop @ xyz_e[:, c] for Dop in (Dr, Ds, Dt)], axis=-1)
                    for c in range(3)], axis=1)
    detJ = np.linalg.det(Jac)
    Jinv = np.linalg.inv(Jac)              # Jinv[q, d, c] = d r_d / d x_c
    gref = np.stack([Dr, Ds, Dt], axis=1)  # gref[q, d, m] = d phi_m / d r_d at q
    gphys = np.einsum("qdc,qdm->qcm", Jinv, gref)
    wq = rho * detJ * h1
    A = np.einsum("q,qcm,qcn->mn", wq, gphys, gphys)
    A += np.diag(h2 * rho * detJ)
    return A, detJ, rho * detJ


def assembled(nx, lx, eps, h1=None, h2=None):
    """Global dense matrix on unique free nodes plus the local->free map.

    h1, h2: None, scalar, or array (nelv, lx^3)."""
    xyz, gid, dirichlet = box(nx, lx, eps)
    E = nx ** 3
    ug = np.unique(gid)
    bnd = np.unique(gid[dirichlet])
    free = np.setdiff1d(ug, bnd)
    pos = -np.ones(ug.max() + 1, np.int64)
    pos[free] = np.arange(len(free))
    A = np.zeros((len(free), len(free)))
    for e in range(E):
        he1 = None if h1 is None else (h1[e] if np.ndim(h1) == 2 else h1)
        he2 = None if h2 is None else (h2[e] if np.ndim(h2) == 2 else h2)
        Ae, _, _ = element_matrix(xyz[e], lx, he1, he2)
        p = pos[gid[e]]
        keep = p >= 0
        A[np.ix_(p[keep], p[keep])] += Ae[np.ix_(keep, keep)]
    return A, pos, gid, xyz


def assembled_full(nx, lx, eps, h1=None, h2=None):
    """Global dense matrix on all unique nodes (no Dirichlet removal)."""
    xyz, gid, _ = box(nx, lx, eps)
    ug = np.unique(gid)
    pos = -np.ones(ug.max() + 1, np.int64)
    pos[ug] = np.arange(len(ug))
    A = np.zeros((len(ug), len(ug)))
    for e in range(nx ** 3):
        he1 = None if h1 is None else (h1[e] if np.ndim(h1) == 2 else h1)
        he2 = None if h2 is None else (h2[e] if np.ndim(h2) == 2 else h2)
        Ae, _, _ = element_matrix(xyz[e], lx, he1, he2)
        p = pos[gid[e]]
        A[np.ix_(p, p)] += Ae
    return A, pos, gid, xyz
