"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds workload parameters and random draws only; it contains none
of the spectral-element arithmetic (no GLL points, no derivative matrix, no
geometry, no gather-scatter), so that both the HIP path and the CPU oracle can
take their inputs from it without sharing method code.

All random draws use numpy ``Generator(PCG64(seed))``.  Seeds: 0 = operand u,
1 = right-hand side, 2 and 3 = the two Gaussian-random-field draws,
11 and 21 = the second and third velocity components' right-hand sides,
31.. = the fixed patterns and 131.. = the per-step noise of a load sequence.

The paper's own workloads (Taylor-Green vortex, pipe, hemisphere meshes and DNS
data) are not available; these box meshes stand in for them with the same
element counts and polynomial orders (64^3 x lx=8 like the TGV verification
mesh, 32^3 x lx=8 close to the 36,480-element pipe, Re = 5000 and dt = 5e-4 of
the scaled-up TGV run).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int            # elements per direction (box of nx^3 hexahedra on [0,1]^3)
    lx: int            # GLL points per direction (polynomial order N = lx-1)
    eps: float         # amplitude of the smooth sine deformation (0: affine)
    h1: object         # "one", a float, or "grf" (h1 = exp(g), g a Gaussian random field)
    h2: float          # mass coefficient (1/dt for the Helmholtz cases)
    rhs: str           # "sine" (manufactured), "uniform" (U[-1,1] load vector)
    rtol: float        # relative residual target (<= 0: fixed iteration count)
    iters: int = 0     # fixed iteration count when rtol <= 0
    nfields: int = 1
    mixed: bool = False
    note: str = ""

    @property
    def nelv(self):
        return self.nx ** 3

    @property
    def n_local(self):
        return self.nelv * self.lx ** 3

    @property
    def n_unique(self):
        return (self.nx * (self.lx - 1) + 1) ** 3


WORKLOADS = {
    "poisson_4x4x4_lx6": Workload(
        "poisson_4x4x4_lx6", 4, 6, 0.0, "one", 0.0, "sine", 0.0, iters=50,
        note="64 affine elements, N=5; ax_helm + gs_op on U[-1,1], 50 Jacobi-PCG steps"),
    "poisson_32x32x32_lx8": Workload(
        "poisson_32x32x32_lx8", 32, 8, 0.05, "one", 0.0, "uniform", 1e-10,
        note="32^3 curved elements, N=7, 16.8M local points; FP64 and mixed solves to 1e-10"),
    "helmholtz_grf_16x16x16_lx8": Workload(
        "helmholtz_grf_16x16x16_lx8", 16, 8, 0.05, "grf", 1000.0, "sine", 1e-12,
        note="variable h1 = exp(GRF), h2 = 1/dt, dt = 1e-3; adjoint gradient vs FD; forward and adjoint "
             "solves to 1e-12, the tightest tolerance an FP64 true residual certifies on this mesh and load "
             "(its rounding floor is ~2e-13)"),
    "poisson_64x64x64_lx8_mixed": Workload(
        "poisson_64x64x64_lx8_mixed", 64, 8, 0.05, "one", 0.0, "sine", 1e-10, mixed=True,
        note="64^3 curved elements, 134M local points; FP32 operator inside FP64 flexible CG"),
    "velocity3_48x48x48_lx12": Workload(
        "velocity3_48x48x48_lx12", 48, 12, 0.05, 1.0 / 5000.0, 1.0 / 5e-4, "uniform", 1e-10,
        nfields=3, mixed=True,
        note="48^3 curved elements, N=11, three velocity Helmholtz solves, Re=5000, dt=5e-4"),
}

# seeds
SEED_U, SEED_RHS, SEED_GRF, SEED_GRF_TARGET = 0, 1, 2, 3
SEED_RHS_FIELDS = (1, 11, 21)
SEED_SEQ, SEED_SEQ_NOISE = 31, 131


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """n draws of U[-1, 1) from PCG64(seed), as FP64 (cast afterwards if asked)."""
    return rng(seed).uniform(-1.0, 1.0, n).astype(dtype, copy=False)


@dataclass(frozen=True)
class GRF:
    """Random-Fourier-feature Gaussian random field
    g(x) = sigma * sqrt(2/M) * sum_m cos(omega_m . x + phi_m),
    omega_m ~ N(0, ell^-2 I), phi_m ~ U[0, 2 pi): a stationary field with unit
    Gaussian correlation of length ell and standard deviation sigma."""
    omega: np.ndarray = field(repr=False)
    phi: np.ndarray = field(repr=False)
    sigma: float = 0.5

    def __call__(self, x, y, z):
        """Field values at the points (x, y, z) (numpy arrays of one shape), FP64.
        Evaluated with torch CPU tensors in chunks of points (all host threads)."""
        import torch

        x = np.asarray(x, np.float64)
        pts = torch.from_numpy(np.stack([x.reshape(-1), np.asarray(y, np.float64).reshape(-1),
                                         np.asarray(z, np.float64).reshape(-1)], axis=1))
        om = torch.from_numpy(np.ascontiguousarray(self.omega.T))      # (3, M)
        ph = torch.from_numpy(self.phi)                                # (M,)
        out = torch.empty(pts.shape[0], dtype=torch.float64)
        chunk = 1 << 15
        for a in range(0, pts.shape[0], chunk):
            out[a:a + chunk] = torch.cos(torch.addmm(ph, pts[a:a + chunk], om)).sum(dim=1)
        amp = self.sigma * math.sqrt(2.0 / len(self.phi))
        return (amp * out.numpy()).reshape(x.shape)


def grf(seed: int, sigma: float = 0.5, ell: float = 0.2, M: int = 512) -> GRF:
    r = rng(seed)
    omega = r.normal(0.0, 1.0 / ell, size=(M, 3))
    phi = r.uniform(0.0, 2.0 * math.pi, size=M)
    return GRF(omega, phi, sigma)


def sine_source(x, y, z):
    """f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z): -lap of the manufactured solution
    u* = sin(pi x) sin(pi y) sin(pi z) (the Poisson problem of Eq. 4-5)."""
    return 3.0 * math.pi ** 2 * np.sin(math.pi * x) * np.sin(math.pi * y) * np.sin(math.pi * z)


def sine_exact(x, y, z):
    return np.sin(math.pi * x) * np.sin(math.pi * y) * np.sin(math.pi * z)


def sequence_load(n: int, k: int, modes: int = 4, dt: float = 0.05, noise: float = 1e-6) -> np.ndarray:
    """Local load vector of step k of a slowly varying sequence, standing in for the
    successive pressure right-hand sides of a time-stepping run: `modes` fixed U[-1,1]
    patterns (seeds SEED_SEQ + j) with amplitudes 1 + 0.5 cos(w_j k dt + j), plus U[-1,1]
    noise of size `noise` drawn afresh each step (seed SEED_SEQ_NOISE + k)."""
    omega = (1.0, 1.7, 2.3, 3.1, 3.7, 4.3, 5.1, 5.9)
    f = np.zeros(n)
    for j in range(modes):
        f += (1.0 + 0.5 * math.cos(omega[j % len(omega)] * k * dt + j)) * uniform(n, SEED_SEQ + j)
    if noise:
        f += noise * uniform(n, SEED_SEQ_NOISE + k)
    return f
