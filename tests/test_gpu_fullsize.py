"""Opt-in full-size runs of the two largest workloads (set SEM_FULL_SIZE=1).

Tolerance of the oracle-recomputed true residual: the solvers stop on their own FP64
evaluation of |b - A x| / |b| <= rtol; an independent FP64 evaluation (the oracle's
operator: other summation order, no FMA) of the same residual differs by up to
~1.5e-11 relative at 134M points (measured), i.e. 15% of rtol = 1e-10, so these
checks use 1.2 * rtol.

Both need minutes of host time for the oracle's own setup (mesh, geometry and a
comparison sort of every local index by global id at 134M and 191M points), so
they are kept out of the default GPU suite; their results are recorded in the
design notes.  Each solution's true residual is recomputed by the oracle's own
FP64 operator.
"""
import os
import sys
import time

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

if os.environ.get("SEM_FULL_SIZE") != "1":
    pytest.skip("full-size runs are opt-in (SEM_FULL_SIZE=1)", allow_module_level=True)

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import workloads  # noqa: E402
from paper_2107_01243_amd import sem  # noqa: E402
from paper_2107_01243_amd import HelmholtzSolve  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def timed_solve(P, b, nfields=1, **kw):
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = sem.pcg_solve(x, b, P.coef, P.msh, P.Xh, P.gs, nfields=nfields, **kw)
    torch.cuda.synchronize()
    return x, info, time.perf_counter() - t0


def test_64cubed_lx8_mixed_vs_fp64():
    """64^3 curved elements, lx = 8 (134M local points), manufactured sine load:
    the mixed solve reaches the FP64 1e-10 residual faster than the FP64 solve."""
    wl = workloads.WORKLOADS["poisson_64x64x64_lx8_mixed"]
    say("[config 64^3] GPU setup")
    P = sem.BoxProblem.build(wl.nx, wl.lx, wl.eps, fp32=True)
    _, B = P.coef.export()
    xyz = P.xyz.view(3, -1)
    f = workloads.sine_source(xyz[0].cpu().numpy(), xyz[1].cpu().numpy(), xyz[2].cpu().numpy())
    b = P.assemble(torch.from_numpy(f).cuda() * B)
    del B, f
    P.xyz = None
    torch.cuda.empty_cache()
    timed_solve(P, b, rtol=1e-4, max_iter=50, raise_on_fail=False)       # warm-up
    x64, i64, t64 = timed_solve(P, b, rtol=wl.rtol, check_every=50)
    xm, im, tm = timed_solve(P, b, rtol=wl.rtol, mixed="reliable", check_every=10)
    xf, iff, tf = timed_solve(P, b, rtol=wl.rtol, mixed="fcg", inner_rtol=1e-4, inner_max_iter=20000,
                              check_every=50)
    say(f"   fp64: {t64:.3f}s {i64[0]['iters']} it; mixed (reliable updates): {tm:.3f}s "
        f"{im[0]['iters']} replacements / {im[0]['inner_iters']} it, speedup {t64 / tm:.2f}; "
        f"mixed (flexible CG): {tf:.3f}s {iff[0]['iters']} outer / {iff[0]['inner_iters']} inner")
    del xf
    assert tm < t64
    X64, XM = x64.cpu().numpy(), xm.cpu().numpy()
    del P, b, x64, xm
    torch.cuda.empty_cache()
    say("[config 64^3] oracle setup")
    O = oracle.Problem(wl.nx, wl.lx, wl.eps, progress=say)
    bo = O.assemble_rhs(O.B * workloads.sine_source(O.x, O.y, O.z))
    for X, info in ((X64, i64[0]), (XM, im[0])):
        tr = O.true_rel_res(X, bo)
        say(f"   oracle true residual {tr:.3e} (solver reported {info['true_rel_res']:.3e})")
        assert tr <= 1.2e-10
    err = np.abs(XM - X64).max() / np.abs(X64).max()
    say(f"   |x_mixed - x_fp64|_inf / |x_fp64|_inf = {err:.2e}")
    assert err <= 1e-5


def test_48cubed_lx12_three_fields_and_gradient():
    """48^3 curved elements, lx = 12 (191M local points per field): three velocity
    Helmholtz solves (h1 = 1/5000, h2 = 1/5e-4) in one batched mixed solve, then the
    h1-gradient of L = 0.5 |u_x - u_t|^2 through the adjoint, checked by central
    differences along a random direction."""
    wl = workloads.WORKLOADS["velocity3_48x48x48_lx12"]
    say("[config 48^3 lx12] GPU setup")
    P = sem.BoxProblem.build(wl.nx, wl.lx, wl.eps, fp32=True)
    P.xyz = None
    h1, h2 = wl.h1, wl.h2
    P.coef.set_helmholtz(h1, h2)
    n = P.n
    bl = np.concatenate([workloads.uniform(n, s) for s in workloads.SEED_RHS_FIELDS])
    b = P.assemble(torch.from_numpy(bl).cuda(), nfields=3)
    x3, info, t = timed_solve(P, b, nfields=3, rtol=wl.rtol, mixed="reliable", check_every=10)
    say(f"   batched mixed solve {t:.3f}s: " + ", ".join(f"{d['iters']}/{d['inner_iters']}" for d in info))
    X3 = x3.view(3, -1).cpu().numpy()
    # gradient on the x component, FP64 forward and adjoint solves
    bx = b[:n].clone()
    ut = (x3[:n] * 1.1).contiguous()
    mult = torch.from_numpy(P.gs.maps()[3].astype(np.float64)).cuda()
    del x3
    torch.cuda.empty_cache()

    def loss(hf):
        u = HelmholtzSolve.apply(hf, bx, P, h2, 1e-13)
        return 0.5 * torch.sum((u - ut) ** 2 / mult)

    hf = torch.full((n,), h1, dtype=torch.float64, device="cuda", requires_grad=True)
    L = loss(hf)
    L.backward()
    dh = torch.from_numpy(workloads.uniform(n, 13)).cuda() * h1
    eps = 1e-6
    with torch.no_grad():
        fd = (float(loss(hf.detach() + eps * dh)) - float(loss(hf.detach() - eps * dh))) / (2 * eps)
    an = float(torch.dot(hf.grad, dh))
    say(f"   gradient: fd {fd:.10e} adjoint {an:.10e}")
    assert abs(fd - an) <= 1e-6 * abs(an)
    del P, b, bx, ut, hf, mult, dh
    torch.cuda.empty_cache()
    say("[config 48^3 lx12] oracle setup")
    O = oracle.Problem(wl.nx, wl.lx, wl.eps, h1=h1, h2=h2, progress=say)
    for f in range(3):
        bo = O.assemble_rhs(bl[f * n:(f + 1) * n])
        tr = O.true_rel_res(X3[f], bo)
        say(f"   field {f}: oracle true residual {tr:.3e} (solver {info[f]['true_rel_res']:.3e})")
        assert tr <= 1.2e-10
