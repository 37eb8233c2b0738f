"""sem_pcg_solve_noalloc (the FP64 Jacobi-PCG solve on the library's fixed device
workspace) against sem_pcg_solve, through the C ABI: two calls in a row, the second on a
smaller problem, each giving the same iteration counts and the same solution bit for bit
as the allocating entry point (same kernels, same Jacobi inverse, same order of
operations); no device memory is taken by the calls; sizes beyond the workspace and
non-resident handles are refused before any launch."""
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import workloads  # noqa: E402
from paper_2107_01243_amd import sem  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(nx, lx, nfields, seed, h1=1.0, h2=0.0):
    P = sem.BoxProblem.build(nx, lx, 0.05)
    P.coef.set_helmholtz(h1, h2)
    f = torch.from_numpy(workloads.uniform(nfields * P.n, seed)).cuda()
    b = P.assemble(f, nfields=nfields)
    return P, b


@pytest.mark.timeout(120)
def test_noalloc_matches_pcg_solve_two_calls():
    cases = ((8, 8, 3, 1.0, 10.0), (4, 6, 1, 1.0, 0.0))  # the second call is smaller
    for nx, lx, nf, h1, h2 in cases:
        say(f"[noalloc] {nx}^3 elements, lx={lx}, {nf} field(s), h1={h1}, h2={h2}")
        P, b = _problem(nx, lx, nf, 1, h1, h2)
        assert P.n * nf <= sem.NOALLOC_MAX_POINTS
        x_ref, info_ref = P.solve(b, nfields=nf, rtol=1e-10, check_every=10)
        x = torch.full_like(b, float("nan"))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        info = sem.pcg_solve_noalloc(x, b, P.coef, P.msh, P.Xh, P.gs, nfields=nf, rtol=1e-10, check_every=10)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        for f in range(nf):
            say(f"   field {f}: {info[f]['iters']} it (allocating entry point {info_ref[f]['iters']}), "
                f"true residual {info[f]['true_rel_res']:.3e}")
            assert info[f]["iters"] == info_ref[f]["iters"]
            assert info[f]["converged"] == 1
            assert info[f]["true_rel_res"] == info_ref[f]["true_rel_res"]
        assert torch.equal(x, x_ref), float((x - x_ref).abs().max())
        # the workspace is held from the first call on; later calls take no memory
        if (nx, lx) != cases[0][:2]:
            assert free1 == free0, (free0, free1)
        del P, b, x, x_ref
        torch.cuda.empty_cache()


@pytest.mark.timeout(60)
def test_noalloc_refuses_oversize_and_nonresident():
    P = sem.BoxProblem.build(12, 8, 0.05)             # 884,736 points
    b3 = torch.zeros(3 * P.n, dtype=torch.float64, device="cuda")
    x3 = torch.zeros_like(b3)
    assert 3 * P.n > sem.NOALLOC_MAX_POINTS
    with pytest.raises(sem.SemError, match="exceeds the allocation-free workspace"):
        sem.pcg_solve_noalloc(x3, b3, P.coef, P.msh, P.Xh, P.gs, nfields=3)
    # a fresh gs handle has never been uploaded
    gs2 = sem.GS(P.msh)
    b = torch.zeros(P.n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(sem.SemError, match="not yet resident"):
        sem.pcg_solve_noalloc(x, b, P.coef, P.msh, P.Xh, gs2)
    # after an allocating call that uses it, the same handle is accepted
    gs2.op(torch.zeros_like(b))
    info = sem.pcg_solve_noalloc(x, b, P.coef, P.msh, P.Xh, gs2)
    assert info[0]["iters"] == 0 and info[0]["converged"] == 1
