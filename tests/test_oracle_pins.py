"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle (``oracle/``) against something other than itself:
closed forms, quadrature exactness, integer counts, exact identities of the
discrete operator (Eq. 9-10), an independent dense numpy brute force
(``tests/brute.py``), the continuous PDE (spectral convergence), and finite
differences.  No GPU is needed.
"""
import json
import math
import os

import numpy as np
import pytest

import brute
import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _ev(s):
    return float(eval(s, {"sqrt": math.sqrt}))


def _cont(P, seed, zero_dirichlet=False):
    """A continuous local vector u_L = Q u_g with u_g ~ U[-1,1] per unique id."""
    ug = workloads.uniform(int(P.glb.max()) + 1, seed)
    u = ug[P.glb]
    if zero_dirichlet:
        u = np.where(P.dirichlet.astype(bool), 0.0, u)
    return u


# ------------------------------------------------------------------ GLL space (Eq. 7-8)
def test_gll_closed_forms():
    g = json.load(open(os.path.join(GOLD, "gll_closed_forms.json")))
    for rule in g["rules"]:
        xi, w = oracle.gll(rule["N"] + 1)
        np.testing.assert_allclose(xi, [_ev(s) for s in rule["points"]], rtol=0, atol=2e-16)
        np.testing.assert_allclose(w, [_ev(s) for s in rule["weights"]], rtol=0, atol=4e-16)


@pytest.mark.parametrize("lx", range(2, 17))
def test_gll_vs_numpy_moments(lx):
    xi, w = oracle.gll(lx)
    xb, wb = brute.gll(lx)
    np.testing.assert_allclose(xi, xb, rtol=0, atol=1e-14)
    np.testing.assert_allclose(w, wb, rtol=0, atol=1e-13)


@pytest.mark.parametrize("lx", [3, 5, 8, 12, 16])
def test_gll_exactness_degree(lx):
    """GLL with N+1 points integrates x^k exactly for k <= 2N-1 and not for k = 2N."""
    N = lx - 1
    xi, w = oracle.gll(lx)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13, k
    k = 2 * N
    assert abs(np.dot(w, xi ** k) - 2.0 / (k + 1)) > 1e-10


def test_dmat_closed_form_N2():
    g = json.load(open(os.path.join(GOLD, "gll_closed_forms.json")))["derivative_N2"]
    D = oracle.deriv_matrix(oracle.gll(3)[0])
    np.testing.assert_allclose(D, [[_ev(s) for s in row] for row in g["D"]], atol=1e-15)


@pytest.mark.parametrize("lx", range(2, 17))
def test_dmat_vs_vandermonde(lx):
    xi, _ = oracle.gll(lx)
    D = oracle.deriv_matrix(xi)
    Db = brute.dmat(brute.gll(lx)[0])
    assert np.abs(D - Db).max() <= 1e-11 * np.abs(Db).max()
    # exact derivative of x^k for k <= N; rows sum to zero
    for k in range(1, lx):
        np.testing.assert_allclose(D @ xi ** k, k * xi ** (k - 1), atol=1e-12 * lx ** 2)
    assert np.abs(D.sum(axis=1)).max() < 1e-12 * lx ** 2


# ------------------------------------------------------------------ mesh and numbering
def test_multiplicity_and_dirichlet_counts():
    cases = json.load(open(os.path.join(GOLD, "box_mesh_counts.json")))["cases"]
    for c in cases:
        m = oracle.box_mesh(c["nx"], c["nx"], c["nx"], c["lx"], 0.05)
        gs = oracle.GS(m["glb"])
        mult = gs.mult()
        for k in (1, 2, 4, 8):
            assert int(np.sum(mult == k)) == k * c[f"mult{k}"], (c, k)
        assert len(np.unique(m["glb"])) == c["unique"]
        assert len(np.unique(m["glb"][m["dirichlet"] == 1])) == c["dirichlet_unique"]
        off, idx, gid = gs.groups()
        assert np.all(np.diff(gid) > 0)
        del m, gs, mult


def test_shared_nodes_coincide_and_walls():
    m = oracle.box_mesh(3, 3, 3, 6, 0.05)
    gs = oracle.GS(m["glb"])
    off, idx, gid = gs.groups()
    for c in ("x", "y", "z"):
        a = m[c]
        for g in range(len(gid)):
            v = a[idx[off[g]:off[g + 1]]]
            assert np.all(v == v[0])
        # indices inside a group ascend
    assert all(np.all(np.diff(idx[off[g]:off[g + 1]]) > 0) for g in range(len(gid)))
    m0 = oracle.box_mesh(3, 3, 3, 6, 0.0)
    on_wall = np.zeros(len(m0["x"]), bool)
    for c in ("x", "y", "z"):
        on_wall |= (m0[c] == 0.0) | (m0[c] == 1.0)
    np.testing.assert_array_equal(on_wall, m0["dirichlet"].astype(bool))


def test_mesh_matches_brute():
    xyz, gid, dr = brute.box(2, 5, 0.05)
    m = oracle.box_mesh(2, 2, 2, 5, 0.05)
    np.testing.assert_array_equal(m["glb"], gid.reshape(-1))
    np.testing.assert_array_equal(m["dirichlet"].astype(bool), dr.reshape(-1))
    for c, name in enumerate("xyz"):
        np.testing.assert_allclose(m[name], xyz[:, :, c].reshape(-1), rtol=0, atol=1e-15)


# ------------------------------------------------------------------ geometry (Eq. 9 G^e)
@pytest.mark.parametrize("nx,lx", [(2, 4), (3, 6), (2, 8)])
def test_affine_geometry_closed_form(nx, lx):
    P = oracle.Problem(nx, lx, 0.0)
    h = 1.0 / nx
    rho = np.tile(np.kron(P.w, np.kron(P.w, P.w)), P.nelv)
    for f in range(3):
        np.testing.assert_allclose(P.G[f], rho * h / 2, rtol=1e-13)
    assert np.abs(P.G[3:]).max() < 1e-15
    np.testing.assert_allclose(P.B, rho * (h / 2) ** 3, rtol=1e-12)


@pytest.mark.parametrize("nx,lx,eps", [(2, 4, 0.0), (4, 6, 0.0), (2, 4, 0.05), (4, 6, 0.05), (2, 8, 0.05)])
def test_volume_is_one(nx, lx, eps):
    """The sine map has det = 1 + eps^2 (...) + eps^3 (...) whose correction terms
    all integrate to zero over the unit cube; GLL quadrature of the
    isoparametric map reproduces the volume 1."""
    P = oracle.Problem(nx, lx, eps)
    assert abs(P.B.sum() - 1.0) < (1e-14 if eps == 0 else 1e-10)


@pytest.mark.parametrize("nx,lx", [(2, 4), (3, 6), (2, 8)])
def test_coordinate_energy_identity_curved(nx, lx):
    """For u = x (the isoparametric coordinate, exact in the space):
    grad u = e_x at every quadrature point, so u^T A_L u = sum B and
    y^T A_L x = 0.  Pins the inverse metric and the G index order."""
    P = oracle.Problem(nx, lx, 0.05)
    X = {"x": P.x, "y": P.y, "z": P.z}
    vol = P.B.sum()
    for a in "xyz":
        Au = P.ax_local(X[a])
        for b in "xyz":
            val = np.dot(X[b], Au)
            if a == b:
                assert abs(val - vol) < 1e-12
            else:
                assert abs(val) < 1e-12


def test_geometry_vs_brute_element():
    P = oracle.Problem(2, 5, 0.05)
    xyz, _, _ = brute.box(2, 5, 0.05)
    for e in range(P.nelv):
        _, detJ, Bb = brute.element_matrix(xyz[e], 5)
        s = slice(e * 125, (e + 1) * 125)
        np.testing.assert_allclose(P.J[s], detJ, rtol=1e-12)
        np.testing.assert_allclose(P.B[s], Bb, rtol=1e-12)


# ------------------------------------------------------------------ ax_helm (Eq. 9)
@pytest.mark.parametrize("lx", [3, 6, 8, 12])
def test_constants_in_nullspace(lx):
    P = oracle.Problem(2, lx, 0.05)
    w = P.ax_local(np.ones(P.n))
    assert np.abs(w).max() < 1e-13 * np.abs(P.G).max() * lx ** 2


def test_symmetric_and_variable_coefficients():
    P = oracle.Problem(3, 6, 0.05)
    u = workloads.uniform(P.n, 0)
    v = workloads.uniform(P.n, 1)
    h1 = 1.0 + 0.5 * workloads.uniform(P.n, 2)
    h2 = 2.0 + workloads.uniform(P.n, 3)
    P.set_coef(h1, h2)
    a = np.dot(v, P.ax_local(u))
    b = np.dot(u, P.ax_local(v))
    assert abs(a - b) <= 1e-13 * abs(a)


def test_assembled_psd_with_constant_nullspace():
    P = oracle.Problem(2, 4, 0.05)
    ids, rep = np.unique(P.glb, return_index=True)
    ng = len(ids)
    pos = np.searchsorted(ids, P.glb)
    A = np.zeros((ng, ng))
    for j in range(ng):
        u = (pos == j).astype(np.float64)
        w = P.gs.op(P.ax_local(u))
        A[:, j] = w[rep]
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > -1e-13 * ev[-1]
    assert ev[1] > 1e-6 * ev[-1]            # exactly one zero mode: the constants
    assert abs(ev[0]) < 1e-12 * ev[-1]


def _poly_energy(a, b, c):
    """int_[0,1]^3 |grad x^a y^b z^c|^2."""
    def m(p):  # int_0^1 t^p
        return 1.0 / (p + 1)
    t = 0.0
    if a: t += a * a * m(2 * a - 2) * m(2 * b) * m(2 * c)
    if b: t += b * b * m(2 * a) * m(2 * b - 2) * m(2 * c)
    if c: t += c * c * m(2 * a) * m(2 * b) * m(2 * c - 2)
    return t


@pytest.mark.parametrize("lx", [4, 5, 8])
def test_energy_exact_on_affine(lx):
    """u^T A_L u = int |grad u|^2 exactly for u in Q_{N-1} on affine elements
    (GLL quadrature exact for degree 2N-1); fails for degree (N,1,0)."""
    N = lx - 1
    P = oracle.Problem(2, lx, 0.0)
    for (a, b, c) in [(N - 1, N - 1, N - 1), (1, 0, 0), (N - 1, 1, 0), (0, N - 1, 2), (N, 0, 0)]:
        u = P.x ** a * P.y ** b * P.z ** c
        e = np.dot(u, P.ax_local(u))
        assert abs(e - _poly_energy(a, b, c)) < 1e-12 * max(1.0, _poly_energy(a, b, c)), (a, b, c)
    if N <= 4:  # the degree-2N quadrature error is visible well above rounding
        u = P.x ** N * P.y
        e = np.dot(u, P.ax_local(u))
        assert abs(e - _poly_energy(N, 1, 0)) > 1e-8


def test_linear_function_interior_rows_vanish_affine():
    P = oracle.Problem(3, 6, 0.0)
    u = 2 * P.x - 3 * P.y + P.z + 0.5
    w = P.gs.op(P.ax_local(u))
    interior = P.dirichlet == 0
    assert np.abs(w[interior]).max() < 1e-13


@pytest.mark.parametrize("nx,lx", [(1, 6), (2, 3), (2, 4)])
def test_operator_vs_dense_brute_force(nx, lx):
    """Oracle's assembled, masked operator equals the numpy chain-rule stiffness
    matrix (curved mesh, variable h1 and h2), on the free unique nodes."""
    eps = 0.05
    P = oracle.Problem(nx, lx, eps)
    h1 = np.exp(0.3 * workloads.uniform(P.n, 5))
    h2 = 3.0 + workloads.uniform(P.n, 6)
    P.set_coef(h1, h2)
    A, pos, gid, _ = brute.assembled(nx, lx, eps, h1.reshape(P.nelv, -1), h2.reshape(P.nelv, -1))
    nf = A.shape[0]
    p_loc = pos[P.glb]
    Ao = np.zeros_like(A)
    rep = np.array([np.flatnonzero(p_loc == j)[0] for j in range(nf)])
    for j in range(nf):
        u = (p_loc == j).astype(np.float64)
        Ao[:, j] = P.apply(u)[rep]
    assert np.abs(Ao - A).max() <= 1e-12 * np.abs(A).max()


# ------------------------------------------------------------------ gather-scatter (Eq. 10)
def test_gs_identities():
    P = oracle.Problem(3, 5, 0.05)
    u = workloads.uniform(P.n, 7)
    g = P.gs.op(u)
    assert abs(np.sum(g / P.mult) - np.sum(u)) < 1e-11
    np.testing.assert_allclose(P.gs.op(g / P.mult), g, rtol=1e-14, atol=1e-14)
    np.testing.assert_array_equal(P.gs.op(np.ones(P.n)), P.mult)


def test_gs_equals_boolean_QQT():
    P = oracle.Problem(2, 4, 0.05)
    ids = np.unique(P.glb)
    Q = (P.glb[:, None] == ids[None, :]).astype(np.float64)   # scatter Q, n_L x n_g
    u = np.floor(workloads.uniform(P.n, 8) * 1000.0)          # integers: sums are exact
    np.testing.assert_array_equal(P.gs.op(u), Q @ (Q.T @ u))


# ------------------------------------------------------------------ Jacobi (Section 4)
def test_jacobi_diagonal_vs_dense():
    nx, lx, eps = 2, 4, 0.05
    P = oracle.Problem(nx, lx, eps)
    h1 = np.exp(0.3 * workloads.uniform(P.n, 5))
    h2 = 3.0 + workloads.uniform(P.n, 6)
    P.set_coef(h1, h2)
    A, pos, _, _ = brute.assembled(nx, lx, eps, h1.reshape(P.nelv, -1), h2.reshape(P.nelv, -1))
    p_loc = pos[P.glb]
    d = P.gs.op(P.diag_local())
    free = p_loc >= 0
    np.testing.assert_allclose(d[free], np.diag(A)[p_loc[free]], rtol=1e-13)
    np.testing.assert_allclose(P.dinv[free], 1.0 / np.diag(A)[p_loc[free]], rtol=1e-13)
    assert np.all(P.dinv[~free] == 0.0)


# ------------------------------------------------------------------ PCG (Section 4)
def test_pcg_config1_matches_dense_solve():
    """64 affine elements, lx=6: 50 Jacobi-PCG steps on the manufactured sine
    load reproduce the dense solve, and the discrete solution is within the
    spectral discretisation error of u* = sin sin sin."""
    wl = workloads.WORKLOADS["poisson_4x4x4_lx6"]
    P = oracle.Problem(wl.nx, wl.lx, wl.eps)
    f = workloads.sine_source(P.x, P.y, P.z)
    b = P.assemble_rhs(P.B * f)
    x, info = P.pcg(b, rtol=0.0, max_iter=wl.iters)
    assert info["iters"] == 50 and info["rel_res"] < 1e-14
    A, pos, _, _ = brute.assembled(wl.nx, wl.lx, wl.eps)
    p_loc = pos[P.glb]
    free = p_loc >= 0
    rep = np.array([np.flatnonzero(p_loc == j)[0] for j in range(A.shape[0])])
    xd = np.linalg.solve(A, b[rep])
    np.testing.assert_allclose(x[free], xd[p_loc[free]], rtol=0, atol=1e-12 * np.abs(xd).max())
    assert np.abs(x - workloads.sine_exact(P.x, P.y, P.z)).max() < 1e-7


def test_spectral_convergence():
    """Manufactured Poisson solution on 2^3 affine elements: the max nodal error
    falls geometrically with N (Eq. 7-9 discretisation of Eq. 4-6)."""
    errs = []
    for lx in range(3, 10):
        P = oracle.Problem(2, lx, 0.0)
        b = P.assemble_rhs(P.B * workloads.sine_source(P.x, P.y, P.z))
        x, info = P.pcg(b, rtol=1e-14)
        assert info["status"] == 0
        errs.append(np.abs(x - workloads.sine_exact(P.x, P.y, P.z)).max())
    errs = np.array(errs)
    assert np.all(errs[1:] < 0.25 * errs[:-1]), errs
    assert errs[-1] < 1e-7


def test_pcg_roundtrip_curved_variable():
    P = oracle.Problem(3, 6, 0.05, h1=1.0, h2=10.0)
    u = _cont(P, 9, zero_dirichlet=True)
    b = P.apply(u)
    x, info = P.pcg(b, rtol=1e-13)
    assert info["status"] == 0
    assert np.abs(x - u).max() < 1e-9
    assert P.true_rel_res(x, b) < 2e-13


def test_pcg_status_codes():
    P = oracle.Problem(2, 5, 0.05)
    b = P.assemble_rhs(workloads.uniform(P.n, 1))
    _, info = P.pcg(b, rtol=1e-12, max_iter=3)
    assert info["status"] == 1 and info["iters"] == 3
    x, info = P.pcg(np.zeros(P.n), rtol=1e-10)
    assert info["status"] == 0 and info["iters"] == 0 and not x.any()


# ------------------------------------------------------------------ adjoint / gradient
def test_adjoint_euler_identity():
    """sum_p h1_p g_p(v, u) = v^T A_L(h1) u for h2 = 0 (Eq. 9 is linear in h1)."""
    P = oracle.Problem(3, 8, 0.05)
    h1 = np.exp(0.5 * workloads.uniform(P.n, 4))
    P.set_coef(h1, 0.0)
    u = workloads.uniform(P.n, 0)
    v = workloads.uniform(P.n, 1)
    g = P.adjoint(u, v)
    lhs = np.dot(h1, g)
    rhs = np.dot(v, P.ax_local(u))
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs)
    # the adjoint is symmetric in (u, v) and g(u, u) >= 0 pointwise (G is SPD)
    np.testing.assert_allclose(P.adjoint(v, u), g, rtol=1e-12, atol=1e-15)
    assert P.adjoint(u, u).min() >= -1e-15


def test_adjoint_central_difference():
    P = oracle.Problem(2, 6, 0.05)
    h1 = np.exp(0.5 * workloads.uniform(P.n, 4))
    u = workloads.uniform(P.n, 0)
    v = workloads.uniform(P.n, 1)
    dh = workloads.uniform(P.n, 2)
    g = P.adjoint(u, v)
    eps = 1e-6
    f = lambda h: np.dot(v, oracle.ax_helm(P.lx, P.D, P.G, P.B, u, h, 0.0))
    fd = (f(h1 + eps * dh) - f(h1 - eps * dh)) / (2 * eps)
    assert abs(fd - np.dot(dh, g)) <= 1e-8 * abs(fd)


def _oracle_loss_grad(P, h1, h2, b, ut, rtol=1e-14):
    P.set_coef(h1, h2)
    u, i1 = P.pcg(b, rtol=rtol)
    assert i1["status"] == 0
    d = u - ut
    L = 0.5 * P.dot(d, d)
    rhs = np.where(P.dirichlet.astype(bool), 0.0, d)
    lam, i2 = P.pcg(rhs, rtol=rtol)
    assert i2["status"] == 0
    return L, -P.adjoint(u, lam)


def test_gradient_vs_dense_finite_differences():
    """dL/dh1 from the oracle's forward + adjoint solves and the h1-adjoint
    contraction equals central differences of a dense brute-force solve."""
    nx, lx, eps, h2 = 2, 3, 0.05, 10.0
    P = oracle.Problem(nx, lx, eps)
    field = workloads.grf(workloads.SEED_GRF)
    h1 = np.exp(field(P.x, P.y, P.z))
    b = P.assemble_rhs(P.B * workloads.sine_source(P.x, P.y, P.z))
    ut = _cont(P, 12, zero_dirichlet=True) * 0.1
    L, grad = _oracle_loss_grad(P, h1, h2, b, ut)

    A0, pos, _, _ = brute.assembled(nx, lx, eps, h1.reshape(P.nelv, -1), h2)
    p_loc = pos[P.glb]
    nf = A0.shape[0]
    rep = np.array([np.flatnonzero(p_loc == j)[0] for j in range(nf)])

    def loss(h):
        A, _, _, _ = brute.assembled(nx, lx, eps, h.reshape(P.nelv, -1), h2)
        u = np.linalg.solve(A, b[rep])
        return 0.5 * np.sum((u - ut[rep]) ** 2)

    assert abs(loss(h1) - L) <= 1e-10 * abs(L)
    rng = np.random.default_rng(0)
    for p in rng.choice(P.n, 12, replace=False):
        e = np.zeros(P.n)
        e[p] = 1e-6 * h1[p]
        fd = (loss(h1 + e) - loss(h1 - e)) / (2e-6 * h1[p])
        assert abs(fd - grad[p]) <= 1e-6 * np.abs(grad).max(), (p, fd, grad[p])


# ------------------------------------------------------------------ projection (Section 4, Table 2)
def _proj_case():
    P = oracle.Problem(2, 5, 0.05)
    X = []
    for sd in (21, 22, 23):
        xs, info = P.pcg(P.assemble_rhs(workloads.uniform(P.n, sd)), rtol=1e-13)
        assert info["status"] == 0
        X.append(xs)
    b = P.assemble_rhs(workloads.uniform(P.n, 24))
    return P, X, b


def test_projection_galerkin_and_exact_recovery():
    """The residual of the projected guess is orthogonal to every stored solution;
    a load whose solution lies in the space is solved exactly; an empty space gives 0."""
    P, X, b = _proj_case()
    x0, r = P.projection(X, b)
    bn = np.sqrt(P.dot(b, b))
    for xi in X:
        assert abs(P.dot(xi, r)) <= 1e-12 * bn * np.sqrt(P.dot(xi, xi))
    x0e, re = P.projection(X, P.apply(X[1]))
    assert np.abs(x0e - X[1]).max() <= 1e-10 * np.abs(X[1]).max()
    assert np.sqrt(P.dot(re, re)) <= 1e-10 * np.sqrt(P.dot(P.apply(X[1]), P.apply(X[1])))
    z, rz = P.projection([], b)
    assert not z.any() and np.array_equal(rz, b)


def test_projection_matches_dense_and_is_optimal():
    """Against an independent dense assembly on the free unique nodes: the same
    x0 = X (X^T A X)^{-1} X^T b, and no other combination of the stored solutions
    is closer to A^{-1} b in the A-norm."""
    P, X, b = _proj_case()
    x0, _ = P.projection(X, b)
    A, pos, _, _ = brute.assembled(2, 5, 0.05)
    p_loc = pos[P.glb]
    free = p_loc >= 0
    rep = np.array([np.flatnonzero(p_loc == j)[0] for j in range(A.shape[0])])
    Xd = np.stack([x[rep] for x in X], axis=1)
    bd = b[rep]
    cd = np.linalg.solve(Xd.T @ A @ Xd, Xd.T @ bd)
    x0d = Xd @ cd
    np.testing.assert_allclose(x0[free], x0d[p_loc[free]], rtol=0, atol=1e-11 * np.abs(x0d).max())
    xs = np.linalg.solve(A, bd)
    e0 = (xs - x0d) @ A @ (xs - x0d)
    rng = np.random.default_rng(7)
    for _ in range(20):
        y = Xd @ (cd + 0.1 * rng.standard_normal(len(X)) * np.abs(cd).max())
        assert (xs - y) @ A @ (xs - y) >= e0


# ------------------------------------------------------------------ GMRES (Section 4, pressure solver)
def test_gmres_minimal_residual_matches_dense_krylov():
    """k steps of (unrestarted) right-preconditioned GMRES give the x in
    x0 + D K_k(A D, r0) (D = point Jacobi) that minimises |b - A x| in the unique-node
    norm: checked against an explicit Krylov basis and a dense least-squares solve with
    an independently assembled operator."""
    P = oracle.Problem(2, 5, 0.05)
    b = P.assemble_rhs(workloads.uniform(P.n, 3))
    A, pos, _, _ = brute.assembled(2, 5, 0.05)
    p_loc = pos[P.glb]
    free = p_loc >= 0
    rep = np.array([np.flatnonzero(p_loc == j)[0] for j in range(A.shape[0])])
    d = P.dinv[rep]
    bd = b[rep]
    for k in (1, 3, 6):
        x, info = P.gmres(b, rtol=1e-30, restart=50, max_iter=k)
        assert info["iters"] == k
        K = [bd]
        for _ in range(k - 1):
            K.append(A @ (d * K[-1]))
        Q, _ = np.linalg.qr(np.stack(K, axis=1))   # basis of K_k(A D, b)
        Y = d[:, None] * Q                          # search space D K_k
        c = np.linalg.lstsq(A @ Y, bd, rcond=None)[0]
        xd = Y @ c
        np.testing.assert_allclose(x[free], xd[p_loc[free]], rtol=0, atol=1e-9 * np.abs(xd).max())


def test_gmres_solves_the_system_with_restarts():
    """Restarted GMRES reaches the tolerance on the true residual and agrees with the
    CG solution of the same SPD system."""
    P = oracle.Problem(3, 5, 0.05)
    b = P.assemble_rhs(workloads.uniform(P.n, 4))
    x, info = P.gmres(b, rtol=1e-10, restart=10)
    assert info["cycles"] > 1
    assert P.true_rel_res(x, b) <= 1e-10
    xc, _ = P.pcg(b, rtol=1e-13)
    assert np.abs(x - xc).max() <= 1e-7 * np.abs(xc).max()


# ------------------------------------------------------------------ two-level Schwarz (Section 4)
def _prolongation(P, nv, cvert, phi):
    """Dense P: local points x coarse vertices (the trilinear basis at every copy)."""
    lx3 = P.lx ** 3
    Pm = np.zeros((P.n, nv))
    for e in range(P.nelv):
        for c in range(8):
            Pm[e * lx3:(e + 1) * lx3, cvert[e, c]] += phi[c]
    return Pm


def test_schwarz_coarse_operator_is_galerkin():
    """A0 equals P^T A P with A an independently assembled dense operator (all unique
    nodes, no mask) and P the trilinear interpolation written out densely."""
    P = oracle.Problem(2, 5, 0.05).schwarz_setup()
    A, pos, gid, _ = brute.assembled_full(2, 5, 0.05)
    nv = P._A0.shape[0]
    Pl = _prolongation(P, nv, P._cvert, P._phi)
    p_loc = pos[P.glb]
    rep = np.array([np.flatnonzero(p_loc == j)[0] for j in range(A.shape[0])])
    Pu = Pl[rep]                           # interpolation onto the unique nodes
    np.testing.assert_allclose(P._A0, Pu.T @ A @ Pu, rtol=0, atol=1e-12 * np.abs(P._A0).max())


def test_schwarz_local_operator_on_affine_elements():
    """On an undeformed box the separable local operator without its extension segments
    is the element's own stiffness matrix (independent chain-rule assembly), and the
    segments add a positive semi-definite term that leaves every coupling between two
    points off the element's faces unchanged."""
    P0 = oracle.Problem(2, 5, 0.0).schwarz_setup(extend=False)
    P1 = oracle.Problem(2, 5, 0.0).schwarz_setup()
    xyz, _, _ = brute.box(2, 5, 0.0)
    for e in (0, 5):
        Ae, _, _ = brute.element_matrix(xyz[e], 5)
        np.testing.assert_allclose(P0._loc[e], Ae, rtol=0, atol=1e-12 * np.abs(Ae).max())
        ext = P1._loc[e] - P0._loc[e]
        assert np.linalg.eigvalsh(ext).min() >= -1e-12 * np.abs(Ae).max()
        lx, N = 5, 4
        idx = np.arange(lx ** 3)
        i, j, k = idx % lx, (idx // lx) % lx, idx // lx ** 2
        inner = ~((i == 0) | (i == N) | (j == 0) | (j == N) | (k == 0) | (k == N))
        assert np.abs(ext[np.ix_(inner, inner)]).max() == 0.0


def _gll_element_1d(lx, L):
    """Stiffness, GLL-quadrature (diagonal) mass and nodes of a degree lx-1 Lagrange
    element on the GLL points of [0, L]: the stiffness integrated exactly by
    Gauss-Legendre quadrature of the basis derivatives, the GLL weights as exact
    integrals of the Lagrange basis (degree N <= 2N - 1 exactness)."""
    N = lx - 1
    xi = np.sort(np.concatenate(([-1.0, 1.0], np.polynomial.legendre.Legendre.basis(N).deriv().roots())))
    x = (xi + 1.0) * L / 2.0
    V = np.vander(x, lx, increasing=True)
    C = np.linalg.inv(V)                           # column j: monomial coefficients of l_j
    q, wq = np.polynomial.legendre.leggauss(lx + 2)
    xq = (q + 1.0) * L / 2.0
    dphi = np.array([np.polynomial.polynomial.polyval(xq, np.polynomial.polynomial.polyder(C[:, j]))
                     for j in range(lx)])         # [basis, quadrature point]
    Km = (dphi * (wq * L / 2.0)) @ dphi.T
    wg = np.array([np.polynomial.polynomial.polyval(x, C[:, j]) for j in range(lx)])  # identity at nodes
    assert np.allclose(wg, np.eye(lx))
    wgl = np.array([np.polynomial.polynomial.polyval(xq, C[:, j]) @ (wq * L / 2.0) for j in range(lx)])
    return Km, np.diag(wgl), x


def _chain_1d(lx, L, segs_lo, segs_hi):
    """Stiffness and lumped mass of a 1-D chain assembled from element matrices: linear
    elements of the lengths segs_lo (listed outward from the element), the GLL element
    of length L, linear elements of the lengths segs_hi (outward); both outermost nodes
    Dirichlet, so the result is restricted to the nodes between them."""
    Km, Mm, _ = _gll_element_1d(lx, L)
    nlo, nhi = len(segs_lo), len(segs_hi)
    n = nlo + lx + nhi                             # one node beyond each segment
    K = np.zeros((n, n))
    M = np.zeros((n, n))
    o = nlo                                        # first element node
    K[o:o + lx, o:o + lx] += Km
    M[o:o + lx, o:o + lx] += Mm

    def seg(a, b, h):
        K[np.ix_([a, b], [a, b])] += np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
        M[np.ix_([a, b], [a, b])] += np.eye(2) * h / 2.0

    for m, h in enumerate(segs_lo):                # node o - m joined to node o - m - 1
        seg(o - m - 1, o - m, h)
    for m, h in enumerate(segs_hi):
        seg(o + lx - 1 + m, o + lx + m, h)
    lo = 1 if nlo > 0 else 0
    hi = n - 1 if nhi > 0 else n
    return K[lo:hi, lo:hi], M[lo:hi, lo:hi]


def _extended_1d(lx, L):
    """Stiffness and (lumped) mass of a 1-D chain, assembled from element matrices and
    then restricted to the middle element's nodes: a linear element of the middle
    element's first GLL spacing at each end (outer node Dirichlet), and the middle
    element (see _gll_element_1d)."""
    _, _, x = _gll_element_1d(lx, L)
    h = x[1] - x[0]
    return _chain_1d(lx, L, [h], [h])


def test_schwarz_extension_matches_assembled_linear_segments():
    """The extension of the local Schwarz operator has the magnitude its reading states:
    on an undeformed box, the oracle's separable local operator equals the Kronecker
    form built from an independent 1-D assembly of the element plus one linear segment
    of the first GLL spacing at each end (Dirichlet beyond), with h1 and h2 both on."""
    for nx, lx in ((2, 4), (1, 6), (3, 8)):
        P = oracle.Problem(nx, lx, 0.0, h1=0.7, h2=3.0).schwarz_setup()
        K, M = _extended_1d(lx, 1.0 / nx)
        ref = 0.7 * (np.kron(M, np.kron(M, K)) + np.kron(M, np.kron(K, M)) + np.kron(K, np.kron(M, M))) \
            + 3.0 * np.kron(M, np.kron(M, M))
        for e in (0, nx ** 3 - 1):
            np.testing.assert_allclose(P._loc[e], ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_schwarz_local_operator_direction_lengths_on_a_stretched_box():
    """On an undeformed box with a different element length per direction (1/2, 1/3, 1/4),
    the separable local operator takes each direction's own length: it equals the
    Kronecker form of three independent 1-D chain assemblies with those lengths, for the
    element-only problem and for the one-point overlap (an interior element: the overlap
    on all six faces).  A direction mix-up in the element lengths fails on this machine though
    not on a cube."""
    lx, h1, h2 = 5, 0.7, 3.0
    nx, ny, nz = 3, 4, 5
    lens = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    e = 1 + nx * (1 + ny * 1)                       # element (1, 1, 1): neighbours on all faces

    def chains(overlap):
        out = []
        for L in lens:
            _, _, x = _gll_element_1d(lx, L)
            d1, d2 = x[1] - x[0], x[2] - x[1]
            segs = [d1, d2] if overlap else [d1]
            out.append(_chain_1d(lx, L, segs, segs))
        return out

    for overlap in (False, True):
        P = oracle.Problem(nx, lx, 0.0, h1=h1, h2=h2, ny=ny, nz=nz).schwarz_setup(overlap=overlap)
        (Kr, Mr), (Ks, Ms), (Kt, Mt) = chains(overlap)
        ref = h1 * (np.kron(Mt, np.kron(Ms, Kr)) + np.kron(Mt, np.kron(Ks, Mr)) + np.kron(Kt, np.kron(Ms, Mr))) \
            + h2 * np.kron(Mt, np.kron(Ms, Mr))
        assert P._loc[e].shape == ref.shape
        np.testing.assert_allclose(P._loc[e], ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_schwarz_overlap_local_operator_matches_assembled_chain():
    """One-point overlap: on an undeformed box the oracle's extended local operator is
    the Kronecker form built from independent 1-D chain assemblies -- beyond a face with
    a neighbour, a first-spacing segment to the extension node and a second-spacing
    segment to a Dirichlet node; beyond a boundary face, the first-spacing segment to a
    Dirichlet node -- for an interior element (overlap on all six faces) and a corner
    element (overlap on its three upper faces only)."""
    nx, h1, h2 = 3, 0.7, 3.0
    for lx in (4, 6):
        P = oracle.Problem(nx, lx, 0.0, h1=h1, h2=h2).schwarz_setup(overlap=True)
        _, _, x = _gll_element_1d(lx, 1.0 / nx)
        d1, d2 = x[1] - x[0], x[2] - x[1]
        for e, lo in ((13, [d1, d2]), (0, [d1])):
            K, M = _chain_1d(lx, 1.0 / nx, lo, [d1, d2])
            ref = h1 * (np.kron(M, np.kron(M, K)) + np.kron(M, np.kron(K, M)) + np.kron(K, np.kron(M, M))) \
                + h2 * np.kron(M, np.kron(M, M))
            assert P._loc[e].shape == ref.shape
            np.testing.assert_allclose(P._loc[e], ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_schwarz_overlap_layer_is_one_spacing_outside():
    """The neighbour points gathered as the extension layer are, on an undeformed box,
    exactly the points one first GLL spacing beyond each face point along the face's
    outward normal (checked with the mesh coordinates, not the global ids), and a face
    has a neighbour exactly when it is inside the box."""
    nx, ny, nz, lx = 3, 2, 2, 5
    P = oracle.Problem(nx, lx, 0.0, ny=ny, nz=nz)
    src = P._extension_sources()
    xyz = np.stack([P.x, P.y, P.z])
    xi = P.xi
    lx3, N = lx ** 3, lx - 1
    nel = (nx, ny, nz)
    for e in range(P.nelv):
        ec = (e % nx, (e // nx) % ny, e // (nx * ny))
        for d in range(3):
            h = (xi[1] - xi[0]) / 2.0 / nel[d]
            for side in (0, 1):
                m = src[e][2 * d + side]
                inside = ec[d] > 0 if side == 0 else ec[d] < nel[d] - 1
                assert (m is not None) == inside
                if m is None:
                    continue
                assert len(m) == lx * lx
                for p, q in m.items():
                    assert (p // lx ** d) % lx == (N if side else 0)
                    step = xyz[:, q] - xyz[:, e * lx3 + p]
                    want = np.zeros(3)
                    want[d] = h if side else -h
                    np.testing.assert_allclose(step, want, rtol=0, atol=1e-14)


def test_schwarz_overlap_single_element_equals_element_solve():
    """With no neighbours the one-point-overlap preconditioner reduces to the
    element-only one (the extension is the first-spacing segment everywhere)."""
    P = oracle.Problem(1, 6, 0.05, h1=1.0, h2=2.0)
    r = P.assemble_rhs(workloads.uniform(P.n, 5))
    z0 = P.schwarz_setup().schwarz_apply(r)
    z1 = P.schwarz_setup(overlap=True).schwarz_apply(r)
    np.testing.assert_allclose(z1, z0, rtol=0, atol=1e-12 * np.abs(z0).max())


def test_schwarz_overlap_reduces_gmres_steps():
    """Giving the local problems the neighbours' residual one point beyond each face
    (minimal overlap) takes GMRES to the tolerance in clearly fewer steps than the
    element-only local problems, on curved meshes of two sizes."""
    for nx, lx in ((4, 6), (3, 8)):
        P = oracle.Problem(nx, lx, 0.05)
        b = P.assemble_rhs(workloads.uniform(P.n, 3))
        P.schwarz_setup()
        x0, i0 = P.gmres(b, rtol=1e-10, restart=30, precond="schwarz")
        P.schwarz_setup(overlap=True)
        x1, i1 = P.gmres(b, rtol=1e-10, restart=30, precond="schwarz")
        assert P.true_rel_res(x1, b) <= 1e-10
        assert i1["iters"] <= 0.85 * i0["iters"], (i0["iters"], i1["iters"])


def test_schwarz_coarse_correction_recovers_coarse_errors():
    """For r = A P u0 (u0 on the free vertices) an exact coarse solve gives back P u0."""
    P = oracle.Problem(3, 5, 0.05).schwarz_setup()
    nv = P._A0.shape[0]
    rng = np.random.default_rng(9)
    u0 = np.where(P._cfree, rng.uniform(-1, 1, nv), 0.0)
    Pl = _prolongation(P, nv, P._cvert, P._phi)
    pu = Pl @ u0
    r = P.apply(pu)
    zc = P.coarse_correction(r, coarse_iters=400)
    np.testing.assert_allclose(zc, pu, rtol=0, atol=1e-9 * np.abs(pu).max())


def test_schwarz_preconditioned_gmres():
    """GMRES with the two-level Schwarz preconditioner meets the tolerance in a small,
    nearly mesh-independent number of steps, well below point Jacobi's."""
    its = []
    for nx in (3, 5):
        P = oracle.Problem(nx, 5, 0.05).schwarz_setup()
        b = P.assemble_rhs(workloads.uniform(P.n, 3))
        x, info = P.gmres(b, rtol=1e-10, restart=40, precond="schwarz")
        assert P.true_rel_res(x, b) <= 1e-10
        xj, ij = P.gmres(b, rtol=1e-10, restart=40)
        assert info["iters"] < 0.4 * ij["iters"]
        its.append(info["iters"])
    assert its[1] <= its[0] + 8


def test_schwarz_coarse_space_interpolates_linear_functions():
    """The coarse basis is the trilinear interpolation of vertex values: on an affine
    mesh the vertex coordinates interpolate to the node coordinates exactly, and every
    interpolated field takes one value on all copies of a global id."""
    P = oracle.Problem(3, 5, 0.0).schwarz_setup()
    nv = P._A0.shape[0]
    Pl = _prolongation(P, nv, P._cvert, P._phi)
    lx3, N = P.lx ** 3, P.lx - 1
    corner = [i + P.lx * (j + P.lx * k) for k in (0, N) for j in (0, N) for i in (0, N)]
    for coord in (P.x, P.y, P.z):
        vx = np.zeros(nv)
        for e in range(P.nelv):
            for c in range(8):
                vx[P._cvert[e, c]] = coord[e * lx3 + corner[c]]
        np.testing.assert_allclose(Pl @ vx, coord, rtol=0, atol=1e-13)
    u = Pl @ np.random.default_rng(2).uniform(-1, 1, nv)
    np.testing.assert_allclose(P.gs.op(u) / P.mult, u, rtol=0, atol=1e-14)
