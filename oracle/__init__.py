"""Plain FP64 CPU oracle for the SEM Helmholtz hot path (arXiv 2107.01243).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
It shares no code with the HIP path.  The arithmetic lives in
``sem_oracle.c`` (plain loops, FP64, ``-O2 -ffp-contract=off``); this module
only marshals numpy arrays into it.

The projection onto previous solutions (``Problem.projection``), flexible GMRES
(``Problem.gmres``) and the two-level Schwarz preconditioner
(``Problem.schwarz_setup`` / ``schwarz_apply``) are written here with numpy on top
of the C operator (small dense systems solved by ``numpy.linalg``).

Every function cites the passage of the paper it follows; the readings taken
where the paper is silent or garbled are listed at the top of ``sem_oracle.c`` for
the C part, and in the docstrings of ``projection``, ``gmres`` and
``schwarz_setup`` (element lengths, extension segments, the one-point overlap,
the coarse space and its fixed-count solve) for the numpy part.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sem_oracle.c")
# SEM_ORACLE_LIB: another build of sem_oracle.c to load instead (the sanitizer test
# loads one built with AddressSanitizer and UndefinedBehaviorSanitizer).
_LIB_OVERRIDE = os.environ.get("SEM_ORACLE_LIB")
_BUILT = os.path.join(_HERE, "liboracle.so")
_LIB = _LIB_OVERRIDE or _BUILT

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile sem_oracle.c into liboracle.so with gcc (FP64, no FP contraction)."""
    if force or not os.path.exists(_BUILT) or os.path.getmtime(_BUILT) < os.path.getmtime(_SRC):
        tmp = _BUILT + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-D_GNU_SOURCE", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _BUILT)
    return _BUILT


_lib = None
_PROGRESS = C.CFUNCTYPE(None, C.c_int, C.c_double)


def set_threads(nthreads: int) -> int:
    """Host threads of the oracle's parallel loops; returns the previous count."""
    return lib().orc_set_threads(int(nthreads))


def lib():
    global _lib
    if _lib is None:
        if not _LIB_OVERRIDE and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        L = C.CDLL(_LIB)
        vp = C.c_void_p
        L.orc_gll.argtypes = [C.c_int, _f64p, _f64p]
        L.orc_deriv_matrix.argtypes = [C.c_int, _f64p, _f64p]
        L.orc_box_mesh.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, _f64p,
                                   _i64p, _u8p, _f64p, _f64p, _f64p]
        L.orc_box_mesh.restype = None
        L.orc_geometry.argtypes = [C.c_int64, C.c_int, _f64p, _f64p, _f64p, _f64p, _f64p,
                                   _f64p, _f64p, _f64p]
        L.orc_geometry.restype = C.c_int64
        L.orc_ax_helm.argtypes = [C.c_int64, C.c_int, _f64p, _f64p, vp, vp, C.c_double,
                                  vp, C.c_double, _f64p, _f64p]
        L.orc_ax_helm.restype = None
        L.orc_ax_adjoint.argtypes = [C.c_int64, C.c_int, _f64p, _f64p, _f64p, _f64p, _f64p]
        L.orc_ax_adjoint.restype = None
        L.orc_gs_create.argtypes = [C.c_int64, _i64p]
        L.orc_gs_create.restype = vp
        L.orc_gs_ngroups.argtypes = [vp]
        L.orc_gs_ngroups.restype = C.c_int64
        L.orc_gs_nentries.argtypes = [vp]
        L.orc_gs_nentries.restype = C.c_int64
        L.orc_gs_groups.argtypes = [vp, _i64p, _i64p, _i64p]
        L.orc_gs_groups.restype = None
        L.orc_gs_op.argtypes = [vp, _f64p]
        L.orc_gs_op.restype = None
        L.orc_gs_free.argtypes = [vp]
        L.orc_gs_free.restype = None
        L.orc_multiplicity.argtypes = [vp, _f64p]
        L.orc_multiplicity.restype = None
        L.orc_apply.argtypes = [C.c_int64, C.c_int, _f64p, _f64p, vp, vp, C.c_double, vp,
                                C.c_double, vp, vp, _f64p, _f64p]
        L.orc_apply.restype = None
        L.orc_diag.argtypes = [C.c_int64, C.c_int, _f64p, _f64p, vp, vp, C.c_double, vp,
                               C.c_double, _f64p]
        L.orc_diag.restype = None
        L.orc_jacobi_dinv.argtypes = [C.c_int64, C.c_int, _f64p, _f64p, vp, vp, C.c_double,
                                      vp, C.c_double, vp, vp, _f64p]
        L.orc_jacobi_dinv.restype = None
        L.orc_wdot.argtypes = [C.c_int64, _f64p, _f64p, _f64p]
        L.orc_wdot.restype = C.c_double
        L.orc_pcg.argtypes = [C.c_int64, C.c_int, _f64p, _f64p, vp, vp, C.c_double, vp,
                              C.c_double, vp, vp, _f64p, _f64p, _f64p, C.c_double, C.c_int,
                              C.POINTER(C.c_int), C.POINTER(C.c_double), _PROGRESS, C.c_int]
        L.orc_pcg.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _coef(h):
    """A coefficient is a python float (scalar) or an FP64 array of n_p values."""
    if h is None:
        return None, 0.0
    if np.isscalar(h):
        return None, float(h)
    a = np.ascontiguousarray(h, dtype=np.float64)
    return a, 0.0


# ---------------------------------------------------------------- space
def gll(lx: int):
    """GLL points and weights (Section 2, Eq. 7-8)."""
    xi = np.zeros(lx)
    w = np.zeros(lx)
    if lib().orc_gll(lx, xi, w) != 0:
        raise ValueError(f"lx={lx} out of range")
    return xi, w


def deriv_matrix(xi):
    """D[i, l] = l_l'(xi_i), the local derivative matrix of Eq. 9."""
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    D = np.zeros((len(xi), len(xi)))
    lib().orc_deriv_matrix(len(xi), xi, D)
    return D


# ---------------------------------------------------------------- mesh
def box_mesh(nx: int, ny: int, nz: int, lx: int, eps: float):
    """Structured box mesh on [0,1]^3, curved by the smooth sine map of amplitude eps.

    Returns dict with glb (int64), dirichlet (uint8), x, y, z (FP64), all n_p long.
    """
    xi, _ = gll(lx)
    n = nx * ny * nz * lx ** 3
    glb = np.zeros(n, np.int64)
    dr = np.zeros(n, np.uint8)
    x = np.zeros(n)
    y = np.zeros(n)
    z = np.zeros(n)
    lib().orc_box_mesh(nx, ny, nz, lx, float(eps), xi, glb, dr, x, y, z)
    return dict(glb=glb, dirichlet=dr, x=x, y=y, z=z)


def geometry(lx: int, D, w, x, y, z):
    """Geometric factors G (6, n_p: G11, G22, G33, G12, G13, G23), B and J (Eq. 9)."""
    n = len(x)
    nelv = n // lx ** 3
    G = np.zeros((6, n))
    B = np.zeros(n)
    J = np.zeros(n)
    bad = lib().orc_geometry(nelv, lx, np.ascontiguousarray(D), np.ascontiguousarray(w),
                             np.ascontiguousarray(x), np.ascontiguousarray(y),
                             np.ascontiguousarray(z), G, B, J)
    if bad:
        raise ValueError(f"{bad} points with non-positive Jacobian")
    return G, B, J


# ---------------------------------------------------------------- operators
def ax_helm(lx, D, G, B, u, h1=1.0, h2=0.0):
    """Unassembled Helmholtz action w = A_L u (Eq. 9-10)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = len(u)
    w = np.zeros(n)
    h1a, h1s = _coef(h1)
    h2a, h2s = _coef(h2)
    Bc = None if B is None else np.ascontiguousarray(B, dtype=np.float64)
    lib().orc_ax_helm(n // lx ** 3, lx, np.ascontiguousarray(D), np.ascontiguousarray(G),
                      _ptr(Bc), _ptr(h1a), h1s, _ptr(h2a), h2s, u, w)
    return w


def ax_adjoint(lx, D, G, u, v):
    """g_p = (D v)_p^T G_p (D u)_p = d(v^T A_L(h1) u)/d h1_p (h1-linearity of Eq. 9)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    g = np.zeros(len(u))
    lib().orc_ax_adjoint(len(u) // lx ** 3, lx, np.ascontiguousarray(D),
                         np.ascontiguousarray(G), u, v, g)
    return g


class GS:
    """Gather-scatter QQ^T (Eq. 10, Algorithm 1 local part), canonical ascending order."""

    def __init__(self, glb):
        self.glb = np.ascontiguousarray(glb, dtype=np.int64)
        self.n = len(self.glb)
        self._h = lib().orc_gs_create(self.n, self.glb)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_gs_free(self._h)
            self._h = None

    def groups(self):
        """(off, idx, gid): groups of local indices sharing a global id with mult >= 2."""
        ng = lib().orc_gs_ngroups(self._h)
        ne = lib().orc_gs_nentries(self._h)
        off = np.zeros(ng + 1, np.int64)
        idx = np.zeros(max(ne, 1), np.int64)
        gid = np.zeros(max(ng, 1), np.int64)
        lib().orc_gs_groups(self._h, off, idx, gid)
        return off, idx[:ne], gid[:ng]

    def op(self, u):
        """Return QQ^T u (a new array)."""
        v = np.array(u, dtype=np.float64, copy=True)
        lib().orc_gs_op(self._h, v)
        return v

    def mult(self):
        m = np.zeros(self.n)
        lib().orc_multiplicity(self._h, m)
        return m


def wdot(a, b, mult):
    """Unique-node inner product sum_L a_L b_L / mult_L."""
    return lib().orc_wdot(len(a), np.ascontiguousarray(a, dtype=np.float64),
                          np.ascontiguousarray(b, dtype=np.float64),
                          np.ascontiguousarray(mult, dtype=np.float64))


class Problem:
    """One discrete Helmholtz problem: space, mesh, geometry, gather-scatter, mask.

    A = mask QQ^T A_L(h1, h2) in local layout (Eq. 9-10 with Eq. 5 imposed by masking).
    """

    def __init__(self, nx, lx, eps=0.0, h1=1.0, h2=0.0, ny=None, nz=None, progress=None):
        say = progress or (lambda msg: None)
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        self.lx = lx
        self.nelv = nx * ny * nz
        self.n = self.nelv * lx ** 3
        self.xi, self.w = gll(lx)
        self.D = deriv_matrix(self.xi)
        m = box_mesh(nx, ny, nz, lx, eps)
        self.glb, self.dirichlet = m["glb"], m["dirichlet"]
        self.x, self.y, self.z = m["x"], m["y"], m["z"]
        say("oracle: mesh done")
        self.G, self.B, self.J = geometry(lx, self.D, self.w, self.x, self.y, self.z)
        say("oracle: geometry done")
        self.gs = GS(self.glb)
        say("oracle: gather-scatter groups done")
        self.mult = self.gs.mult()
        self.set_coef(h1, h2)
        say("oracle: Jacobi diagonal done")

    def set_coef(self, h1, h2):
        self.h1, self.h2 = h1, h2
        self._h1a, self._h1s = _coef(h1)
        self._h2a, self._h2s = _coef(h2)
        self.dinv = np.zeros(self.n)
        lib().orc_jacobi_dinv(self.nelv, self.lx, self.D, self.G, _ptr(self.B),
                              _ptr(self._h1a), self._h1s, _ptr(self._h2a), self._h2s,
                              self.gs._h, _ptr(self.dirichlet), self.dinv)

    def ax_local(self, u):
        return ax_helm(self.lx, self.D, self.G, self.B, u, self.h1, self.h2)

    def apply(self, u):
        """w = mask QQ^T A_L u."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        w = np.zeros(self.n)
        lib().orc_apply(self.nelv, self.lx, self.D, self.G, _ptr(self.B), _ptr(self._h1a),
                        self._h1s, _ptr(self._h2a), self._h2s, self.gs._h,
                        _ptr(self.dirichlet), u, w)
        return w

    def diag_local(self):
        d = np.zeros(self.n)
        lib().orc_diag(self.nelv, self.lx, self.D, self.G, _ptr(self.B), _ptr(self._h1a),
                       self._h1s, _ptr(self._h2a), self._h2s, d)
        return d

    def assemble_rhs(self, f_local):
        """b = mask QQ^T f: a local load vector summed onto the unique nodes."""
        b = self.gs.op(f_local)
        b[self.dirichlet.astype(bool)] = 0.0
        return b

    def pcg(self, b, x0=None, rtol=1e-10, max_iter=100000, progress=None, every=100):
        """Jacobi-PCG (Section 4 velocity solver).  rtol <= 0: exactly max_iter steps.
        progress(iteration, rel_res), if given, is called every `every` iterations."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        it = C.c_int(0)
        rr = C.c_double(0.0)
        cb = _PROGRESS(progress) if progress is not None else _PROGRESS()
        st = lib().orc_pcg(self.nelv, self.lx, self.D, self.G, _ptr(self.B), _ptr(self._h1a),
                           self._h1s, _ptr(self._h2a), self._h2s, self.gs._h,
                           _ptr(self.dirichlet), self.dinv, b, x, float(rtol), int(max_iter),
                           C.byref(it), C.byref(rr), cb, int(every))
        return x, dict(status=st, iters=it.value, rel_res=rr.value)

    def dot(self, a, b):
        return wdot(a, b, self.mult)

    def projection(self, X, b):
        """Initial guess from previous solutions (Section 4 and Table 2: the pressure
        solve keeps a space of previous solutions, after Nek5000).  Definition: the
        best approximation of A^{-1} b from span(X) in the A-norm, x0 = sum_i c_i X_i
        with (X^T A X) c = X^T b in the unique-node inner product -- equivalently the
        Galerkin condition (X_i, b - A x0) = 0.  Returns (x0, r = b - A x0)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        if len(X) == 0:
            return np.zeros(self.n), b.copy()
        AX = [self.apply(x) for x in X]
        G = np.array([[self.dot(xi, axj) for axj in AX] for xi in X])
        rhs = np.array([self.dot(xi, b) for xi in X])
        c = np.linalg.solve(G, rhs)
        x0 = np.zeros(self.n)
        for ci, xi in zip(c, X):
            x0 += ci * xi
        return x0, b - self.apply(x0)

    # -------------------------------------------------------------- two-level Schwarz
    def schwarz_setup(self, extend=True, overlap=False):
        """Data of the two-level additive overlapping Schwarz preconditioner of the
        pressure solve (Section 4: M^{-1} = R0^T A0^{-1} R0 + sum_k Rk^T Ak~^{-1} Rk;
        coarse grid on linear elements).  Local problem k: element k's lx^3 points with
        homogeneous Dirichlet conditions one first-GLL-spacing beyond each face; Ak~ is the
        separable box operator h1 (Mt x Ms x Kr + Mt x Ks x Mr + Kt x Ms x Mr) + h2 Mt x Ms x Mr
        with, per direction, the element's GLL stiffness and mass for the length
        L = 2 / sqrt(mean over the element of G_dd / B) plus one linear segment of the
        first-spacing length at each end (extend=False drops the segments: the element
        alone, for checks).  Coarse space: trilinear functions of the element vertices;
        A0 = P^T A P (Galerkin) on the free vertices.  h1, h2 scalars.

        overlap=True: the minimal overlap of one point.  Beyond every face that element k
        shares with a neighbour, the local problem also holds the layer of the
        neighbour's points one GLL index inside it: along that direction the 1-D
        operator gains a free extension node, joined to the face point by the
        first-spacing segment and held by a Dirichlet condition one second-GLL-spacing
        (J (xi_2 - xi_1)) beyond it; faces without a neighbour keep the extend=True
        segment.  The local right-hand side is the residual on the element's points and,
        on the extension layers, the neighbour's residual; the box's edge and corner
        points (outside the element in two or three directions) get zero.
        schwarz_apply then keeps each local solution on the element's own points only
        (restricted additive Schwarz) before the sum over shared points."""
        if not (np.isscalar(self.h1) and np.isscalar(self.h2)):
            raise ValueError("the Schwarz preconditioner takes scalar h1, h2")
        lx, N, E = self.lx, self.lx - 1, self.nelv
        xi, w, D = self.xi, self.w, self.D
        Kref = D.T @ np.diag(w) @ D          # 1-D stiffness on [-1, 1]
        dref = xi[1] - xi[0]                 # first GLL spacing on [-1, 1]
        dref2 = xi[min(2, N)] - xi[min(2, N) - 1]  # second spacing (the first when lx = 2)
        G = np.asarray(self.G).reshape(6, E, lx ** 3)
        B = np.asarray(self.B).reshape(E, lx ** 3)
        self._overlap = bool(overlap)
        src = self._extension_sources() if overlap else None
        self._loc = []
        self._ov = []
        for e in range(E):
            Ks, Ms, ranges = [], [], []
            for d in range(3):
                L = 2.0 / np.sqrt(np.mean(G[d, e] / B[e]))
                J = L / 2.0
                h, h2 = J * dref, J * dref2  # extension segment, and the one beyond
                lo = bool(overlap) and src[e][2 * d] is not None
                hi = bool(overlap) and src[e][2 * d + 1] is not None
                o = int(lo)
                nd = lx + int(lo) + int(hi)
                K = np.zeros((nd, nd))
                M = np.zeros((nd, nd))
                K[o:o + lx, o:o + lx] = Kref / J
                M[o:o + lx, o:o + lx] = np.diag(w * J)
                for has, f, xn in ((lo, o, o - 1), (hi, o + N, o + N + 1)):
                    if has:
                        K[np.ix_([xn, f], [xn, f])] += np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
                        M[xn, xn] += h / 2.0 + h2 / 2.0
                        M[f, f] += h / 2.0
                        K[xn, xn] += 1.0 / h2
                    elif extend:
                        K[f, f] += 1.0 / h
                        M[f, f] += h / 2.0
                Ks.append(K)
                Ms.append(M)
                ranges.append(np.arange(-int(lo), lx + int(hi)))
            # point (i, j, k) at i + lx j + lx^2 k: kron(t, s, r)
            Kr, Ksd, Kt = Ks
            Mr, Msd, Mt = Ms
            A = self.h1 * (np.kron(Mt, np.kron(Msd, Kr)) + np.kron(Mt, np.kron(Ksd, Mr)) +
                           np.kron(Kt, np.kron(Msd, Mr))) + self.h2 * np.kron(Mt, np.kron(Msd, Mr))
            self._loc.append(A)
            if overlap:
                # box points (I, J, K), I fastest: where each takes its right-hand side
                I = np.tile(ranges[0], len(ranges[1]) * len(ranges[2]))
                Jc = np.tile(np.repeat(ranges[1], len(ranges[0])), len(ranges[2]))
                Kc = np.repeat(ranges[2], len(ranges[0]) * len(ranges[1]))
                out = [(c < 0) | (c > N) for c in (I, Jc, Kc)]
                nout = out[0].astype(int) + out[1] + out[2]
                own = nout == 0
                gather = np.full(I.size, -1, dtype=np.int64)
                gather[own] = e * lx ** 3 + (I + lx * (Jc + lx * Kc))[own]
                for q in np.flatnonzero(nout == 1):
                    c = [I[q], Jc[q], Kc[q]]
                    d = [out[0][q], out[1][q], out[2][q]].index(True)
                    side = int(c[d] > N)
                    c[d] = N if side else 0
                    gather[q] = src[e][2 * d + side][c[0] + lx * (c[1] + lx * c[2])]
                self._ov.append((np.linalg.inv(A), gather, own))
        # coarse space: vertices = global ids of the element corners
        corner = [i + lx * (j + lx * k) for k in (0, N) for j in (0, N) for i in (0, N)]
        cg = np.array([[self.glb[e * lx ** 3 + c] for c in corner] for e in range(E)])
        vid, cidx = np.unique(cg, return_inverse=True)
        self._cvert = cidx.reshape(E, 8)
        nv = len(vid)
        dirv = np.zeros(nv, bool)
        for e in range(E):
            for c in range(8):
                dirv[self._cvert[e, c]] = self.dirichlet[e * lx ** 3 + corner[c]] != 0
        self._cfree = ~dirv
        l0, l1 = (1.0 - xi) / 2.0, (1.0 + xi) / 2.0
        phi1 = [l0, l1]
        # phi[c][p]: trilinear basis of corner c = a + 2 b + 4 c at point p of an element
        self._phi = np.array([np.kron(phi1[cc], np.kron(phi1[bb], phi1[aa]))
                              for cc in (0, 1) for bb in (0, 1) for aa in (0, 1)])
        A0 = np.zeros((nv, nv))
        probes = np.tile(self._phi[:, None, :], (1, E, 1)).reshape(8, -1)
        for c in range(8):
            wc = self.ax_local(probes[c]).reshape(E, lx ** 3)
            for e in range(E):
                for c2 in range(8):
                    A0[self._cvert[e, c2], self._cvert[e, c]] += self._phi[c2] @ wc[e]
        self._A0 = A0
        return self

    def schwarz_apply(self, r, coarse_iters=10):
        """z = M^{-1} r for an assembled, masked residual r: the local solves (on the
        element's own points) summed over the shared points and averaged by multiplicity,
        plus the coarse correction P e0,
        e0 from coarse_iters Jacobi-CG steps on A0 e0 = P^T r (from e0 = 0); masked."""
        lx, E = self.lx, self.nelv
        r = np.asarray(r, dtype=np.float64)
        if self._overlap:
            zl = np.zeros((E, lx ** 3))
            for e, (Ainv, gather, own) in enumerate(self._ov):
                rhs = np.where(gather >= 0, r[np.maximum(gather, 0)], 0.0)
                zl[e] = (Ainv @ rhs)[own]
            zl = zl.reshape(-1)
        else:
            rl = r.reshape(E, lx ** 3)
            zl = np.stack([np.linalg.solve(self._loc[e], rl[e]) for e in range(E)]).reshape(-1)
        z = self.gs.op(zl) / self.mult
        out = z + self.coarse_correction(r, coarse_iters)
        out[self.dirichlet.astype(bool)] = 0.0
        return out

    def _extension_sources(self):
        """The neighbour points that extend each element's Schwarz subdomain by one
        point (Section 4, overlapping subdomains of the additive Schwarz method).
        For element e and face (d, side) (face index 2 d + side; the face's points
        have local coordinate d equal to 0, or lx - 1 for side 1): None when no other
        element holds every global id of the face, else a dict from each face point's
        local index p to the index, in the whole local layout, of its extension point --
        in that neighbour, the point adjacent (one GLL index away) to the copy of p whose
        global id is not one of e's.  Brute force over global ids; any orientation."""
        lx, N, E, lx3 = self.lx, self.lx - 1, self.nelv, self.lx ** 3
        g = np.asarray(self.glb).reshape(E, lx3)
        ids = [set(g[e].tolist()) for e in range(E)]
        holders = {}
        for e in range(E):
            for v in ids[e]:
                holders.setdefault(v, set()).add(e)
        where = [{v: p for p, v in enumerate(g[e].tolist())} for e in range(E)]
        out = []
        for e in range(E):
            faces = []
            for d in range(3):
                for side in (0, 1):
                    pts = [p for p in range(lx3) if (p // lx ** d) % lx == (N if side else 0)]
                    common = set.intersection(*(holders[g[e, p]] for p in pts)) - {e}
                    if not common:
                        faces.append(None)
                        continue
                    (e2,) = common
                    m = {}
                    for p in pts:
                        q = where[e2][g[e, p]]
                        cand = []
                        for dd in range(3):
                            c = (q // lx ** dd) % lx
                            for s in (-1, 1):
                                if 0 <= c + s <= N and g[e2, q + s * lx ** dd] not in ids[e]:
                                    cand.append(q + s * lx ** dd)
                        (q2,) = cand
                        m[p] = e2 * lx3 + q2
                    faces.append(m)
            out.append(faces)
        return out

    def coarse_correction(self, r, coarse_iters=10):
        """P e0 with e0 from coarse_iters Jacobi-CG steps on A0 e0 = P^T r, e0 = 0 first."""
        lx, E = self.lx, self.nelv
        # r0 = P^T r over unique points (local copies weighted by 1 / mult)
        rw = (np.asarray(r) / self.mult).reshape(E, lx ** 3)
        nv = self._A0.shape[0]
        r0 = np.zeros(nv)
        for e in range(E):
            for c in range(8):
                r0[self._cvert[e, c]] += self._phi[c] @ rw[e]
        f = self._cfree
        A0 = self._A0[np.ix_(f, f)]
        e0 = np.zeros(nv)
        if coarse_iters > 0 and f.any():
            bvec = r0[f]
            dg = 1.0 / np.diag(A0)
            xk = np.zeros_like(bvec)
            rk = bvec.copy()
            zk = dg * rk
            pk = zk.copy()
            rz = rk @ zk
            for _ in range(coarse_iters):
                if rz == 0.0:
                    break
                q = A0 @ pk
                a = rz / (pk @ q)
                xk += a * pk
                rk -= a * q
                zk = dg * rk
                rz_new = rk @ zk
                pk = zk + (rz_new / rz) * pk
                rz = rz_new
            e0[f] = xk
        return np.stack([e0[self._cvert[e]] @ self._phi for e in range(E)]).reshape(-1)

    def gmres(self, b, rtol=1e-10, restart=30, max_iter=100000, x0=None, precond="jacobi", coarse_iters=10):
        """Flexible GMRES(m) with right preconditioning (point Jacobi, or the two-level
        Schwarz preconditioner of schwarz_apply) -- the Krylov solver
        of the paper's pressure equation (Section 4, Table 2) -- in the unique-node inner
        product, following Saad, Iterative Methods for Sparse Linear Systems, Alg. 9.6:
        Arnoldi by modified Gram-Schmidt, the small least-squares problem solved by
        numpy.linalg.lstsq at every step, restart from the true residual.  Returns
        (x, {"iters": Arnoldi steps, "cycles": ..., "rel_res": |b - A x| / |b|})."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        norm = lambda v: np.sqrt(self.dot(v, v))
        bn = norm(b)
        total, cycles = 0, 0
        while True:
            r = b - self.apply(x)
            beta = norm(r)
            rel = beta / bn if bn > 0 else 0.0
            if rel <= rtol or total >= max_iter:
                break
            cycles += 1
            V, Z = [r / beta], []
            H = np.zeros((restart + 1, restart))
            y = np.zeros(0)
            for j in range(restart):
                z = self.dinv * V[j] if precond == "jacobi" else self.schwarz_apply(V[j], coarse_iters)
                Z.append(z)
                w = self.apply(z)
                for i in range(j + 1):
                    H[i, j] = self.dot(w, V[i])
                    w = w - H[i, j] * V[i]
                H[j + 1, j] = norm(w)
                total += 1
                e1 = np.zeros(j + 2)
                e1[0] = beta
                y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
                res = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y)
                if res <= rtol * bn or total >= max_iter or H[j + 1, j] == 0.0:
                    break
                V.append(w / H[j + 1, j])
            for yi, zi in zip(y, Z):
                x = x + yi * zi
        return x, {"iters": total, "cycles": cycles, "rel_res": rel}

    def true_rel_res(self, x, b):
        r = b - self.apply(x)
        return np.sqrt(self.dot(r, r)) / np.sqrt(self.dot(b, b))

    def adjoint(self, u, v):
        return ax_adjoint(self.lx, self.D, self.G, u, v)
