"""ctypes binding of libsem (include/sem.h): argument marshalling only.

Every numeric step runs in the HIP kernels of libsem.so; torch supplies device
memory (tensor storage) and the current HIP stream.  If libsem.so is absent the
import of this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsem.so")

SEM_OK, SEM_ERR_INVALID, SEM_ERR_OOM, SEM_ERR_HIP = 0, -1, -2, -3
SEM_ERR_NOT_CONVERGED, SEM_ERR_BREAKDOWN, SEM_ERR_UNSUPPORTED = -4, -5, -6
SEM_F64, SEM_F32 = 0, 1
SEM_COEF_F32 = 1
_NAMES = {0: "SEM_OK", -1: "SEM_ERR_INVALID", -2: "SEM_ERR_OOM", -3: "SEM_ERR_HIP",
          -4: "SEM_ERR_NOT_CONVERGED", -5: "SEM_ERR_BREAKDOWN", -6: "SEM_ERR_UNSUPPORTED"}


class SemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class PcgParams(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int), ("check_every", C.c_int),
                ("mixed", C.c_int), ("inner_rtol", C.c_double), ("inner_max_iter", C.c_int),
                ("use_x0", C.c_int), ("delta", C.c_double), ("variant", C.c_int)]


class GmresParams(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int), ("restart", C.c_int), ("precond", C.c_int),
                ("use_x0", C.c_int), ("coarse_iters", C.c_int)]


class PcgInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("inner_iters", C.c_int), ("converged", C.c_int),
                ("rel_res", C.c_double), ("true_rel_res", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = C.c_void_p
_SIGS = {
    "sem_space_create": ([C.c_int, C.POINTER(_vp)], C.c_int),
    "sem_space_get": ([_vp, _vp, _vp, _vp], C.c_int),
    "sem_space_destroy": ([_vp], None),
    "sem_box_mesh": ([C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, _vp, _vp, _vp], C.c_int),
    "sem_mesh_create": ([C.c_int64, C.c_int, _vp, _vp, C.POINTER(_vp)], C.c_int),
    "sem_mesh_size": ([_vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "sem_mesh_destroy": ([_vp], None),
    "sem_gs_create": ([_vp, C.POINTER(_vp)], C.c_int),
    "sem_gs_sizes": ([_vp, _vp, _vp, _vp], C.c_int),
    "sem_gs_export_maps": ([_vp, _vp, _vp, _vp, _vp], C.c_int),
    "sem_gs_destroy": ([_vp], None),
    "sem_gs_op": ([_vp, C.c_int, _vp, C.c_int, _vp], C.c_int),
    "sem_mask": ([_vp, C.c_int, _vp, C.c_int, _vp], C.c_int),
    "sem_coef_create": ([_vp, _vp, _vp, C.c_uint, _vp, C.POINTER(_vp)], C.c_int),
    "sem_coef_create_from_G": ([_vp, _vp, _vp, _vp, C.c_uint, _vp, C.POINTER(_vp)], C.c_int),
    "sem_coef_set_helmholtz": ([_vp, _vp, C.c_double, _vp, C.c_double, _vp], C.c_int),
    "sem_coef_export": ([_vp, _vp, _vp, _vp], C.c_int),
    "sem_coef_destroy": ([_vp], None),
    "sem_ax_helm": ([_vp, _vp, _vp, _vp, _vp, C.c_int, C.c_int, _vp], C.c_int),
    "sem_ax_helm_adjoint": ([_vp, _vp, _vp, _vp, _vp, _vp, C.c_int, _vp], C.c_int),
    "sem_jacobi_inverse": ([_vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "sem_pcg_solve": ([_vp, _vp, C.c_int, _vp, _vp, _vp, _vp, C.POINTER(PcgParams),
                       C.POINTER(PcgInfo), _vp], C.c_int),
    "sem_pcg_solve_noalloc": ([_vp, _vp, C.c_int, _vp, _vp, _vp, _vp, C.POINTER(PcgParams),
                               C.POINTER(PcgInfo), _vp], C.c_int),
    "sem_stream_triad": ([_vp, _vp, _vp, C.c_double, C.c_int64, _vp], C.c_int),
    "sem_gmres_solve": ([_vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(GmresParams), C.POINTER(PcgInfo), _vp],
                        C.c_int),
    "sem_schwarz_apply": ([_vp, _vp, _vp, _vp, _vp, _vp, C.c_int, C.c_int, _vp], C.c_int),
    "sem_proj_create": ([_vp, _vp, _vp, _vp, C.c_int, C.POINTER(_vp)], C.c_int),
    "sem_proj_size": ([_vp, _vp, _vp, _vp], C.c_int),
    "sem_proj_reset": ([_vp], C.c_int),
    "sem_proj_project": ([_vp, _vp, _vp, _vp, _vp], C.c_int),
    "sem_proj_update": ([_vp, _vp, _vp, _vp, _vp], C.c_int),
    "sem_proj_solve": ([_vp, _vp, _vp, C.POINTER(PcgParams), C.POINTER(PcgInfo), _vp], C.c_int),
    "sem_proj_destroy": ([_vp], None),
    "sem_last_error": ([], C.c_char_p),
    "sem_version": ([], C.c_char_p),
    "sem_rtol_margin": ([], C.c_double),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2107_01243_amd.build`")
    L = C.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


_L = _load()

# Every solver iterates to RTOL_MARGIN * rtol by its own FP64 true residual
# (SEM_RTOL_MARGIN of sem.h), so other FP64 evaluations of it also meet rtol.
RTOL_MARGIN = float(_L.sem_rtol_margin())


def lib():
    return _L


def _check(status):
    if status != SEM_OK:
        raise SemError(status, _L.sem_last_error().decode(errors="replace"))


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


def _ptr(t):
    return None if t is None else _vp(t.data_ptr())


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(_vp)


def _dtype(t):
    if t.dtype == torch.float64:
        return SEM_F64
    if t.dtype == torch.float32:
        return SEM_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev(t, n=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} values, expected {n}")
    return t


# ---------------------------------------------------------------- handles
class Space:
    """GLL space Xh (Section 2, Eq. 7-9)."""

    def __init__(self, lx: int):
        h = _vp()
        _check(_L.sem_space_create(lx, C.byref(h)))
        self._h = h
        self.lx = lx
        self.xi = np.zeros(lx)
        self.w = np.zeros(lx)
        self.D = np.zeros((lx, lx))
        _check(_L.sem_space_get(h, _np_ptr(self.xi), _np_ptr(self.w), _np_ptr(self.D)))

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "_h", None) and _L is not None:
            _L.sem_space_destroy(self._h)
            self._h = None


def box_mesh(nx: int, ny: int, nz: int, lx: int, eps: float):
    """Synthetic curved box mesh (host arrays): glb int64, dirichlet uint8, xyz (3, n_p)."""
    n = nx * ny * nz * lx ** 3
    glb = np.empty(n, np.int64)
    dr = np.empty(n, np.uint8)
    xyz = np.empty((3, n), np.float64)
    _check(_L.sem_box_mesh(nx, ny, nz, lx, float(eps), _np_ptr(glb), _np_ptr(dr), _np_ptr(xyz)))
    return dict(glb=glb, dirichlet=dr, xyz=xyz)


class Mesh:
    """msh: element count, global ids and Dirichlet flags."""

    def __init__(self, nelv: int, lx: int, glb: np.ndarray, dirichlet: np.ndarray | None = None):
        glb = np.ascontiguousarray(glb, dtype=np.int64)
        if glb.size != nelv * lx ** 3:
            raise ValueError("glb has the wrong length")
        d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
        h = _vp()
        _check(_L.sem_mesh_create(nelv, lx, _np_ptr(glb), _np_ptr(d), C.byref(h)))
        self._h = h
        self.nelv, self.lx, self.n = nelv, lx, glb.size

    def sizes(self):
        v = [C.c_int64(), C.c_int(), C.c_int64(), C.c_int64(), C.c_int64()]
        _check(_L.sem_mesh_size(self._h, *[C.byref(x) for x in v]))
        return dict(nelv=v[0].value, lx=v[1].value, n_local=v[2].value, n_unique=v[3].value,
                    n_dirichlet_local=v[4].value)

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "_h", None) and _L is not None:
            _L.sem_mesh_destroy(self._h)
            self._h = None


class GS:
    """Gather-scatter QQ^T (Eq. 10, Section 3.2)."""

    def __init__(self, msh: Mesh):
        h = _vp()
        _check(_L.sem_gs_create(msh._h, C.byref(h)))
        self._h = h
        self.msh = msh

    def sizes(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(_L.sem_gs_sizes(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def maps(self):
        npairs, nblocks, nbe = self.sizes()
        pairs = np.empty(max(2 * npairs, 1), np.int32)
        ptr = np.empty(nblocks + 1, np.int64)
        idx = np.empty(max(nbe, 1), np.int32)
        mult = np.empty(self.msh.n, np.uint8)
        _check(_L.sem_gs_export_maps(self._h, _np_ptr(pairs), _np_ptr(ptr), _np_ptr(idx), _np_ptr(mult)))
        return pairs[:2 * npairs].reshape(-1, 2), ptr, idx[:nbe], mult

    def op(self, u: torch.Tensor, nfields: int = 1, stream=None):
        """u <- QQ^T u in place."""
        _dev(u, nfields * self.msh.n, "u")
        _check(_L.sem_gs_op(_ptr(u), nfields, self._h, _dtype(u), _stream(stream)))
        return u

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "_h", None) and _L is not None:
            _L.sem_gs_destroy(self._h)
            self._h = None


class Coef:
    """coef: geometric factors G (Eq. 9), mass B, Helmholtz h1 / h2."""

    def __init__(self, Xh: Space, msh: Mesh, xyz: torch.Tensor | None = None,
                 G: torch.Tensor | None = None, B: torch.Tensor | None = None,
                 fp32: bool = False, stream=None):
        h = _vp()
        flags = SEM_COEF_F32 if fp32 else 0
        if xyz is not None:
            _dev(xyz, 3 * msh.n, "xyz")
            _check(_L.sem_coef_create(Xh._h, msh._h, _ptr(xyz), flags, _stream(stream), C.byref(h)))
        else:
            _dev(G, 6 * msh.n, "G")
            _dev(B, msh.n, "B")
            _check(_L.sem_coef_create_from_G(Xh._h, msh._h, _ptr(G), _ptr(B), flags, _stream(stream),
                                             C.byref(h)))
        self._h = h
        self.Xh, self.msh, self.fp32 = Xh, msh, fp32
        self.h1 = 1.0
        self.h2 = 0.0

    def set_helmholtz(self, h1=1.0, h2=0.0, stream=None):
        """h1 / h2: python floats, or FP64 device tensors with n_p values (copied)."""
        n = self.msh.n
        h1p = _ptr(_dev(h1, n, "h1")) if isinstance(h1, torch.Tensor) else None
        h2p = _ptr(_dev(h2, n, "h2")) if isinstance(h2, torch.Tensor) else None
        for t in (h1, h2):
            if isinstance(t, torch.Tensor) and t.dtype != torch.float64:
                raise TypeError("h1/h2 fields must be float64")
        s1 = 0.0 if h1p is not None else float(h1)
        s2 = 0.0 if h2p is not None else float(h2)
        _check(_L.sem_coef_set_helmholtz(self._h, h1p, s1, h2p, s2, _stream(stream)))
        # own copies, so that helmholtz() can restore exactly what the handle holds
        self.h1 = h1.detach().clone() if isinstance(h1, torch.Tensor) else s1
        self.h2 = h2.detach().clone() if isinstance(h2, torch.Tensor) else s2

    def helmholtz(self):
        """(h1, h2) as the handle holds them: floats, or FP64 device tensors (copies)."""
        return self.h1, self.h2

    def export(self, stream=None):
        n = self.msh.n
        G = torch.empty(6 * n, dtype=torch.float64, device="cuda")
        B = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(_L.sem_coef_export(self._h, _ptr(G), _ptr(B), _stream(stream)))
        return G, B

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "_h", None) and _L is not None:
            _L.sem_coef_destroy(self._h)
            self._h = None


# ---------------------------------------------------------------- operators
def ax_helm(w, u, coef: Coef, msh: Mesh, Xh: Space, nfields: int = 1, stream=None):
    """w = A_L u (Eq. 9), unassembled; Listing 1 argument order."""
    _dev(u, nfields * msh.n, "u")
    _dev(w, nfields * msh.n, "w")
    if u.dtype != w.dtype:
        raise TypeError("u and w must share a dtype")
    _check(_L.sem_ax_helm(_ptr(w), _ptr(u), coef._h, msh._h, Xh._h, nfields, _dtype(u), _stream(stream)))
    return w


def ax_helm_adjoint(g, u, v, coef: Coef, msh: Mesh, Xh: Space, stream=None):
    """g_p = (D v)_p^T G_p (D u)_p = d(v^T A_L(h1) u)/d h1_p."""
    for t, nm in ((g, "g"), (u, "u"), (v, "v")):
        _dev(t, msh.n, nm)
    _check(_L.sem_ax_helm_adjoint(_ptr(g), _ptr(u), _ptr(v), coef._h, msh._h, Xh._h, _dtype(u),
                                  _stream(stream)))
    return g


def mask(u, msh: Mesh, nfields: int = 1, stream=None):
    _dev(u, nfields * msh.n, "u")
    _check(_L.sem_mask(_ptr(u), nfields, msh._h, _dtype(u), _stream(stream)))
    return u


def jacobi_inverse(coef: Coef, msh: Mesh, Xh: Space, gs: GS, stream=None):
    d = torch.empty(msh.n, dtype=torch.float64, device="cuda")
    _check(_L.sem_jacobi_inverse(_ptr(d), coef._h, msh._h, Xh._h, gs._h, _stream(stream)))
    return d


MIXED_MODES = {False: 0, True: 1, 0: 0, 1: 1, 2: 2, "fp64": 0, "reliable": 1, "fcg": 2}


def pcg_solve(x, b, coef: Coef, msh: Mesh, Xh: Space, gs: GS, nfields: int = 1, rtol: float = 1e-10,
              max_iter: int = 100000, check_every: int = 25, mixed=False,
              inner_rtol: float = 1e-4, inner_max_iter: int = 2000, use_x0: bool = False,
              delta: float = 0.5, single_reduction: bool = False, stream=None,
              raise_on_fail: bool = True):
    """Solve mask QQ^T A_L x = b (Section 4 Jacobi-PCG).  mixed: False / "fp64" (FP64
    PCG), True / "reliable" (FP32 PCG with FP64 reliable updates), "fcg" (FP64 flexible
    CG around an FP32 Jacobi-PCG).  single_reduction (FP64 only): Chronopoulos-Gear
    form with one reduction phase per iteration.  Returns one info dict per field."""
    _dev(x, nfields * msh.n, "x")
    _dev(b, nfields * msh.n, "b")
    if x.dtype != torch.float64 or b.dtype != torch.float64:
        raise TypeError("x and b must be float64")
    P = PcgParams(float(rtol), int(max_iter), int(check_every), MIXED_MODES[mixed], float(inner_rtol),
                  int(inner_max_iter), int(bool(use_x0)), float(delta), int(bool(single_reduction)))
    info = (PcgInfo * nfields)()
    st = _L.sem_pcg_solve(_ptr(x), _ptr(b), nfields, coef._h, msh._h, Xh._h, gs._h, C.byref(P), info,
                          _stream(stream))
    out = [info[f].as_dict() for f in range(nfields)]
    for d in out:
        d["status"] = st
    if st != SEM_OK and raise_on_fail:
        raise SemError(st, _L.sem_last_error().decode(errors="replace"))
    return out


def pcg_solve_noalloc(x, b, coef: Coef, msh: Mesh, Xh: Space, gs: GS, nfields: int = 1, rtol: float = 1e-10,
                      max_iter: int = 100000, check_every: int = 25, use_x0: bool = False, stream=None,
                      raise_on_fail: bool = True):
    """The FP64 Jacobi-PCG solve of pcg_solve on the library's fixed device workspace
    (no device allocation; n_p * nfields <= NOALLOC_MAX_POINTS; the gs handle must
    already be resident, e.g. after one gs_op).  Returns one info dict per field."""
    _dev(x, nfields * msh.n, "x")
    _dev(b, nfields * msh.n, "b")
    if x.dtype != torch.float64 or b.dtype != torch.float64:
        raise TypeError("x and b must be float64")
    P = PcgParams(float(rtol), int(max_iter), int(check_every), 0, 1e-4, 1, int(bool(use_x0)), 0.0, 0)
    info = (PcgInfo * nfields)()
    st = _L.sem_pcg_solve_noalloc(_ptr(x), _ptr(b), nfields, coef._h, msh._h, Xh._h, gs._h, C.byref(P), info,
                                  _stream(stream))
    out = [info[f].as_dict() for f in range(nfields)]
    for d in out:
        d["status"] = st
    if st != SEM_OK and raise_on_fail:
        raise SemError(st, _L.sem_last_error().decode(errors="replace"))
    return out


# SEM_NOALLOC_MAX_POINTS of sem.h
NOALLOC_MAX_POINTS = 1 << 21

GMRES_PRECOND = {"jacobi": 0, "schwarz": 1, "schwarz_overlap": 2}


def gmres_solve(x, b, coef: Coef, msh: Mesh, Xh: Space, gs: GS, rtol: float = 1e-10, max_iter: int = 100000,
                restart: int = 30, precond: str = "jacobi", use_x0: bool = False, coarse_iters: int = 10,
                stream=None, raise_on_fail: bool = True):
    """Flexible GMRES(restart) for mask QQ^T A_L x = b (the paper's pressure Krylov
    solver, Section 4).  Returns an info dict (iters = Arnoldi steps, inner_iters =
    cycles)."""
    _dev(x, msh.n, "x")
    _dev(b, msh.n, "b")
    if x.dtype != torch.float64 or b.dtype != torch.float64:
        raise TypeError("x and b must be float64")
    P = GmresParams(float(rtol), int(max_iter), int(restart), GMRES_PRECOND[precond], int(bool(use_x0)),
                    int(coarse_iters))
    info = PcgInfo()
    st = _L.sem_gmres_solve(_ptr(x), _ptr(b), coef._h, msh._h, Xh._h, gs._h, C.byref(P), C.byref(info),
                            _stream(stream))
    d = info.as_dict()
    d["status"] = st
    if st != SEM_OK and raise_on_fail:
        raise SemError(st, _L.sem_last_error().decode(errors="replace"))
    return d


def schwarz_apply(z, r, coef: Coef, msh: Mesh, Xh: Space, gs: GS, coarse_iters: int = 10, overlap: bool = False,
                  stream=None):
    """z = M0^{-1} r, the two-level additive Schwarz preconditioner (Section 4); with
    overlap, the local problems extend one point into the face neighbours."""
    _dev(z, msh.n, "z")
    _dev(r, msh.n, "r")
    _check(_L.sem_schwarz_apply(_ptr(z), _ptr(r), coef._h, msh._h, Xh._h, gs._h, int(coarse_iters),
                                int(bool(overlap)), _stream(stream)))
    return z


class Projection:
    """Space of up to max_vectors previous solutions of one scalar system, used for
    initial guesses (Section 4 and Table 2: 20 previous pressure solutions)."""

    def __init__(self, coef: Coef, msh: Mesh, Xh: Space, gs: GS, max_vectors: int = 20):
        h = _vp()
        _check(_L.sem_proj_create(coef._h, msh._h, Xh._h, gs._h, int(max_vectors), C.byref(h)))
        self._h = h
        self._keep = (coef, msh, Xh, gs)   # the handle points at these
        self.n = msh.n

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "_h", None) and _L is not None:
            _L.sem_proj_destroy(self._h)
            self._h = None

    def size(self):
        """(vectors held, capacity, restarts)."""
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        _check(_L.sem_proj_size(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def reset(self):
        _check(_L.sem_proj_reset(self._h))

    def project(self, b, stream=None):
        """(x0, r = b - A x0): best A-norm approximation of A^{-1} b from the space."""
        _dev(b, self.n, "b")
        x0 = torch.empty_like(b)
        r = torch.empty_like(b)
        _check(_L.sem_proj_project(self._h, _ptr(x0), _ptr(r), _ptr(b), _stream(stream)))
        return x0, r

    def update(self, x, x0, stream=None) -> bool:
        """Add the solution x (whose projection was x0); False if it added nothing."""
        _dev(x, self.n, "x")
        _dev(x0, self.n, "x0")
        added = C.c_int()
        _check(_L.sem_proj_update(self._h, _ptr(x), _ptr(x0), C.byref(added), _stream(stream)))
        return bool(added.value)

    def solve(self, b, rtol: float = 1e-10, max_iter: int = 100000, check_every: int = 25, mixed=False,
              inner_rtol: float = 1e-4, inner_max_iter: int = 2000, delta: float = 0.5, stream=None,
              raise_on_fail: bool = True):
        """x = x0 + dx with A dx = b - A x0 solved by PCG; x joins the space."""
        _dev(b, self.n, "b")
        x = torch.empty_like(b)
        P = PcgParams(float(rtol), int(max_iter), int(check_every), MIXED_MODES[mixed], float(inner_rtol),
                      int(inner_max_iter), 0, float(delta))
        info = PcgInfo()
        st = _L.sem_proj_solve(_ptr(x), _ptr(b), self._h, C.byref(P), C.byref(info), _stream(stream))
        d = info.as_dict()
        d["status"] = st
        if st != SEM_OK and raise_on_fail:
            raise SemError(st, _L.sem_last_error().decode(errors="replace"))
        return x, d


def stream_triad(a, b, c, s: float, stream=None):
    """a = b + s c (FP64 device vectors): the STREAM-triad bandwidth probe."""
    for t, nm in ((a, "a"), (b, "b"), (c, "c")):
        _dev(t, a.numel(), nm)
        if t.dtype != torch.float64:
            raise TypeError("triad vectors must be float64")
    _check(_L.sem_stream_triad(_ptr(a), _ptr(b), _ptr(c), float(s), a.numel(), _stream(stream)))
    return a


# ---------------------------------------------------------------- convenience
@dataclass
class BoxProblem:
    """A synthetic curved box problem resident on the current GPU."""
    Xh: Space
    msh: Mesh
    gs: GS
    coef: Coef
    xyz: torch.Tensor      # (3, n_p) FP64 device
    glb: np.ndarray
    dirichlet: np.ndarray
    nx: int
    lx: int

    @property
    def n(self):
        return self.msh.n

    @property
    def mult(self):
        """Multiplicity of every local point (FP64 device tensor, cached)."""
        m = getattr(self, "_mult", None)
        if m is None:
            m = torch.from_numpy(self.gs.maps()[3].astype(np.float64)).to("cuda")
            self._mult = m
        return m

    @classmethod
    def build(cls, nx: int, lx: int, eps: float = 0.05, fp32: bool = False, ny=None, nz=None):
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        Xh = Space(lx)
        m = box_mesh(nx, ny, nz, lx, eps)
        msh = Mesh(nx * ny * nz, lx, m["glb"], m["dirichlet"])
        gs = GS(msh)
        xyz = torch.from_numpy(m["xyz"]).to("cuda")
        coef = Coef(Xh, msh, xyz=xyz, fp32=fp32)
        return cls(Xh, msh, gs, coef, xyz, m["glb"], m["dirichlet"], nx, lx)

    def ax(self, u, nfields=1, out=None):
        w = torch.empty_like(u) if out is None else out
        return ax_helm(w, u, self.coef, self.msh, self.Xh, nfields)

    def apply(self, u, nfields=1):
        """mask QQ^T A_L u."""
        w = self.ax(u, nfields)
        self.gs.op(w, nfields)
        return mask(w, self.msh, nfields)

    def assemble(self, f_local, nfields=1):
        """b = mask QQ^T f (copy)."""
        b = f_local.clone()
        self.gs.op(b, nfields)
        return mask(b, self.msh, nfields)

    def solve(self, b, nfields=1, **kw):
        x = torch.zeros_like(b)
        info = pcg_solve(x, b, self.coef, self.msh, self.Xh, self.gs, nfields=nfields, **kw)
        return x, info

    def adjoint(self, u, v):
        g = torch.empty_like(u)
        return ax_helm_adjoint(g, u, v, self.coef, self.msh, self.Xh)

    def gmres(self, b, **kw):
        x = torch.zeros_like(b)
        info = gmres_solve(x, b, self.coef, self.msh, self.Xh, self.gs, **kw)
        return x, info

    def projection(self, max_vectors: int = 20) -> Projection:
        return Projection(self.coef, self.msh, self.Xh, self.gs, max_vectors)
