"""CPU-only checks of libsem: exported symbols, host-side setup and error paths.

No kernel is launched here.  The GLL space, the synthetic box mesh and the
gather-scatter maps are host code in the library, so they are compared with the
oracle on the CPU (maps bit-exact, including the 32^3 x lx=8 mesh at full size).
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sem.h")
LIB = os.path.join(ROOT, "paper_2107_01243_amd", "libsem.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsem.so not built")


@pytest.fixture(scope="module")
def L():
    from paper_2107_01243_amd import sem
    return sem.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sem_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 20
    for nm in names:
        assert hasattr(L, nm), nm


def test_version_and_error_string(L):
    assert L.sem_version().startswith(b"libsem")
    sp = C.c_void_p()
    assert L.sem_space_create(1, C.byref(sp)) == -1
    assert b"lx=1" in L.sem_last_error()
    assert L.sem_space_create(17, C.byref(sp)) == -1


@pytest.mark.parametrize("lx", range(2, 17))
def test_space_matches_oracle(lx):
    from paper_2107_01243_amd import sem
    Xh = sem.Space(lx)
    xi, w = oracle.gll(lx)
    D = oracle.deriv_matrix(xi)
    np.testing.assert_allclose(Xh.xi, xi, rtol=0, atol=2e-16)
    np.testing.assert_allclose(Xh.w, w, rtol=0, atol=4e-16)
    assert np.abs(Xh.D - D).max() <= 1e-14 * np.abs(D).max()


@pytest.mark.parametrize("nx,ny,nz,lx,eps", [(4, 4, 4, 6, 0.0), (3, 2, 5, 8, 0.05), (2, 2, 2, 12, 0.05), (1, 1, 1, 2, 0.05)])
def test_box_mesh_matches_oracle(nx, ny, nz, lx, eps):
    from paper_2107_01243_amd import sem
    m = sem.box_mesh(nx, ny, nz, lx, eps)
    o = oracle.box_mesh(nx, ny, nz, lx, eps)
    np.testing.assert_array_equal(m["glb"], o["glb"])
    np.testing.assert_array_equal(m["dirichlet"], o["dirichlet"])
    for c, nm in enumerate("xyz"):
        np.testing.assert_allclose(m["xyz"][c], o[nm], rtol=0, atol=4e-16)


def _oracle_split(glb):
    """Oracle groups split into the library's pair / block lists."""
    gs = oracle.GS(glb)
    off, idx, _ = gs.groups()
    sizes = np.diff(off)
    two = np.flatnonzero(sizes == 2)
    pairs = np.stack([idx[off[two]], idx[off[two] + 1]], axis=1) if len(two) else np.zeros((0, 2), np.int64)
    big = np.flatnonzero(sizes > 2)
    blk_idx = np.concatenate([idx[off[g]:off[g + 1]] for g in big]) if len(big) else np.zeros(0, np.int64)
    blk_ptr = np.concatenate([[0], np.cumsum(sizes[big])])
    return pairs, blk_ptr, blk_idx, gs.mult()


def _check_maps(glb, dirichlet, nelv, lx):
    from paper_2107_01243_amd import sem
    msh = sem.Mesh(nelv, lx, glb, dirichlet)
    gs = sem.GS(msh)
    pairs, ptr, idx, mult = gs.maps()
    opairs, optr, oidx, omult = _oracle_split(glb)
    np.testing.assert_array_equal(pairs, opairs)
    np.testing.assert_array_equal(ptr, optr)
    np.testing.assert_array_equal(idx, oidx)
    np.testing.assert_array_equal(mult, omult.astype(np.uint8))
    return msh, gs


@pytest.mark.parametrize("nx,lx", [(4, 6), (3, 8), (2, 12), (1, 5), (5, 3)])
def test_gs_maps_bit_exact(nx, lx):
    m = oracle.box_mesh(nx, nx, nx, lx, 0.05)
    _check_maps(m["glb"], m["dirichlet"], nx ** 3, lx)


def test_gs_maps_full_size_32cubed_lx8():
    m = oracle.box_mesh(32, 32, 32, 8, 0.05)
    msh, gs = _check_maps(m["glb"], m["dirichlet"], 32 ** 3, 8)
    npairs, nblocks, nbe = gs.sizes()
    assert npairs == 3500148
    assert nblocks == 559302 + 29791
    assert nbe == 4 * 559302 + 8 * 29791
    s = msh.sizes()
    assert s["n_unique"] == 11390625 and s["n_local"] == 16777216


def test_gs_maps_general_ids():
    """Scrambled, sparse global ids exercise the comparison-sort path."""
    m = oracle.box_mesh(3, 3, 3, 4, 0.0)
    rng = np.random.default_rng(4)
    ids = np.unique(m["glb"])
    relabel = dict(zip(ids, rng.choice(10 ** 12, len(ids), replace=False)))
    glb = np.array([relabel[g] for g in m["glb"]], np.int64)
    _check_maps(glb, None, 27, 4)


def test_host_error_paths():
    from paper_2107_01243_amd import sem
    m = oracle.box_mesh(2, 2, 2, 4, 0.0)
    with pytest.raises(sem.SemError, match="INVALID"):
        sem.Mesh(8, 4, np.where(np.arange(512) == 3, -1, m["glb"]), None)
    bad = m["dirichlet"].copy()
    g0 = m["glb"][np.flatnonzero(np.bincount(m["glb"])[m["glb"]] >= 2)[0]]
    copies = np.flatnonzero(m["glb"] == g0)
    bad[copies[0]] = 1 - bad[copies[1]]
    msh = sem.Mesh(8, 4, m["glb"], bad)
    with pytest.raises(sem.SemError, match="Dirichlet"):
        sem.GS(msh)
    many = np.zeros(4 ** 3 * 5, np.int64)   # 320 copies of one id
    with pytest.raises(sem.SemError, match="255"):
        sem.GS(sem.Mesh(5, 4, many, None))
    with pytest.raises(sem.SemError):
        sem.box_mesh(2, 2, 2, 20, 0.0)
    with pytest.raises(sem.SemError):
        sem.box_mesh(0, 2, 2, 4, 0.0)
