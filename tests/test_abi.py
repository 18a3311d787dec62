"""The C-ABI library loads and exports every function declared in
include/ibvt.h; host-only calls behave (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ibvt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^(?:int|void|const char\s*\*)\s*(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1810_13046_amd import ibvt
    return ibvt.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    from paper_1810_13046_amd import ibvt
    assert sorted(ibvt.EXPORTED) == names


def test_exported_set_equals_declared_set(lib):
    """The library's dynamic symbol table holds the declared calls and
    nothing else (no internal helper is reachable through the ABI)."""
    import shutil
    import subprocess
    from paper_1810_13046_amd import ibvt
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-D", "--defined-only", ibvt.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines()
                       if len(ln.split()) >= 3 and ln.split()[1] in ("T", "W", "D", "B", "V")})
    assert exported == declared_functions()


def test_status_strings(lib):
    for st in range(8):
        assert lib.ibvt_status_string(st)
    assert lib.ibvt_status_string(0) == b"ok"


def test_lattice_coords_follow_staggering(oracle_mod):
    """Host-side lattice of each component equals the oracle's reading of
    the staggered grid (faces along d, midpoints elsewhere)."""
    import workloads as wl
    from paper_1810_13046_amd import lattice_coords
    faces = [wl.uniform_faces(8), wl.stretched_faces(12, 4.0), wl.uniform_faces(5, 0.0, 2.0)]
    for d in range(3):
        got = lattice_coords(faces, d)
        want = oracle_mod.lattice(faces, d)
        for e in range(3):
            assert np.array_equal(got[e], want[e])


def test_invalid_arguments_rejected_on_host(lib):
    from paper_1810_13046_amd import ibvt
    out = ctypes.c_void_p()
    # NULL grid
    st = lib.assemble_coupling(None, None, 0, 0, None, ctypes.byref(out))
    assert st == 1 and not out.value
    # non-increasing faces
    faces = [np.array([0.0, 0.5, 0.4, 1.0]), np.linspace(0, 1, 4), np.linspace(0, 1, 4)]
    g, keep = ibvt._grid_struct(faces)
    m = ibvt._Mesh()
    m.n_vert, m.n_tet, m.X, m.tets = 4, 1, 8, 8   # never dereferenced: grid fails first
    st = lib.assemble_coupling(ctypes.byref(g), ctypes.byref(m), 0, 0, None, ctypes.byref(out))
    assert st == 1
    assert b"increasing" in lib.ibvt_last_error()
    # bad precision on a valid grid
    faces = [np.linspace(0, 1, 4)] * 3
    g, keep = ibvt._grid_struct(faces)
    st = lib.assemble_coupling(ctypes.byref(g), ctypes.byref(m), 7, 0, None, ctypes.byref(out))
    assert st == 1
    # too few cells for the cell-centre lattices
    faces = [np.array([0.0, 1.0]), np.linspace(0, 1, 4), np.linspace(0, 1, 4)]
    g, keep = ibvt._grid_struct(faces)
    n = ctypes.c_int64()
    assert lib.ibvt_lattice_coords(ctypes.byref(g), 0, 0, None, ctypes.byref(n)) == 1
    # NULL handle
    assert lib.coupling_info(None, None) == 1
    lib.coupling_free(None)


def test_planar_lattice_coords_follow_staggering(oracle_mod):
    """Planar lattices (ibvt_lattice_coords_2d) equal the 2D oracle's."""
    from oracle import plane
    import workloads as wl
    from paper_1810_13046_amd import lattice_coords
    faces = [wl.uniform_faces(9), wl.stretched_faces(7, 3.0, -1.0, 1.0)]
    for d in range(2):
        got = lattice_coords(faces, d)
        want = plane.lattice(faces, d)
        assert len(got) == 2
        for e in range(2):
            assert np.array_equal(got[e], want[e])


def test_planar_invalid_arguments_rejected_on_host(lib):
    from paper_1810_13046_amd import ibvt
    out = ctypes.c_void_p()
    assert lib.assemble_coupling_2d(None, None, 0, 0, None, ctypes.byref(out)) == 1
    faces = [np.array([0.0, 0.5, 0.4, 1.0]), np.linspace(0, 1, 4)]
    g, keep = ibvt._grid_struct(faces)
    m = ibvt._Mesh2d()
    m.n_vert, m.n_tri, m.X, m.tris = 3, 1, 8, 8   # never dereferenced: grid fails first
    assert lib.assemble_coupling_2d(ctypes.byref(g), ctypes.byref(m), 0, 0, None,
                                    ctypes.byref(out)) == 1
    assert b"increasing" in lib.ibvt_last_error()
    faces = [np.linspace(0, 1, 4)] * 2
    g, keep = ibvt._grid_struct(faces)
    assert lib.assemble_coupling_2d(ctypes.byref(g), ctypes.byref(m), 7, 0, None,
                                    ctypes.byref(out)) == 1
    assert lib.assemble_coupling_2d(ctypes.byref(g), ctypes.byref(m), 0, 64, None,
                                    ctypes.byref(out)) == 1
    n = ctypes.c_int64()
    assert lib.ibvt_lattice_coords_2d(ctypes.byref(g), 2, 0, None, ctypes.byref(n)) == 1
    assert not out.value
