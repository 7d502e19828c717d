"""The C-ABI library loads on a host without a GPU and exports every entry
point declared in include/hts.h (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2103_00081_amd", "libhts.so")
HDR = os.path.join(ROOT, "include", "hts.h")


def declared():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"\b(hts_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["hts_create_mesh", "hts_set_materials", "hts_apply_operator", "hts_solve_step",
                 "hts_advance"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libhts.so missing: run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_exports():
    import paper_2103_00081_amd as hts
    assert sorted(hts.EXPORTS) == declared()
    L = hts.load()
    o = hts.default_opts()
    assert o.rtol == 1e-8 and o.gmres_restart == 30


def test_error_paths_without_device():
    """Argument validation happens before any device work."""
    import paper_2103_00081_amd as hts
    L = hts.load()
    h = ctypes.c_void_p()
    assert L.hts_create_mesh(None, ctypes.byref(h)) == -1
    d = hts.MeshDesc()
    d.degree = 3
    assert L.hts_create_mesh(ctypes.byref(d), ctypes.byref(h)) == -1
    assert b"degree" in L.hts_last_error()
    assert L.hts_apply_operator(None, 0, 0, 1.0, None, None) == -1


def test_graded_mesh_validation_without_device():
    """Graded axes must span the box with strictly increasing edges."""
    import numpy as np
    import paper_2103_00081_amd as hts
    L = hts.load()
    h = ctypes.c_void_p()

    def desc(edges_x, degree=1):
        d = hts.MeshDesc()
        d.degree = degree
        for k in range(3):
            d.origin[k] = 0.0
            d.extent[k] = 10.0
            d.ncells[k] = 4
        d.edges[0] = edges_x.ctypes.data
        return d

    bad_order = np.array([0.0, 3.0, 2.0, 6.0, 10.0])
    assert L.hts_create_mesh(ctypes.byref(desc(bad_order)), ctypes.byref(h)) == -1
    assert b"increase" in L.hts_last_error()
    short = np.array([0.0, 1.0, 2.0, 6.0, 9.0])
    assert L.hts_create_mesh(ctypes.byref(desc(short)), ctypes.byref(h)) == -1
    assert b"span" in L.hts_last_error()


def test_mesh_size_limit_without_device():
    """A mesh with 2^29 nodes or more is refused before any device work (the
    operator kernels address one FP64 vector with 32-bit byte offsets)."""
    import paper_2103_00081_amd as hts
    L = hts.load()
    h = ctypes.c_void_p()
    d = hts.MeshDesc()
    d.degree = 1
    for k, n in enumerate((1000, 1000, 600)):   # 1001 * 1001 * 601 > 2^29 nodes
        d.origin[k] = 0.0
        d.extent[k] = 100.0
        d.ncells[k] = n
    assert L.hts_create_mesh(ctypes.byref(d), ctypes.byref(h)) == -1
    assert b"too large" in L.hts_last_error()


def test_hexahedral_mesh_validation_without_device():
    """Node coordinates need degree 1 and no graded edges; every cell must
    have det J > 0 at its Gauss points and finite coordinates.  All refused
    before any device work."""
    import numpy as np
    import paper_2103_00081_amd as hts
    import synth
    L = hts.load()
    h = ctypes.c_void_p()
    n = (4, 3, 2)

    def desc(xyz, degree=1, edges=None):
        d = hts.MeshDesc()
        d.degree = degree
        for k in range(3):
            d.origin[k] = 0.0
            d.extent[k] = 10.0
            d.ncells[k] = n[k]
        d.coords = xyz.ctypes.data
        if edges is not None:
            d.edges[0] = edges.ctypes.data
        return d

    xyz = np.ascontiguousarray(synth.terrain_coords((0.0, 0.0, 0.0), (10.0, 10.0, 10.0), n,
                                                    top_amp=1.0, bottom_amp=0.5))
    assert L.hts_create_mesh(ctypes.byref(desc(xyz, degree=2)), ctypes.byref(h)) == -1
    assert b"degree 1" in L.hts_last_error()
    edges = np.linspace(0.0, 10.0, n[0] + 1)
    assert L.hts_create_mesh(ctypes.byref(desc(xyz, edges=edges)), ctypes.byref(h)) == -1
    assert b"either" in L.hts_last_error()
    # swap two node planes: every cell between them turns inside out
    inv = xyz.reshape(n[2] + 1, -1, 3).copy()
    inv[[0, 1]] = inv[[1, 0]]
    inv = np.ascontiguousarray(inv.reshape(-1, 3))
    assert L.hts_create_mesh(ctypes.byref(desc(inv)), ctypes.byref(h)) == -1
    assert b"inverted" in L.hts_last_error()
    bad = xyz.copy()
    bad[5, 1] = np.nan
    assert L.hts_create_mesh(ctypes.byref(desc(bad)), ctypes.byref(h)) == -1
    assert b"finite" in L.hts_last_error()
