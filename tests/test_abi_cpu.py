"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/dg.h declares, rejects bad meshes before any HIP call, and its
host-built reference tables (quadrature rules and basis) agree with the
oracle's independently built ones."""
import os
import re

import numpy as np
import pytest

import oracle as O
from oracle import quadrature as Q
from paper_1601_07944_amd import binding as B
from paper_1601_07944_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "dg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = B.load()
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTS) == names


def good_mesh():
    return W.square_mesh(3, 1.0, 0.1, 0)


def test_validate_accepts_good_meshes():
    for m in (good_mesh(), W.delaunay_mesh(50, 3), W.square_mesh(1, 1.0, 0.0, 0)):
        assert B.validate(2, m.vxy, m.nbr_elem, m.nbr_side) == 0, B.last_error()


def test_validate_rejects_bad_order():
    m = good_mesh()
    for p in (0, 6, -1):
        assert B.validate(p, m.vxy, m.nbr_elem, m.nbr_side) == -3


def test_validate_rejects_clockwise_element():
    m = good_mesh()
    v = m.vxy.copy()
    v[4] = v[4][[0, 2, 1]]
    assert B.validate(1, v, m.nbr_elem, m.nbr_side) == -2
    assert "element 4" in B.last_error()


def test_validate_rejects_asymmetric_neighbours():
    m = good_mesh()
    nb = m.nbr_elem.copy()
    nb[0, 0], nb[0, 1] = nb[0, 1], nb[0, 0]
    assert B.validate(1, m.vxy, nb, m.nbr_side) == -2


def test_validate_rejects_mismatched_edge():
    m = good_mesh()
    v = m.vxy.copy()
    v[0, 0, 0] += 1e-3  # move one copy of a shared vertex
    assert B.validate(1, v, m.nbr_elem, m.nbr_side) == -2


def test_validate_boundary_codes():
    # box meshes with every kind of boundary are accepted; unknown codes are not
    box = W.box_mesh(5, 4, 1.0, 1.0, 0.2, 1, bc=(W.BC_WALL, W.BC_OUTFLOW, W.BC_STATE, W.BC_WALL))
    assert B.validate(2, box.vxy, box.nbr_elem, box.nbr_side) == 0
    nb = box.nbr_elem.copy()
    nb[nb == W.BC_OUTFLOW] = -4
    assert B.validate(2, box.vxy, nb, box.nbr_side) == -4
    # an interior side may not be half of a boundary: the neighbour must point back
    m = good_mesh()
    nb = m.nbr_elem.copy()
    nb[2, 1] = -1
    assert B.validate(1, m.vxy, nb, m.nbr_side) == -2


def test_validate_rejects_out_of_range():
    m = good_mesh()
    nb = m.nbr_elem.copy()
    nb[2, 1] = 10**6
    assert B.validate(1, m.vxy, nb, m.nbr_side) == -2
    ns = m.nbr_side.copy()
    ns[1, 1] = 3
    assert B.validate(1, m.vxy, m.nbr_elem, ns) == -2


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_library_tables_match_oracle(p):
    t = B.reference_tables(p)
    r, s, w = Q.triangle_rule(p)
    # same rule (point order may differ): match points
    key_lib = np.array(sorted(zip(t["r"], t["s"], t["w"])))
    key_orc = np.array(sorted(zip(r, s, w)))
    assert np.abs(key_lib - key_orc).max() < 1e-15
    gx, gw = Q.gauss_legendre(p + 1)
    assert np.abs(t["gx"] - gx).max() < 1e-15 and np.abs(t["gw"] - gw).max() < 1e-15
    assert np.all(t["gx"][::-1] == -t["gx"]) and np.all(t["gw"][::-1] == t["gw"])
    phi, dr, ds = O.basis(p, t["r"], t["s"])
    assert np.abs(t["phi"] - phi).max() < 1e-13
    assert np.abs(t["dphidr"] - dr).max() < 1e-12
    assert np.abs(t["dphids"] - ds).max() < 1e-12
    for q in range(3):
        x = t["gx"]
        rr, ss = {0: ((1 + x) / 2, 0 * x), 1: ((1 - x) / 2, (1 + x) / 2), 2: (0 * x, (1 - x) / 2)}[q]
        assert np.abs(t["phi_side"][q] - O.basis(p, rr, ss)[0]).max() < 1e-13


def test_validate_rejects_empty_mesh():
    # zero elements: an error, not an empty operator
    empty = np.zeros((0, 3, 2))
    assert B.validate(1, empty, np.zeros((0, 3), dtype=np.int64), np.zeros((0, 3), dtype=np.int8)) == -1


def test_validate_rejects_degenerate_element():
    # a triangle of zero area (collinear vertices) is rejected like an
    # inverted one
    m = good_mesh()
    v = m.vxy.copy()
    v[0, 2] = 0.5 * (v[0, 0] + v[0, 1])
    assert B.validate(1, v, m.nbr_elem, m.nbr_side) == -2


def test_null_and_bad_arguments_are_errors_not_crashes():
    lib = B.load()
    import ctypes

    out = ctypes.c_void_p()
    m = good_mesh()
    vxy = np.ascontiguousarray(m.vxy)
    # null arrays
    assert lib.dg_mesh_create(1, m.n_elem, None, None, None, 1.4, ctypes.byref(out)) == -1
    # order outside 1..5 is rejected before any device call
    nb = np.ascontiguousarray(m.nbr_elem, dtype=np.int64)
    ns = np.ascontiguousarray(m.nbr_side, dtype=np.int8)
    assert lib.dg_mesh_create(6, m.n_elem, vxy.ctypes.data, nb.ctypes.data, ns.ctypes.data, 1.4, ctypes.byref(out)) == -3
    # the entry points refuse a null mesh
    assert lib.dg_rhs(None, None, None, 0, None, None) == -1
    assert lib.dg_set_surface_mode(None, 0) == -1
    assert lib.dg_set_stream_concurrency(None, 1) == -1
    assert lib.dg_set_boundary_state(None, None) == -1
    assert b"null" in lib.dg_last_error()


def test_binding_fails_loudly_without_the_library(tmp_path):
    # no CPU fallback: a missing library is an error
    saved = B._lib
    B._lib = None
    try:
        with pytest.raises(RuntimeError):
            B.load(str(tmp_path / "libdgmi.so"))
    finally:
        B._lib = saved
