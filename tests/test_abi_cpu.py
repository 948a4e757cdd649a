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


def test_validate_rejects_meshes_beyond_32bit_indexing():
    # the kernels index per-element arrays with 32-bit offsets: a mesh whose
    # largest padded field offset reaches 2^31 is refused before any array
    # is read (so tiny placeholder arrays are enough here)
    v = np.zeros((1, 3, 2))
    nb = np.zeros((1, 3), dtype=np.int64)
    ns = np.zeros((1, 3), dtype=np.int8)
    lib = B.load()
    for p in (1, 3, 5):
        np_ = (p + 1) * (p + 2) // 2
        per_elem = max(4 * np_, 12 * (p + 1))
        n_bad = (2**31) // per_elem + 64
        assert lib.dg_mesh_validate(p, n_bad, v.ctypes.data, nb.ctypes.data, ns.ctypes.data) == -4
        assert "32-bit" in B.last_error()
    # and an element count beyond int32 altogether
    assert lib.dg_mesh_validate(1, 2**31 + 5, v.ctypes.data, nb.ctypes.data, ns.ctypes.data) == -4


class _FakeMesh(B.DGMesh):
    """A DGMesh whose argument checks can run without a GPU: no library
    handle (any call that got past the checks would fail on it)."""

    def __init__(self, n=10, p=2):
        import torch

        np_ = (p + 1) * (p + 2) // 2
        npad = (n + 63) // 64 * 64
        info = B.dg_info()
        info.p, info.n_modes, info.n_vol_points, info.n_edge_points = p, np_, 6, p + 1
        info.n_elem, info.n_elem_pad, info.state_len = n, npad, npad * 4 * np_
        info.ws_rhs, info.ws_step, info.ws_vjp = 1000, 2000, 3000
        self.info, self.p, self.n, self.np, self.nq = info, p, n, np_, 6
        self.device = torch.device("cpu")
        self._h = None
        self._lib = None
        self._ws = None

    def close(self):
        pass


def test_binding_rejects_bad_tensors_before_any_launch():
    import torch

    dm = _FakeMesh()
    good = torch.zeros(dm.info.state_len, dtype=torch.float64)
    bad = [
        ("float32", torch.zeros(dm.info.state_len, dtype=torch.float32)),
        ("short", torch.zeros(dm.info.state_len - 1, dtype=torch.float64)),
        ("user layout", torch.zeros(dm.n * 4 * dm.np, dtype=torch.float64)),
        ("strided", torch.zeros(2 * dm.info.state_len, dtype=torch.float64)[::2]),
        ("meta device", torch.zeros(dm.info.state_len, dtype=torch.float64, device="meta")),
    ]
    calls = [
        lambda t: dm.rhs(t, out=good, ws=torch.zeros(1000, dtype=torch.uint8)),
        lambda t: dm.rhs(good, out=t, ws=torch.zeros(1000, dtype=torch.uint8)),
        lambda t: dm.rk_step(t, 0.1, ws=torch.zeros(2000, dtype=torch.uint8)),
        lambda t: dm.advance(t, 3, 0.1, dt_dev=torch.zeros(1, dtype=torch.float64),
                             ws=torch.zeros(2000, dtype=torch.uint8)),
        lambda t: dm.max_dt(t, 0.1, dt_dev=torch.zeros(1, dtype=torch.float64),
                            ws=torch.zeros(1000, dtype=torch.uint8)),
        lambda t: dm.rhs_vjp(good, t, out=good),
        lambda t: dm.rk_step_vjp(good, t, 0.1, out=good, ws=torch.zeros(3000, dtype=torch.uint8)),
        lambda t: dm.rk_step_stages(good, t, good, 0.1, ws=torch.zeros(2000, dtype=torch.uint8)),
        lambda t: dm.limit(t),
        lambda t: dm.unpack(t),
        lambda t: dm.eval_points(t),
    ]
    for call in calls:
        for name, t in bad:
            with pytest.raises(ValueError):
                call(t)
    # user-layout arguments and the small ones
    with pytest.raises(ValueError):
        dm.pack(torch.zeros(dm.n * 4 * dm.np, dtype=torch.float32), out=good)
    with pytest.raises(ValueError):
        dm.pack(torch.zeros(dm.n * 4 * dm.np + 1, dtype=torch.float64), out=good)
    with pytest.raises(ValueError):
        dm.project(torch.zeros(dm.n * dm.nq * 4, dtype=torch.float32), out=good)
    with pytest.raises(ValueError):
        dm.unpack(good, out=torch.zeros(dm.n * 4 * dm.np - 1, dtype=torch.float64))
    with pytest.raises(ValueError):  # workspace too small
        dm.rk_step(good, 0.1, ws=torch.zeros(1999, dtype=torch.uint8))
    with pytest.raises(ValueError):  # a step-length history shorter than the steps
        dm.advance(good, 3, 0.1, dt_dev=torch.zeros(1, dtype=torch.float64), dt_hist=torch.zeros(2, dtype=torch.float64),
                   ws=torch.zeros(2000, dtype=torch.uint8))
    with pytest.raises(ValueError):
        dm.advance(good, -1, 0.1)
    with pytest.raises(ValueError):  # one stage state without the other
        dm.rk_step_vjp(good, good, 0.1, u1=good, out=good, ws=torch.zeros(3000, dtype=torch.uint8))
    with pytest.raises(ValueError):
        B.check_tensor(np.zeros(3), "x", torch.device("cpu"))


def test_stale_library_is_detected(monkeypatch, tmp_path):
    # ensure_built() rebuilds unless the library was built from exactly the
    # current sources: the recorded hash is compared, not file times
    from paper_1601_07944_amd import build as Bd

    lib = tmp_path / "libdgmi.so"
    stamp = tmp_path / "libdgmi.so.sources.json"
    lib.write_bytes(b"")
    monkeypatch.setattr(Bd, "LIB", str(lib))
    monkeypatch.setattr(Bd, "STAMP", str(stamp))
    calls = []
    monkeypatch.setattr(Bd, "build", lambda *a, **k: calls.append(1) or str(lib))
    assert Bd.built_hash() is None
    Bd.ensure_built()  # no record of its sources
    assert calls == [1]
    stamp.write_text('{"source_sha256_16": "0000000000000000"}')
    Bd.ensure_built()  # built from other sources
    assert calls == [1, 1]
    stamp.write_text('{"source_sha256_16": "%s"}' % Bd.source_hash())
    Bd.ensure_built()  # current
    assert calls == [1, 1]
    assert len(Bd.source_hash()) == 16
    assert any(f.endswith("dg_kernels.h") for f in Bd.source_files())
