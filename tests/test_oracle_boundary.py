"""Pins of the oracle's domain boundaries (Section "Surface Integration
Kernel": a boundary edge's right-hand state is a ghost state that depends on
the kind of boundary; Section "Mesh Connectivity": boundary sides carry a
negative code).  CPU only.

  * solid wall = mirror symmetry: on a box with walls at x = 0 and x = lx
    (periodic in y), the right-hand side equals that of the periodic mesh
    doubled by its mirror image about x = 0, restricted to the box, for
    mirror-symmetric data — this pins the wall against the (separately
    pinned) periodic operator;
  * outflow: for a polynomial state whose flux the rules integrate exactly,
    the right-hand side is the projection of -div F(u) on every element,
    boundary elements included (the outflow ghost passes the physical flux
    through, with no dissipation);
  * prescribed state: a free stream prescribed on all sides is kept exactly;
  * closed walls conserve mass and energy; a gas at rest stays at rest.
"""
import numpy as np
import pytest

import oracle as O
from paper_1601_07944_amd import workloads as W
from test_oracle_operator import exact_dudt, linear_state

LX = 1.0


def mirror_data(x, y):
    # even in x (rho, rho v, E) and odd in x (rho u), period 2 LX in x and 1 in y
    cx, sx = np.cos(np.pi * x / LX), np.sin(np.pi * x / LX)
    rho = 1.0 + 0.2 * cx * np.sin(2 * np.pi * y) + 0.1 * np.cos(2 * np.pi * x / LX)
    u = 0.3 * sx + 0.05 * np.sin(2 * np.pi * x / LX) * np.cos(2 * np.pi * y)
    v = 0.2 * cx + 0.1 * np.sin(2 * np.pi * y)
    p = 1.0 + 0.1 * cx * np.cos(2 * np.pi * y)
    return W.primitive_to_conserved(rho, u, v, p)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_wall_is_mirror_symmetry(p):
    box = W.box_mesh(6, 5, LX, 1.0, 0.2, 3, bc=(W.BC_WALL, W.BC_WALL, 0, 0))
    dbl = W.mirror_doubled_x(box, LX)
    ob, od = O.Oracle(box, p), O.Oracle(dbl, p)
    Cb = ob.project(mirror_data)
    Cd = od.project(mirror_data)
    assert np.array_equal(Cb, Cd[: box.n_elem])
    Rb = ob.rhs(Cb)
    Rd = od.rhs(Cd)[: box.n_elem]
    assert np.abs(Rb - Rd).max() <= 1e-12 * np.abs(Rd).max()
    # the walls matter: a box with outflow sides gives something else
    bo = W.box_mesh(6, 5, LX, 1.0, 0.2, 3, bc=(W.BC_OUTFLOW, W.BC_OUTFLOW, 0, 0))
    assert np.abs(O.Oracle(bo, p).rhs(Cb) - Rb).max() > 1e-3 * np.abs(Rb).max()


@pytest.mark.parametrize("p", [2, 3, 4])
def test_outflow_polynomial_state_exact(p):
    box = W.box_mesh(5, 4, 1.0, 1.0, 0.2, 5, bc=(W.BC_OUTFLOW,) * 4)
    orc = O.Oracle(box, p)
    C = orc.project(linear_state)
    R = orc.rhs(C)
    rng = np.random.default_rng(p)
    rs = rng.uniform(0.05, 0.45, size=(2, 5))
    Rh = orc.eval(R, rs[0], rs[1])
    xy = orc.map_points(rs[0], rs[1])
    ex = exact_dudt(xy[..., 0], xy[..., 1])
    assert np.abs(Rh - ex).max() < 1e-11 * np.abs(ex).max()


@pytest.mark.parametrize("p", [1, 3])
def test_prescribed_free_stream_is_kept(p):
    box = W.box_mesh(5, 4, 1.0, 1.0, 0.2, 6, bc=(W.BC_STATE,) * 4)
    orc = O.Oracle(box, p)
    U = W.free_stream(np.zeros(1), np.zeros(1), rho=1.2, u=0.4, v=-0.3, p=0.9)[0]
    orc.set_bc_state(U)
    C = orc.project(W.free_stream, rho=1.2, u=0.4, v=-0.3, p=0.9)
    assert np.abs(orc.rhs(C)).max() < 1e-12
    # a different prescribed state drives the boundary elements
    orc.set_bc_state(U * 1.1)
    R = orc.rhs(C)
    touches = (box.nbr_elem < 0).any(axis=1)
    assert np.abs(R[touches]).max() > 1e-3 and np.abs(R[~touches]).max() < 1e-12


@pytest.mark.parametrize("p", [1, 2, 3])
def test_closed_walls_conserve_mass_and_energy(p):
    box = W.box_mesh(6, 6, 1.0, 1.0, 0.2, 7, bc=(W.BC_WALL,) * 4)
    orc = O.Oracle(box, p)
    C = W.random_state(box.n_elem, orc.np, seed=p)
    R = orc.rhs(C)
    det = orc.det()
    rate = (det[:, None] * R[:, :, 0]).sum(0)
    scale = (det[:, None] * np.abs(R[:, :, 0])).sum(0)
    assert abs(rate[0]) < 1e-13 * scale[0] and abs(rate[3]) < 1e-13 * scale[3]
    assert abs(rate[1]) > 1e-6 * scale[1]  # the walls push on the gas: momentum is not conserved
    rest = orc.project(W.free_stream, u=0.0, v=0.0)
    assert np.abs(orc.rhs(rest)).max() < 1e-12


def test_outflow_free_stream_is_kept():
    box = W.box_mesh(5, 5, 1.0, 1.0, 0.2, 8, bc=(W.BC_OUTFLOW,) * 4)
    orc = O.Oracle(box, 2)
    C = orc.project(W.free_stream, u=0.7, v=0.2)
    assert np.abs(orc.rhs(C)).max() < 1e-12


ADJ_BOXES = {"walls": (W.BC_WALL,) * 4, "outflow": (W.BC_OUTFLOW,) * 4, "state": (W.BC_STATE,) * 4,
             "channel": (W.BC_STATE, W.BC_OUTFLOW, W.BC_WALL, W.BC_WALL)}


def flowing(x, y):
    # nonzero normal velocity on every side of the unit box
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    return W.primitive_to_conserved(rho, 0.3 + 0.1 * np.cos(2 * np.pi * y), -0.2 + 0.1 * np.sin(2 * np.pi * x),
                                    1.0 + 0.1 * np.cos(2 * np.pi * (x + y)))


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("kind", sorted(ADJ_BOXES))
def test_adjoint_through_ghost_states_complex_step(kind, p):
    # <Rbar, J d> from complex-step derivatives of the forward operator (its
    # ghost states included) equals <J^T Rbar, d> from the hand-written
    # adjoint, whose boundary sides go back through the ghost's Jacobian
    box = W.box_mesh(5, 4, 1.0, 1.0, 0.2, 11, bc=ADJ_BOXES[kind])
    orc = O.Oracle(box, p)
    orc.set_bc_state(W.primitive_to_conserved(np.array(1.2), np.array(0.4), np.array(-0.1), np.array(1.1)).reshape(4))
    C = orc.project(flowing) + 0.01 * W.random_state(box.n_elem, orc.np, seed=p)
    rng = np.random.default_rng(30 + p)
    for _ in range(2):
        d = rng.normal(size=C.shape)
        Rb = rng.normal(size=C.shape)
        Jd = orc.rhs_complex(C + 1e-30j * d).imag / 1e-30
        lhs = np.sum(Rb * Jd)
        rhs = np.sum(orc.rhs_vjp(C, Rb) * d)
        assert abs(lhs - rhs) <= 1e-13 * np.abs(Rb * Jd).sum(), (lhs, rhs)


def test_adjoint_step_on_a_channel_finite_differences():
    box = W.box_mesh(6, 5, 1.0, 1.0, 0.2, 12, bc=ADJ_BOXES["channel"])
    orc = O.Oracle(box, 2)
    C = orc.project(flowing)
    dt, _ = orc.max_dt(C, 0.3 / 5)
    rng = np.random.default_rng(5)
    d = rng.normal(size=C.shape)
    ub = rng.normal(size=C.shape)
    eps = 1e-6
    fd = (orc.rk3_step(C + eps * d, dt) - orc.rk3_step(C - eps * d, dt)) / (2 * eps)
    assert abs(np.sum(ub * fd) - np.sum(orc.rk3_step_vjp(C, dt, ub) * d)) <= 1e-8 * np.abs(ub * fd).sum()
