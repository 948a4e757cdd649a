"""Pins of the oracle's DG operator, projection, time step and SSP-RK3
(test infrastructure).  Each test checks the oracle against something fixed
by the mathematics, not against itself:

* projection reproduces polynomials of degree <= p (mass = det J * I);
* a constant state has zero right-hand side (free stream: metric terms and
  the divergence identity, eq. (2ddg0));
* element means change only through edge fluxes that cancel pairwise
  (conservation on periodic meshes);
* for polynomial states whose flux the quadrature integrates exactly, the
  right-hand side equals the exact time derivative -div F(u) of the Euler
  equations (eq. (euler));
* the discrete solution does not depend on how each element numbers its
  vertices, and commutes with rotations and translations of the plane
  (side mappings and the reversed edge points of the Surface Integration
  Kernel section);
* the CFL step has its closed form on right isosceles triangles;
* the three-stage SSP Runge-Kutta step converges at third order in dt.
"""
import functools

import numpy as np
import pytest

import oracle as O
from paper_1601_07944_amd import workloads as W

O.set_threads(4)


def det_of(mesh):
    X = mesh.vxy
    return (X[:, 1, 0] - X[:, 0, 0]) * (X[:, 2, 1] - X[:, 0, 1]) - (X[:, 2, 0] - X[:, 0, 0]) * (X[:, 1, 1] - X[:, 0, 1])


def to_reference(mesh, xy):
    """Reference coordinates (r, s) of physical points xy[N, k, 2] per element."""
    X = mesh.vxy
    a = X[:, 1] - X[:, 0]
    b = X[:, 2] - X[:, 0]
    d = a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]
    rel = xy - X[:, None, 0]
    r = (rel[..., 0] * b[:, None, 1] - rel[..., 1] * b[:, None, 0]) / d[:, None]
    s = (a[:, None, 0] * rel[..., 1] - a[:, None, 1] * rel[..., 0]) / d[:, None]
    return r, s


def eval_at_physical(orc, mesh, C, xy):
    """U_h at physical points xy[N, k, 2] (one set of points per element)."""
    r, s = to_reference(mesh, xy)
    out = np.empty(xy.shape[:2] + (4,))
    for k in range(xy.shape[1]):
        # evaluate each element at its own reference point k
        phi, _, _ = O.basis(orc.p, r[:, k], s[:, k])
        out[:, k] = np.einsum("nmj,nj->nm", C, phi)
    return out


def meshes_small():
    return [W.square_mesh(6, 1.0, 0.2, 11), W.delaunay_mesh(60, 12)]


# ---------------------------------------------------------------- projection
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_projection_reproduces_polynomials(p):
    mesh = W.square_mesh(4, 1.0, 0.2, 3)
    orc = O.Oracle(mesh, p)
    rng = np.random.default_rng(p)
    coef = rng.normal(size=(4, p + 1, p + 1))

    def poly(x, y):
        out = np.zeros(np.shape(x) + (4,))
        for a in range(p + 1):
            for b in range(p + 1 - a):
                out += coef[:, a, b] * (x**a * y**b)[..., None]
        return out

    C = orc.project(poly)
    rs = rng.uniform(0.05, 0.45, size=(2, 7))
    Uh = orc.eval(C, rs[0], rs[1])
    xy = orc.map_points(rs[0], rs[1])
    ue = poly(xy[..., 0], xy[..., 1])
    assert np.abs(Uh - ue).max() < 1e-12 * np.abs(ue).max()


# ---------------------------------------------------------------- free stream
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_free_stream_is_exact(p):
    for mesh in meshes_small():
        orc = O.Oracle(mesh, p)
        C = orc.project(W.free_stream)
        R = orc.rhs(C)
        # scale: max |F| * max(l / det J)
        X = mesh.vxy
        lmax = np.max(np.linalg.norm(X[:, [1, 2, 0]] - X, axis=2))
        scale = 3.0 * lmax / det_of(mesh).min()
        assert np.abs(R).max() < 1e-13 * scale, (p, mesh.name, np.abs(R).max())


def test_free_stream_stays_constant_over_steps():
    mesh = W.square_mesh(8, 10.0, 0.2, 1)
    orc = O.Oracle(mesh, 3)
    C0 = orc.project(W.free_stream)
    C = C0.copy()
    dt, rc = orc.max_dt(C, 0.3 / 7)
    assert rc == 0
    for _ in range(100):
        C = orc.rk3_step(C, dt)
    assert np.abs(C - C0).max() < 1e-13 * np.abs(C0).max()


# ---------------------------------------------------------------- conservation
@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_conservation_per_call(p):
    for mesh in meshes_small():
        orc = O.Oracle(mesh, p)
        C = W.random_state(mesh.n_elem, orc.np, seed=p)
        R = orc.rhs(C)
        terms = det_of(mesh)[:, None] * R[:, :, 0]
        assert np.all(np.abs(terms.sum(0)) < 1e-13 * np.abs(terms).sum(0))


def test_conservation_over_steps():
    mesh = W.delaunay_mesh(100, 7)
    orc = O.Oracle(mesh, 2)
    C = orc.project(W.density_jump)
    det = det_of(mesh)
    tot0 = (det[:, None] * C[:, :, 0]).sum(0)
    dt, _ = orc.max_dt(C, 0.3 / 5)
    for _ in range(30):
        C = orc.rk3_step(C, dt)
    tot = (det[:, None] * C[:, :, 0]).sum(0)
    assert np.all(np.abs(tot - tot0) < 1e-12 * np.abs(tot0))


# ------------------------------------------------- linear advection reduction
def test_linear_advection_invariants():
    # u = v = 0.5 and p = 1 everywhere: the state stays on the manifold
    # rho u = rho/2, rho v = rho/2, E = 2.5 + rho/4 (a pure contact wave)
    mesh = W.delaunay_mesh(80, 4)
    orc = O.Oracle(mesh, 2)
    C = orc.project(W.density_jump)
    dt, _ = orc.max_dt(C, 0.3 / 5)
    for _ in range(20):
        C = orc.rk3_step(C, dt)
    e0 = np.zeros(orc.np)
    e0[0] = 2.5 / np.sqrt(2.0)
    assert np.abs(C[:, 1] - 0.5 * C[:, 0]).max() < 1e-13
    assert np.abs(C[:, 2] - 0.5 * C[:, 0]).max() < 1e-13
    assert np.abs(C[:, 3] - 0.25 * C[:, 0] - e0).max() < 1e-13


# --------------------------------------------- exact divergence, poly states
def euler_flux_np(U, gamma=1.4):
    rho, mx, my, E = U[..., 0], U[..., 1], U[..., 2], U[..., 3]
    u = mx / rho
    v = my / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    Fx = np.stack([mx, mx * u + p, mx * v, u * (E + p)], axis=-1)
    Fy = np.stack([my, my * u, my * v + p, v * (E + p)], axis=-1)
    return Fx, Fy


def linear_state(x, y):
    rho = 1.3 + 0 * x
    mx = 0.2 + 0.3 * x - 0.25 * y
    my = -0.1 + 0.15 * x + 0.35 * y
    E = 3.0 + 0.4 * x + 0.2 * y
    return np.stack([rho, mx, my, E], axis=-1)


def exact_dudt(x, y):
    # -div F(u) by complex-step derivatives of the flux along x and y
    h = 1e-30
    Fx, _ = euler_flux_np(linear_state(x + 1j * h, y + 0j))
    _, Fy = euler_flux_np(linear_state(x + 0j, y + 1j * h))
    return -(Fx.imag + Fy.imag) / h


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_polynomial_state_gives_exact_time_derivative(p):
    # rho constant, momenta and energy linear: the flux is a cubic, the
    # volume rule (degree 2p) and the edge rule (degree 2p+1) integrate the
    # weak form exactly for p >= 2, the traces are continuous so the
    # dissipation term vanishes, and the divergence theorem gives
    # R = projection of -div F(u) = -div F(u) (a quadratic).
    mesh = W.square_mesh(6, 1.0, 0.2, 21)
    orc = O.Oracle(mesh, p)
    C = orc.project(linear_state)
    R = orc.rhs(C)
    # elements away from the periodic seam (the state is not periodic)
    cen = mesh.centroids()
    inner = np.all((cen > 1.5 / 6) & (cen < 1 - 1.5 / 6), axis=1)
    rng = np.random.default_rng(p)
    rs = rng.uniform(0.05, 0.45, size=(2, 5))
    Rh = orc.eval(R, rs[0], rs[1])[inner]
    xy = orc.map_points(rs[0], rs[1])[inner]
    ex = exact_dudt(xy[..., 0], xy[..., 1])
    assert np.abs(Rh - ex).max() < 1e-11 * np.abs(ex).max(), np.abs(Rh - ex).max()


# ---------------------------------------- relabel / rotation / translation
def relabel(mesh, shift):
    """Cyclically rotate the local vertex numbering of every element by
    shift[i] in {0,1,2}: new vertex q = old vertex q+shift."""
    N = mesh.n_elem
    idx = (np.arange(3)[None, :] + shift[:, None]) % 3
    vxy = np.take_along_axis(mesh.vxy, idx[:, :, None], axis=1)
    nbr = np.take_along_axis(mesh.nbr_elem, idx, axis=1)
    old_side = np.take_along_axis(mesh.nbr_side.astype(np.int64), idx, axis=1)
    nsd = (old_side - shift[nbr]) % 3
    return W.Mesh(vxy, nbr, nsd.astype(np.int8), mesh.period, mesh.name + "_relabel")


@pytest.mark.parametrize("p", [1, 2, 3])
def test_vertex_relabel_invariance(p):
    mesh = W.square_mesh(6, 10.0, 0.2, 4)
    rng = np.random.default_rng(9)
    shift = rng.integers(0, 3, size=mesh.n_elem)
    m2 = relabel(mesh, shift)
    results = []
    for m in (mesh, m2):
        orc = O.Oracle(m, p)
        C = orc.project(W.isentropic_vortex)
        for _ in range(5):
            C = orc.rk3_step(C, 0.01)
        results.append((orc, m, C))
    # compare U_h at the same physical points (centroid and a corner-ish point)
    xy = np.stack([mesh.vxy.mean(1), 0.6 * mesh.vxy[:, 0] + 0.2 * mesh.vxy[:, 1] + 0.2 * mesh.vxy[:, 2]], axis=1)
    U1 = eval_at_physical(results[0][0], results[0][1], results[0][2], xy)
    U2 = eval_at_physical(results[1][0], results[1][1], results[1][2], xy)
    assert np.abs(U1 - U2).max() < 1e-12 * np.abs(U1).max()


def test_rotation_and_translation_covariance():
    p = 2
    mesh = W.square_mesh(6, 10.0, 0.2, 5)
    # rotate the plane by 90 degrees: (x, y) -> (-y, x); velocity rotates too
    vr = np.stack([-mesh.vxy[..., 1], mesh.vxy[..., 0]], axis=-1)
    mrot = W.Mesh(vr, mesh.nbr_elem, mesh.nbr_side, mesh.period)
    shift = np.array([0.37, -1.21])
    mtr = W.Mesh(mesh.vxy + shift, mesh.nbr_elem, mesh.nbr_side, mesh.period)
    vort = functools.partial(W.isentropic_vortex, vel=(1.0, 0.5))
    vort_rot = functools.partial(W.isentropic_vortex, vel=(-0.5, 1.0), center=(-5.0, 5.0))
    vort_tr = functools.partial(W.isentropic_vortex, vel=(1.0, 0.5), center=(5.0 + shift[0], 5.0 + shift[1]))
    out = []
    for m, fn in ((mesh, vort), (mrot, vort_rot), (mtr, vort_tr)):
        orc = O.Oracle(m, p)
        C = orc.project(fn)
        for _ in range(4):
            C = orc.rk3_step(C, 0.01)
        out.append(orc.eval(C, np.array([1 / 3, 0.2]), np.array([1 / 3, 0.6])))
    U0, Ur, Ut = out
    rot = np.stack([Ur[..., 0], Ur[..., 2], -Ur[..., 1], Ur[..., 3]], axis=-1)  # rotate momentum back
    assert np.abs(rot - U0).max() < 1e-12 * np.abs(U0).max()
    assert np.abs(Ut - U0).max() < 1e-12 * np.abs(U0).max()


# ---------------------------------------------------------------- time step
def test_cfl_time_step_closed_form():
    n, L = 5, 2.0
    mesh = W.square_mesh(n, L, 0.0, 0)
    orc = O.Oracle(mesh, 1)
    C = orc.project(functools.partial(W.free_stream, rho=1.2, u=0.3, v=-0.4, p=0.8))
    dt, rc = orc.max_dt(C, 0.1)
    h = L / n
    r_in = h * (1.0 - np.sqrt(0.5))  # right isosceles triangle with legs h
    lam = 0.5 + np.sqrt(1.4 * 0.8 / 1.2)
    assert rc == 0 and abs(dt - 0.1 * r_in / lam) < 1e-14 * dt
    C[3, 0, 0] = -1.0  # negative density mean
    dt, rc = orc.max_dt(C, 0.1)
    assert rc == -1 and np.isnan(dt)


def test_ssp_rk3_is_third_order():
    mesh = W.square_mesh(8, 10.0, 0.1, 2)
    orc = O.Oracle(mesh, 2)
    C0 = orc.project(W.isentropic_vortex)
    dt0, _ = orc.max_dt(C0, 0.3 / 5)
    T = 8 * dt0

    def run(nsteps):
        C = C0.copy()
        for _ in range(nsteps):
            C = orc.rk3_step(C, T / nsteps)
        return C

    ref = run(256)
    errs = [np.abs(run(n) - ref).max() for n in (8, 16, 32)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.8), rates
