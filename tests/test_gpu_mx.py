"""The FP64 stage kernel with its contractions on the matrix cores
(dg_set_matrix_cores) against the CPU oracle, through the C ABI.

Same bars as the vector-ALU kernels: relative L2 error <= 1e-11 for the
right-hand side and for SSP-RK3 steps; the fused step length of dg_advance
equal to the oracle's to 1e-14.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_07944_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-11
WALL, OUT, STATE = W.BC_WALL, W.BC_OUTFLOW, W.BC_STATE
# (left, right, bottom, top); 0 on both sides of a direction = periodic
BOXES = {"walls": (WALL, WALL, WALL, WALL), "channel": (STATE, OUT, WALL, WALL),
         "x_walls_y_periodic": (WALL, WALL, 0, 0)}
U_FAR = W.primitive_to_conserved(np.array(1.2), np.array(0.4), np.array(-0.1), np.array(1.1)).reshape(4)


def case(msg):
    print(f"[gpu case] {msg}", file=sys.stderr, flush=True)


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def mx_mesh(mesh, p, on=True):
    from paper_1601_07944_amd import binding as B

    dm = B.DGMesh.from_mesh(mesh, p)
    dm.set_matrix_cores(on)
    return dm


def flow(x, y):
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    u = 0.3 + 0.1 * np.cos(2 * np.pi * y)
    v = -0.2 + 0.1 * np.sin(2 * np.pi * x)
    p = 1.0 + 0.1 * np.cos(2 * np.pi * (x + y))
    return W.primitive_to_conserved(rho, u, v, p)


MESHES = {
    "square23_j0.2": lambda: W.square_mesh(23, 1.0, 0.2, 5),  # 1058 elements: ragged last workgroup
    "delaunay517": lambda: W.delaunay_mesh(517, 6),  # 1034 elements, unstructured
    "two": lambda: W.square_mesh(1, 1.0, 0.0, 0),  # 2 elements: every side borders the other
}


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("mname", sorted(MESHES))
def test_rhs_random_state(mname, p):
    mesh = MESHES[mname]()
    orc = O.Oracle(mesh, p)
    C = W.random_state(mesh.n_elem, orc.np, seed=20 + p)
    case(f"dg_rhs matrix cores p={p} mesh={mname} N={mesh.n_elem}")
    dm = mx_mesh(mesh, p)
    got = dm.unpack(dm.rhs(dm.pack(dev(C)))).cpu().numpy()
    ref = orc.rhs(C)
    err = rel_l2(got, ref)
    worst = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= TOL and worst <= 10 * TOL, (err, worst)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("kind", sorted(BOXES))
def test_boundary_rhs_and_steps(kind, p):
    import torch

    mesh = W.box_mesh(14, 12, 1.0, 1.0, 0.2, 4, bc=BOXES[kind])  # 336 elements
    orc = O.Oracle(mesh, p)
    orc.set_bc_state(U_FAR)
    dm = mx_mesh(mesh, p)
    dm.set_boundary_state(U_FAR)
    C = orc.project(flow) + 0.01 * W.random_state(mesh.n_elem, orc.np, seed=p)
    case(f"dg_rhs + 5 dg_rk_step matrix cores box={kind} p={p}")
    got = dm.unpack(dm.rhs(dm.pack(dev(C)))).cpu().numpy()
    assert rel_l2(got, orc.rhs(C)) <= TOL
    C0 = orc.project(flow)
    dt, _ = orc.max_dt(C0, 0.3 / (2 * p + 1))
    Cg = dm.pack(dev(C0))
    ref = C0
    for _ in range(5):
        dm.rk_step(Cg, dt)
        ref = orc.rk3_step(ref, dt)
    torch.cuda.synchronize()
    assert rel_l2(dm.unpack(Cg).cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("p", [1, 3, 4, 5])
def test_advance_fused_step_length(p):
    # dg_advance with the step length fused into stages 3 and 1 (per-64-element
    # minima of the matrix-core stage 3): the step lengths and states follow the
    # oracle's max_dt + rk3_step
    import torch

    mesh = W.delaunay_mesh(700, 30 + p)  # 1,400 triangles
    orc = O.Oracle(mesh, p)
    C0 = orc.project(W.smooth_density)
    cfl = 0.3 / (2 * p + 1)
    dm = mx_mesh(mesh, p)
    Cg = dm.pack(dev(C0))
    nsteps = 4
    hist = torch.zeros(nsteps, dtype=torch.float64, device=Cg.device)
    case(f"dg_advance x{nsteps} matrix cores p={p} N={mesh.n_elem}")
    dm.advance(Cg, nsteps, cfl, dt_hist=hist)
    ref = C0
    dts = []
    for _ in range(nsteps):
        dt, rc = orc.max_dt(ref, cfl)
        assert rc == 0
        dts.append(dt)
        ref = orc.rk3_step(ref, dt)
    torch.cuda.synchronize()
    assert np.allclose(hist.cpu().numpy(), dts, rtol=1e-13, atol=0)
    assert rel_l2(dm.unpack(Cg).cpu().numpy(), ref) <= TOL


def test_advance_with_separate_final_pass():
    # above 4,096 per-64-element minima (262,144 elements) the step length
    # takes a separate final pass: bitwise equal to max_dt + rk_step on the
    # same kernel
    import torch

    mesh = W.square_mesh(370, 1.0, 0.2, 3)  # 273,800 triangles
    p = 1
    dm = mx_mesh(mesh, p)
    xy = dm.quad_points().cpu().numpy()
    C0 = dm.project(dev(W.smooth_density(xy[..., 0], xy[..., 1])))
    cfl = 0.3 / 3
    nsteps = 3
    case(f"dg_advance x{nsteps} matrix cores p=1 N={mesh.n_elem} (separate final pass)")
    Ca = C0.clone()
    hist = torch.zeros(nsteps, dtype=torch.float64, device=Ca.device)
    dm.advance(Ca, nsteps, cfl, dt_hist=hist)
    Cs = C0.clone()
    ref = []
    for _ in range(nsteps):
        dt_dev, dt = dm.max_dt(Cs, cfl)
        ref.append(dt)
        dm.rk_step(Cs, dt_dev=dt_dev)
    torch.cuda.synchronize()
    assert np.array_equal(hist.cpu().numpy(), np.asarray(ref))
    assert torch.equal(Ca, Cs)


@pytest.mark.parametrize("p", [2, 4])
def test_rk4_stages(p):
    # the general Runge-Kutta stage (RK4) through the matrix-core kernel
    import torch

    mesh = W.delaunay_mesh(300, 40 + p)
    orc = O.Oracle(mesh, p)
    C0 = orc.project(W.smooth_density)
    dt, _ = orc.max_dt(C0, 0.3 / (2 * p + 1))
    dm = mx_mesh(mesh, p)
    dm.set_integrator(2)
    Cg = dm.pack(dev(C0))
    ref = C0
    case(f"RK4 x3 matrix cores p={p}")
    for _ in range(3):
        dm.rk_step(Cg, dt)
        ref = orc.rk_step(ref, dt, "rk4")
    torch.cuda.synchronize()
    assert rel_l2(dm.unpack(Cg).cpu().numpy(), ref) <= TOL


def test_switch_is_validated():
    from paper_1601_07944_amd import binding as B

    dm = mx_mesh(W.square_mesh(2, 1.0, 0.0, 0), 2)
    case("dg_set_matrix_cores argument check")
    assert dm._lib.dg_set_matrix_cores(dm._h, 2) == -1  # DG_EINVAL
    assert dm._lib.dg_set_matrix_cores(dm._h, -2) == -1
    dm.set_matrix_cores(False)
    dm.set_matrix_cores(None)


@pytest.mark.parametrize("p,auto_mx", [(2, False), (3, True), (4, True), (5, True)])
def test_automatic_choice(p, auto_mx):
    # on a mesh below DG_LANES4_MAX_ELEMENTS the automatic choice runs the
    # matrix-core kernel at p = 3..5 (bitwise the forced kernel), and an
    # explicit lane count keeps the vector-ALU kernel
    import torch

    from paper_1601_07944_amd import binding as B

    mesh = W.delaunay_mesh(600, 50 + p)
    orc = O.Oracle(mesh, p)
    C = W.random_state(mesh.n_elem, orc.np, seed=p)
    case(f"automatic matrix-core choice p={p}")
    auto = B.DGMesh.from_mesh(mesh, p)
    forced = mx_mesh(mesh, p, True)
    vec = mx_mesh(mesh, p, False)
    vec.set_lanes(4)
    four = B.DGMesh.from_mesh(mesh, p)
    four.set_lanes(4)
    k = 16 if auto_mx else 4
    assert auto.kernel_choice() == (k, k)
    assert auto.adjoint_kernel() == (16 if p in (3, 4) else 4)
    assert forced.adjoint_kernel() == 16 and vec.adjoint_kernel() == 4
    assert forced.kernel_choice() == (16, 16) and vec.kernel_choice() == (4, 4) and four.kernel_choice() == (4, 4)
    Cg = auto.pack(dev(C))
    Ra, Rm, Rv, R4 = auto.rhs(Cg), forced.rhs(Cg), vec.rhs(Cg), four.rhs(Cg)
    torch.cuda.synchronize()
    assert torch.equal(Ra, Rm if auto_mx else Rv)
    assert torch.equal(R4, Rv)
    for R in (Ra, Rm, Rv):
        assert rel_l2(auto.unpack(R).cpu().numpy(), orc.rhs(C)) <= TOL


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_mixed_rhs_bound_and_conservation(p):
    # the mixed form on the matrix cores: within the mixed bound of the FP64
    # oracle (3e-5 relative L2 for one right-hand side), and the element
    # means conservative to FP64 rounding (bitwise equal FP32 edge fluxes)
    mesh = W.delaunay_mesh(900, 4)
    orc = O.Oracle(mesh, p)
    C = orc.project(W.density_jump)
    dm = mx_mesh(mesh, p)
    case(f"dg_rhs DG_MIXED matrix cores p={p} N={mesh.n_elem}")
    R = dm.unpack(dm.rhs(dm.pack(dev(C)), prec=1)).cpu().numpy()
    err = rel_l2(R, orc.rhs(C))
    print(f"mixed matrix-core rhs p={p} rel L2 {err:.2e}", file=sys.stderr, flush=True)
    assert err <= 3e-5
    terms = orc.det()[:, None] * R[:, :, 0]
    assert np.all(np.abs(terms.sum(0)) < 1e-13 * np.abs(terms).sum(0))


@pytest.mark.parametrize("p", [1, 3, 4, 5])
def test_mixed_100_steps(p):
    import torch

    mesh = W.delaunay_mesh(2000, 2)
    orc = O.Oracle(mesh, p)
    C0 = orc.project(W.smooth_density)
    dm = mx_mesh(mesh, p)
    Cg = dm.pack(dev(C0))
    cfl = 0.3 / (2 * p + 1)
    case(f"dg_rk_step DG_MIXED matrix cores p={p} 100 steps N={mesh.n_elem}")
    Co = C0
    tot0 = (orc.det()[:, None] * C0[:, :, 0]).sum(0)
    for _ in range(100):
        dt, _ = orc.max_dt(Co, cfl)
        Co = orc.rk3_step(Co, dt)
        dm.rk_step(Cg, dt, prec=1)
    got = dm.unpack(Cg).cpu().numpy()
    torch.cuda.synchronize()
    err = rel_l2(got, Co)
    print(f"mixed matrix-core 100 steps p={p} rel L2 {err:.2e}", file=sys.stderr, flush=True)
    assert err <= 1e-5
    tot = (orc.det()[:, None] * got[:, :, 0]).sum(0)
    assert np.all(np.abs(tot - tot0) <= 1e-12 * np.abs(tot0))


@pytest.mark.parametrize("p", [2, 4, 5])
@pytest.mark.parametrize("kind", sorted(BOXES))
def test_mixed_boundaries_and_fused_step_length(kind, p):
    # mixed form with domain boundaries: one right-hand side within 3e-5, and
    # dg_advance (step length fused into the stages) equal to max_dt + rk_step
    import torch

    mesh = W.box_mesh(14, 12, 1.0, 1.0, 0.2, 4, bc=BOXES[kind])
    orc = O.Oracle(mesh, p)
    orc.set_bc_state(U_FAR)
    dm = mx_mesh(mesh, p)
    dm.set_boundary_state(U_FAR)
    C = orc.project(flow)
    case(f"DG_MIXED matrix cores box={kind} p={p}")
    got = dm.unpack(dm.rhs(dm.pack(dev(C)), prec=1)).cpu().numpy()
    assert rel_l2(got, orc.rhs(C)) <= 3e-5
    C0 = dm.pack(dev(C))
    cfl = 0.3 / (2 * p + 1)
    Ca = C0.clone()
    dm.advance(Ca, 4, cfl, prec=1)
    Cs = C0.clone()
    for _ in range(4):
        dt_dev, _ = dm.max_dt(Cs, cfl)
        dm.rk_step(Cs, dt_dev=dt_dev, prec=1)
    torch.cuda.synchronize()
    assert torch.equal(Ca, Cs)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("mname", sorted(MESHES))
def test_adjoint_rhs_vjp(mname, p):
    # the adjoint on the matrix cores (forced on): the VJP of the right-hand
    # side against the oracle's hand-written adjoint, 1e-11
    mesh = MESHES[mname]()
    orc = O.Oracle(mesh, p)
    C = W.random_state(mesh.n_elem, orc.np, seed=30 + p)
    Rb = np.random.default_rng(30 + p).normal(size=C.shape)
    dm = mx_mesh(mesh, p)
    case(f"dg_rhs_vjp matrix cores p={p} {mname}")
    got = dm.unpack(dm.rhs_vjp(dm.pack(dev(C)), dm.pack(dev(Rb)))).cpu().numpy()
    assert rel_l2(got, orc.rhs_vjp(C, Rb)) <= TOL


@pytest.mark.parametrize("p", [1, 3, 4])
def test_adjoint_rk_step_vjp(p):
    # the adjoint of one SSP-RK3 step (stage modes 1..3) with stored and with
    # recomputed stage states
    mesh = W.delaunay_mesh(700, 9)
    orc = O.Oracle(mesh, p)
    C = orc.project(W.density_jump)
    dt, _ = orc.max_dt(C, 0.3 / (2 * p + 1))
    ub = np.random.default_rng(p).normal(size=C.shape)
    dm = mx_mesh(mesh, p)
    Cg, ubg = dm.pack(dev(C)), dm.pack(dev(ub))
    ref = orc.rk3_step_vjp(C, dt, ub)
    case(f"dg_rk_step_vjp matrix cores p={p}")
    got = dm.unpack(dm.rk_step_vjp(Cg, ubg, dt)).cpu().numpy()
    assert rel_l2(got, ref) <= TOL
    u1, u2 = dm.empty_state(), dm.empty_state()
    Cw = Cg.clone()
    dm.rk_step_stages(Cw, u1, u2, dt)
    got = dm.unpack(dm.rk_step_vjp(Cg, ubg, dt, u1=u1, u2=u2)).cpu().numpy()
    assert rel_l2(got, ref) <= TOL


@pytest.mark.parametrize("p", [2, 3, 5])
@pytest.mark.parametrize("kind", sorted(BOXES))
def test_adjoint_through_ghost_states(kind, p):
    mesh = W.box_mesh(14, 12, 1.0, 1.0, 0.2, 4, bc=BOXES[kind])
    orc = O.Oracle(mesh, p)
    orc.set_bc_state(U_FAR)
    dm = mx_mesh(mesh, p)
    dm.set_boundary_state(U_FAR)
    C = orc.project(flow) + 0.01 * W.random_state(mesh.n_elem, orc.np, seed=p)
    Rb = np.random.default_rng(40 + p).normal(size=C.shape)
    case(f"dg_rhs_vjp matrix cores box={kind} p={p}")
    got = dm.unpack(dm.rhs_vjp(dm.pack(dev(C)), dm.pack(dev(Rb)))).cpu().numpy()
    assert rel_l2(got, orc.rhs_vjp(C, Rb)) <= TOL


@pytest.mark.parametrize("p", [3, 4])
def test_rk2_stages(p):
    # the paper's RK2 (general stages) through the matrix-core kernel
    import torch

    mesh = W.delaunay_mesh(500, 60 + p)
    orc = O.Oracle(mesh, p)
    C0 = orc.project(W.smooth_density)
    dt, _ = orc.max_dt(C0, 0.3 / (2 * p + 1))
    dm = mx_mesh(mesh, p)
    dm.set_integrator(1)
    Cg = dm.pack(dev(C0))
    ref = C0
    case(f"RK2 x5 matrix cores p={p}")
    for _ in range(5):
        dm.rk_step(Cg, dt)
        ref = orc.rk_step(ref, dt, "rk2")
    torch.cuda.synchronize()
    assert rel_l2(dm.unpack(Cg).cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("p", [3, 5])
def test_mixed_rk4(p):
    # RK4 in the mixed form on the matrix cores: within the mixed bound for
    # states (1e-5 after 20 steps)
    import torch

    mesh = W.delaunay_mesh(900, 34)
    orc = O.Oracle(mesh, p)
    C0 = orc.project(W.smooth_density)
    dt, _ = orc.max_dt(C0, 0.3 / (2 * p + 1))
    dm = mx_mesh(mesh, p)
    dm.set_integrator(2)
    Cg = dm.pack(dev(C0))
    ref = C0
    case(f"mixed RK4 x20 matrix cores p={p}")
    for _ in range(20):
        dm.rk_step(Cg, dt, prec=1)
        ref = orc.rk_step(ref, dt, "rk4")
    torch.cuda.synchronize()
    assert rel_l2(dm.unpack(Cg).cpu().numpy(), ref) <= 1e-5


def test_limited_steps():
    # SSP-RK3 with the Barth-Jespersen limiter after every stage, the stages
    # on the matrix cores (forced at p=1)
    import torch

    mesh = W.delaunay_mesh(800, 33)
    orc = O.Oracle(mesh, 1)
    C0 = orc.project(W.density_jump)
    dt, _ = orc.max_dt(C0, 0.1)
    dm = mx_mesh(mesh, 1)
    dm.set_limiter(1)
    Cg = dm.pack(dev(C0))
    ref = C0
    case("limited SSP-RK3 x15 matrix cores p=1")
    for _ in range(15):
        dm.rk_step(Cg, dt)
        ref = orc.rk3_step(ref, dt, limit=True)
    torch.cuda.synchronize()
    assert rel_l2(dm.unpack(Cg).cpu().numpy(), ref) <= TOL
