"""GPU adjoint (dg_rhs_vjp, dg_rk_step_vjp, the checkpointed torch
autograd Function) against the oracle's hand-written adjoint, complex-step
derivatives of the oracle's forward operator, and finite differences of the
GPU forward path.

Bars: 1e-11 relative L2 against the oracle's adjoint (FP64); dot-product
test 1e-12; central differences (eps = 1e-6) along 8 seeded directions
within 1e-6 relative."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_07944_amd import workloads as W

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[gpu case] {msg}", file=sys.stderr, flush=True)


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_mesh(mesh, p, lanes=0):
    if lanes == 1 and p >= 4:
        pytest.skip("one lane per element is refused from p = 4 on (DG_EUNSUPPORTED)")
    from paper_1601_07944_amd import binding as B

    dm = B.DGMesh.from_mesh(mesh, p)
    dm.set_lanes(lanes)
    return dm


MESHES = {"delaunay600": lambda: W.delaunay_mesh(600, 5), "square20": lambda: W.square_mesh(20, 1.0, 0.2, 6)}


@pytest.mark.parametrize("lanes", [1, 4])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("mname", sorted(MESHES))
def test_rhs_vjp_matches_oracle(p, mname, lanes):
    mesh = MESHES[mname]()
    orc = O.Oracle(mesh, p)
    C = W.random_state(mesh.n_elem, orc.np, seed=p)
    Rb = np.random.default_rng(p).normal(size=C.shape)
    dm = gpu_mesh(mesh, p, lanes)
    case(f"dg_rhs_vjp p={p} {mname} lanes={lanes}")
    got = dm.unpack(dm.rhs_vjp(dm.pack(dev(C)), dm.pack(dev(Rb)))).cpu().numpy()
    ref = orc.rhs_vjp(C, Rb)
    assert rel_l2(got, ref) <= 1e-11


@pytest.mark.parametrize("p", [1, 3, 5])
def test_rhs_vjp_dot_product_complex_step(p):
    mesh = W.delaunay_mesh(500, 8)
    orc = O.Oracle(mesh, p)
    rng = np.random.default_rng(20 + p)
    C = W.random_state(mesh.n_elem, orc.np, seed=p)
    d = rng.normal(size=C.shape)
    Rb = rng.normal(size=C.shape)
    Jd = orc.rhs_complex(C + 1e-30j * d).imag / 1e-30
    dm = gpu_mesh(mesh, p)
    case(f"dot-product test p={p}")
    vjp = dm.unpack(dm.rhs_vjp(dm.pack(dev(C)), dm.pack(dev(Rb)))).cpu().numpy()
    lhs, rhs = np.sum(Rb * Jd), np.sum(vjp * d)
    assert abs(lhs - rhs) <= 1e-12 * np.abs(Rb * Jd).sum()


@pytest.mark.parametrize("lanes", [1, 4])
@pytest.mark.parametrize("stored", [False, True])
@pytest.mark.parametrize("p", [1, 3])
def test_rk_step_vjp_matches_oracle(p, stored, lanes):
    import torch

    mesh = W.delaunay_mesh(700, 9)
    orc = O.Oracle(mesh, p)
    C = orc.project(W.density_jump)
    dt, _ = orc.max_dt(C, 0.3 / (2 * p + 1))
    ub = np.random.default_rng(p).normal(size=C.shape)
    dm = gpu_mesh(mesh, p, lanes)
    case(f"dg_rk_step_vjp p={p} stored_stages={stored} lanes={lanes}")
    Cg = dm.pack(dev(C))
    ubg = dm.pack(dev(ub))
    if stored:
        u1, u2 = dm.empty_state(), dm.empty_state()
        Cw = Cg.clone()
        dm.rk_step_stages(Cw, u1, u2, dt)
        out = dm.rk_step_vjp(Cg, ubg, dt, u1=u1, u2=u2)
        # dg_rk_step_stages advances like dg_rk_step, bit for bit
        Cr = Cg.clone()
        dm.rk_step(Cr, dt)
        torch.cuda.synchronize()
        assert torch.equal(Cr, Cw)
    else:
        out = dm.rk_step_vjp(Cg, ubg, dt)
    got = dm.unpack(out).cpu().numpy()
    assert rel_l2(got, orc.rk3_step_vjp(C, dt, ub)) <= 1e-11


def oracle_objective_gradient(orc, C0, dt, nsteps):
    from test_oracle_adjoint import pressure_objective

    states = [C0]
    for _ in range(nsteps):
        states.append(orc.rk3_step(states[-1], dt))
    J, g = pressure_objective(orc, None, states[-1])
    for n in range(nsteps - 1, -1, -1):
        g = orc.rk3_step_vjp(states[n], dt, g)
    return J, g


def test_checkpointed_adjoint_matches_oracle_512():
    # the adjoint workload on the oracle's 512-element mesh: p=2, smooth
    # data, 200 SSP-RK3 steps with fixed dt, checkpoint every 20
    import torch

    from paper_1601_07944_amd import adjoint as A

    mesh = W.square_mesh(16, 1.0, 0.2, 30)
    p = 2
    orc = O.Oracle(mesh, p)
    C0 = orc.project(W.smooth_density)
    dt, _ = orc.max_dt(C0, 0.3 / (2 * p + 1))
    nsteps = 200
    case("checkpointed adjoint vs oracle, 512 elements, 200 steps")
    Jo, go = oracle_objective_gradient(orc, C0, dt, nsteps)
    dm = gpu_mesh(mesh, p)
    C0g = dm.pack(dev(C0)).requires_grad_(True)
    CN = A.run_steps(C0g, dm, dt, nsteps, 20)
    J, gN = A.pressure_disk_objective(dm, CN.detach())
    CN.backward(gN)
    g = dm.unpack(C0g.grad.detach()).cpu().numpy()
    torch.cuda.synchronize()
    assert abs(float(J) - Jo) <= 1e-12 * abs(Jo)
    assert rel_l2(g, go) <= 1e-11


def test_adjoint_gradient_finite_differences_131072():
    # 256 x 256 x 2 = 131,072 jittered triangles, p=2, smooth data, 200 steps
    # with fixed dt, checkpoint every 20; J = pressure over the disk r < 0.1
    # about (0.5, 0.5); central differences eps = 1e-6 along 8 seeded
    # N(0,1) directions
    import torch

    from paper_1601_07944_amd import adjoint as A

    mesh = W.square_mesh(256, 1.0, 0.2, 3)
    p = 2
    dm = gpu_mesh(mesh, p)
    xy = dm.quad_points().cpu().numpy()
    C0 = dm.project(dev(W.smooth_density(xy[..., 0], xy[..., 1])))
    _, dt = dm.max_dt(C0, 0.3 / (2 * p + 1))
    nsteps = 200
    case("adjoint FD check, 131072 elements, 200 steps, 8 directions")
    x = C0.clone().requires_grad_(True)
    CN = A.run_steps(x, dm, dt, nsteps, 20)
    J0, gN = A.pressure_disk_objective(dm, CN.detach())
    CN.backward(gN)
    g = x.grad.detach()

    def J_of(C):
        C = C.clone()
        for _ in range(nsteps):
            dm.rk_step(C, dt)
        return float(A.pressure_disk_objective(dm, C)[0])

    eps = 1e-6
    worst = 0.0
    for s in range(100, 108):
        d = torch.from_numpy(np.random.default_rng(s).normal(size=(mesh.n_elem, 4, dm.np))).cuda()
        dint = dm.pack(d)
        fd = (J_of(C0 + eps * dint) - J_of(C0 - eps * dint)) / (2 * eps)
        ad = float(torch.sum(g * dint))
        worst = max(worst, abs(fd - ad) / abs(fd))
        print(f"direction {s}: fd {fd:.10e} adjoint {ad:.10e}", file=sys.stderr, flush=True)
    assert worst <= 1e-6, worst


@pytest.mark.parametrize("p", [1, 3, 4])
def test_rk_step_stages_to(p):
    # the out-of-place stage states of the reverse sweep: u1, u2 bit for bit
    # those of dg_rk_step_stages, the input untouched, the new state equal
    # to dg_rk_step's to rounding (its last stage is the general form)
    import torch

    from paper_1601_07944_amd import binding as B

    mesh = W.delaunay_mesh(700, 19)
    orc = O.Oracle(mesh, p)
    C = orc.project(W.density_jump)
    dt, _ = orc.max_dt(C, 0.3 / (2 * p + 1))
    dm = gpu_mesh(mesh, p, 0)
    Cg = dm.pack(dev(C))
    case(f"dg_rk_step_stages_to p={p}")
    u1, u2, Cn = dm.empty_state(), dm.empty_state(), dm.empty_state()
    C_in = Cg.clone()
    dm.rk_step_stages_to(C_in, Cn, u1, u2, dt)
    v1, v2 = dm.empty_state(), dm.empty_state()
    Cw = Cg.clone()
    dm.rk_step_stages(Cw, v1, v2, dt)
    torch.cuda.synchronize()
    assert torch.equal(C_in, Cg)
    assert torch.equal(u1, v1) and torch.equal(u2, v2)
    assert float(torch.linalg.norm(Cn - Cw) / torch.linalg.norm(Cw)) <= 1e-15
    assert rel_l2(dm.unpack(Cn).cpu().numpy(), orc.rk3_step(C, dt)) <= 1e-11
    with pytest.raises(B.DGError):
        dm.rk_step_stages_to(C_in, C_in, u1, u2, dt)


@pytest.mark.parametrize("p", [2, 3])
def test_keep_all_adjoint_equals_checkpointed(p):
    # every = 0 (the forward pass keeps every step's stage states with
    # dg_rk_step_stages_to, no recomputation) against the checkpointed sweep:
    # with one segment (every >= nsteps) the sweep recomputes the same
    # out-of-place steps from C0, so the gradients agree bit for bit; with
    # checkpoints every 5 steps, taken from dg_rk_step (whose last stage
    # rounds differently), within 1e-12; the same cotangent of C_N seeds all
    # three; C_N within 1e-14; choose_every picks 0 when the states fit
    import torch

    from paper_1601_07944_amd import adjoint as A

    mesh = W.delaunay_mesh(900, 60 + p)
    dm = gpu_mesh(mesh, p)
    xy = dm.quad_points().cpu().numpy()
    C0 = dm.project(dev(W.smooth_density(xy[..., 0], xy[..., 1])))
    _, dt = dm.max_dt(C0, 0.3 / (2 * p + 1))
    nsteps = 23
    case(f"keep-all adjoint vs checkpointed, p={p}, {mesh.n_elem} elements, {nsteps} steps")
    grads, outs, gN = {}, {}, None
    for every in (nsteps, 5, 0):
        x = C0.clone().requires_grad_(True)
        CN = A.run_steps(x, dm, dt, nsteps, every)
        if gN is None:  # one cotangent of C_N for all three sweeps
            _, gN = A.pressure_disk_objective(dm, CN.detach())
        CN.backward(gN)
        grads[every] = x.grad.detach().clone()
        outs[every] = CN.detach().clone()
    torch.cuda.synchronize()

    def rel(a, b):
        return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))

    assert rel(outs[0], outs[nsteps]) <= 1e-14
    assert torch.equal(grads[0], grads[nsteps])
    assert rel(grads[0], grads[5]) <= 1e-12
    assert A.choose_every(dm, nsteps) == 0
    assert A.choose_every(dm, 10**9) == 20
    with pytest.raises(ValueError):
        A.run_steps(C0.clone().requires_grad_(True), dm, dt, 3, -1)
