"""The benchmark's headline workload at full size against the oracle, whole
state: the periodic unit-square Delaunay triangulation of 2,000,000 uniform
random points (seed 4, 4,000,000 triangles) with the density jump on the
smooth density wave.  The oracle runs its element loop on the host cores
(OpenMP, a few seconds per right-hand side).

For p = 1..5 (one lane per element up to p = 3 at this size, the
matrix-core kernel at p = 4, four lanes and the matrix-core mixed kernel at
p = 5): one dg_rhs, and one dg_advance step in the launch configuration the
benchmark times (step length from the per-block minima, fused into the stage
kernels), FP64 within 1e-11 relative L2 of the oracle and the step length
within 1e-14; the mixed form's step within 1e-5 (its stated bound for
states); and the increment of one step ten times the CFL step.  At p = 3
and 4 also the adjoint of the right-hand side (the matrix-core adjoint
kernel).

At p = 1 also one step with the Barth-Jespersen limiter after every stage
(the limiter workload the benchmark times).  And a channel of the same size
class with all three boundary kinds (2,000,000 triangles, p = 4: the
matrix-core kernel's boundary variants).

The mixed form's right-hand side is held to 1e-4 here (2e-4 at p = 5), not
to the 3e-5 of the 1,800-element meshes of the mixed-precision tests: its
FP32 traces and fluxes are rounded relative to their own size (about 1),
while the right-hand side of an element is their difference across it,
which shrinks with the element; on this mesh (median inradius 1.7e-4, the
thinnest triangles 1.6e-7) the measured error is 3.2e-5, 4.5e-5, 6.6e-5,
6.6e-5 and 9.7e-5 of the right-hand side's L2 norm at p = 1..5 (growing
with the order), and the state after a step still differs from the oracle's by
3-4e-11.
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_07944_amd import workloads as W

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[gpu case] {msg}", file=sys.stderr, flush=True)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def mesh():
    case("headline mesh: Delaunay triangulation of 2,000,000 points, seed 4")
    m = W.delaunay_mesh(2_000_000, 4)
    assert m.n_elem == 4_000_000
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    O.set_threads(min(cores, 16))
    return m


# the stage kernels the automatic choice runs on this mesh (FP64, mixed):
# one lane per element up to p = 3, the matrix cores at p = 4, four lanes in
# FP64 and the matrix cores in the mixed form at p = 5
KERNELS = {1: (1, 1), 2: (1, 1), 3: (1, 1), 4: (16, 16), 5: (4, 16)}
# the mixed form's right-hand-side bound on this mesh (module docstring)
MIXED_RHS = {1: 1e-4, 2: 1e-4, 3: 1e-4, 4: 1e-4, 5: 2e-4}


@pytest.mark.parametrize("p", [3, 4, 1, 2, 5])
def test_headline_rhs_and_fused_step(mesh, p):
    import torch

    from paper_1601_07944_amd import binding as B

    orc = O.Oracle(mesh, p)
    C0 = orc.project(W.density_jump)
    dm = B.DGMesh.from_mesh(mesh, p)
    kernel = dm.kernel_choice()
    assert kernel == KERNELS[p]
    case(f"headline dg_rhs + dg_advance x1 p={p} N={mesh.n_elem} stage kernels {kernel}")
    Cg = dm.pack(torch.from_numpy(C0).cuda())
    R = dm.unpack(dm.rhs(Cg)).cpu().numpy()
    Ro = orc.rhs(C0)
    err = rel_l2(R, Ro)
    print(f"headline p={p} dg_rhs rel L2 {err:.2e}", file=sys.stderr, flush=True)
    assert err <= 1e-11
    R = dm.unpack(dm.rhs(Cg, prec=B.DG_MIXED)).cpu().numpy()
    err = rel_l2(R, Ro)
    print(f"headline p={p} dg_rhs mixed rel L2 {err:.2e}", file=sys.stderr, flush=True)
    assert err <= MIXED_RHS[p]
    del R, Ro

    cfl = 0.3 / (2 * p + 1)
    dto, rc = orc.max_dt(C0, cfl)
    assert rc == 0
    ref = orc.rk3_step(C0, dto)
    for prec, tol in ((B.DG_FP64, 1e-11), (B.DG_MIXED, 1e-5)):
        A = Cg.clone()
        hist = torch.empty(1, dtype=torch.float64, device=A.device)
        dm.advance(A, 1, cfl, dt_hist=hist, prec=prec)
        got = dm.unpack(A).cpu().numpy()
        torch.cuda.synchronize()
        dtg = float(hist.cpu()[0])
        err = rel_l2(got, ref)
        print(f"headline p={p} prec={prec} dg_advance step rel L2 {err:.2e}, dt {dtg:.17g} vs {dto:.17g}",
              file=sys.stderr, flush=True)
        assert abs(dtg - dto) <= 1e-14 * dto
        assert err <= tol
        del A, got
    del ref

    # the CFL step is set by the mesh's thinnest triangles and barely moves
    # the state; a step ten times longer (still inside the SSP-RK3 stability
    # region there) gives increments of ~5e-6 of the state, compared as
    # increments: FP64 within 1e-10 (the right-hand side's 1e-11 plus the
    # cancellation of C0 + increment - C0), the mixed form within its
    # right-hand-side bound on this mesh
    h = 10.0 * dto
    inc = orc.rk3_step(C0, h) - C0
    for prec, tol in ((B.DG_FP64, 1e-10), (B.DG_MIXED, MIXED_RHS[p])):
        A = Cg.clone()
        dm.rk_step(A, h, prec=prec)
        got = dm.unpack(A).cpu().numpy() - C0
        torch.cuda.synchronize()
        err = rel_l2(got, inc)
        print(f"headline p={p} prec={prec} dg_rk_step (10x the CFL step) increment rel L2 {err:.2e}, "
              f"|increment| / |state| {np.linalg.norm(inc) / np.linalg.norm(C0):.1e}", file=sys.stderr, flush=True)
        assert err <= tol
        del A, got
    dm.close()


@pytest.mark.parametrize("p", [3, 4])
def test_headline_adjoint(mesh, p):
    # the adjoint the benchmark times at this point (the matrix-core kernel at
    # p=3, also the automatic choice at p=4): dg_rhs_vjp of the whole state
    # against the oracle's hand-written adjoint (serial, ten to twenty seconds
    # here), 1e-11
    import torch

    from paper_1601_07944_amd import binding as B

    orc = O.Oracle(mesh, p)
    C0 = orc.project(W.density_jump)
    Rb = np.random.default_rng(11).normal(size=C0.shape)
    dm = B.DGMesh.from_mesh(mesh, p)
    assert dm.adjoint_kernel() == 16
    case(f"headline dg_rhs_vjp p={p} N={mesh.n_elem}")
    got = dm.unpack(dm.rhs_vjp(dm.pack(torch.from_numpy(C0).cuda()), dm.pack(torch.from_numpy(Rb).cuda())))
    got = got.cpu().numpy()
    ref = orc.rhs_vjp(C0, Rb)
    err = rel_l2(got, ref)
    print(f"headline p={p} dg_rhs_vjp rel L2 {err:.2e}", file=sys.stderr, flush=True)
    assert err <= 1e-11
    dm.close()


def test_channel_2m_p4_boundaries_full_size():
    # a channel at the headline's size class: 1000 x 1000 x 2 = 2,000,000
    # jittered triangles (0.2h, seed 4), prescribed state on the left,
    # outflow on the right, walls at the bottom and top, smooth flow, p=4
    # (the matrix-core kernel's boundary variants, every stage): dg_rhs and
    # one dg_advance step (step length fused into the stages) against the
    # oracle, FP64 within 1e-11 and the step length within 1e-14, the mixed
    # step within 1e-5
    import torch

    from paper_1601_07944_amd import binding as B

    WALL, OUT, STATE = W.BC_WALL, W.BC_OUTFLOW, W.BC_STATE
    u_far = W.primitive_to_conserved(np.array(1.2), np.array(0.4), np.array(-0.1), np.array(1.1)).reshape(4)

    def flow(x, y):
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
        u = 0.3 + 0.1 * np.cos(2 * np.pi * y)
        v = -0.2 + 0.1 * np.sin(2 * np.pi * x)
        p = 1.0 + 0.1 * np.cos(2 * np.pi * (x + y))
        return W.primitive_to_conserved(rho, u, v, p)

    p = 4
    m = W.box_mesh(1000, 1000, 1.0, 1.0, 0.2, 4, bc=(STATE, OUT, WALL, WALL))
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    O.set_threads(min(cores, 16))
    orc = O.Oracle(m, p)
    orc.set_bc_state(u_far)
    C0 = orc.project(flow)
    dm = B.DGMesh.from_mesh(m, p)
    dm.set_boundary_state(u_far)
    assert dm.kernel_choice() == (16, 16)
    case(f"channel dg_rhs + dg_advance x1 p={p} N={m.n_elem}")
    Cg = dm.pack(torch.from_numpy(C0).cuda())
    R = dm.unpack(dm.rhs(Cg)).cpu().numpy()
    err = rel_l2(R, orc.rhs(C0))
    print(f"channel p={p} dg_rhs rel L2 {err:.2e}", file=sys.stderr, flush=True)
    assert err <= 1e-11
    del R
    cfl = 0.3 / (2 * p + 1)
    dto, rc = orc.max_dt(C0, cfl)
    assert rc == 0
    ref = orc.rk3_step(C0, dto)
    for prec, tol in ((B.DG_FP64, 1e-11), (B.DG_MIXED, 1e-5)):
        A = Cg.clone()
        hist = torch.empty(1, dtype=torch.float64, device=A.device)
        dm.advance(A, 1, cfl, dt_hist=hist, prec=prec)
        got = dm.unpack(A).cpu().numpy()
        torch.cuda.synchronize()
        dtg = float(hist.cpu()[0])
        err = rel_l2(got, ref)
        print(f"channel p={p} prec={prec} dg_advance step rel L2 {err:.2e}, dt {dtg:.17g} vs {dto:.17g}",
              file=sys.stderr, flush=True)
        assert abs(dtg - dto) <= 1e-14 * dto
        assert err <= tol
        del A, got
    dm.close()


def test_headline_limited_step_p1(mesh):
    # the limiter workload the benchmark times at this size (p=1, the
    # Barth-Jespersen limiter after every stage, CFL 0.1): one dg_advance
    # step against the oracle's limited SSP-RK3 step, FP64 within 1e-11,
    # the step length within 1e-14; the limiter changes the step
    import torch

    from paper_1601_07944_amd import binding as B

    p = 1
    orc = O.Oracle(mesh, p)
    C0 = orc.project(W.density_jump)
    dto, rc = orc.max_dt(C0, 0.1)
    assert rc == 0
    ref = orc.rk3_step(C0, dto, limit=True)
    dm = B.DGMesh.from_mesh(mesh, p)
    dm.set_limiter(dm.LIMITER_BJ)
    case(f"headline limited dg_advance x1 p={p} N={mesh.n_elem}")
    A = dm.pack(torch.from_numpy(C0).cuda())
    hist = torch.empty(1, dtype=torch.float64, device=A.device)
    dm.advance(A, 1, 0.1, dt_hist=hist)
    got = dm.unpack(A).cpu().numpy()
    torch.cuda.synchronize()
    dtg = float(hist.cpu()[0])
    err = rel_l2(got, ref)
    effect = rel_l2(orc.rk3_step(C0, dto), ref)
    print(f"headline limited step rel L2 {err:.2e}, dt {dtg:.17g} vs {dto:.17g}, limiter effect {effect:.1e}",
          file=sys.stderr, flush=True)
    assert abs(dtg - dto) <= 1e-14 * dto
    assert err <= 1e-11
    assert effect > 1e-9
    dm.close()
