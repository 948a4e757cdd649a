"""GPU check of dg_rk_step_noalloc, the step without a workspace (stage
states in the library's static device scratch), against dg_rk_step with a
caller-owned workspace: the same launches, so equal bit for bit.  Two calls
in a row on one GPU, the second on a smaller mesh, so the second call runs
over scratch that still holds the first call's (larger) stage states; then
the size limit."""
import sys

import numpy as np
import pytest

from paper_1601_07944_amd import workloads as W

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20  # DG_NOALLOC_SCRATCH_BYTES


def case(msg):
    print(f"[gpu case] {msg}", file=sys.stderr, flush=True)


def setup(mesh, p, lanes, init):
    if lanes == 1 and p >= 4:
        pytest.skip("one lane per element is refused from p = 4 on (DG_EUNSUPPORTED)")
    import torch

    from paper_1601_07944_amd import binding as B

    dm = B.DGMesh.from_mesh(mesh, p)
    dm.set_lanes(lanes)
    xy = dm.quad_points().cpu().numpy()
    C0 = dm.project(torch.from_numpy(np.ascontiguousarray(init(xy[..., 0], xy[..., 1]))).cuda())
    return dm, C0


def steps_both_ways(dm, C0, p, prec, nsteps):
    """nsteps steps with dg_rk_step_noalloc and with dg_rk_step, each step
    with the device CFL step length of its own state."""
    import torch

    cfl = 0.3 / (2 * p + 1)
    A, Bst = C0.clone(), C0.clone()
    dta = torch.empty(1, dtype=torch.float64, device="cuda")
    dtb = torch.empty(1, dtype=torch.float64, device="cuda")
    for _ in range(nsteps):
        dm.max_dt(A, cfl, dt_dev=dta, to_host=False)
        dm.rk_step_noalloc(A, dt_dev=dta, prec=prec)
        dm.max_dt(Bst, cfl, dt_dev=dtb, to_host=False)
        dm.rk_step(Bst, dt_dev=dtb, prec=prec)
    torch.cuda.synchronize()
    return A, Bst


@pytest.mark.parametrize("lanes", [0, 1, 4])  # 0: the automatic choice (matrix cores at p = 3, 5 here)
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("p", [1, 3, 5])
def test_noalloc_step_equals_workspace_step(p, prec, lanes):
    import torch

    # first call: 12,800 triangles; second: 512 (a ragged 2-block tail)
    big = W.square_mesh(80, 1.0, 0.2, 41 + p)
    small = W.square_mesh(16, 1.0, 0.2, 51 + p)
    for mesh, nsteps in ((big, 3), (small, 2)):
        case(f"dg_rk_step_noalloc p={p} prec={prec} lanes={lanes} n={mesh.n_elem}")
        dm, C0 = setup(mesh, p, lanes, W.density_jump)
        state_bytes = dm.info.state_len * 8
        assert 2 * state_bytes <= SCRATCH_BYTES
        A, Bst = steps_both_ways(dm, C0, p, prec, nsteps)
        assert torch.isfinite(A).all()
        assert not torch.equal(A, C0)
        assert torch.equal(A, Bst), f"max |diff| {float((A - Bst).abs().max()):.3e}"
        dm.close()


def test_noalloc_rk4_and_limiter():
    """The integrator and limiter settings apply as in dg_rk_step (RK4 keeps
    its running sum in the scratch as well)."""
    import torch

    mesh = W.square_mesh(40, 1.0, 0.2, 61)
    for p, integrator, limiter in ((2, 2, 0), (1, 0, 1), (1, 1, 1)):
        case(f"dg_rk_step_noalloc p={p} integrator={integrator} limiter={limiter}")
        dm, C0 = setup(mesh, p, 0, W.density_jump)
        dm.set_integrator(integrator)
        dm.set_limiter(limiter)
        A, Bst = steps_both_ways(dm, C0, p, 0, 3)
        assert torch.equal(A, Bst)
        dm.close()


def test_noalloc_refuses_meshes_beyond_the_scratch():
    import torch

    from paper_1601_07944_amd import binding as B

    # 235 x 235 x 2 = 110,450 triangles at p = 3: two states of 35.4 MB > 64 MiB
    mesh = W.square_mesh(235, 1.0, 0.2, 71)
    case(f"dg_rk_step_noalloc over the limit n={mesh.n_elem}")
    dm, C0 = setup(mesh, 3, 0, W.density_jump)
    assert 2 * dm.info.state_len * 8 > SCRATCH_BYTES
    C = C0.clone()
    with pytest.raises(B.DGError) as ei:
        dm.rk_step_noalloc(C, dt=1e-4)
    assert ei.value.code == -4 and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.equal(C, C0)  # nothing launched
    # the edge-wise surface mode is refused as well
    small = W.square_mesh(8, 1.0, 0.2, 72)
    ds, Cs = setup(small, 2, 0, W.density_jump)
    ds.set_surface_mode(ds.SURFACE_EDGEWISE)
    with pytest.raises(B.DGError) as ei:
        ds.rk_step_noalloc(Cs, dt=1e-4)
    assert ei.value.code == -4
    dm.close()
    ds.close()
