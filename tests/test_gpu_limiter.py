"""GPU Barth-Jespersen limiter (p = 1, Section "Limiting Kernel") through the
C ABI against the oracle's limiter, on its own (dg_limit) and inside limited
SSP-RK3 steps (dg_rk_step, dg_advance with dg_set_limiter).

Bar: 1e-11 relative L2 over all coefficients (FP64); dg_advance equals
dg_max_dt + dg_rk_step bit for bit with the limiter on, as without it."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_07944_amd import workloads as W
from test_oracle_limiter import rough_state

pytestmark = pytest.mark.gpu
BJ = 1


def case(msg):
    print(f"[gpu case] {msg}", file=sys.stderr, flush=True)


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_mesh(mesh, p, lanes=0):
    from paper_1601_07944_amd import binding as B

    dm = B.DGMesh.from_mesh(mesh, p)
    dm.set_lanes(lanes)
    return dm


MESHES = {
    "delaunay700": lambda: W.delaunay_mesh(700, 13),
    "square23": lambda: W.square_mesh(23, 1.0, 0.2, 14),
    "two": lambda: W.square_mesh(1, 1.0, 0.0, 0),
}


@pytest.mark.parametrize("state", ["rough", "mild", "jump"])
@pytest.mark.parametrize("mname", sorted(MESHES))
def test_limit_matches_oracle(mname, state):
    mesh = MESHES[mname]()
    orc = O.Oracle(mesh, 1)
    if state == "rough":
        C = rough_state(mesh.n_elem, 21)
    elif state == "mild":
        C = W.random_state(mesh.n_elem, 3, seed=22)
    else:
        C = orc.project(W.density_jump)
    dm = gpu_mesh(mesh, 1)
    case(f"dg_limit {mname} {state}")
    got = dm.unpack(dm.limit(dm.pack(dev(C)))).cpu().numpy()
    ref = orc.limit(C)
    assert np.array_equal(got[:, :, 0], C[:, :, 0])
    assert rel_l2(got, ref) <= 1e-11


@pytest.mark.parametrize("lanes", [1, 4])
def test_limited_steps_match_oracle(lanes):
    import torch

    mesh = W.delaunay_mesh(900, 15)
    orc = O.Oracle(mesh, 1)
    C0 = orc.project(W.density_jump)
    dt, _ = orc.max_dt(C0, 0.1)
    dm = gpu_mesh(mesh, 1, lanes)
    dm.set_limiter(BJ)
    case(f"limited dg_rk_step x20 lanes={lanes}")
    Cg = dm.pack(dev(C0))
    ref = C0
    dm.timing(True)
    for _ in range(20):
        dm.rk_step(Cg, dt)
        ref = orc.rk3_step(ref, dt, limit=True)
    torch.cuda.synchronize()
    dm.timing(False)
    kt = dm.timing_read()
    assert rel_l2(dm.unpack(Cg).cpu().numpy(), ref) <= 1e-11
    # a limiter pass after every stage
    assert kt["limit"][1] == 60, kt
    # and it is not the unlimited step
    un = C0
    for _ in range(20):
        un = orc.rk3_step(un, dt)
    assert rel_l2(un, ref) > 1e-6


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("lanes", [1, 4])
def test_limited_advance_equals_max_dt_plus_rk_step(lanes, prec):
    import torch

    mesh = W.delaunay_mesh(1100, 16)
    orc = O.Oracle(mesh, 1)
    C0 = orc.project(W.density_jump)
    dm = gpu_mesh(mesh, 1, lanes)
    dm.set_limiter(BJ)
    case(f"limited dg_advance lanes={lanes} prec={prec}")
    A = dm.pack(dev(C0))
    Bst = A.clone()
    hist = torch.empty(10, dtype=torch.float64, device="cuda")
    dm.advance(A, 10, 0.1, dt_hist=hist, prec=prec)
    dt_dev = torch.empty(1, dtype=torch.float64, device="cuda")
    ref_hist = []
    for _ in range(10):
        dm.max_dt(Bst, 0.1, dt_dev=dt_dev, to_host=False)
        ref_hist.append(dt_dev.clone())
        dm.rk_step(Bst, dt_dev=dt_dev, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(A, Bst)
    assert torch.equal(hist, torch.cat(ref_hist))


def test_limiter_errors():
    from paper_1601_07944_amd import binding as B

    mesh = W.square_mesh(4, 1.0, 0.1, 0)
    dm2 = gpu_mesh(mesh, 2)
    C2 = dm2.pack(dev(W.random_state(mesh.n_elem, dm2.np, 1)))
    case("limiter error paths")
    with pytest.raises(B.DGError) as ei:
        dm2.set_limiter(BJ)
    assert ei.value.code == -4
    with pytest.raises(B.DGError) as ei:
        dm2.limit(C2)
    assert ei.value.code == -4
    dm1 = gpu_mesh(mesh, 1)
    with pytest.raises(B.DGError) as ei:
        dm1.set_limiter(7)
    assert ei.value.code == -1
    dm1.set_limiter(BJ)
    C1 = dm1.pack(dev(W.random_state(mesh.n_elem, 3, 2)))
    with pytest.raises(B.DGError) as ei:
        dm1.rk_step_vjp(C1, C1.clone(), 1e-3)
    assert ei.value.code == -4
    dm1.set_surface_mode(dm1.SURFACE_EDGEWISE)
    with pytest.raises(B.DGError) as ei:
        dm1.rk_step(C1, 1e-3)
    assert ei.value.code == -4
