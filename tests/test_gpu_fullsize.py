"""GPU checks of the code paths that only large meshes reach, at sizes the
oracle cannot follow step by step: the step-length reduction of dg_advance
when its per-block minima are too many to be reduced inside the first stage
kernel (a separate final pass), compared bit for bit with dg_max_dt +
dg_rk_step, and its first step length against the oracle's."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_07944_amd import workloads as W

pytestmark = pytest.mark.gpu

FUSE_MAX = 4096  # per-block minima that the first stage kernel reduces itself


def case(msg):
    print(f"[gpu case] {msg}", file=sys.stderr, flush=True)


@pytest.mark.parametrize(
    "p,n_side,prec",
    [
        (1, 388, 0),  # 301,088 elements: 4,705 stage-3 minima > 4,096
        (4, 388, 0),
        (1, 725, 0),  # 1,051,250 elements: also the first step's 4,107 minima
        (1, 725, 1),
    ],
)
def test_advance_with_separate_final_pass(p, n_side, prec):
    import torch

    from paper_1601_07944_amd import binding as B

    mesh = W.square_mesh(n_side, 1.0, 0.2, 21)
    case(f"dg_advance separate final pass p={p} n={mesh.n_elem} prec={prec}")
    dm = B.DGMesh.from_mesh(mesh, p)
    dm.set_lanes(4)
    assert dm.info.n_elem_pad // 64 > FUSE_MAX
    first_separate = (dm.n + 255) // 256 > FUSE_MAX
    assert first_separate == (n_side == 725)
    xy = dm.quad_points().cpu().numpy()
    C0 = dm.project(torch.from_numpy(np.ascontiguousarray(W.density_jump(xy[..., 0], xy[..., 1]))).cuda())
    del xy
    cfl = 0.3 / (2 * p + 1)
    nsteps = 3
    A = C0.clone()
    hist = torch.empty(nsteps, dtype=torch.float64, device="cuda")
    dm.advance(A, nsteps, cfl, dt_hist=hist, prec=prec)
    Bst = C0.clone()
    dt_dev = torch.empty(1, dtype=torch.float64, device="cuda")
    ref_hist = []
    for _ in range(nsteps):
        dm.max_dt(Bst, cfl, dt_dev=dt_dev, to_host=False)
        ref_hist.append(dt_dev.clone())
        dm.rk_step(Bst, dt_dev=dt_dev, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(hist, torch.cat(ref_hist))
    assert torch.equal(A, Bst)
    assert torch.isfinite(A).all()
    # the first step length against the oracle's reduction of the same state
    orc = O.Oracle(mesh, p)
    dt_orc, _ = orc.max_dt(dm.unpack(C0).cpu().numpy(), cfl)
    assert abs(hist[0].item() - dt_orc) <= 1e-14 * dt_orc
    dm.close()
