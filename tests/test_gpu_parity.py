"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

FP64 bar: relative L2 error <= 1e-11 over all coefficients in the user
layout, and every element's coefficients within 1e-11 of the state's scale.
Integer / layout work (pack, unpack, permutation) is compared bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1601_07944_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-11


def case(msg):
    print(f"[gpu case] {msg}", file=sys.stderr, flush=True)


def torch_mod():
    import torch

    return torch


ELEMENTWISE, EDGEWISE, COLOURED = 0, 1, 2
# surface organisation and work-items per element of the element-wise path
# (third entry: volume integral on a second stream, edge-wise mode)
SURFACE = {"elementwise1": (ELEMENTWISE, 1), "elementwise4": (ELEMENTWISE, 4), "edgewise": (EDGEWISE, 0),
           "edgewise2streams": (EDGEWISE, 0, 1), "coloured": (COLOURED, 0)}


def gpu_mesh(mesh, p, surface=(ELEMENTWISE, 0)):
    from paper_1601_07944_amd import binding as B

    if surface[1] == 1 and p >= 4:
        pytest.skip("one lane per element is refused from p = 4 on (DG_EUNSUPPORTED)")

    dm = B.DGMesh.from_mesh(mesh, p)
    dm.set_surface_mode(surface[0])
    dm.set_lanes(surface[1])
    if len(surface) > 2:
        dm.set_stream_concurrency(surface[2])
    return dm


def to_dev(a):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def check_close(got, ref, tol=TOL):
    err = rel_l2(got, ref)
    scale = np.abs(ref).max()
    worst = np.abs(got - ref).max() / scale
    assert err <= tol and worst <= 10 * tol, (err, worst)
    return err


def gpu_rhs(mesh, p, C_user, surface=(ELEMENTWISE, 0)):
    dm = gpu_mesh(mesh, p, surface)
    C = dm.pack(to_dev(C_user))
    R = dm.rhs(C)
    out = dm.unpack(R).cpu().numpy()
    torch_mod().cuda.synchronize()
    return out


MESHES = {
    "square23_j0.2": lambda: W.square_mesh(23, 1.0, 0.2, 5),  # 1058 elements: 16 full blocks + ragged tail
    "delaunay517": lambda: W.delaunay_mesh(517, 6),  # 1034 elements, unstructured
}


@pytest.mark.parametrize("surface", sorted(SURFACE))
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("mname", sorted(MESHES))
def test_rhs_random_state(p, mname, surface):
    mesh = MESHES[mname]()
    orc = O.Oracle(mesh, p)
    C = W.random_state(mesh.n_elem, orc.np, seed=10 + p)
    case(f"dg_rhs p={p} mesh={mname} N={mesh.n_elem} seed={10 + p} surface={surface}")
    got = gpu_rhs(mesh, p, C, SURFACE[surface])
    check_close(got, orc.rhs(C))


@pytest.mark.parametrize("p", [1, 3])
def test_rhs_vortex_small_config(p):
    mesh = W.square_mesh(16, 10.0, 0.1, 0)  # 512 triangles on [0,10]^2
    orc = O.Oracle(mesh, p)
    C = orc.project(W.isentropic_vortex)
    case(f"dg_rhs vortex p={p} N=512")
    check_close(gpu_rhs(mesh, p, C), orc.rhs(C))


def test_rhs_full_size_p3_vortex():
    # the 32,768-triangle p=3 vortex workload, whole state against the oracle
    mesh = W.square_mesh(128, 10.0, 0.2, 1)
    orc = O.Oracle(mesh, 3)
    C = orc.project(W.isentropic_vortex)
    case("dg_rhs vortex p=3 N=32768 (full size)")
    check_close(gpu_rhs(mesh, 3, C), orc.rhs(C))


@pytest.mark.parametrize("surface", sorted(SURFACE))
@pytest.mark.parametrize("n,seed", [(1, 0), (32, 7), (33, 8), (1100, 9)])
def test_rhs_edge_sizes(n, seed, surface):
    # 2 elements (every side borders the other), exactly 64, 66, and 2200
    # elements (8 full 256-element workgroups + a ragged one: exercises the
    # XCD remap with a grid padded to a multiple of 8)
    mesh = W.square_mesh(1, 1.0, 0.0, 0) if n == 1 else W.delaunay_mesh(n, seed)
    for p in (1, 4):
        orc = O.Oracle(mesh, p)
        C = W.random_state(mesh.n_elem, orc.np, seed=seed)
        case(f"dg_rhs p={p} N={mesh.n_elem} surface={surface}")
        check_close(gpu_rhs(mesh, p, C, SURFACE[surface]), orc.rhs(C))


def test_pack_unpack_bit_exact():
    torch = torch_mod()
    mesh = W.delaunay_mesh(300, 2)
    for p in (1, 5):
        dm = gpu_mesh(mesh, p)
        C = np.random.default_rng(p).normal(size=(mesh.n_elem, 4, dm.np))
        case(f"dg_pack/dg_unpack p={p} N={mesh.n_elem}")
        back = dm.unpack(dm.pack(to_dev(C))).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(back, C)


@pytest.mark.parametrize("p", [1, 3, 5])
def test_quad_points_and_projection(p):
    mesh = W.square_mesh(9, 10.0, 0.2, 4)
    orc = O.Oracle(mesh, p)
    dm = gpu_mesh(mesh, p)
    case(f"dg_quad_points/dg_project p={p}")
    xy = dm.quad_points().cpu().numpy()
    # the library may order the points of its rule differently: compare sets
    xo = orc.quad_points()
    a = np.sort(xy[..., 0] * 1e3 + xy[..., 1], axis=1)
    b = np.sort(xo[..., 0] * 1e3 + xo[..., 1], axis=1)
    assert np.abs(a - b).max() < 1e-10
    u = W.isentropic_vortex(xy[..., 0], xy[..., 1])
    Cg = dm.unpack(dm.project(to_dev(u))).cpu().numpy()
    Co = orc.project(W.isentropic_vortex)
    check_close(Cg, Co, 1e-13)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_max_dt(p):
    mesh = W.delaunay_mesh(400, 9)
    orc = O.Oracle(mesh, p)
    C = orc.project(W.density_jump)
    dm = gpu_mesh(mesh, p)
    case(f"dg_max_dt p={p}")
    _, dt = dm.max_dt(dm.pack(to_dev(C)), 0.3 / (2 * p + 1))
    ref, rc = orc.max_dt(C, 0.3 / (2 * p + 1))
    assert rc == 0 and abs(dt - ref) <= 1e-14 * ref


def test_max_dt_nonphysical():
    from paper_1601_07944_amd import binding as B

    mesh = W.square_mesh(8, 1.0, 0.1, 1)
    orc = O.Oracle(mesh, 2)
    C = orc.project(W.smooth_density)
    C[17, 0, 0] = -0.5
    dm = gpu_mesh(mesh, 2)
    case("dg_max_dt non-physical mean")
    with pytest.raises(B.DGError) as ei:
        dm.max_dt(dm.pack(to_dev(C)), 0.1)
    assert ei.value.code == -7
    dt_dev, _ = dm.max_dt(dm.pack(to_dev(C)), 0.1, to_host=False)
    assert np.isnan(dt_dev.cpu().numpy()[0])


@pytest.mark.parametrize("surface", sorted(SURFACE))
def test_rk_step_vortex_to_t1_small_config(surface):
    # 512 triangles, p=1, isentropic vortex, SSP-RK3 with CFL 0.3/(2p+1) to t=1
    torch = torch_mod()
    mesh = W.square_mesh(16, 10.0, 0.1, 0)
    p = 1
    orc = O.Oracle(mesh, p)
    Co = orc.project(W.isentropic_vortex)
    dm = gpu_mesh(mesh, p, SURFACE[surface])
    Cg = dm.pack(to_dev(Co))
    t, T, cfl = 0.0, 1.0, 0.3 / (2 * p + 1)
    steps = 0
    case(f"dg_rk_step vortex p=1 N=512 to t=1 surface={surface}")
    while t < T - 1e-14:
        dto, _ = orc.max_dt(Co, cfl)
        _, dtg = dm.max_dt(Cg, cfl)
        assert abs(dtg - dto) <= 1e-12 * dto
        dt = min(dto, T - t)
        Co = orc.rk3_step(Co, dt)
        dm.rk_step(Cg, dt)
        t += dt
        steps += 1
    got = dm.unpack(Cg).cpu().numpy()
    torch.cuda.synchronize()
    assert steps > 100
    check_close(got, Co)


@pytest.mark.parametrize("surface", sorted(SURFACE))
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_ssp3_steps_every_order(p, surface):
    # ten SSP-RK3 steps of the vortex at every order and in every kernel
    # organisation (the one-lane kernels run with register spills at p >= 4)
    torch = torch_mod()
    mesh = W.delaunay_mesh(650, 40 + p)
    orc = O.Oracle(mesh, p)
    C0 = orc.project(W.isentropic_vortex, center=(0.5, 0.5), period=1.0, beta=1.0)
    dt, _ = orc.max_dt(C0, 0.3 / (2 * p + 1))
    dm = gpu_mesh(mesh, p, SURFACE[surface])
    case(f"dg_rk_step x10 p={p} surface={surface}")
    Cg = dm.pack(to_dev(C0))
    ref = C0
    for _ in range(10):
        dm.rk_step(Cg, dt)
        ref = orc.rk3_step(ref, dt)
    got = dm.unpack(Cg).cpu().numpy()
    torch.cuda.synchronize()
    check_close(got, ref)


def test_rk_step_device_dt_matches_host_dt():
    # the step length read from device memory (dg_max_dt output) gives the
    # same result bit for bit as the host value
    torch = torch_mod()
    mesh = W.delaunay_mesh(700, 3)
    orc = O.Oracle(mesh, 3)
    C0 = orc.project(W.density_jump)
    dm = gpu_mesh(mesh, 3)
    case("dg_rk_step device dt vs host dt p=3")
    A = dm.pack(to_dev(C0))
    Bst = A.clone()
    for _ in range(3):
        dt_dev, dt = dm.max_dt(A, 0.3 / 7)
        dm.rk_step(A, dt_dev=dt_dev)
        dm.rk_step(Bst, dt)
    torch.cuda.synchronize()
    assert torch.equal(A, Bst)
    ref = C0
    for _ in range(3):
        dt, _ = orc.max_dt(ref, 0.3 / 7)
        ref = orc.rk3_step(ref, dt)
    check_close(dm.unpack(A).cpu().numpy(), ref)


def test_bitwise_deterministic_across_streams():
    torch = torch_mod()
    mesh = W.delaunay_mesh(2000, 11)
    p = 2
    orc = O.Oracle(mesh, p)
    C0 = W.random_state(mesh.n_elem, orc.np, seed=3)
    dm = gpu_mesh(mesh, p)
    case("determinism p=2 two streams")
    C = dm.pack(to_dev(C0))
    r1 = dm.rhs(C).clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ws2 = torch.empty(dm.info.ws_rhs, dtype=torch.uint8, device="cuda")
        r2 = dm.rhs(C, ws=ws2, stream=s)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2)


@pytest.mark.parametrize("p", [1, 3, 5])
def test_surface_strategies_agree_and_conserve(p):
    # the two surface organisations give the same operator up to rounding;
    # element means change only through edge fluxes that cancel pairwise
    torch = torch_mod()
    mesh = W.delaunay_mesh(1500, 21)
    orc = O.Oracle(mesh, p)
    C = W.random_state(mesh.n_elem, orc.np, seed=5)
    case(f"surface strategies p={p}")
    a = gpu_rhs(mesh, p, C, SURFACE["elementwise1"])
    b = gpu_rhs(mesh, p, C, SURFACE["edgewise"])
    c = gpu_rhs(mesh, p, C, SURFACE["elementwise4"])
    d = gpu_rhs(mesh, p, C, SURFACE["coloured"])
    check_close(a, b, 1e-13)
    check_close(c, b, 1e-13)
    check_close(d, b, 1e-13)
    det = orc.det()
    for R in (a, b, c, d):
        terms = det[:, None] * R[:, :, 0]
        assert np.all(np.abs(terms.sum(0)) < 1e-13 * np.abs(terms).sum(0))


@pytest.mark.parametrize("p", [1, 3, 5])
def test_edge_colouring(p):
    # at most five colours; the coloured edges add into shared accumulators,
    # so a missed conflict would show as run-to-run differences: two runs
    # of ten steps agree bit for bit, and with the oracle
    torch = torch_mod()
    mesh = W.delaunay_mesh(1500, 50 + p)
    orc = O.Oracle(mesh, p)
    C0 = orc.project(W.density_jump)
    dt, _ = orc.max_dt(C0, 0.3 / (2 * p + 1))
    dm = gpu_mesh(mesh, p, SURFACE["coloured"])
    assert 3 <= dm.info.n_colours <= 5
    case(f"coloured edges x10 twice p={p} colours={dm.info.n_colours}")
    runs = []
    for _ in range(2):
        Cg = dm.pack(to_dev(C0))
        for _ in range(10):
            dm.rk_step(Cg, dt)
        runs.append(Cg)
    torch.cuda.synchronize()
    assert torch.equal(runs[0], runs[1])
    ref = C0
    for _ in range(10):
        ref = orc.rk3_step(ref, dt)
    check_close(dm.unpack(runs[0]).cpu().numpy(), ref)


@pytest.mark.parametrize("n,p", [(256, 1), (2000, 3), (16384, 2)])
def test_two_streams_equal_one_stream(n, p):
    # the edge-wise path with the volume integral on a second stream gives
    # the one-stream results bit for bit (right-hand side and ten steps,
    # twice), and its volume kernel shows up in the per-launch timing
    torch = torch_mod()
    mesh = W.delaunay_mesh(n, 60 + p)
    orc = O.Oracle(mesh, p)
    C0 = orc.project(W.density_jump)
    dt, _ = orc.max_dt(C0, 0.3 / (2 * p + 1))
    one = gpu_mesh(mesh, p, SURFACE["edgewise"])
    two = gpu_mesh(mesh, p, SURFACE["edgewise2streams"])
    case(f"edge-wise two streams vs one N={mesh.n_elem} p={p}")
    Cg = one.pack(to_dev(C0))
    assert torch.equal(one.rhs(Cg), two.rhs(Cg))
    two.timing(True)
    for _ in range(2):
        A, Bst = Cg.clone(), Cg.clone()
        for _ in range(10):
            one.rk_step(A, dt)
            two.rk_step(Bst, dt)
        torch.cuda.synchronize()
        assert torch.equal(A, Bst)
    kt = two.timing_read()
    two.timing(False)
    assert kt["volume"][1] == 60 and kt["element"][1] == 60 and kt["edge"][1] == 60


def test_full_size_p3_step_sampled():
    # the benchmark's launch configuration: 32,768 triangles, p=3, one
    # SSP-RK3 step with dt from dg_max_dt on the device; whole state checked
    torch = torch_mod()
    mesh = W.square_mesh(128, 10.0, 0.2, 1)
    orc = O.Oracle(mesh, 3)
    C0 = orc.project(W.isentropic_vortex)
    dm = gpu_mesh(mesh, 3)
    case("bench configuration: one step p=3 N=32768")
    Cg = dm.pack(to_dev(C0))
    ws = dm.workspace("step")
    dt_dev = torch.empty(1, dtype=torch.float64, device="cuda")
    dm.max_dt(Cg, 0.3 / 7, dt_dev=dt_dev, to_host=False, ws=ws)
    dm.rk_step(Cg, dt_dev=dt_dev, ws=ws)
    got = dm.unpack(Cg).cpu().numpy()
    dt, _ = orc.max_dt(C0, 0.3 / 7)
    check_close(got, orc.rk3_step(C0, dt))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("lanes", [1, 4])
def test_advance_equals_max_dt_plus_rk_step(lanes, prec):
    # dg_advance (step length fused into the stage kernels on the 4-lane
    # path) gives bit for bit the steps of dg_max_dt + dg_rk_step, and the
    # step-length history
    torch = torch_mod()
    mesh = W.delaunay_mesh(1600, 13)
    p = 3
    orc = O.Oracle(mesh, p)
    C0 = orc.project(W.density_jump)
    dm = gpu_mesh(mesh, p, (ELEMENTWISE, lanes))
    case(f"dg_advance lanes={lanes} prec={prec}")
    A = dm.pack(to_dev(C0))
    Bst = A.clone()
    cfl = 0.3 / 7
    hist = torch.empty(7, dtype=torch.float64, device="cuda")
    dm.advance(A, 7, cfl, dt_hist=hist, prec=prec)
    ref_hist = []
    dt_dev = torch.empty(1, dtype=torch.float64, device="cuda")
    for _ in range(7):
        dm.max_dt(Bst, cfl, dt_dev=dt_dev, to_host=False)
        ref_hist.append(dt_dev.clone())
        dm.rk_step(Bst, dt_dev=dt_dev, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(A, Bst)
    assert torch.equal(hist, torch.cat(ref_hist))
    if prec == 0:
        ref = C0
        for _ in range(7):
            ref = orc.rk3_step(ref, orc.max_dt(ref, cfl)[0])
        check_close(dm.unpack(A).cpu().numpy(), ref)


@pytest.mark.parametrize("p", [4, 5])
def test_one_lane_refused_from_p4(p):
    """From p = 4 on an element's coefficients and accumulators exceed one
    lane's registers: dg_set_lanes_per_element(1) is refused, four lanes and
    the automatic choice stay accepted, and the mesh keeps working."""
    from paper_1601_07944_amd import binding as B

    mesh = W.square_mesh(8, 1.0, 0.1, 3)
    dm = B.DGMesh.from_mesh(mesh, p)
    with pytest.raises(B.DGError) as ei:
        dm.set_lanes(1)
    assert ei.value.code == -4 and "p = 4" in str(ei.value)
    dm.set_lanes(4)
    dm.set_lanes(0)
    C = dm.pack(to_dev(W.random_state(mesh.n_elem, dm.np, 5)))
    R = dm.rhs(C)
    assert bool(torch_mod().isfinite(R).all())
    dm.close()
