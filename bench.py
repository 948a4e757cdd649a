#!/usr/bin/env python3
"""Throughput of the modal DG hot path on one MI355X.

Workload: isentropic vortex on the periodic square [0,10]^2, 128 x 128
squares split into 32,768 triangles (vertices jittered by up to 0.2h, seed
1), p = 3 (10 modes, 12-point degree-6 volume rule, 4 Gauss points per
edge), FP64.  One step is the whole hot path: the CFL time-step reduction
on the device followed by one SSP-RK3 step (three right-hand sides, each
one fused kernel: surface flux on each element's sides, volume integral,
inverse mass, stage update).

value = DOF-updates/s = N_elem * N_p * 4 variables * 3 RHS evaluations per
step / seconds per step, with the state resident in HBM.

Prints ONE JSON line.  Extra objects:
  roofline      the dominant kernel's algorithmic bytes per launch over its
                average launch time, against the 8 TB/s HBM peak: the timed
                region (HIP events on the library's stream around K steps of
                dg_advance, whose launches are the 3K stage kernels and one
                step-length reduction) less that reduction's time, over 3K;
                a second pass with an event pair around every launch gives
                the per-kernel split (the pairs add ~2 us per launch);
  cpu_baseline  the CPU oracle (serial C, OpenMP element loop) timed on this
                host on a bounded sample of the same workload;
  rhs_only      dg_rhs alone, DOF-updates/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "DOF-updates/s of DG RHS at p=3, FP64 vs mixed; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0


GEOMETRY_BYTES = 5 * 8 + 3 * (3 * 8 + 4) + 4  # adj(J), 1/det J; per side normal, half length, neighbour; sides


def algorithmic_bytes_stage_kernel(n_elem: int, n_modes: int, stage0_reads: float) -> float:
    """Bytes the method itself must move in one fused stage launch: read the
    stage state and write the new one (2 x 8 B x 4 x N_p per element), read
    the stage-0 state in stages 2 and 3 (stage0_reads = launches that read
    it / launches), and read the element's geometry and connectivity
    (GEOMETRY_BYTES).  Re-reads of neighbour coefficients for the edge
    traces are implementation traffic and are not counted."""
    per_elem = 8.0 * 4 * n_modes * (2.0 + stage0_reads) + GEOMETRY_BYTES
    return per_elem * n_elem


STAGE_SOURCE_END = "// ---------------------------------------------------------------- limiter"


def stage_source_digest() -> str:
    """sha256 prefix of what the stage kernels are compiled from: the kernel
    header up to the limiter section (physics, helpers, the fused stage
    kernels) and the compiler flags."""
    import hashlib

    from paper_1601_07944_amd import build as Bd

    src = open(os.path.join(HERE, "paper_1601_07944_amd", "csrc", "dg_kernels.h")).read()
    text = src[: src.index(STAGE_SOURCE_END)] + "\n".join(Bd.FLAGS)
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM bytes per launch measured with rocprofv3 counters, if the summary
    in profiles/ was taken from the current stage-kernel source."""
    path = os.path.join(HERE, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
        ent = rec.get(kernel)
        if not ent or ent.get("source_sha256_16") != stage_source_digest():
            return None
        return ent.get("bytes_per_launch")
    except Exception:
        return None


def cpu_baseline(mesh, p, seconds: float):
    """Oracle SSP-RK3 steps on the same mesh and state for about `seconds`."""
    import numpy as np

    import oracle as O
    from paper_1601_07944_amd import workloads as W

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = O.set_threads(cores)
    orc = O.Oracle(mesh, p)
    C = orc.project(W.isentropic_vortex)
    dt, _ = orc.max_dt(C, 0.3 / (2 * p + 1))
    steps = 0
    t0 = time.perf_counter()
    while True:
        orc.max_dt(C, 0.3 / (2 * p + 1))
        C = orc.rk3_step(C, dt)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 1000:
            break
    dof = mesh.n_elem * orc.np * 4
    assert np.isfinite(C).all()
    return {
        "value": dof * 3 * steps / el,
        "unit": "DOF-updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{steps} SSP-RK3 steps (+ CFL reduction) of the same {mesh.n_elem}-triangle p={p} vortex state, "
        f"{el:.1f} s wall",
    }


def two_stream_edgewise(steps: int):
    """The paper's suggestion for meshes too small to fill the device: the
    volume and surface kernels of the edge-wise organisation on two streams.
    SSP-RK3 steps of the density jump, p = 3, on jittered unit-square meshes
    of 512 to 32,768 triangles, one stream against two (same results bit for
    bit), with the fused element-wise step beside them."""
    import numpy as np
    import torch

    from paper_1601_07944_amd import binding as B
    from paper_1601_07944_amd import workloads as W

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    rows = []
    for n in (16, 32, 64, 128):
        mesh = W.square_mesh(n, 1.0, 0.2, 7)
        dm = B.DGMesh.from_mesh(mesh, 3)
        xy = dm.quad_points().cpu().numpy()
        C0 = dm.project(torch.from_numpy(np.ascontiguousarray(W.density_jump(xy[..., 0], xy[..., 1]))).cuda())
        ws = dm.workspace("step")
        dt_dev, _ = dm.max_dt(C0, 0.3 / 7)
        row = {"n_elem": dm.n}
        for name, surface, conc in (("elementwise", dm.SURFACE_ELEMENTWISE, 0), ("edgewise_1stream", dm.SURFACE_EDGEWISE, 0),
                                    ("edgewise_2streams", dm.SURFACE_EDGEWISE, 1)):
            dm.set_surface_mode(surface)
            dm.set_stream_concurrency(conc)
            C = C0.clone()
            for _ in range(5):
                dm.rk_step(C, dt_dev=dt_dev, ws=ws)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(steps):
                dm.rk_step(C, dt_dev=dt_dev, ws=ws)
            e1.record()
            torch.cuda.synchronize()
            row[name] = e0.elapsed_time(e1) / steps
        rows.append(row)
        dm.close()
    return {"workload": "density jump, p=3, jittered unit square, fixed dt, ms per SSP-RK3 step", "steps": steps,
            "rows": rows}


def limiter_overhead(steps: int):
    """The paper's limiter benchmark (Section "Limiting"): p = 1 steps with
    and without the Barth-Jespersen limiter after every RK stage, here on
    128 x 128 x 2 = 32,768 jittered triangles of the unit square with the
    density jump across r < 0.25 (a discontinuity the limiter acts on)."""
    import numpy as np
    import torch

    from paper_1601_07944_amd import binding as B
    from paper_1601_07944_amd import workloads as W

    mesh = W.square_mesh(128, 1.0, 0.2, 5)
    dm = B.DGMesh.from_mesh(mesh, 1)
    xy = dm.quad_points().cpu().numpy()
    C0 = dm.project(torch.from_numpy(np.ascontiguousarray(W.density_jump(xy[..., 0], xy[..., 1]))).cuda())
    ws = dm.workspace("step")
    dt_dev = torch.empty(1, dtype=torch.float64, device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    res = {}
    for name, lim in (("unlimited", B.DGMesh.LIMITER_NONE), ("limited", B.DGMesh.LIMITER_BJ)):
        dm.set_limiter(lim)
        C = C0.clone()
        dm.advance(C, 5, 0.1, dt_dev=dt_dev, ws=ws)
        torch.cuda.synchronize()
        e0.record()
        dm.advance(C, steps, 0.1, dt_dev=dt_dev, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / steps
    dm.timing(True)
    dm.advance(C0.clone(), 10, 0.1, dt_dev=dt_dev, ws=ws)
    torch.cuda.synchronize()
    dm.timing(False)
    kt = dm.timing_read()
    dm.close()
    return {
        "workload": "density jump, periodic unit square, 32,768 jittered triangles, p=1, CFL 0.1",
        "steps": steps,
        "ms_per_step_unlimited": res["unlimited"],
        "ms_per_step_limited": res["limited"],
        "overhead": res["limited"] / res["unlimited"] - 1.0,
        "limit_kernel_us": kt["limit"][0] / max(1, kt["limit"][1]) * 1e3,
    }


def run_scale(args):
    """Per-order throughput at scale (one JSON line with a list): periodic
    unit square, density jump across r < 0.25 about (0.5, 0.5) on the smooth
    density wave (u = v = 0.5, p = 1), or the smooth wave alone
    (--data smooth), FP64 and mixed precision, K steps each; the stage
    kernel's algorithmic bytes per launch over its mean launch time against
    the HBM peak, and the mixed form's state difference to FP64 after the
    K steps."""
    import numpy as np
    import torch

    from paper_1601_07944_amd import binding as B
    from paper_1601_07944_amd import workloads as W

    B.load()
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    if args.mesh == "delaunay":
        mesh = W.delaunay_mesh(args.n_tri // 2, 4)
    else:
        n = int(round((args.n_tri / 2) ** 0.5))
        mesh = W.square_mesh(n, 1.0, 0.2, 4)
    t_mesh = time.perf_counter() - t0
    print(f"[scale] mesh {mesh.name}: {mesh.n_elem} triangles in {t_mesh:.1f} s", file=sys.stderr, flush=True)
    res = []
    for p in [int(x) for x in args.orders.split(",")]:
        dm = B.DGMesh.from_mesh(mesh, p)
        xy = dm.quad_points().cpu().numpy()
        init = W.smooth_density if args.data == "smooth" else W.density_jump
        C0 = dm.project(torch.from_numpy(np.ascontiguousarray(init(xy[..., 0], xy[..., 1]))).to(dev))
        del xy
        ws = dm.workspace("step")
        dt_dev = torch.empty(1, dtype=torch.float64, device=dev)
        cfl = 0.3 / (2 * p + 1)
        dof = dm.n * dm.np * 4
        row = {"p": p, "n_elem": dm.n, "dof": dof}
        finals = {}
        variants = [("fp64", B.DG_FP64, 0, 0), ("mixed", B.DG_MIXED, 0, 0)]
        if not args.no_lane_variants:
            variants += [("fp64_lanes1", B.DG_FP64, 1, 0), ("fp64_lanes4", B.DG_FP64, 4, 0)]
        if args.surface_variants:
            variants += [("fp64_edgewise", B.DG_FP64, 0, dm.SURFACE_EDGEWISE),
                         ("fp64_coloured", B.DG_FP64, 0, dm.SURFACE_COLOURED)]
        for name, prec, lanes, surface in variants:
            dm.set_lanes(lanes)
            dm.set_surface_mode(surface)
            C = C0.clone()

            def step(k=1):
                dm.advance(C, k, cfl, dt_dev=dt_dev, prec=prec, ws=ws)

            Cw = C0.clone()  # warm-up on a copy, so that C takes exactly K steps
            dm.advance(Cw, 2, cfl, dt_dev=dt_dev, prec=prec, ws=ws)
            del Cw
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            step(args.steps)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            if name in ("fp64", "mixed"):
                finals[name] = C.clone()
            dm.timing(True)
            step(min(args.steps, 10))
            torch.cuda.synchronize()
            dm.timing(False)
            kt = dm.timing_read()
            dm.set_surface_mode(dm.SURFACE_ELEMENTWISE)
            if surface:
                row[name] = {"value": dof * 3 / (ms * 1e-3), "ms_per_step": ms,
                             "kernel_ms_per_launch": {k: v[0] / v[1] for k, v in kt.items() if v[1]}}
                if surface == dm.SURFACE_COLOURED:
                    row[name]["colours"] = int(dm.info.n_colours)
                print(f"[scale] p={p} {name}: {row[name]}", file=sys.stderr, flush=True)
                del C
                continue
            st_ms = kt["stage"][0] / kt["stage"][1]
            ach = algorithmic_bytes_stage_kernel(dm.n, dm.np, 2.0 / 3.0) / (st_ms * 1e-3) / 1e9
            row[name] = {
                "value": dof * 3 / (ms * 1e-3),
                "ms_per_step": ms,
                "stage_ms": st_ms,
                "dt_ms": (kt["dt"][0] / kt["dt"][1]) if kt["dt"][1] else 0.0,
                "stage_hbm_GBs_algorithmic": ach,
                "frac_hbm": ach / HBM_PEAK_GBS,
            }
            print(f"[scale] p={p} {name}: {row[name]}", file=sys.stderr, flush=True)
            del C
        row["mixed_speedup"] = row["fp64"]["ms_per_step"] / row["mixed"]["ms_per_step"]
        row["mixed_rel_l2_vs_fp64"] = float(torch.linalg.norm(finals["mixed"] - finals["fp64"]) /
                                            torch.linalg.norm(finals["fp64"]))
        print(f"[scale] p={p} mixed speedup {row['mixed_speedup']:.3f}, state difference "
              f"{row['mixed_rel_l2_vs_fp64']:.2e}", file=sys.stderr, flush=True)
        del finals
        res.append(row)
        dm.close()
        del C0, ws
        torch.cuda.empty_cache()
    out = {
        "workload": f"{'smooth density wave' if args.data == 'smooth' else 'density jump on the smooth wave'}, "
        f"periodic unit square, {mesh.n_elem} triangles ({args.mesh}), SSP-RK3 steps with device CFL step",
        "steps": args.steps,
        "orders": res,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument(
        "--counter-pass",
        action="store_true",
        help="for rocprofv3 --pmc runs: a few steps of the workload, then a 256 MiB device copy of known size "
        "(the calibration kernel for FETCH_SIZE / WRITE_SIZE); prints nothing else",
    )
    ap.add_argument("--counter-prec", choices=["fp64", "mixed"], default="fp64",
                    help="precision of the counter pass's steps")
    ap.add_argument("--workload", choices=["vortex", "scale"], default="vortex",
                    help="vortex: the 32,768-triangle p=3 headline workload (default); scale: per-order sweep at scale")
    ap.add_argument("--mesh", choices=["square", "delaunay"], default="square", help="scale workload mesh")
    ap.add_argument("--n-tri", type=int, default=4_000_000, help="scale workload triangles")
    ap.add_argument("--orders", default="1,2,3,4,5", help="scale workload orders")
    ap.add_argument("--data", choices=["jump", "smooth"], default="jump", help="scale workload initial data")
    ap.add_argument("--no-lane-variants", action="store_true", help="scale workload: automatic lanes only")
    ap.add_argument("--surface-variants", action="store_true",
                    help="scale workload: also time the edge-wise and coloured surface modes (FP64)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(
            "bench.py measures one GPU: the path runs on a single MI355X; a multi-GPU run "
            "(element partition + halo exchange) is not implemented.",
            file=sys.stderr,
        )
        sys.exit(2)

    from paper_1601_07944_amd import build as Bd

    Bd.ensure_built()
    if args.workload == "scale":
        run_scale(args)
        return

    import numpy as np
    import torch

    from paper_1601_07944_amd import binding as B
    from paper_1601_07944_amd import workloads as W

    B.load()  # raises if the HIP library is not built
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    p = 3
    mesh = W.square_mesh(128, 10.0, 0.2, 1)
    dm = B.DGMesh.from_mesh(mesh, p)
    xy = dm.quad_points().cpu().numpy()
    u = torch.from_numpy(np.ascontiguousarray(W.isentropic_vortex(xy[..., 0], xy[..., 1]))).to(dev)
    C = dm.project(u)
    ws = dm.workspace("step")
    dt_dev = torch.empty(1, dtype=torch.float64, device=dev)
    cfl = 0.3 / (2 * p + 1)
    dof = dm.n * dm.np * 4

    def steps_prec(state, prec, k):
        # k steps of the whole hot path: CFL step length on the device, then
        # one SSP-RK3 step (three fused stages), in one library call
        dm.advance(state, k, cfl, dt_dev=dt_dev, prec=prec, ws=ws)

    def step_prec(state, prec):
        steps_prec(state, prec, 1)

    def step():
        step_prec(C, B.DG_FP64)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.counter_pass:
        for _ in range(args.steps):
            step_prec(C, B.DG_MIXED if args.counter_prec == "mixed" else B.DG_FP64)
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)  # 256 MiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"counter_pass": True, "steps": args.steps, "copy_bytes": a.numel() * 8}), flush=True)
        return

    # timed region
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    steps_prec(C, B.DG_FP64, args.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps

    # the same K steps again with a pair of HIP events around every kernel
    # launch (on the stream the kernels run on): per-kernel durations
    dm.timing(True)
    torch.cuda.synchronize()
    e0.record()
    steps_prec(C, B.DG_FP64, args.steps)
    e1.record()
    torch.cuda.synchronize()
    dm.timing(False)
    kt = dm.timing_read()
    ms_step_events = e0.elapsed_time(e1) / args.steps
    _, dt_host = dm.max_dt(C, cfl)
    assert np.isfinite(dt_host) and dt_host > 0

    # dg_rhs alone
    R = dm.empty_state()
    rws = dm.workspace("step")
    for _ in range(5):
        dm.rhs(C, out=R, ws=rws)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        dm.rhs(C, out=R, ws=rws)
    e1.record()
    torch.cuda.synchronize()
    ms_rhs = e0.elapsed_time(e1) / args.steps

    kernels = {
        k: {"ms_per_launch": (ms / n if n else None), "launches": n, "share": ms / max(1e-30, sum(v[0] for v in kt.values()))}
        for k, (ms, n) in kt.items()
        if n
    }
    dominant = max(kt, key=lambda k: kt[k][0])
    st_ms, st_n = kt["stage"]
    assert st_n == 3 * args.steps, kt
    launch_ms = (ms_step * args.steps - kt["dt"][0]) / (3 * args.steps)
    ach = algorithmic_bytes_stage_kernel(dm.n, dm.np, 2.0 / 3.0) / (launch_ms * 1e-3) / 1e9
    traffic = load_traffic("stage")

    # mixed precision (FP32 contractions/fluxes, FP64 means, update, dt):
    # same steps, and its error after K steps against the FP64 path
    C64 = C.clone()
    Cmx = C.clone()
    for _ in range(5):
        step_prec(Cmx, B.DG_MIXED)
    Cmx.copy_(C64)
    torch.cuda.synchronize()
    e0.record()
    steps_prec(Cmx, B.DG_MIXED, args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms_step_mixed = e0.elapsed_time(e1) / args.steps
    steps_prec(C64, B.DG_FP64, args.steps)
    torch.cuda.synchronize()
    mixed_err = float(torch.linalg.norm(Cmx - C64) / torch.linalg.norm(C64))

    # adjoint: reverse sweep over the same number of steps with a fixed dt
    # (checkpoint every 20 steps, segment recomputation keeping the stage
    # states, then the step adjoints) against the forward steps
    from paper_1601_07944_amd import adjoint as A

    nadj = max(20, min(args.steps, 200) // 20 * 20)
    Ca = C.clone()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(nadj):
        dm.rk_step(Ca, dt_host)
    e1.record()
    torch.cuda.synchronize()
    ms_fwd = e0.elapsed_time(e1)
    ckpts = []
    Ca = C.clone()
    for n in range(nadj):
        if n % 20 == 0:
            ckpts.append(Ca.clone())
        dm.rk_step(Ca, dt_host)
    gN = torch.randn_like(Ca)
    A.backward_sweep(dm, ckpts[:1], dt_host, 20, 20, gN)  # warm-up
    torch.cuda.synchronize()
    e0.record()
    A.backward_sweep(dm, ckpts, dt_host, nadj, 20, gN)
    e1.record()
    torch.cuda.synchronize()
    ms_rev = e0.elapsed_time(e1)
    # the step adjoints alone (stage states already stored)
    Cs, u1s, u2s = C.clone(), dm.empty_state(), dm.empty_state()
    dm.rk_step_stages(Cs, u1s, u2s, dt_host)
    g = gN.clone()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(nadj):
        g = dm.rk_step_vjp(C, g, dt_host, u1=u1s, u2=u2s)
    e1.record()
    torch.cuda.synchronize()
    ms_vjp = e0.elapsed_time(e1)

    # the other element-wise variant (1 or 4 work-items per element)
    auto4 = dm.info.n_elem <= 1048576 or p >= 4
    lanes_alt = 1 if auto4 else 4
    dm.set_lanes(lanes_alt)
    steps_prec(C, B.DG_FP64, 5)
    torch.cuda.synchronize()
    e0.record()
    steps_prec(C, B.DG_FP64, args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms_step_alt = e0.elapsed_time(e1) / args.steps
    dm.set_lanes(0)

    # the paper's edge-wise organisation (3 kernels per RHS), same steps
    dm.set_surface_mode(dm.SURFACE_EDGEWISE)
    steps_prec(C, B.DG_FP64, 5)
    torch.cuda.synchronize()
    e0.record()
    steps_prec(C, B.DG_FP64, args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms_step_edge = e0.elapsed_time(e1) / args.steps

    # coloured edges: one launch per colour, lifts added in place
    dm.set_surface_mode(dm.SURFACE_COLOURED)
    steps_prec(C, B.DG_FP64, 5)
    torch.cuda.synchronize()
    e0.record()
    steps_prec(C, B.DG_FP64, args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms_step_col = e0.elapsed_time(e1) / args.steps
    dm.set_surface_mode(dm.SURFACE_ELEMENTWISE)

    limiter = limiter_overhead(args.steps)
    streams = two_stream_edgewise(args.steps)

    out = {
        "metric": METRIC,
        "value": dof * 3 / (ms_step * 1e-3),
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "isentropic vortex, periodic [0,10]^2, 32,768 jittered triangles (0.2h, seed 1), p=3, "
            "FP64; step = CFL reduction + SSP-RK3 step (3 RHS)",
            "n_elem": dm.n,
            "p": p,
            "dof": dof,
        },
        "roofline": {
            "kernel": "k_stage4<3, 1..3, double> (fused RHS: surface + volume + 1/det J + SSP-RK3 stage)",
            "launch_us": launch_ms * 1e3,
            "launch_us_with_event_pairs": st_ms / st_n * 1e3,
            "bound": "hbm",
            "achieved": ach,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS,
            "traffic": traffic,
            "dominant_kernel_by_time": dominant,
        },
        "kernels": kernels,
        "ms_per_step_with_kernel_events": ms_step_events,
        "surface_edgewise": {"ms_per_step": ms_step_edge, "value": dof * 3 / (ms_step_edge * 1e-3)},
        "surface_coloured": {"ms_per_step": ms_step_col, "value": dof * 3 / (ms_step_col * 1e-3),
                             "colours": int(dm.info.n_colours)},
        "edgewise_two_streams": streams,
        "lanes_per_element": {"headline": 4 if auto4 else 1, "alternative": lanes_alt,
                              "alternative_ms_per_step": ms_step_alt},
        "wall_s_timed_region": wall,
        "rhs_only": {"value": dof / (ms_rhs * 1e-3), "unit": "DOF-updates/s", "ms_per_call": ms_rhs},
        "mixed": {
            "value": dof * 3 / (ms_step_mixed * 1e-3),
            "ms_per_step": ms_step_mixed,
            "speedup_vs_fp64": ms_step / ms_step_mixed,
            "rel_l2_vs_fp64_after_steps": mixed_err,
            "steps": args.steps,
        },
        "adjoint_forward_ratio": {
            "ratio": ms_rev / ms_fwd,
            "ratio_without_recompute": ms_vjp / ms_fwd,
            "steps": nadj,
            "checkpoint_every": 20,
            "ms_forward": ms_fwd,
            "ms_reverse": ms_rev,
        },
    }
    out["limiter_overhead"] = limiter
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mesh, p, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
