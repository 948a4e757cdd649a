#!/usr/bin/env python3
"""Throughput of the modal DG hot path on one MI355X.

Headline workload: periodic Delaunay triangulation of 2,000,000 uniform
random points in the unit square (seed 4), exactly 4,000,000 triangles; the
density jump across r < 0.25 about (0.5, 0.5) on the smooth density wave
(u = v = 0.5, p = 1); p = 3 (10 modes, 12-point degree-6 volume rule, 4
Gauss points per edge); FP64.  The state (1.28 GB) is far larger than every
cache, so the stage kernels stream it from HBM.  One step is the whole hot
path: the CFL time-step reduction on the device followed by one SSP-RK3 step
(three right-hand sides, each one fused kernel: surface flux on each
element's sides, volume integral, inverse mass, stage update).

value = DOF-updates/s = N_elem * N_p * 4 variables * 3 RHS evaluations per
step / seconds per step, with the state resident in HBM.

Prints ONE JSON line.  Extra objects:
  roofline       the stage kernel's algorithmic bytes per launch over its
                 mean launch time (the timed region, HIP events on the
                 library's stream around K steps of dg_advance, less the
                 step-length reductions it contains, over 3K launches),
                 against the 8 TB/s HBM peak; `traffic` is the HBM bytes
                 per launch that rocprofv3 counters measured for the same
                 kernel source on this workload (null when the source has
                 changed since);
  cpu_baseline   the CPU oracle (serial C, OpenMP element loop) evaluating
                 the right-hand side of the same mesh and state on this
                 host's cores, and on one core;
  mixed          the same steps in mixed precision, and its state
                 difference to FP64;
  rhs_only       dg_rhs alone;
  adjoint_forward_ratio  reverse sweep (checkpoint every 20 steps, segment
                 recomputation) over 50 steps of this workload against the
                 forward steps, with and without recomputation, and with
                 every step's stage states kept by the forward pass in
                 device memory (192 GB here; skipped if they do not fit);
  orders         p = 1..5 on this mesh, FP64 and mixed, 50 steps each:
                 DOF-updates/s, stage launch time, algorithmic HBM fraction;
                 at p = 1 also the limiter's cost;
  adjoint_131072 the adjoint ratio on 131,072 jittered triangles, p = 2,
                 smooth data, 200 steps with a checkpoint every 20;
  mixed_workload FP64 against mixed precision on the 2,000,000-triangle
                 Delaunay mesh (1,000,000 points, seed 2), smooth data,
                 p = 2 and 4, 100 steps;
  cache_resident the 32,768-triangle isentropic vortex at p = 3 (state
                 10.5 MB, inside the 256 MB last-level cache), with the
                 other surface organisations and the limiter at p = 1;
  boundary_mesh  a 2,000,000-triangle channel (inflow, outflow, walls) at
                 p = 4: the automatic choice against the vector-ALU kernel.
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

# adj(J) (4) and 1/det J; per side: unit normal (2) and half length, the
# neighbour index; the neighbours' side indices
GEOMETRY_BYTES = 5 * 8 + 3 * (3 * 8 + 4) + 4

TARGET_POINTS, TARGET_SEED = 2_000_000, 4  # 4,000,000 triangles
TARGET_WORKLOAD = (
    "density jump (rho x0.5 inside r<0.25 about (0.5,0.5)) on the smooth density wave, periodic unit-square "
    "Delaunay triangulation of 2,000,000 uniform random points (seed 4), 4,000,000 triangles, p=3, FP64; "
    "step = device CFL reduction + SSP-RK3 step (3 fused RHS stage kernels)"
)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes_stage_kernel(n_elem: int, n_modes: int, stage0_reads: float) -> float:
    """Bytes the method itself must move in one fused stage launch: read the
    stage state and write the new one (2 x 8 B x 4 x N_p per element), read
    the stage-0 state in stages 2 and 3 (stage0_reads = launches that read
    it / launches), and read the element's geometry and connectivity
    (GEOMETRY_BYTES).  Re-reads of neighbour coefficients for the edge
    traces are implementation traffic and are not counted."""
    per_elem = 8.0 * 4 * n_modes * (2.0 + stage0_reads) + GEOMETRY_BYTES
    return per_elem * n_elem


def stage_source_digest() -> str:
    """sha256 prefix of what the stage kernels are compiled from: the kernel
    sources (the header and the per-order units) and the compiler flags."""
    import hashlib

    from paper_1601_07944_amd import build as Bd

    h = hashlib.sha256()
    for f in Bd.source_files():
        if os.path.basename(f).startswith("dg_kernels"):
            with open(f, "rb") as fh:
                h.update(fh.read())
    h.update(json.dumps([Bd.FLAGS, Bd.FILE_FLAGS]).encode())
    return h.hexdigest()[:16]


def load_traffic(key: str):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/
    traffic.json), if they were taken from the current kernel source."""
    path = os.path.join(HERE, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            ent = json.load(f).get(key)
        if not ent or ent.get("source_sha256_16") != stage_source_digest():
            return None
        return ent.get("bytes_per_launch")
    except (OSError, ValueError):
        return None


def stage_kernel(dm, prec) -> int:
    """The stage kernel the library's current choice runs for this precision:
    1 or 4 lanes per element, or 16 (FP64 on the matrix cores)."""
    from paper_1601_07944_amd import binding as B

    fp64, mixed = dm.kernel_choice()
    return fp64 if prec == B.DG_FP64 else mixed


def adjoint_kernel_name(dm, p):
    k = dm.adjoint_kernel()
    what = "adjoint of the fused RHS / SSP-RK3 stage"
    if k == 16:
        return f"k_stage_vjp_mx<{p}, 1..3> ({what}, 16 x 16 x 4 matrix products, 16 elements per wavefront)"
    if k == 4:
        return f"k_stage_vjp4<{p}, 1..3> ({what}, 4 lanes per element)"
    return f"k_stage_vjp<{p}, 1..3> ({what}, 1 lane per element)"


def stage_kernel_name(dm, p, prec=0):
    k = stage_kernel(dm, prec)
    t = "double" if prec == 0 else "float"
    what = "fused RHS: surface + volume + 1/det J + SSP-RK3 stage"
    if k == 16:
        return f"k_stage_mx<{p}, 1..3, {t}> ({what}, 16 x 16 x 4 matrix products, 16 elements per wavefront)"
    if k == 4:
        return f"k_stage4<{p}, 1..3, {t}> ({what}, 4 lanes per element)"
    return f"k_stage<{p}, 1..3, {t}> ({what}, 1 lane per element)"


class Timer:
    def __init__(self):
        import torch

        self.torch = torch
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def __call__(self, fn):
        """Milliseconds of fn()'s GPU work on the current stream."""
        self.torch.cuda.synchronize()
        self.e0.record()
        fn()
        self.e1.record()
        self.torch.cuda.synchronize()
        return self.e0.elapsed_time(self.e1)


def make_state(dm, init, dev):
    import numpy as np
    import torch

    xy = dm.quad_points().cpu().numpy()
    u = torch.from_numpy(np.ascontiguousarray(init(xy[..., 0], xy[..., 1]))).to(dev)
    del xy
    C = dm.project(u)
    del u
    return C


def advance_throughput(dm, C0, p, prec, steps, warmup, split_steps=10):
    """K steps of dg_advance (CFL step on the device + SSP-RK3) timed with
    HIP events, then a second pass with an event pair around every launch
    for the per-kernel split.  Returns (dict, final state)."""
    import torch

    from paper_1601_07944_amd import binding as B

    tm = Timer()
    cfl = 0.3 / (2 * p + 1)
    dt_dev = torch.empty(1, dtype=torch.float64, device=C0.device)
    ws = dm.workspace("step")
    if warmup:
        Cw = C0.clone()
        dm.advance(Cw, warmup, cfl, dt_dev=dt_dev, prec=prec, ws=ws)
        del Cw
    C = C0.clone()
    t0 = time.perf_counter()
    ms = tm(lambda: dm.advance(C, steps, cfl, dt_dev=dt_dev, prec=prec, ws=ws)) / steps
    wall = time.perf_counter() - t0
    # per-launch split over a few more steps (on a copy: C keeps exactly K steps)
    Cs = C.clone()
    dm.timing(True)
    ms_split = tm(lambda: dm.advance(Cs, split_steps, cfl, dt_dev=dt_dev, prec=prec, ws=ws)) / split_steps
    dm.timing(False)
    kt = dm.timing_read()
    del Cs
    st_ms, st_n = kt["stage"]
    dof = dm.n * dm.np * 4
    out = {
        "value": dof * 3 / (ms * 1e-3),
        "ms_per_step": ms,
        "ms_per_step_with_kernel_events": ms_split,
        "wall_s_timed_region": wall,
        "kernel": stage_kernel_name(dm, p, prec),
        "precision": "fp64" if prec == B.DG_FP64 else "mixed",
        "kernel_ms_per_step": {k: v[0] / split_steps for k, v in kt.items() if v[1]},
    }
    if st_n == 3 * split_steps:
        # the fused stage kernels: one launch per RK stage
        dt_per_step = kt["dt"][0] / split_steps  # separate reductions (none when fused into the stages)
        launch_ms = (ms - dt_per_step) / 3.0
        ach = algorithmic_bytes_stage_kernel(dm.n, dm.np, 2.0 / 3.0) / (launch_ms * 1e-3) / 1e9
        out.update({
            "stage_launch_us": launch_ms * 1e3,
            "stage_launch_us_with_event_pairs": st_ms / st_n * 1e3,
            "dt_reduction_us_per_step": dt_per_step * 1e3,
            "stage_hbm_GBs_algorithmic": ach,
            "frac_hbm": ach / HBM_PEAK_GBS,
        })
    return out, C


def adjoint_ratio(dm, C0, dt, nsteps, every):
    """Reverse sweep over nsteps SSP-RK3 steps with a fixed step length
    (checkpoint every `every` steps, each segment recomputed keeping its
    stage states, then the step adjoints) against the forward steps; and the
    step adjoints alone (stage states already stored)."""
    import torch

    from paper_1601_07944_amd import adjoint as A

    tm = Timer()
    Ca = C0.clone()
    dm.rk_step(Ca, dt)  # warm-up
    Ca = C0.clone()

    def fwd():
        for _ in range(nsteps):
            dm.rk_step(Ca, dt)

    ms_fwd = tm(fwd)
    ckpts = []
    Ca = C0.clone()
    for n in range(nsteps):
        if n % every == 0:
            ckpts.append(Ca.clone())
        dm.rk_step(Ca, dt)
    gN = torch.randn(Ca.shape, dtype=Ca.dtype, device=Ca.device, generator=torch.Generator(Ca.device).manual_seed(7))
    del Ca
    A.backward_sweep(dm, ckpts[:1], dt, min(every, nsteps), every, gN)  # warm-up
    torch.cuda.empty_cache()
    ms_rev = tm(lambda: A.backward_sweep(dm, ckpts, dt, nsteps, every, gN))
    del ckpts
    torch.cuda.empty_cache()
    Cs, u1s, u2s = C0.clone(), dm.empty_state(), dm.empty_state()
    dm.rk_step_stages(Cs, u1s, u2s, dt)
    g = [gN.clone()]

    def vjps():
        for _ in range(nsteps):
            g[0] = dm.rk_step_vjp(C0, g[0], dt, u1=u1s, u2=u2s)

    ms_vjp = tm(vjps)
    del Cs, u1s, u2s, g
    torch.cuda.empty_cache()
    # every step's stage states kept by the forward pass itself (3 nsteps
    # states in device memory, every = 0): the reverse sweep is then the step
    # adjoints alone; a first pass fills the allocator's cache
    need = 3 * nsteps * int(dm.info.state_len) * 8
    if A.choose_every(dm, nsteps) == 0:
        box = {}

        def fwd_keep():
            box["CN"], box["tape"] = A.forward_keep_all(dm, box.pop("C"), dt, nsteps)

        def rev_keep():
            box["g"] = A.backward_tape(dm, box.pop("tape"), dt, gN)

        times = []
        for _ in range(2):
            box.clear()
            box["C"] = C0.clone()
            t_f = tm(fwd_keep)
            t_r = tm(rev_keep)
            times.append((t_f, t_r))
        box.clear()
        ms_fk, ms_rk = times[-1]
        keep = {
            "ratio": ms_rk / ms_fwd,
            "forward_keeping_over_forward": ms_fk / ms_fwd,
            "ms_forward_keeping": ms_fk,
            "ms_reverse": ms_rk,
            "state_bytes": need,
        }
    else:
        free, _ = torch.cuda.mem_get_info()
        keep = {"skipped": f"needs {need / 1e9:.1f} GB of device memory, {free / 1e9:.1f} GB free"}
    torch.cuda.empty_cache()
    return {
        "ratio": ms_rev / ms_fwd,
        "ratio_without_recompute": ms_vjp / ms_fwd,
        "steps": nsteps,
        "checkpoint_every": every,
        "ms_forward": ms_fwd,
        "ms_reverse": ms_rev,
        "ms_step_adjoints_only": ms_vjp,
        "keep_all_stage_states": keep,
    }


def stream_copy(nbytes=2 << 30, reps=5):
    """Device-to-device copy of nbytes (torch's copy kernel), HIP events over
    reps copies: bytes read + written per second, the practical HBM ceiling
    beside the 8 TB/s peak."""
    import torch

    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    tm = Timer()
    ms = tm(lambda: [b.copy_(a) for _ in range(reps)]) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_moved": 2 * nbytes, "ms": ms, "GBs": 2 * nbytes / (ms * 1e-3) / 1e9}


def cpu_baseline(mesh, p, init, dof, n_all=3):
    """The oracle's right-hand side of the same mesh and state: n_all calls
    on every host core this process may use, then one call on one core."""
    import numpy as np

    import oracle as O

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    orc = O.Oracle(mesh, p)
    C = orc.project(init)
    used = O.set_threads(cores)
    t0 = time.perf_counter()
    for _ in range(n_all):
        R = orc.rhs(C)
    t_all = (time.perf_counter() - t0) / n_all
    O.set_threads(1)
    t0 = time.perf_counter()
    R = orc.rhs(C)
    t_one = time.perf_counter() - t0
    O.set_threads(cores)
    assert np.isfinite(R).all()
    return {
        "value": dof / t_all,
        "unit": "DOF-updates/s",
        "cores": used,
        "kind": "oracle",
        "sample": f"{n_all} right-hand-side evaluations of the same {mesh.n_elem}-triangle p={p} state on {used} "
        f"threads ({t_all:.2f} s each), plus one on 1 thread",
        "single_core": {"value": dof / t_one, "s_per_rhs": t_one},
        "s_per_rhs": t_all,
    }


def limiter_cost(dm, C0, steps):
    """The paper's limiter benchmark (Section "Limiting"): p = 1 steps with
    and without the Barth-Jespersen limiter after every RK stage."""
    import torch

    tm = Timer()
    dt_dev = torch.empty(1, dtype=torch.float64, device=C0.device)
    ws = dm.workspace("step")
    res = {}
    for name, lim in (("unlimited", dm.LIMITER_NONE), ("limited", dm.LIMITER_BJ)):
        dm.set_limiter(lim)
        C = C0.clone()
        dm.advance(C, 3, 0.1, dt_dev=dt_dev, ws=ws)
        res[name] = tm(lambda: dm.advance(C, steps, 0.1, dt_dev=dt_dev, ws=ws)) / steps
        del C
    C = C0.clone()
    dm.timing(True)
    dm.advance(C, 5, 0.1, dt_dev=dt_dev, ws=ws)
    torch.cuda.synchronize()
    dm.timing(False)
    kt = dm.timing_read()
    dm.set_limiter(dm.LIMITER_NONE)
    return {
        "steps": steps,
        "ms_per_step_unlimited": res["unlimited"],
        "ms_per_step_limited": res["limited"],
        "overhead": res["limited"] / res["unlimited"] - 1.0,
        "limit_kernel_us": kt["limit"][0] / max(1, kt["limit"][1]) * 1e3,
    }


def orders_sweep(mesh, headline_p3, mixed_p3, steps, dev):
    """p = 1..5 on the headline mesh, FP64 and mixed precision."""
    import torch

    from paper_1601_07944_amd import binding as B
    from paper_1601_07944_amd import workloads as W

    rows = []
    for p in (1, 2, 3, 4, 5):
        if p == 3:
            row = {"p": 3, "n_elem": mesh.n_elem, "dof": mesh.n_elem * 40, "fp64": headline_p3, "mixed": mixed_p3}
        else:
            dm = B.DGMesh.from_mesh(mesh, p)
            C0 = make_state(dm, W.density_jump, dev)
            row = {"p": p, "n_elem": dm.n, "dof": dm.n * dm.np * 4}
            r64, C64 = advance_throughput(dm, C0, p, B.DG_FP64, steps, 2)
            rmx, Cmx = advance_throughput(dm, C0, p, B.DG_MIXED, steps, 2)
            rmx["rel_l2_vs_fp64_after_steps"] = float(torch.linalg.norm(Cmx - C64) / torch.linalg.norm(C64))
            del C64, Cmx
            row["fp64"], row["mixed"] = r64, rmx
            if p == 1:
                row["limiter"] = limiter_cost(dm, C0, steps)
            dm.close()
            del C0, dm
            torch.cuda.empty_cache()
        row["mixed_speedup"] = row["fp64"]["ms_per_step"] / row["mixed"]["ms_per_step"]
        row["kernel"] = row["fp64"]["kernel"]
        log(f"p={p}: fp64 {row['fp64']['value']:.3e} DOF/s ({row['fp64']['ms_per_step']:.3f} ms/step, "
            f"frac {row['fp64']['frac_hbm']:.3f}), mixed x{row['mixed_speedup']:.3f}")
        rows.append(row)
    return rows


def adjoint_131072(dev):
    from paper_1601_07944_amd import binding as B
    from paper_1601_07944_amd import workloads as W

    mesh = W.square_mesh(256, 1.0, 0.2, 3)
    p = 2
    dm = B.DGMesh.from_mesh(mesh, p)
    C0 = make_state(dm, W.smooth_density, dev)
    _, dt = dm.max_dt(C0, 0.3 / (2 * p + 1))
    r = adjoint_ratio(dm, C0, dt, 200, 20)
    r["workload"] = ("smooth density wave, periodic unit square, 256x256x2 = 131,072 triangles jittered by 0.2h "
                     "(seed 3), p=2, FP64, fixed dt")
    r["adjoint_kernel"] = adjoint_kernel_name(dm, p)
    r["forward_kernel"] = stage_kernel_name(dm, p)
    dm.close()
    return r


def mixed_workload(steps, dev):
    import torch

    from paper_1601_07944_amd import binding as B
    from paper_1601_07944_amd import workloads as W

    t0 = time.perf_counter()
    mesh = W.delaunay_mesh(1_000_000, 2)
    log(f"mixed workload mesh: {mesh.n_elem} triangles in {time.perf_counter() - t0:.1f} s")
    rows = []
    for p in (2, 4):
        dm = B.DGMesh.from_mesh(mesh, p)
        C0 = make_state(dm, W.smooth_density, dev)
        r64, C64 = advance_throughput(dm, C0, p, B.DG_FP64, steps, 2)
        rmx, Cmx = advance_throughput(dm, C0, p, B.DG_MIXED, steps, 2)
        rows.append({
            "p": p,
            "n_elem": dm.n,
            "fp64": r64,
            "mixed": rmx,
            "mixed_speedup": r64["ms_per_step"] / rmx["ms_per_step"],
            "rel_l2_vs_fp64_after_steps": float(torch.linalg.norm(Cmx - C64) / torch.linalg.norm(C64)),
        })
        log(f"mixed workload p={p}: speedup {rows[-1]['mixed_speedup']:.3f}, "
            f"difference {rows[-1]['rel_l2_vs_fp64_after_steps']:.2e}")
        dm.close()
        del C0, C64, Cmx, dm
        torch.cuda.empty_cache()
    return {"workload": ("smooth density wave, periodic unit-square Delaunay triangulation of 1,000,000 uniform random "
                         "points (seed 2), 2,000,000 triangles"), "steps": steps, "orders": rows}


def two_stream_edgewise(steps):
    """The paper's suggestion for meshes too small to fill the device: the
    volume and surface kernels of the edge-wise organisation on two streams.
    SSP-RK3 steps of the density jump, p = 3, on jittered unit-square meshes
    of 512 to 32,768 triangles, one stream against two (same results bit for
    bit), with the fused element-wise step beside them."""
    import torch

    from paper_1601_07944_amd import binding as B
    from paper_1601_07944_amd import workloads as W

    tm = Timer()
    rows = []
    for n in (16, 32, 64, 128):
        mesh = W.square_mesh(n, 1.0, 0.2, 7)
        dm = B.DGMesh.from_mesh(mesh, 3)
        C0 = make_state(dm, W.density_jump, torch.device("cuda", 0))
        ws = dm.workspace("step")
        dt_dev, _ = dm.max_dt(C0, 0.3 / 7)
        row = {"n_elem": dm.n}
        for name, surface, conc in (("elementwise", dm.SURFACE_ELEMENTWISE, 0),
                                    ("edgewise_1stream", dm.SURFACE_EDGEWISE, 0),
                                    ("edgewise_2streams", dm.SURFACE_EDGEWISE, 1)):
            dm.set_surface_mode(surface)
            dm.set_stream_concurrency(conc)
            C = C0.clone()
            for _ in range(3):
                dm.rk_step(C, dt_dev=dt_dev, ws=ws)

            def run():
                for _ in range(steps):
                    dm.rk_step(C, dt_dev=dt_dev, ws=ws)

            row[name] = tm(run) / steps
        rows.append(row)
        dm.close()
    return {"workload": "density jump, p=3, jittered unit square, fixed dt, ms per SSP-RK3 step", "steps": steps,
            "rows": rows}


def cache_resident(steps, dev):
    """The 32,768-triangle isentropic vortex at p = 3 (10.5 MB state, inside
    the last-level cache), the other surface organisations and lane counts,
    and the limiter at p = 1 on 32,768 triangles."""
    from paper_1601_07944_amd import binding as B
    from paper_1601_07944_amd import workloads as W

    p = 3
    mesh = W.square_mesh(128, 10.0, 0.2, 1)
    dm = B.DGMesh.from_mesh(mesh, p)
    C0 = make_state(dm, W.isentropic_vortex, dev)
    res, C = advance_throughput(dm, C0, p, B.DG_FP64, steps, 5)
    res["workload"] = ("isentropic vortex, periodic [0,10]^2, 128x128x2 = 32,768 triangles jittered by 0.2h (seed 1), "
                       "p=3, FP64; the state (10.5 MB) stays in the last-level cache")
    rmx, _ = advance_throughput(dm, C0, p, B.DG_MIXED, steps, 5)
    res["mixed"] = {"ms_per_step": rmx["ms_per_step"], "speedup_vs_fp64": res["ms_per_step"] / rmx["ms_per_step"]}
    # the other FP64 stage kernels on the same workload (an explicit lane
    # count selects the vector-ALU kernels)
    res["alternatives"] = {}
    for lanes in (4, 1):
        dm.set_lanes(lanes)
        ra, _ = advance_throughput(dm, C0, p, B.DG_FP64, steps, 3)
        res["alternatives"][ra["kernel"]] = {"ms_per_step": ra["ms_per_step"], "stage_launch_us": ra.get("stage_launch_us")}
    dm.set_lanes(0)
    for name, mode in (("surface_edgewise", dm.SURFACE_EDGEWISE), ("surface_coloured", dm.SURFACE_COLOURED)):
        dm.set_surface_mode(mode)
        rs, _ = advance_throughput(dm, C0, p, B.DG_FP64, steps, 3)
        res[name] = {"ms_per_step": rs["ms_per_step"], "value": rs["value"]}
    dm.set_surface_mode(dm.SURFACE_ELEMENTWISE)
    dm.close()
    lmesh = W.square_mesh(128, 1.0, 0.2, 5)
    dl = B.DGMesh.from_mesh(lmesh, 1)
    Cl = make_state(dl, W.density_jump, dev)
    res["limiter_p1_32768"] = limiter_cost(dl, Cl, steps)
    dl.close()
    res["edgewise_two_streams"] = two_stream_edgewise(steps)
    return res


def counter_pass(args):
    """For rocprofv3 --pmc runs: --steps steps of the headline workload (or
    the cache-resident one) for every order in --p and every precision in
    --counter-prec, then a 256 MiB device copy of known size, the
    calibration kernel for FETCH_SIZE / WRITE_SIZE."""
    import torch

    from paper_1601_07944_amd import binding as B
    from paper_1601_07944_amd import workloads as W

    dev = torch.device("cuda", 0)
    if args.counter_workload == "cache_resident":
        mesh, init = W.square_mesh(128, 10.0, 0.2, 1), W.isentropic_vortex
    else:
        mesh, init = W.delaunay_mesh(TARGET_POINTS, TARGET_SEED), W.density_jump
    dt_dev = torch.empty(1, dtype=torch.float64, device=dev)
    for p in [int(x) for x in str(args.p).split(",")]:
        dm = B.DGMesh.from_mesh(mesh, p)
        C0 = make_state(dm, init, dev)
        for name in args.counter_prec.split(","):
            prec = B.DG_MIXED if name == "mixed" else B.DG_FP64
            C = C0.clone()
            dm.advance(C, args.steps, 0.3 / (2 * p + 1), dt_dev=dt_dev, prec=prec)
            torch.cuda.synchronize()
            log(f"counter pass: p={p} {name} {args.steps} steps")
            del C
        if args.counter_adjoint:
            # --steps step adjoints (stage states stored, fixed dt)
            _, dt = dm.max_dt(C0, 0.3 / (2 * p + 1))
            u1, u2 = dm.empty_state(), dm.empty_state()
            Cs = C0.clone()
            dm.rk_step_stages(Cs, u1, u2, dt)
            g = torch.ones_like(C0)
            for _ in range(args.steps):
                g = dm.rk_step_vjp(C0, g, dt, u1=u1, u2=u2)
            torch.cuda.synchronize()
            log(f"counter pass: p={p} {args.steps} step adjoints")
            del Cs, u1, u2, g
        dm.close()
        del C0, dm
        torch.cuda.empty_cache()
    a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)  # 256 MiB
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"counter_pass": True, "p": args.p, "prec": args.counter_prec, "n_elem": mesh.n_elem,
                      "steps": args.steps, "copy_bytes": a.numel() * 8,
                      "stage_source_sha256_16": stage_source_digest()}), flush=True)


def boundary_mesh(steps, dev):
    """A channel with every boundary kind: 1000 x 1000 x 2 = 2,000,000
    jittered triangles (0.2h, seed 4) on the unit square, prescribed state on
    the left, outflow on the right, walls at the bottom and top, smooth flow,
    p = 4: the stage launch time of the automatic choice (the matrix-core
    kernel's boundary variants) against the vector-ALU kernel, FP64 and
    mixed."""
    import numpy as np
    import torch

    from paper_1601_07944_amd import binding as B
    from paper_1601_07944_amd import workloads as W

    def flow(x, y):
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
        u = 0.3 + 0.1 * np.cos(2 * np.pi * y)
        v = -0.2 + 0.1 * np.sin(2 * np.pi * x)
        p = 1.0 + 0.1 * np.cos(2 * np.pi * (x + y))
        return W.primitive_to_conserved(rho, u, v, p)

    p = 4
    mesh = W.box_mesh(1000, 1000, 1.0, 1.0, 0.2, 4, bc=(W.BC_STATE, W.BC_OUTFLOW, W.BC_WALL, W.BC_WALL))
    dm = B.DGMesh.from_mesh(mesh, p)
    dm.set_boundary_state(W.primitive_to_conserved(np.array(1.2), np.array(0.4), np.array(-0.1),
                                                   np.array(1.1)).reshape(4))
    C0 = make_state(dm, flow, dev)
    res = {"workload": "channel, 2,000,000 jittered triangles, inflow / outflow / walls, smooth flow",
           "n_elem": dm.n, "p": p, "steps": steps}
    for prec, name in ((B.DG_FP64, "fp64"), (B.DG_MIXED, "mixed")):
        row = {}
        for label, mx in (("automatic", None), ("vector_alu", False)):
            dm.set_matrix_cores(mx)
            r, _ = advance_throughput(dm, C0, p, prec, steps, 3)
            row[label] = {"kernel": stage_kernel_name(dm, p, prec), "stage_launch_us": r["stage_launch_us"],
                          "ms_per_step": r["ms_per_step"]}
        dm.set_matrix_cores(None)
        row["speedup"] = row["vector_alu"]["stage_launch_us"] / row["automatic"]["stage_launch_us"]
        res[name] = row
    dm.close()
    del C0, dm
    torch.cuda.empty_cache()
    return res


def section(out, name, fn):
    """Runs one extra measurement; a Python error there is recorded in its
    place instead of losing the whole line."""
    t0 = time.perf_counter()
    log(f"{name} ...")
    try:
        out[name] = fn()
    except Exception as e:  # noqa: BLE001 -- the headline must still print
        out[name] = {"error": f"{type(e).__name__}: {e}"}
        log(f"{name} failed: {e}")
    log(f"{name} done in {time.perf_counter() - t0:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--sweep-steps", type=int, default=50, help="steps per order and precision in the order sweep")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline, mixed and rhs_only only")
    ap.add_argument("--counter-pass", action="store_true",
                    help="for rocprofv3 --pmc runs: --steps steps, then a 256 MiB copy; prints nothing else")
    ap.add_argument("--counter-prec", default="fp64", help="fp64, mixed or both (comma-separated)")
    ap.add_argument("--counter-adjoint", action="store_true",
                    help="counter pass: also --steps step adjoints (SSP-RK3, stage states stored)")
    ap.add_argument("--counter-workload", choices=["target", "cache_resident"], default="target")
    ap.add_argument("--p", default="3", help="orders of the counter pass (comma-separated)")
    ap.add_argument("--only", choices=["boundary_mesh"],
                    help="run only this extra measurement (for profiling it) and print its JSON object")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the path runs on a single MI355X; a multi-GPU run "
              "(element partition + halo exchange) is not implemented.", file=sys.stderr)
        sys.exit(2)

    from paper_1601_07944_amd import build as Bd

    Bd.ensure_built()
    import torch

    from paper_1601_07944_amd import binding as B
    from paper_1601_07944_amd import workloads as W

    B.load()  # raises if the HIP library is not built
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.only == "boundary_mesh":
        print(json.dumps({"boundary_mesh": boundary_mesh(min(args.steps, 20), dev)}), flush=True)
        return
    if args.counter_pass:
        counter_pass(args)
        return

    p = 3
    t0 = time.perf_counter()
    mesh = W.delaunay_mesh(TARGET_POINTS, TARGET_SEED)
    log(f"headline mesh: {mesh.n_elem} triangles in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    dm = B.DGMesh.from_mesh(mesh, p)
    C0 = make_state(dm, W.density_jump, dev)
    log(f"dg_mesh_create + projection: {time.perf_counter() - t0:.1f} s")
    dof = dm.n * dm.np * 4

    head, C64 = advance_throughput(dm, C0, p, B.DG_FP64, args.steps, args.warmup)
    log(f"headline: {head['value']:.4e} DOF-updates/s, {head['ms_per_step']:.3f} ms/step, "
        f"stage {head['stage_launch_us']:.1f} us, frac {head['frac_hbm']:.3f}")
    mixed, Cmx = advance_throughput(dm, C0, p, B.DG_MIXED, args.steps, args.warmup)
    mixed["speedup_vs_fp64"] = head["ms_per_step"] / mixed["ms_per_step"]
    mixed["rel_l2_vs_fp64_after_steps"] = float(torch.linalg.norm(Cmx - C64) / torch.linalg.norm(C64))
    mixed["steps"] = args.steps
    log(f"mixed: x{mixed['speedup_vs_fp64']:.3f}, difference {mixed['rel_l2_vs_fp64_after_steps']:.2e}")
    del Cmx
    _, dt_host = dm.max_dt(C64, 0.3 / 7)
    assert dt_host > 0
    del C64

    # dg_rhs alone
    tm = Timer()
    R = dm.empty_state()
    rws = dm.workspace("rhs")
    for _ in range(3):
        dm.rhs(C0, out=R, ws=rws)
    nr = max(5, args.steps)

    def rhs_calls():
        for _ in range(nr):
            dm.rhs(C0, out=R, ws=rws)

    ms_rhs = tm(rhs_calls) / nr
    del R

    launch_ms = head["stage_launch_us"] * 1e-3
    ach = head["stage_hbm_GBs_algorithmic"]
    log("stream copy ...")
    tkey = f"stage_p3_delaunay4m_{ {1: 'lanes1', 4: 'lanes4', 16: 'mx'}[stage_kernel(dm, B.DG_FP64)] }"
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": TARGET_WORKLOAD, "n_elem": dm.n, "p": p, "dof": dof},
        "roofline": {
            "kernel": stage_kernel_name(dm, p),
            "bound": "hbm",
            "achieved": ach,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS,
            "traffic": load_traffic(tkey),
            "algorithmic_bytes_per_launch": algorithmic_bytes_stage_kernel(dm.n, dm.np, 2.0 / 3.0),
            "launch_us": launch_ms * 1e3,
            "launch_us_with_event_pairs": head["stage_launch_us_with_event_pairs"],
        },
        "stream_copy": stream_copy(),
        "fp64": head,
        "mixed": mixed,
        "rhs_only": {"value": dof / (ms_rhs * 1e-3), "unit": "DOF-updates/s", "ms_per_call": ms_rhs},
        "library_source_sha256_16": Bd.source_hash(),
    }
    if not args.quick:
        section(out, "adjoint_forward_ratio", lambda: dict(adjoint_ratio(dm, C0, dt_host, 50, 20),
                                                           workload="the headline workload, fixed dt",
                                                           adjoint_kernel=adjoint_kernel_name(dm, p),
                                                           forward_kernel=stage_kernel_name(dm, p)))
    dm.close()
    del C0, dm
    torch.cuda.empty_cache()
    if not args.quick:
        section(out, "orders", lambda: orders_sweep(mesh, head, mixed, args.sweep_steps, dev))
        if not args.no_cpu_baseline:
            section(out, "cpu_baseline", lambda: cpu_baseline(mesh, p, W.density_jump, dof))
        del mesh
        section(out, "adjoint_131072", lambda: adjoint_131072(dev))
        section(out, "mixed_workload", lambda: mixed_workload(100, dev))
        section(out, "cache_resident", lambda: cache_resident(min(args.steps, 50), dev))
        section(out, "boundary_mesh", lambda: boundary_mesh(20, dev))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
