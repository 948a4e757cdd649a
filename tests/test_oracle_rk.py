"""Pins of the oracle's classic Runge-Kutta steps (Section "Time-stepping":
explicit RK of order two and four), CPU only.

  * temporal order: on a fixed semi-discrete problem (vortex, p=2), errors
    against a fine-step solution fall like dt^2 (Heun) and dt^4 (classic
    RK4) — a dropped or misweighted stage lowers the order;
  * conservation of the means and free-stream preservation;
  * the limited variants end on a fixed point of the limiter.
"""
import numpy as np
import pytest

import oracle as O
from paper_1601_07944_amd import workloads as W


@pytest.mark.parametrize("scheme,order", [("rk2", 2), ("rk4", 4)])
def test_temporal_order(scheme, order):
    mesh = W.square_mesh(8, 10.0, 0.1, 2)
    orc = O.Oracle(mesh, 2)
    C0 = orc.project(W.isentropic_vortex)
    dt0, _ = orc.max_dt(C0, 0.3 / 5)
    T = 12 * dt0

    def run(nsteps):
        C = C0.copy()
        for _ in range(nsteps):
            C = orc.rk_step(C, T / nsteps, scheme)
        return C

    ref = run(256)
    # coarse enough that the fourth-order errors stay far above rounding
    errs = [np.abs(run(n) - ref).max() for n in (4, 8, 16)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > order - 0.2), rates
    assert np.all(rates < order + 0.6), rates


@pytest.mark.parametrize("scheme", ["rk2", "rk4"])
def test_conservation_and_free_stream(scheme):
    mesh = W.delaunay_mesh(200, 4)
    orc = O.Oracle(mesh, 3)
    det = orc.det()
    C = orc.project(W.isentropic_vortex, center=(0.5, 0.5), period=1.0, beta=0.5)
    dt, _ = orc.max_dt(C, 0.3 / 7)
    C1 = orc.rk_step(C, dt, scheme)
    tot0 = (det[:, None] * C[:, :, 0]).sum(0)
    tot1 = (det[:, None] * C1[:, :, 0]).sum(0)
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * (det[:, None] * np.abs(C[:, :, 0])).sum(0))
    F = orc.project(W.free_stream)
    dtf, _ = orc.max_dt(F, 0.3 / 7)
    assert np.abs(orc.rk_step(F, dtf, scheme) - F).max() < 1e-13


@pytest.mark.parametrize("scheme", ["rk2", "rk4"])
def test_limited_step_ends_on_limiter_fixed_point(scheme):
    mesh = W.delaunay_mesh(300, 6)
    orc = O.Oracle(mesh, 1)
    C = orc.project(W.density_jump)
    dt, _ = orc.max_dt(C, 0.1)
    C1 = orc.rk_step(C, dt, scheme, limit=True)
    assert np.abs(orc.limit(C1) - C1).max() <= 1e-14 * np.abs(C1).max()
    assert np.abs(C1 - orc.rk_step(C, dt, scheme)).max() > 1e-8
