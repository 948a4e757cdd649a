"""Convergence of the oracle's scheme on the isentropic vortex (test
infrastructure).

The vortex is an exact smooth solution of the Euler equations (eq. (euler)).
With the free stream at rest it is steady and the error is purely spatial:
order p+1 is expected (the paper's convergence table shows rates near p+1 at
steady state).  Advected with the free stream, the proven rate of upwind-type
DG on general triangulations is p+1/2 (and is sharp); the observed rate lies
between the two.  The time step is that of the finest mesh on every level,
so the SSP-RK3 error stays below the spatial one.
"""
import functools

import numpy as np
import pytest

import oracle as O
from paper_1601_07944_amd import workloads as W

O.set_threads(8)


def run_levels(p, vel, T, ns=(16, 32, 64)):
    fn = functools.partial(W.isentropic_vortex, vel=vel)
    fine = W.square_mesh(ns[-1], 10.0, 0.2, 1)
    of = O.Oracle(fine, p)
    dt, _ = of.max_dt(of.project(fn), 0.3 / (2 * p + 1))
    nsteps = int(np.ceil(T / dt))
    dt = T / nsteps
    errs = []
    for n in ns:
        m = W.square_mesh(n, 10.0, 0.2, 1)
        orc = O.Oracle(m, p)
        C = orc.project(fn)
        for _ in range(nsteps):
            C = orc.rk3_step(C, dt)
        c = np.array([5.0 + vel[0] * T, 5.0 + vel[1] * T])
        mask = ((m.centroids() - c) ** 2).sum(1) < 9.0
        errs.append(orc.l2_error(C, fn, mask=mask, t=T)[0])
    errs = np.array(errs)
    return np.log2(errs[:-1] / errs[1:]), errs


@pytest.mark.parametrize("p", [1, 2, 3])
def test_steady_vortex_order_p_plus_1(p):
    rates, errs = run_levels(p, (0.0, 0.0), 0.2)
    assert rates[-1] >= p + 1 - 0.3, (rates, errs)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_advected_vortex_order(p):
    rates, errs = run_levels(p, (1.0, 1.0), 0.2)
    assert rates[-1] >= p + 0.5 - 0.1, (rates, errs)
