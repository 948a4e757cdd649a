"""CPU oracle of the modal DG method -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never imports it, and it imports nothing from the product path: the only
shared module is the seeded input generator (meshes and initial data).

The arithmetic lives in dg_oracle.c (plain serial FP64 C, element by
element, every edge flux evaluated from both sides) and quadrature.py (the
quadrature rules from their moment equations).  This file only builds that C
file with gcc and marshals arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import quadrature

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dg_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile dg_oracle.c with gcc (-O2, no fast-math, OpenMP loop pragmas)."""
    srcs = [_SRC, os.path.join(_HERE, "dg_oracle_forward.inc")]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in srcs):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _configure(lib):
    lib.orc_create.restype = ctypes.c_void_p
    lib.orc_create.argtypes = [
        ctypes.c_int,
        ctypes.c_int64,
        _dp,
        ctypes.POINTER(ctypes.c_int64),
        ctypes.POINTER(ctypes.c_int8),
        ctypes.c_double,
        ctypes.c_int,
        _dp,
        _dp,
        _dp,
        ctypes.c_int,
        _dp,
        _dp,
    ]
    lib.orc_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_rhs.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.orc_project.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.orc_quad_points.argtypes = [ctypes.c_void_p, _dp]
    lib.orc_map_points.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]
    lib.orc_eval.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, _dp, _dp, _dp]
    lib.orc_det.argtypes = [ctypes.c_void_p, _dp]
    lib.orc_max_dt.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, _dp]
    lib.orc_max_dt.restype = ctypes.c_int
    lib.orc_rk3_step.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double]
    lib.orc_limit_bj.argtypes = [ctypes.c_void_p, _dp]
    lib.orc_limit_bj.restype = ctypes.c_int
    lib.orc_rk3_step_limited.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double]
    lib.orc_rk3_step_limited.restype = ctypes.c_int
    lib.orc_rk_step.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, ctypes.c_int, ctypes.c_int]
    lib.orc_rk_step.restype = ctypes.c_int
    lib.orc_set_bc_state.argtypes = [ctypes.c_void_p, _dp]
    lib.orc_basis.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
    _cp = ctypes.POINTER(ctypes.c_double * 2)
    lib.orc_cs_rhs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.orc_rhs_vjp.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.orc_rk3_step_vjp.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, _dp, _dp]
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_set_threads.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def source() -> str:
    """The oracle's C source as one file (the forward include inlined), for
    compiling modified copies in the mutation tests."""
    with open(_SRC) as f:
        src = f.read()
    with open(os.path.join(_HERE, "dg_oracle_forward.inc")) as f:
        inc = f.read()
    return src.replace('#include "dg_oracle_forward.inc"', inc)


def load_variant(src: str, path: str):
    """Compile a modified copy of the oracle source to `path` and load it.
    Used only by the mutation tests, which plant a mistake in a copy of the
    oracle and check that the pins catch it."""
    cpath = path[:-3] + ".c"
    with open(cpath, "w") as f:
        f.write(src)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", path, cpath, "-lm"], check=True)
    return _configure(ctypes.CDLL(path))


def _p(a):
    return a.ctypes.data_as(_dp)


def n_modes(p: int) -> int:
    return (p + 1) * (p + 2) // 2


def basis(p: int, r, s):
    """phi, dphi/dr, dphi/ds at points (r, s): arrays [npts, np]."""
    lib = _load()
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    s = np.atleast_1d(np.asarray(s, dtype=np.float64))
    np_ = n_modes(p)
    phi = np.empty((r.size, np_))
    dr = np.empty((r.size, np_))
    ds = np.empty((r.size, np_))
    for k in range(r.size):
        lib.orc_basis(p, float(r[k]), float(s[k]), _p(phi[k]), _p(dr[k]), _p(ds[k]))
    return phi, dr, ds


def set_threads(n: int) -> int:
    """Set the OpenMP thread count of the element loop; returns the count."""
    return _load().orc_set_threads(int(n))


class Oracle:
    """Reference DG operator on one mesh at order p (user layout [N][4][Np])."""

    def __init__(self, mesh, p: int, gamma: float = 1.4, lib=None):
        lib = lib if lib is not None else _load()
        self.p = p
        self.np = n_modes(p)
        self.n = mesh.n_elem
        self.gamma = gamma
        self.qr, self.qs, self.qw = quadrature.triangle_rule(p)
        self.gx, self.gw = quadrature.gauss_legendre(p + 1)
        self.nq = self.qr.size
        self.ne = self.gx.size
        self._keep = [mesh.vxy, mesh.nbr_elem, mesh.nbr_side]
        ctx = lib.orc_create(
            p,
            self.n,
            _p(mesh.vxy),
            mesh.nbr_elem.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            mesh.nbr_side.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
            gamma,
            self.nq,
            _p(self.qr),
            _p(self.qs),
            _p(self.qw),
            self.ne,
            _p(self.gx),
            _p(self.gw),
        )
        if not ctx:
            raise ValueError("oracle: unsupported order")
        self.has_boundary = bool((mesh.nbr_elem < 0).any())
        self._ctx = ctypes.c_void_p(ctx)
        self._lib = lib

    def __del__(self):
        try:
            self._lib.orc_destroy(self._ctx)
        except Exception:
            pass

    def _state(self, C):
        C = np.ascontiguousarray(C, dtype=np.float64)
        assert C.shape == (self.n, 4, self.np), C.shape
        return C

    def rhs(self, C):
        C = self._state(C)
        R = np.empty_like(C)
        self._lib.orc_rhs(self._ctx, _p(C), _p(R))
        return R

    def rhs_complex(self, C):
        """The forward operator on a complex state (complex-step derivatives:
        Im R(C + i h d) / h = (dR/dC) d to rounding for tiny h)."""
        C = np.ascontiguousarray(C, dtype=np.complex128)
        assert C.shape == (self.n, 4, self.np)
        R = np.empty_like(C)
        self._lib.orc_cs_rhs(self._ctx, C.ctypes.data, R.ctypes.data)
        return R

    def set_bc_state(self, U):
        """Conserved state (rho, rho u, rho v, E) of boundary code -3."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (4,)
        self._lib.orc_set_bc_state(self._ctx, _p(U))

    def rhs_vjp(self, C, Rbar):
        """Hand-written adjoint: (dR/dC)^T Rbar (boundary sides through their
        ghost states)."""
        C = self._state(C)
        Rbar = self._state(Rbar)
        Cb = np.empty_like(C)
        self._lib.orc_rhs_vjp(self._ctx, _p(C), _p(Rbar), _p(Cb))
        return Cb

    def rk3_step_vjp(self, C, dt, ubar):
        """Adjoint of one SSP-RK3 step with fixed dt."""
        C = self._state(C)
        ubar = self._state(ubar)
        Cb = np.empty_like(C)
        self._lib.orc_rk3_step_vjp(self._ctx, _p(C), float(dt), _p(ubar), _p(Cb))
        return Cb

    def quad_points(self):
        xy = np.empty((self.n, self.nq, 2))
        self._lib.orc_quad_points(self._ctx, _p(xy))
        return xy

    def map_points(self, r, s):
        r = np.ascontiguousarray(r, dtype=np.float64)
        s = np.ascontiguousarray(s, dtype=np.float64)
        xy = np.empty((self.n, r.size, 2))
        self._lib.orc_map_points(self._ctx, r.size, _p(r), _p(s), _p(xy))
        return xy

    def project_values(self, u):
        """Project point values u[N][nq][4] given at quad_points()."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        assert u.shape == (self.n, self.nq, 4)
        C = np.empty((self.n, 4, self.np))
        self._lib.orc_project(self._ctx, _p(u), _p(C))
        return C

    def project(self, fn, **kw):
        xy = self.quad_points()
        return self.project_values(fn(xy[..., 0], xy[..., 1], **kw))

    def eval(self, C, r, s):
        C = self._state(C)
        r = np.ascontiguousarray(r, dtype=np.float64)
        s = np.ascontiguousarray(s, dtype=np.float64)
        out = np.empty((self.n, r.size, 4))
        self._lib.orc_eval(self._ctx, _p(C), r.size, _p(r), _p(s), _p(out))
        return out

    def det(self):
        d = np.empty(self.n)
        self._lib.orc_det(self._ctx, _p(d))
        return d

    def max_dt(self, C, cfl):
        C = self._state(C)
        dt = np.empty(1)
        rc = self._lib.orc_max_dt(self._ctx, _p(C), float(cfl), _p(dt))
        return float(dt[0]), rc

    def rk3_step(self, C, dt, limit=False):
        """One SSP-RK3 step; with limit=True (p = 1 only) the Barth-Jespersen
        limiter is applied after every stage and to the new state."""
        C = self._state(C).copy()
        if limit:
            if self._lib.orc_rk3_step_limited(self._ctx, _p(C), float(dt)) != 0:
                raise ValueError("the limiter is defined for p = 1 only")
        else:
            self._lib.orc_rk3_step(self._ctx, _p(C), float(dt))
        return C

    def rk_step(self, C, dt, scheme, limit=False):
        """One step of the paper's classic RK integrators: scheme "rk2"
        (Heun) or "rk4"; "ssp3" is rk3_step."""
        if scheme == "ssp3":
            return self.rk3_step(C, dt, limit)
        C = self._state(C).copy()
        if self._lib.orc_rk_step(self._ctx, _p(C), float(dt), {"rk2": 1, "rk4": 2}[scheme], int(limit)) != 0:
            raise ValueError("unsupported scheme / limiter combination")
        return C

    def limit(self, C):
        """Barth-Jespersen slope limiter (p = 1): a limited copy of C."""
        C = self._state(C).copy()
        if self._lib.orc_limit_bj(self._ctx, _p(C)) != 0:
            raise ValueError("the limiter is defined for p = 1 only")
        return C

    # -- error norms -------------------------------------------------------
    def l2_error(self, C, exact, mask=None, **kw):
        """Per-variable L2 error of U_h against exact(x, y, **kw), using a
        collapsed Gauss-Jacobi product rule with (p+3)^2 points per element
        (exact for polynomials of degree <= 2p+4)."""
        from scipy.special import roots_jacobi

        n1 = self.p + 3
        a, wa = roots_jacobi(n1, 0.0, 0.0)
        b, wb = roots_jacobi(n1, 1.0, 0.0)
        # (xi, eta) in [-1,1]^2 -> r = (1+xi)(1-eta)/4, s = (1+eta)/2; dr ds = (1-eta)/8 dxi deta
        XI, ETA = np.meshgrid(a, b, indexing="ij")
        W = np.outer(wa, wb) / 8.0  # the (1-eta) factor is in the Jacobi weight
        r = ((1 + XI) * (1 - ETA) / 4).ravel()
        s = ((1 + ETA) / 2).ravel()
        w = W.ravel()
        Uh = self.eval(C, r, s)
        xy = self.map_points(r, s)
        ue = exact(xy[..., 0], xy[..., 1], **kw)
        d2 = ((Uh - ue) ** 2 * w[None, :, None]).sum(axis=1) * self.det()[:, None]
        if mask is not None:
            d2 = d2[mask]
        return np.sqrt(d2.sum(axis=0))
