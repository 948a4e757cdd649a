"""ctypes binding of libdgmi (include/dg.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; this module
passes device pointers of torch tensors and the current HIP stream through
the C ABI and turns status codes into exceptions.  It never computes any
part of the method itself and has no CPU fallback: if libdgmi.so is missing
or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgmi.so")

DG_FP64 = 0
DG_MIXED = 1

STATUS = {
    0: "DG_OK",
    -1: "DG_EINVAL",
    -2: "DG_EMESH",
    -3: "DG_EORDER",
    -4: "DG_EUNSUPPORTED",
    -5: "DG_ENOMEM",
    -6: "DG_EHIP",
    -7: "DG_ENONPHYS",
}

# Every symbol include/dg.h declares.
EXPORTS = [
    "dg_mesh_validate",
    "dg_mesh_create",
    "dg_mesh_destroy",
    "dg_mesh_info",
    "dg_quad_points",
    "dg_project",
    "dg_pack",
    "dg_unpack",
    "dg_rhs",
    "dg_max_dt",
    "dg_rk_step",
    "dg_rk_step_noalloc",
    "dg_advance",
    "dg_rhs_vjp",
    "dg_rk_step_vjp",
    "dg_rk_step_stages",
    "dg_rk_step_stages_to",
    "dg_eval_points",
    "dg_quad_weights",
    "dg_set_lanes_per_element",
    "dg_set_matrix_cores",
    "dg_set_surface_mode",
    "dg_set_stream_concurrency",
    "dg_set_boundary_state",
    "dg_set_integrator",
    "dg_set_limiter",
    "dg_limit",
    "dg_timing_enable",
    "dg_timing_read",
    "dg_reference_tables",
    "dg_matrix_core_tables",
    "dg_last_error",
]


class DGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class dg_info(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_int),
        ("n_modes", ctypes.c_int),
        ("n_vol_points", ctypes.c_int),
        ("n_edge_points", ctypes.c_int),
        ("n_elem", ctypes.c_int64),
        ("n_elem_pad", ctypes.c_int64),
        ("n_edges", ctypes.c_int64),
        ("state_len", ctypes.c_int64),
        ("ws_rhs", ctypes.c_int64),
        ("ws_step", ctypes.c_int64),
        ("ws_vjp", ctypes.c_int64),
        ("n_colours", ctypes.c_int64),
        ("stage_fp64", ctypes.c_int),
        ("stage_mixed", ctypes.c_int),
        ("adjoint", ctypes.c_int),
    ]


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


def load(path: str = LIB_PATH):
    """Load libdgmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it first (python -m paper_1601_07944_amd.build)")
    # torch first: it must bring up the HIP runtime before the library's
    # code objects are registered with it
    import torch  # noqa: F401

    lib = ctypes.CDLL(path)
    i32, i64 = ctypes.c_int, ctypes.c_int64
    lib.dg_last_error.restype = ctypes.c_char_p
    lib.dg_mesh_validate.argtypes = [i32, i64, _vp, _vp, _vp]
    lib.dg_mesh_create.argtypes = [i32, i64, _vp, _vp, _vp, ctypes.c_double, ctypes.POINTER(_vp)]
    lib.dg_mesh_destroy.argtypes = [_vp]
    lib.dg_mesh_info.argtypes = [_vp, ctypes.POINTER(dg_info)]
    lib.dg_quad_points.argtypes = [_vp, _vp, _vp]
    lib.dg_project.argtypes = [_vp, _vp, _vp, _vp]
    lib.dg_pack.argtypes = [_vp, _vp, _vp, _vp]
    lib.dg_unpack.argtypes = [_vp, _vp, _vp, _vp]
    lib.dg_rhs.argtypes = [_vp, _vp, _vp, i32, _vp, _vp]
    lib.dg_max_dt.argtypes = [_vp, _vp, ctypes.c_double, _vp, _dp, _vp, _vp]
    lib.dg_rk_step.argtypes = [_vp, _vp, ctypes.c_double, _vp, i32, _vp, _vp]
    lib.dg_rk_step_noalloc.argtypes = [_vp, _vp, ctypes.c_double, _vp, i32, _vp]
    lib.dg_advance.argtypes = [_vp, _vp, i64, ctypes.c_double, _vp, _vp, i32, _vp, _vp]
    lib.dg_rhs_vjp.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    lib.dg_rk_step_vjp.argtypes = [_vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.dg_rk_step_stages.argtypes = [_vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp]
    lib.dg_rk_step_stages_to.argtypes = [_vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp]
    lib.dg_eval_points.argtypes = [_vp, _vp, _vp, _vp]
    lib.dg_quad_weights.argtypes = [_vp, _vp, _vp]
    lib.dg_set_lanes_per_element.argtypes = [_vp, i32]
    lib.dg_set_matrix_cores.argtypes = [_vp, i32]
    lib.dg_set_surface_mode.argtypes = [_vp, i32]
    lib.dg_set_stream_concurrency.argtypes = [_vp, i32]
    lib.dg_set_boundary_state.argtypes = [_vp, _dp]
    lib.dg_set_integrator.argtypes = [_vp, i32]
    lib.dg_set_limiter.argtypes = [_vp, i32]
    lib.dg_limit.argtypes = [_vp, _vp, _vp]
    lib.dg_timing_enable.argtypes = [_vp, i32]
    lib.dg_timing_read.argtypes = [_vp, _dp, ctypes.POINTER(i64), i32]
    lib.dg_reference_tables.argtypes = [i32, _dp, i64]
    lib.dg_reference_tables.restype = i64
    lib.dg_matrix_core_tables.argtypes = [i32, i32, _dp, i64]
    lib.dg_matrix_core_tables.restype = i64
    for name in EXPORTS:
        getattr(lib, name).restype = getattr(lib, name).restype or i32
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise DGError(rc, load().dg_last_error().decode())
    return rc


def last_error() -> str:
    return load().dg_last_error().decode()


def validate(p, vxy, nbr_elem, nbr_side):
    """Host-only mesh check (no HIP call); returns the status code."""
    vxy = np.ascontiguousarray(vxy, dtype=np.float64)
    nbr_elem = np.ascontiguousarray(nbr_elem, dtype=np.int64)
    nbr_side = np.ascontiguousarray(nbr_side, dtype=np.int8)
    return load().dg_mesh_validate(p, vxy.shape[0], vxy.ctypes.data, nbr_elem.ctypes.data, nbr_side.ctypes.data)


def reference_tables(p: int) -> dict:
    """Host-only: the library's quadrature rules and basis tables."""
    np_ = (p + 1) * (p + 2) // 2
    cap = 4096
    buf = np.zeros(cap)
    n = load().dg_reference_tables(p, buf.ctypes.data_as(_dp), cap)
    if n < 0:
        _check(int(n))
    nq = {1: 3, 2: 6, 3: 12, 4: 16, 5: 25}[p]
    ne = p + 1
    o = 0

    def take(k):
        nonlocal o
        a = buf[o : o + k].copy()
        o += k
        return a

    out = dict(r=take(nq), s=take(nq), w=take(nq), gx=take(ne), gw=take(ne))
    out["phi"] = take(nq * np_).reshape(nq, np_)
    out["dphidr"] = take(nq * np_).reshape(nq, np_)
    out["dphids"] = take(nq * np_).reshape(nq, np_)
    out["phi_side"] = take(3 * ne * np_).reshape(3, ne, np_)
    assert o == n
    return out


def matrix_core_tables(p: int, fp64: bool) -> "np.ndarray":
    """Host-only: the matrix-core kernels' table operands, [blocks][64]."""
    cap = 1 << 16
    buf = np.zeros(cap)
    n = load().dg_matrix_core_tables(p, 1 if fp64 else 0, buf.ctypes.data_as(_dp), cap)
    if n < 0:
        _check(int(n))
    return buf[:n].reshape(-1, 64).copy()


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def check_tensor(t, name, device, numel=None, min_numel=None, dtype="float64", min_bytes=None):
    """Raise ValueError unless t is a contiguous torch tensor on `device`
    with the given dtype ("float64", or None for any) and exactly `numel`
    elements (or at least `min_numel` elements, or at least `min_bytes`
    bytes).  Every entry point checks its tensors with this before any
    launch: a kernel handed a host pointer, a tensor of another dtype or a
    buffer that is too short would read or write outside it."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if t.device != device:
        raise ValueError(f"{name}: tensor is on {t.device}, the mesh is on {device}")
    if dtype is not None and t.dtype != getattr(torch, dtype):
        raise ValueError(f"{name}: dtype {t.dtype}, expected torch.{dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor is not contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected at least {min_numel}")
    if min_bytes is not None and t.numel() * t.element_size() < min_bytes:
        raise ValueError(f"{name}: {t.numel() * t.element_size()} bytes, expected at least {min_bytes}")
    return t


class DGMesh:
    """A mesh on the current device (dg_mesh_create); torch tensors carry
    all device memory.  States passed to rhs / rk_step / max_dt are in the
    library's internal layout (see pack / unpack)."""

    def __init__(self, p, vxy, nbr_elem, nbr_side, gamma=1.4):
        import torch

        lib = load()
        vxy = np.ascontiguousarray(vxy, dtype=np.float64)
        nbr_elem = np.ascontiguousarray(nbr_elem, dtype=np.int64)
        nbr_side = np.ascontiguousarray(nbr_side, dtype=np.int8)
        h = _vp()
        _check(lib.dg_mesh_create(p, vxy.shape[0], vxy.ctypes.data, nbr_elem.ctypes.data, nbr_side.ctypes.data,
                                  float(gamma), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        info = dg_info()
        _check(lib.dg_mesh_info(h, ctypes.byref(info)))
        self.info = info
        self.p = p
        self.n = info.n_elem
        self.np = info.n_modes
        self.nq = info.n_vol_points
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._ws = None

    @classmethod
    def from_mesh(cls, mesh, p, gamma=1.4):
        return cls(p, mesh.vxy, mesh.nbr_elem, mesh.nbr_side, gamma)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dg_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- argument checks (before any launch) --------------------------------
    def _state(self, t, name):
        return check_tensor(t, name, self.device, numel=int(self.info.state_len))

    def _ws_check(self, t, nbytes, name="ws"):
        return check_tensor(t, name, self.device, dtype=None, min_bytes=int(nbytes))

    def _dt(self, t, name="dt_dev", count=1):
        return check_tensor(t, name, self.device, min_numel=count)

    # -- allocation helpers (torch owns device memory) --------------------
    def empty_state(self):
        import torch

        return torch.empty(self.info.state_len, dtype=torch.float64, device=self.device)

    def workspace(self, kind="step"):
        import torch

        nbytes = self.info.ws_step if kind == "step" else self.info.ws_rhs
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._ws

    # -- entry points -------------------------------------------------------
    def quad_points(self, stream=None):
        import torch

        xy = torch.empty((self.n, self.nq, 2), dtype=torch.float64, device=self.device)
        _check(self._lib.dg_quad_points(self._h, _ptr(xy), _stream(stream)))
        return xy

    def project(self, u, out=None, stream=None):
        out = self.empty_state() if out is None else self._state(out, "out")
        check_tensor(u, "u", self.device, numel=self.n * self.nq * 4)
        _check(self._lib.dg_project(self._h, _ptr(u), _ptr(out), _stream(stream)))
        return out

    def pack(self, C_user, out=None, stream=None):
        out = self.empty_state() if out is None else self._state(out, "out")
        check_tensor(C_user, "C_user", self.device, numel=self.n * 4 * self.np)
        _check(self._lib.dg_pack(self._h, _ptr(C_user), _ptr(out), _stream(stream)))
        return out

    def unpack(self, C, out=None, stream=None):
        import torch

        self._state(C, "C")
        if out is None:
            out = torch.empty((self.n, 4, self.np), dtype=torch.float64, device=self.device)
        check_tensor(out, "out", self.device, numel=self.n * 4 * self.np)
        _check(self._lib.dg_unpack(self._h, _ptr(C), _ptr(out), _stream(stream)))
        return out

    def rhs(self, C, out=None, prec=DG_FP64, ws=None, stream=None):
        self._state(C, "C")
        out = self.empty_state() if out is None else self._state(out, "out")
        ws = self.workspace("rhs") if ws is None else self._ws_check(ws, self.info.ws_rhs)
        _check(self._lib.dg_rhs(self._h, _ptr(C), _ptr(out), prec, _ptr(ws), _stream(stream)))
        return out

    def max_dt(self, C, cfl, dt_dev=None, to_host=True, ws=None, stream=None):
        """Returns (dt_dev tensor, host float or None)."""
        import torch

        self._state(C, "C")
        dt_dev = torch.empty(1, dtype=torch.float64, device=self.device) if dt_dev is None else self._dt(dt_dev)
        ws = self.workspace("rhs") if ws is None else self._ws_check(ws, self.info.ws_rhs)
        host = ctypes.c_double(0.0)
        _check(self._lib.dg_max_dt(self._h, _ptr(C), float(cfl), _ptr(dt_dev),
                                   ctypes.byref(host) if to_host else None, _ptr(ws), _stream(stream)))
        return dt_dev, (host.value if to_host else None)

    KERNELS = ("traces", "edge", "element", "dt", "stage", "vjp", "limit", "volume")
    SURFACE_ELEMENTWISE = 0
    SURFACE_EDGEWISE = 1
    SURFACE_COLOURED = 2

    def set_lanes(self, lanes: int):
        """Work-items per element in the element-wise kernels: 0 (auto), 1 or 4."""
        _check(self._lib.dg_set_lanes_per_element(self._h, int(lanes)))

    def kernel_choice(self):
        """Stage kernels of the current choice, (FP64, mixed precision): 1 or 4
        lanes per element, or 16 (16 x 16 x 4 matrix products)."""
        info = dg_info()
        _check(self._lib.dg_mesh_info(self._h, ctypes.byref(info)))
        return info.stage_fp64, info.stage_mixed

    def adjoint_kernel(self):
        """Adjoint stage kernel of the current choice: 1 or 4 lanes per
        element, or 16 (16 x 16 x 4 matrix products)."""
        info = dg_info()
        _check(self._lib.dg_mesh_info(self._h, ctypes.byref(info)))
        return info.adjoint

    def set_matrix_cores(self, on):
        """FP64 stages with their contractions on the matrix cores: True, False,
        or None (automatic, the default)."""
        _check(self._lib.dg_set_matrix_cores(self._h, -1 if on is None else (1 if on else 0)))

    def set_surface_mode(self, mode: int):
        _check(self._lib.dg_set_surface_mode(self._h, int(mode)))

    def set_stream_concurrency(self, on: bool):
        """Edge-wise mode: volume integral on a second stream (bitwise equal)."""
        _check(self._lib.dg_set_stream_concurrency(self._h, 1 if on else 0))

    def set_boundary_state(self, U):
        """Conserved state (rho, rho u, rho v, E) of boundary code DG_BC_STATE."""
        import numpy as np

        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (4,)
        _check(self._lib.dg_set_boundary_state(self._h, U.ctypes.data_as(_dp)))

    RK_SSP3, RK2, RK4 = 0, 1, 2

    def set_integrator(self, scheme: int):
        """dg_rk_step / dg_advance scheme: 0 SSP-RK3, 1 Heun (RK2), 2 classic RK4."""
        _check(self._lib.dg_set_integrator(self._h, int(scheme)))

    LIMITER_NONE, LIMITER_BJ = 0, 1

    def set_limiter(self, limiter: int):
        """0: no limiting; 1: Barth-Jespersen (p = 1) after every RK stage."""
        _check(self._lib.dg_set_limiter(self._h, int(limiter)))

    def limit(self, C, stream=None):
        """Barth-Jespersen limiter (p = 1) applied once, in place; returns C."""
        self._state(C, "C")
        _check(self._lib.dg_limit(self._h, _ptr(C), _stream(stream)))
        return C

    def timing(self, on: bool):
        _check(self._lib.dg_timing_enable(self._h, 1 if on else 0))

    def timing_read(self):
        """{kernel kind: (total ms, launches)} since the last read (waits)."""
        nk = len(self.KERNELS)
        ms = (ctypes.c_double * nk)()
        cnt = (ctypes.c_int64 * nk)()
        _check(self._lib.dg_timing_read(self._h, ms, cnt, nk))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.KERNELS)}

    def advance(self, C, nsteps, cfl, dt_dev=None, dt_hist=None, prec=DG_FP64, ws=None, stream=None):
        """nsteps SSP-RK3 steps with the device CFL step length (in place)."""
        import torch

        if int(nsteps) < 0:
            raise ValueError(f"nsteps = {nsteps} < 0")
        self._state(C, "C")
        dt_dev = torch.empty(1, dtype=torch.float64, device=self.device) if dt_dev is None else self._dt(dt_dev)
        if dt_hist is not None:
            self._dt(dt_hist, "dt_hist", max(1, int(nsteps)))
        ws = self.workspace("step") if ws is None else self._ws_check(ws, self.info.ws_step)
        _check(self._lib.dg_advance(self._h, _ptr(C), int(nsteps), float(cfl), _ptr(dt_dev),
                                    _ptr(dt_hist) if dt_hist is not None else None, prec, _ptr(ws), _stream(stream)))
        return dt_dev

    def rhs_vjp(self, C, Rbar, out=None, stream=None):
        self._state(C, "C")
        self._state(Rbar, "Rbar")
        out = self.empty_state() if out is None else self._state(out, "out")
        _check(self._lib.dg_rhs_vjp(self._h, _ptr(C), _ptr(Rbar), _ptr(out), None, _stream(stream)))
        return out

    def rk_step_stages(self, C, u1, u2, dt=0.0, dt_dev=None, ws=None, stream=None):
        self._state(C, "C")
        self._state(u1, "u1")
        self._state(u2, "u2")
        if dt_dev is not None:
            self._dt(dt_dev)
        ws = self.workspace("step") if ws is None else self._ws_check(ws, self.info.ws_step)
        _check(self._lib.dg_rk_step_stages(self._h, _ptr(C), float(dt), _ptr(dt_dev) if dt_dev is not None else None,
                                           _ptr(u1), _ptr(u2), _ptr(ws), _stream(stream)))
        return C

    def rk_step_stages_to(self, C, Cnext, u1, u2, dt=0.0, dt_dev=None, ws=None, stream=None):
        """dg_rk_step_stages with the new state written to Cnext (C unchanged)."""
        self._state(C, "C")
        self._state(Cnext, "Cnext")
        self._state(u1, "u1")
        self._state(u2, "u2")
        if dt_dev is not None:
            self._dt(dt_dev)
        ws = self.workspace("step") if ws is None else self._ws_check(ws, self.info.ws_step)
        _check(self._lib.dg_rk_step_stages_to(self._h, _ptr(C), _ptr(Cnext), float(dt),
                                              _ptr(dt_dev) if dt_dev is not None else None, _ptr(u1), _ptr(u2),
                                              _ptr(ws), _stream(stream)))
        return Cnext

    def rk_step_vjp(self, C, ubar, dt=0.0, dt_dev=None, u1=None, u2=None, out=None, ws=None, stream=None):
        import torch

        self._state(C, "C")
        self._state(ubar, "ubar")
        if (u1 is None) != (u2 is None):
            raise ValueError("pass both stage states u1 and u2, or neither")
        if u1 is not None:
            self._state(u1, "u1")
            self._state(u2, "u2")
        if dt_dev is not None:
            self._dt(dt_dev)
        out = self.empty_state() if out is None else self._state(out, "out")
        if ws is None:
            if getattr(self, "_ws_vjp", None) is None:
                self._ws_vjp = torch.empty(self.info.ws_vjp, dtype=torch.uint8, device=self.device)
            ws = self._ws_vjp
        else:
            self._ws_check(ws, self.info.ws_vjp)
        _check(self._lib.dg_rk_step_vjp(self._h, _ptr(C), float(dt), _ptr(dt_dev) if dt_dev is not None else None,
                                        _ptr(u1) if u1 is not None else None, _ptr(u2) if u2 is not None else None,
                                        _ptr(ubar), _ptr(out), _ptr(ws), _stream(stream)))
        return out

    def eval_points(self, C, out=None, stream=None):
        import torch

        self._state(C, "C")
        out = torch.empty((self.n, self.nq, 4), dtype=torch.float64, device=self.device) if out is None else out
        check_tensor(out, "out", self.device, numel=self.n * self.nq * 4)
        _check(self._lib.dg_eval_points(self._h, _ptr(C), _ptr(out), _stream(stream)))
        return out

    def quad_weights(self, out=None, stream=None):
        import torch

        out = torch.empty((self.n, self.nq), dtype=torch.float64, device=self.device) if out is None else out
        check_tensor(out, "out", self.device, numel=self.n * self.nq)
        _check(self._lib.dg_quad_weights(self._h, _ptr(out), _stream(stream)))
        return out

    def rk_step(self, C, dt=0.0, dt_dev=None, prec=DG_FP64, ws=None, stream=None):
        self._state(C, "C")
        if dt_dev is not None:
            self._dt(dt_dev)
        ws = self.workspace("step") if ws is None else self._ws_check(ws, self.info.ws_step)
        _check(self._lib.dg_rk_step(self._h, _ptr(C), float(dt), _ptr(dt_dev) if dt_dev is not None else None, prec,
                                    _ptr(ws), _stream(stream)))
        return C

    def rk_step_noalloc(self, C, dt=0.0, dt_dev=None, prec=DG_FP64, stream=None):
        """dg_rk_step_noalloc: one step with the stage states in the
        library's static device scratch (no workspace, nothing allocated)."""
        self._state(C, "C")
        if dt_dev is not None:
            self._dt(dt_dev)
        _check(self._lib.dg_rk_step_noalloc(self._h, _ptr(C), float(dt), _ptr(dt_dev) if dt_dev is not None else None,
                                            prec, _stream(stream)))
        return C
