"""Seeded synthetic inputs: periodic triangle meshes and initial data.

This module holds no part of the discontinuous Galerkin method itself (no
basis, quadrature, geometry, flux or time stepping).  It only produces the
inputs that both the HIP path and the CPU oracle consume:

* meshes as per-element vertex coordinates plus neighbour connectivity, in
  the form the paper's mesh description uses (Section "Mesh Connectivity":
  every element knows the element across each of its three sides); vertices
  are counter-clockwise so that the element map of eq. (2dmap) has a
  positive Jacobian determinant;
* the conserved variables (rho, rho*u, rho*v, E) of the test problems at
  arbitrary physical points (Euler equations, eq. (euler), ideal gas).

Periodicity lives entirely in the connectivity: every element stores its own
unwrapped vertex coordinates, and an element on the wrap seam simply names
its periodic neighbour.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


# ---------------------------------------------------------------------------
# meshes
# ---------------------------------------------------------------------------
class Mesh:
    """Triangle mesh in the element-neighbour form.

    vxy      float64 [N, 3, 2]  vertices, counter-clockwise, unwrapped
    nbr_elem int64   [N, 3]     element across local side q (v_q -> v_{q+1})
    nbr_side int8    [N, 3]     that neighbour's local side index (0..2)
    period   float              side length of the periodic square
    """

    def __init__(self, vxy, nbr_elem, nbr_side, period, name=""):
        self.vxy = np.ascontiguousarray(vxy, dtype=np.float64)
        self.nbr_elem = np.ascontiguousarray(nbr_elem, dtype=np.int64)
        self.nbr_side = np.ascontiguousarray(nbr_side, dtype=np.int8)
        self.period = float(period)
        self.name = name

    @property
    def n_elem(self) -> int:
        return self.vxy.shape[0]

    def centroids(self) -> np.ndarray:
        return self.vxy.mean(axis=1)


def square_mesh(n: int, length: float = 1.0, jitter: float = 0.0, seed: int = 0) -> Mesh:
    """Periodic n x n lattice on [0, length)^2, each square split along the
    diagonal (i, j) -> (i+1, j+1) into two triangles.

    Every periodic lattice vertex is displaced per coordinate by an
    independent U[-jitter*h, jitter*h] draw (h = length/n); the periodic
    copies of a vertex get the same displacement.  Element numbering:
    square (i, j) holds elements 2*(j*n+i) (lower-right triangle A) and
    2*(j*n+i)+1 (upper-left triangle B).
    """
    h = length / n
    rng = np.random.default_rng(seed)
    disp = rng.uniform(-jitter * h, jitter * h, size=(n, n, 2)) if jitter > 0 else np.zeros((n, n, 2))

    def vert(i, j):
        # unwrapped lattice position plus the displacement of its periodic image
        return np.stack([i * h + disp[i % n, j % n, 0], j * h + disp[i % n, j % n, 1]], axis=-1)

    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")  # ii[j, i] = i
    ii = ii.ravel()
    jj = jj.ravel()
    sq = jj * n + ii
    N = 2 * n * n
    vxy = np.empty((N, 3, 2))
    a = 2 * sq
    b = 2 * sq + 1
    vxy[a, 0] = vert(ii, jj)
    vxy[a, 1] = vert(ii + 1, jj)
    vxy[a, 2] = vert(ii + 1, jj + 1)
    vxy[b, 0] = vert(ii, jj)
    vxy[b, 1] = vert(ii + 1, jj + 1)
    vxy[b, 2] = vert(ii, jj + 1)

    def sqid(i, j):
        return (j % n) * n + (i % n)

    nbr = np.empty((N, 3), dtype=np.int64)
    nsd = np.empty((N, 3), dtype=np.int8)
    # A(i,j): side 0 bottom   <-> B(i, j-1) side 1 (top)
    #         side 1 right    <-> B(i+1, j) side 2 (left)
    #         side 2 diagonal <-> B(i, j)   side 0
    nbr[a, 0] = 2 * sqid(ii, jj - 1) + 1
    nsd[a, 0] = 1
    nbr[a, 1] = 2 * sqid(ii + 1, jj) + 1
    nsd[a, 1] = 2
    nbr[a, 2] = b
    nsd[a, 2] = 0
    # B(i,j): side 0 diagonal <-> A(i, j)   side 2
    #         side 1 top      <-> A(i, j+1) side 0
    #         side 2 left     <-> A(i-1, j) side 1
    nbr[b, 0] = a
    nsd[b, 0] = 2
    nbr[b, 1] = 2 * sqid(ii, jj + 1)
    nsd[b, 1] = 0
    nbr[b, 2] = 2 * sqid(ii - 1, jj)
    nsd[b, 2] = 1
    return Mesh(vxy, nbr, nsd, length, name=f"square{n}x{n}x2_j{jitter}_s{seed}")


# boundary codes in place of a neighbour (Section "Mesh Connectivity":
# boundary edges store a negative integer naming their kind of boundary)
BC_WALL, BC_OUTFLOW, BC_STATE = -1, -2, -3


def box_mesh(nx: int, ny: int, lx: float = 1.0, ly: float = 1.0, jitter: float = 0.0, seed: int = 0,
             bc=(BC_WALL, BC_WALL, 0, 0)) -> Mesh:
    """nx x ny lattice on [0, lx] x [0, ly], each square split along the
    diagonal (i, j) -> (i+1, j+1) as in square_mesh.  bc = (left, right,
    bottom, top): a negative boundary code for each side of the box, or 0 on
    both sides of a direction for periodicity in it.  Interior vertices are
    jittered by U[-jitter*h, jitter*h] per coordinate; vertices on a
    non-periodic side keep their normal coordinate (straight boundaries).
    Boundary sides get nbr_elem = the code and nbr_side = -1."""
    left, right, bottom, top = bc
    px = left == 0 and right == 0
    py = bottom == 0 and top == 0
    assert (left == 0) == (right == 0) and (bottom == 0) == (top == 0)
    hx, hy = lx / nx, ly / ny
    rng = np.random.default_rng(seed)
    disp = rng.uniform(-jitter, jitter, size=(nx + 1, ny + 1, 2)) if jitter > 0 else np.zeros((nx + 1, ny + 1, 2))
    disp[..., 0] *= hx
    disp[..., 1] *= hy
    if px:
        disp[nx, :] = disp[0, :]
    else:
        disp[0, :, 0] = 0.0
        disp[nx, :, 0] = 0.0
    if py:
        disp[:, ny] = disp[:, 0]
    else:
        disp[:, 0, 1] = 0.0
        disp[:, ny, 1] = 0.0

    def vert(i, j):
        ii_, jj_ = (i % nx if px else i), (j % ny if py else j)
        return np.stack([i * hx + disp[ii_, jj_, 0], j * hy + disp[ii_, jj_, 1]], axis=-1)

    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ii = ii.ravel()
    jj = jj.ravel()
    sq = jj * nx + ii
    N = 2 * nx * ny
    a, b = 2 * sq, 2 * sq + 1
    vxy = np.empty((N, 3, 2))
    vxy[a, 0], vxy[a, 1], vxy[a, 2] = vert(ii, jj), vert(ii + 1, jj), vert(ii + 1, jj + 1)
    vxy[b, 0], vxy[b, 1], vxy[b, 2] = vert(ii, jj), vert(ii + 1, jj + 1), vert(ii, jj + 1)

    def sqid(i, j):
        return (j % ny) * nx + (i % nx)

    nbr = np.empty((N, 3), dtype=np.int64)
    nsd = np.empty((N, 3), dtype=np.int8)
    nbr[a, 0], nsd[a, 0] = 2 * sqid(ii, jj - 1) + 1, 1
    nbr[a, 1], nsd[a, 1] = 2 * sqid(ii + 1, jj) + 1, 2
    nbr[a, 2], nsd[a, 2] = b, 0
    nbr[b, 0], nsd[b, 0] = a, 2
    nbr[b, 1], nsd[b, 1] = 2 * sqid(ii, jj + 1), 0
    nbr[b, 2], nsd[b, 2] = 2 * sqid(ii - 1, jj), 1
    if not py:
        m = jj == 0
        nbr[a[m], 0], nsd[a[m], 0] = bottom, -1
        m = jj == ny - 1
        nbr[b[m], 1], nsd[b[m], 1] = top, -1
    if not px:
        m = ii == nx - 1
        nbr[a[m], 1], nsd[a[m], 1] = right, -1
        m = ii == 0
        nbr[b[m], 2], nsd[b[m], 2] = left, -1
    name = f"box{nx}x{ny}_bc{left}{right}{bottom}{top}_j{jitter}_s{seed}"
    return Mesh(vxy, nbr, nsd, max(lx, ly), name=name)


def mirror_doubled_x(box: Mesh, lx: float) -> Mesh:
    """The periodic mesh on [-lx, lx) x [0, ly) made of a box mesh whose
    left and right sides (x = 0 and x = lx) are boundaries and its mirror
    image about x = 0, with period 2 lx in x; elements 0..N-1 are the box's,
    N..2N-1 their mirror images.  A mirrored element lists its vertices as
    (v0, v2, v1) mirrored, so it stays counter-clockwise; its sides 0, 1, 2
    are the mirrors of the original's sides 2, 1, 0.  Across x = 0 and
    across the seam x = lx ~ -lx every boundary side meets the mirror image
    of its own element."""
    N = box.n_elem
    side_map = np.array([2, 1, 0])  # mirrored element's side s <-> original side side_map[s]
    vm = box.vxy[:, [0, 2, 1], :].copy()
    vm[..., 0] *= -1.0
    vxy = np.concatenate([box.vxy, vm])
    nbr = np.empty((2 * N, 3), dtype=np.int64)
    nsd = np.empty((2 * N, 3), dtype=np.int8)
    inv = side_map  # involution: original side q <-> mirrored side inv[q]
    for q in range(3):
        nb = box.nbr_elem[:, q]
        ns = box.nbr_side[:, q].astype(np.int64)
        interior = nb >= 0
        # original elements
        nbr[:N, q] = np.where(interior, nb, np.arange(N) + N)
        nsd[:N, q] = np.where(interior, ns, inv[q])
        # mirrored elements: side inv[q] of element N+i mirrors side q of i
        nbr[N:, inv[q]] = np.where(interior, nb + N, np.arange(N))
        nsd[N:, inv[q]] = np.where(interior, inv[np.where(interior, ns, 0)], q)
    assert (box.nbr_elem[box.nbr_elem < 0] != 0).all()
    return Mesh(vxy, nbr, nsd, 2 * lx, name=box.name + "_mirrored")


def delaunay_mesh(n_points: int, seed: int, length: float = 1.0, margin: float | None = None) -> Mesh:
    """Periodic Delaunay triangulation of n_points seeded uniform points in
    [0, length)^2.

    The points are replicated into a band of width `margin` around the
    square, triangulated with Qhull, and the triangles whose centroid lies in
    [0, length)^2 are kept.  On the torus a triangulation has exactly twice as
    many triangles as vertices; that count is asserted, which also checks
    that the band was wide enough.
    """
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    P = rng.uniform(0.0, length, size=(n_points, 2))
    if margin is None:
        margin = min(0.5 * length, 12.0 * length / np.sqrt(n_points))
    shifts = [(dx, dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1)]
    pts, base, off = [], [], []
    for dx, dy in shifts:
        Q = P + np.array([dx, dy]) * length
        keep = (
            (Q[:, 0] >= -margin) & (Q[:, 0] < length + margin) & (Q[:, 1] >= -margin) & (Q[:, 1] < length + margin)
        )
        idx = np.nonzero(keep)[0]
        pts.append(Q[idx])
        base.append(idx)
        off.append(np.tile(np.array([dx, dy], dtype=np.int64), (idx.size, 1)))
    pts = np.concatenate(pts)
    base = np.concatenate(base)
    off = np.concatenate(off)
    tri = Delaunay(pts)
    S = tri.simplices.astype(np.int64)  # [T, 3]
    X = pts[S]  # [T, 3, 2]
    # counter-clockwise orientation
    cross = (X[:, 1, 0] - X[:, 0, 0]) * (X[:, 2, 1] - X[:, 0, 1]) - (X[:, 1, 1] - X[:, 0, 1]) * (
        X[:, 2, 0] - X[:, 0, 0]
    )
    flip = cross < 0
    S[flip] = S[flip][:, [0, 2, 1]]
    X = pts[S]
    cen = X.mean(axis=1)
    cell = np.floor(cen / length).astype(np.int64)  # periodic cell of the centroid
    inside = (cell[:, 0] == 0) & (cell[:, 1] == 0)
    kept = np.nonzero(inside)[0]
    T = kept.size
    if T != 2 * n_points:
        raise RuntimeError(f"periodic Delaunay: {T} triangles for {n_points} points (expected {2 * n_points})")

    # Key every triangle (any periodic copy) by its base vertex ids and the
    # vertex offsets relative to the cell of its centroid, rotated so that the
    # smallest base id comes first (rotation keeps the CCW order).
    def keys(tris):
        b = base[S[tris]]  # [t, 3]
        o = off[S[tris]] - cell[tris][:, None, :]  # [t, 3, 2], entries in [-2, 2]
        r = np.argmin(b, axis=1)
        idx = (r[:, None] + np.arange(3)[None, :]) % 3
        b = np.take_along_axis(b, idx, axis=1)
        o = np.take_along_axis(o, idx[:, :, None], axis=1)
        oc = (o[:, :, 0] + 2) * 5 + (o[:, :, 1] + 2)
        k1 = b[:, 0] * n_points + b[:, 1]
        k2 = b[:, 2] * 15625 + oc[:, 0] * 625 + oc[:, 1] * 25 + oc[:, 2]
        return np.ascontiguousarray(np.stack([k1, k2], axis=1)).view(np.dtype((np.void, 16))).ravel()

    kk = keys(kept)
    order = np.argsort(kk)
    ksorted = kk[order]
    nbr = np.empty((T, 3), dtype=np.int64)
    nsd = np.empty((T, 3), dtype=np.int8)
    # local side q of a triangle runs v_q -> v_{q+1}; Qhull's neighbors[t][k]
    # is the triangle opposite vertex k, i.e. across side (k+1) % 3.
    Nb = tri.neighbors[kept]
    for q in range(3):
        nt = Nb[:, (q + 2) % 3]
        if np.any(nt < 0):
            raise RuntimeError("periodic Delaunay: band too narrow (hull edge reached)")
        kn = keys(nt)
        pos = np.searchsorted(ksorted, kn)
        pos = np.minimum(pos, T - 1)
        if np.any(ksorted[pos] != kn):
            raise RuntimeError("periodic Delaunay: neighbour copy not found (band too narrow)")
        nbr[:, q] = order[pos]
    vb = base[S[kept]]  # base ids per kept triangle in its CCW order
    for q in range(3):
        u = vb[:, q]
        v = vb[:, (q + 1) % 3]
        nb = nbr[:, q]
        found = np.full(T, -1, dtype=np.int64)
        for qq in range(3):
            a = vb[nb, qq]
            c = vb[nb, (qq + 1) % 3]
            m = (a == v) & (c == u)
            found[m & (found < 0)] = qq
        if np.any(found < 0):
            raise RuntimeError("periodic Delaunay: neighbour side not found")
        nsd[:, q] = found
    return Mesh(X[kept], nbr, nsd, length, name=f"delaunay{n_points}_s{seed}")


# ---------------------------------------------------------------------------
# initial data and exact solutions (conserved variables rho, rho u, rho v, E)
# ---------------------------------------------------------------------------
def primitive_to_conserved(rho, u, v, p, gamma=GAMMA):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E], axis=-1)


def isentropic_vortex(x, y, t=0.0, beta=5.0, center=(5.0, 5.0), vel=(1.0, 1.0), period=10.0, gamma=GAMMA):
    """Isentropic vortex advected with the free stream (rho=1, u=v=1, p=1).

    The centre moves with the free stream and is taken at its periodic image
    nearest to (x, y).  Returns conserved variables [..., 4].
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    cx = center[0] + vel[0] * t
    cy = center[1] + vel[1] * t
    dx = x - cx
    dy = y - cy
    dx -= period * np.round(dx / period)
    dy -= period * np.round(dy / period)
    r2 = dx * dx + dy * dy
    e = np.exp(0.5 * (1.0 - r2))
    u = vel[0] - beta / (2.0 * np.pi) * dy * e
    v = vel[1] + beta / (2.0 * np.pi) * dx * e
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * np.pi * np.pi) * e * e
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho**gamma
    return primitive_to_conserved(rho, u, v, p, gamma)


def smooth_density(x, y, t=0.0, period=1.0, gamma=GAMMA):
    """rho = 1 + 0.2 sin(2 pi x) sin(2 pi y), u = v = 0.5, p = 1, advected
    exactly with velocity (0.5, 0.5) (a contact wave: u, v, p stay constant)."""
    x = np.asarray(x, dtype=np.float64) - 0.5 * t
    y = np.asarray(y, dtype=np.float64) - 0.5 * t
    k = 2.0 * np.pi / period
    rho = 1.0 + 0.2 * np.sin(k * x) * np.sin(k * y)
    one = np.ones_like(rho)
    return primitive_to_conserved(rho, 0.5 * one, 0.5 * one, one, gamma)


def density_jump(x, y, t=0.0, period=1.0, gamma=GAMMA):
    """smooth_density scaled by 0.5 inside the circle r < 0.25 about
    (0.5, 0.5) (equal pressure, equal velocity), advected with (0.5, 0.5)."""
    x = np.asarray(x, dtype=np.float64) - 0.5 * t
    y = np.asarray(y, dtype=np.float64) - 0.5 * t
    xs = np.mod(x, period)
    ys = np.mod(y, period)
    k = 2.0 * np.pi / period
    rho = 1.0 + 0.2 * np.sin(k * xs) * np.sin(k * ys)
    r2 = (xs - 0.5 * period) ** 2 + (ys - 0.5 * period) ** 2
    rho = np.where(r2 < (0.25 * period) ** 2, 0.5 * rho, rho)
    one = np.ones_like(rho)
    return primitive_to_conserved(rho, 0.5 * one, 0.5 * one, one, gamma)


def free_stream(x, y, rho=1.0, u=0.3, v=-0.2, p=0.9, gamma=GAMMA):
    x = np.asarray(x, dtype=np.float64)
    one = np.ones_like(x)
    return primitive_to_conserved(rho * one, u * one, v * one, p * one, gamma)


def random_state(n_elem: int, n_modes: int, seed: int, amp: float = 0.05) -> np.ndarray:
    """Random modal coefficients in the user layout [N][4][Np] around a
    physical state: mode 0 carries a positive mean (rho ~ 1, p ~ 1), the
    higher modes are small U[-amp, amp] 0.6^degree perturbations so that the
    traces stay physical.  Mode 0 of the orthonormal basis is the constant sqrt(2),
    so the cell average is sqrt(2) * c_0."""
    rng = np.random.default_rng(seed)
    # modes are ordered by total degree d; perturbations decay like 0.6^d so
    # that edge traces stay physical up to p = 5
    deg = np.concatenate([np.full(d + 1, d) for d in range(n_modes)])[:n_modes]
    C = rng.uniform(-amp, amp, size=(n_elem, 4, n_modes)) * 0.6 ** deg
    rho = 1.0 + 0.1 * rng.uniform(-1, 1, size=n_elem)
    u = 0.3 * rng.uniform(-1, 1, size=n_elem)
    v = 0.3 * rng.uniform(-1, 1, size=n_elem)
    p = 1.0 + 0.1 * rng.uniform(-1, 1, size=n_elem)
    U = primitive_to_conserved(rho, u, v, p)
    C[:, :, 0] = U / np.sqrt(2.0)
    return C


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------
WORKLOADS = {
    # 512 triangles, p=1, isentropic vortex on [0,10]^2, jitter 0.1h, seed 0
    "vortex_p1_512": dict(mesh=("square", 16, 10.0, 0.1, 0), p=1, data="vortex"),
    # 32,768 triangles, p=3, isentropic vortex on [0,10]^2, jitter 0.2h, seed 1
    "vortex_p3_32768": dict(mesh=("square", 128, 10.0, 0.2, 1), p=3, data="vortex"),
    # 131,072 triangles, p=2, smooth data on the unit square, jitter 0.2h, seed 3
    "smooth_p2_131072": dict(mesh=("square", 256, 1.0, 0.2, 3), p=2, data="smooth"),
}


def make_mesh(spec) -> Mesh:
    kind = spec[0]
    if kind == "square":
        _, n, length, jit, seed = spec
        return square_mesh(n, length, jit, seed)
    if kind == "delaunay":
        _, npts, seed = spec
        return delaunay_mesh(npts, seed)
    raise ValueError(kind)


def initial_data(name: str):
    return {
        "vortex": isentropic_vortex,
        "smooth": smooth_density,
        "jump": density_jump,
        "free": free_stream,
    }[name]
