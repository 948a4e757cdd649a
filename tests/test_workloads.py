"""Invariants of the seeded mesh generators (CPU)."""
import numpy as np
import pytest

from paper_1601_07944_amd import workloads as W


def check_mesh(m):
    N = m.n_elem
    nb, ns = m.nbr_elem, m.nbr_side.astype(np.int64)
    assert np.all((nb >= 0) & (nb < N)) and np.all((ns >= 0) & (ns < 3))
    assert np.all(nb[nb, ns] == np.arange(N)[:, None])  # symmetric neighbours
    assert np.all(ns[nb, ns] == np.arange(3)[None, :])
    X = m.vxy
    det = (X[:, 1, 0] - X[:, 0, 0]) * (X[:, 2, 1] - X[:, 0, 1]) - (X[:, 2, 0] - X[:, 0, 0]) * (X[:, 1, 1] - X[:, 0, 1])
    assert np.all(det > 0)  # counter-clockwise
    # the two copies of an edge have equal length and opposite direction up
    # to a period shift
    q = np.arange(3)
    e = X[:, (q + 1) % 3] - X[:, q]
    en = e[nb, ns]
    assert np.allclose(e, -en, atol=1e-12 * m.period)
    # total area = period^2
    assert abs(det.sum() / 2 - m.period**2) < 1e-10 * m.period**2


@pytest.mark.parametrize("n,L,jit,seed", [(1, 1.0, 0.0, 0), (2, 1.0, 0.1, 0), (16, 10.0, 0.1, 0), (7, 1.0, 0.2, 3)])
def test_square_mesh(n, L, jit, seed):
    m = W.square_mesh(n, L, jit, seed)
    assert m.n_elem == 2 * n * n
    check_mesh(m)


@pytest.mark.parametrize("npts,seed", [(30, 1), (500, 2), (5000, 4)])
def test_periodic_delaunay(npts, seed):
    m = W.delaunay_mesh(npts, seed)
    assert m.n_elem == 2 * npts  # Euler characteristic of the torus
    check_mesh(m)
    # Delaunay: no vertex of a neighbour lies strictly inside a circumcircle
    X = m.vxy
    a, b, c = X[:, 0], X[:, 1], X[:, 2]
    d = 2 * (a[:, 0] * (b[:, 1] - c[:, 1]) + b[:, 0] * (c[:, 1] - a[:, 1]) + c[:, 0] * (a[:, 1] - b[:, 1]))
    sq = (X**2).sum(-1)
    ux = (sq[:, 0] * (b[:, 1] - c[:, 1]) + sq[:, 1] * (c[:, 1] - a[:, 1]) + sq[:, 2] * (a[:, 1] - b[:, 1])) / d
    uy = (sq[:, 0] * (c[:, 0] - b[:, 0]) + sq[:, 1] * (a[:, 0] - c[:, 0]) + sq[:, 2] * (b[:, 0] - a[:, 0])) / d
    R2 = (a[:, 0] - ux) ** 2 + (a[:, 1] - uy) ** 2
    for q in range(3):
        nb = m.nbr_elem[:, q]
        opp = X[nb, (m.nbr_side[:, q].astype(int) + 2) % 3]  # neighbour's vertex off the shared edge
        # shift the neighbour copy next to this element
        shift = X[:, q] - X[nb, (m.nbr_side[:, q].astype(int) + 1) % 3]
        o = opp + shift
        assert np.all((o[:, 0] - ux) ** 2 + (o[:, 1] - uy) ** 2 >= R2 * (1 - 1e-9))


def test_seeded_and_deterministic():
    a = W.square_mesh(8, 1.0, 0.2, 5)
    b = W.square_mesh(8, 1.0, 0.2, 5)
    assert np.array_equal(a.vxy, b.vxy)
    c = W.delaunay_mesh(200, 9)
    d = W.delaunay_mesh(200, 9)
    assert np.array_equal(c.vxy, d.vxy) and np.array_equal(c.nbr_elem, d.nbr_elem)
