"""Pins of the oracle's orthonormal modal basis (test infrastructure).

The paper uses an orthonormal basis of the polynomials of degree <= p on the
reference triangle, so that the mass matrix is the identity (Section "The
Discontinuous Galerkin Method", around eq. (2ddg0)); its slopes are modes 2
and 3 at p = 1 (limiter section).
"""
import numpy as np
import pytest
from scipy.special import roots_jacobi

import oracle as O


def product_rule(n):
    # collapsed Gauss-Jacobi product rule on the reference triangle, exact to
    # degree 2n-1 (independent of the oracle's own rule)
    a, wa = roots_jacobi(n, 0.0, 0.0)
    b, wb = roots_jacobi(n, 1.0, 0.0)
    XI, ETA = np.meshgrid(a, b, indexing="ij")
    return ((1 + XI) * (1 - ETA) / 4).ravel(), ((1 + ETA) / 2).ravel(), (np.outer(wa, wb) / 8).ravel()


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_gram_is_identity(p):
    r, s, w = product_rule(p + 2)
    phi, _, _ = O.basis(p, r, s)
    G = (phi * w[:, None]).T @ phi
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-13


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_hierarchical_degrees(p):
    # modes are ordered by total degree: a mode of degree d is orthogonal to
    # every monomial of degree < d, and the block of degree d has d+1 modes
    r, s, w = product_rule(p + 2)
    phi, _, _ = O.basis(p, r, s)
    j = 0
    for d in range(p + 1):
        for _ in range(d + 1):
            for a in range(d):
                for b in range(d - a):
                    assert abs(np.sum(w * phi[:, j] * r**a * s**b)) < 1e-13
            j += 1
    # and each mode of degree d is not orthogonal to all degree-d monomials
    j = 0
    for d in range(p + 1):
        for _ in range(d + 1):
            m = max(abs(np.sum(w * phi[:, j] * r**a * s ** (d - a))) for a in range(d + 1))
            assert m > 1e-6
            j += 1


def test_first_modes_closed_form():
    rng = np.random.default_rng(5)
    r = rng.uniform(0, 0.5, 20)
    s = rng.uniform(0, 0.5, 20)
    phi, dr, ds = O.basis(3, r, s)
    assert np.allclose(phi[:, 0], np.sqrt(2.0), atol=1e-15)
    assert np.allclose(phi[:, 1], 2 * np.sqrt(3.0) * (2 * r + s - 1), atol=1e-14)
    assert np.allclose(phi[:, 2], 2 * (3 * s - 1), atol=1e-14)
    assert np.allclose(dr[:, 1], 4 * np.sqrt(3.0)) and np.allclose(ds[:, 1], 2 * np.sqrt(3.0))
    assert np.allclose(dr[:, 2], 0.0) and np.allclose(ds[:, 2], 6.0)


@pytest.mark.parametrize("p", [1, 3, 5])
def test_gradient_by_finite_differences(p):
    rng = np.random.default_rng(p)
    r = rng.uniform(0.05, 0.45, 15)
    s = rng.uniform(0.05, 0.45, 15)
    h = 1e-6
    _, dr, ds = O.basis(p, r, s)
    fd_r = (O.basis(p, r + h, s)[0] - O.basis(p, r - h, s)[0]) / (2 * h)
    fd_s = (O.basis(p, r, s + h)[0] - O.basis(p, r, s - h)[0]) / (2 * h)
    scale = np.abs(dr).max()
    assert np.abs(fd_r - dr).max() < 1e-7 * scale
    assert np.abs(fd_s - ds).max() < 1e-7 * scale


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_divergence_identity(p):
    # int_T grad phi dr ds = sum over sides of int_side phi n ds
    r, s, w = product_rule(p + 2)
    _, dr, ds = O.basis(p, r, s)
    vol = np.stack([(w[:, None] * dr).sum(0), (w[:, None] * ds).sum(0)])
    x, wx = np.polynomial.legendre.leggauss(p + 2)
    t = 0.5 * (1 + x)
    sur = np.zeros_like(vol)
    # side (0,0)->(1,0): normal (0,-1), length 1
    sur[1] -= 0.5 * (wx[:, None] * O.basis(p, t, 0 * t)[0]).sum(0)
    # side (1,0)->(0,1): normal (1,1)/sqrt2, length sqrt2
    ph = O.basis(p, 1 - t, t)[0]
    sur[0] += 0.5 * (wx[:, None] * ph).sum(0)
    sur[1] += 0.5 * (wx[:, None] * ph).sum(0)
    # side (0,1)->(0,0): normal (-1,0), length 1
    sur[0] -= 0.5 * (wx[:, None] * O.basis(p, 0 * t, t)[0]).sum(0)
    assert np.abs(vol - sur).max() < 1e-12
