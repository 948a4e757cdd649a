"""Pins of the oracle's quadrature rules (test infrastructure).

Volume rule: symmetric rule of order 2p (Section "Volume Integration
Kernel"), point counts printed in the Kernel Runtime Distribution section.
Edge rule: (p+1)-point Gauss-Legendre (Section "Surface Integration Kernel").
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import quadrature as Q

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "point_counts.json")))


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_triangle_rule_exact_monomials(p):
    # brute force on the reference triangle: int r^a s^b = a! b! / (a+b+2)!
    r, s, w = Q.triangle_rule(p)
    for a in range(2 * p + 1):
        for b in range(2 * p + 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = np.sum(w * r**a * s**b)
            assert abs(got / exact - 1.0) < 5e-15, (p, a, b, got, exact)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_triangle_rule_not_exact_beyond_2p(p):
    # the rule is of degree exactly 2p (a degree 2p+2 monomial is missed)
    r, s, w = Q.triangle_rule(p)
    errs = []
    d = 2 * p + 2
    for a in range(d + 1):
        b = d - a
        exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
        errs.append(abs(np.sum(w * r**a * s**b) / exact - 1.0))
    assert max(errs) > 1e-8


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_triangle_rule_symmetric_interior_positive(p):
    r, s, w = Q.triangle_rule(p)
    l1 = 1.0 - r - s
    assert np.all(w > 0) and np.all(r > 0) and np.all(s > 0) and np.all(l1 > 0)
    assert abs(w.sum() - 0.5) < 1e-15
    pts = np.stack([l1, r, s], axis=1)
    key = lambda P, W: np.array(sorted(map(tuple, np.round(np.c_[P[:, 1:], W], 13))))
    base = key(pts, w)
    for perm in ([1, 2, 0], [2, 0, 1], [0, 2, 1], [1, 0, 2], [2, 1, 0]):
        assert np.allclose(key(pts[:, perm], w), base, atol=1e-13)


def test_point_counts_match_paper():
    for p, n in GOLD["volume_points"].items():
        assert Q.triangle_rule(int(p))[0].size == n
    for p, n in GOLD["surface_points_per_triangle"].items():
        assert 3 * Q.gauss_legendre(int(p) + 1)[0].size == n


def test_p1_rule_is_interior_orbit():
    # p=1: the degree-2 rule with one S21 orbit at barycentric (2/3,1/6,1/6),
    # not the edge-midpoint rule of the same degree
    r, s, w = Q.triangle_rule(1)
    assert np.allclose(sorted(zip(r, s)), sorted([(1 / 6, 1 / 6), (2 / 3, 1 / 6), (1 / 6, 2 / 3)]), atol=1e-15)
    assert np.allclose(w, 1 / 6, atol=1e-16)


def test_p3_rule_is_the_named_root():
    # two degree-6 12-point S21,S21,S111 rules exist; the named one has an
    # orbit at a ~ 0.0631 and weights ~ 0.0254 / 0.0584 / 0.0414
    r, s, w = Q.triangle_rule(3)
    assert np.isclose(min(r.min(), s.min(), (1 - r - s).min()), 0.0531450498448, atol=1e-10)
    assert np.allclose(sorted(set(np.round(w, 10))), [0.0254224532, 0.0414255378, 0.0583931379], atol=1e-10)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_gauss_legendre(n):
    x, w = Q.gauss_legendre(n)
    ref_x, ref_w = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, ref_x, atol=2e-16) and np.allclose(w, ref_w, atol=2e-16)
    assert np.all(x[::-1] == -x) and np.all(w[::-1] == w)
    for d in range(2 * n):
        exact = 0.0 if d % 2 else 2.0 / (d + 1)
        assert abs(np.sum(w * x**d) - exact) < 1e-15
