"""Oracle quadrature rules (test infrastructure only; see oracle/__init__.py).

Volume rule.  The paper integrates the volume term with symmetric triangle
rules of order 2p (Section "Volume Integration Kernel"; the Kernel Runtime
Distribution section fixes 3 points at p=1 and 16 at p=4).  The cited rule
tables are not part of the text, so the rule is defined here by its
properties: fully symmetric under the six vertex permutations, exact for all
polynomials of total degree <= 2p on the reference triangle
{(0,0),(1,0),(0,1)}, all points strictly inside, all weights positive, with
the orbit structure of the classical minimal rules:

    p : points : orbits                        approximate orbit parameters
    1 :   3    : S21                           a=0.167
    2 :   6    : 2 x S21                       a=0.0916, 0.446
    3 :  12    : 2 x S21 + S111                a=0.0631, 0.249; (0.636, 0.310)
    4 :  16    : S3 + 3 x S21 + S111           a=0.459, 0.171, 0.0505; (0.00839, 0.263)
    5 :  25    : S3 + 2 x S21 + 3 x S111       a=0.486, 0.109; (0.142, 0.308),
                                               (0.0250, 0.247), (0.00954, 0.0668)

An S21 orbit with parameter a holds the barycentric points (a, a, 1-2a) and
their permutations; an S111 orbit with (a, b) the six permutations of
(a, b, 1-a-b).  Several rules of one degree can share an orbit structure (at
p=3 there are two), so the approximate parameters name the rule; Newton's
method on the moment equations int r^i s^j = i! j! / (i+j+2)! then fixes it
to rounding (the equations are solved in an orthogonal polynomial basis,
where they are well conditioned).  Weights sum to the reference area 1/2.

Edge rule.  (p+1)-point Gauss-Legendre on [-1, 1] (Section "Surface
Integration Kernel"), taken from numpy and symmetrised so that node k and
node p-k are exact negatives and carry bitwise equal weights; the two
elements of an edge then see identical point sets in opposite order.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy.special import eval_jacobi

# orbit structure (n_S3, n_S21, n_S111) and rough parameters per p
_ORBITS = {
    1: ((0, 1, 0), [(0.167,)], [0.1667]),
    2: ((0, 2, 0), [(0.0916,), (0.446,)], [0.055, 0.112]),
    3: ((0, 2, 1), [(0.0631,), (0.249,), (0.636, 0.310)], [0.0254, 0.0584, 0.0414]),
    4: ((1, 3, 1), [(0.459,), (0.171,), (0.0505,), (0.00839, 0.263)], [0.0722, 0.0475, 0.0516, 0.0162, 0.0136]),
    5: (
        (1, 2, 3),
        [(0.486,), (0.109,), (0.142, 0.308), (0.0250, 0.247), (0.00954, 0.0668)],
        [0.0454, 0.0184, 0.0227, 0.0364, 0.0142, 0.0047],
    ),
}


def _expand(struct, params):
    """Points (r, s) and weights of a symmetric rule from its orbit params."""
    n3, n21, n111 = struct
    pts, wts = [], []
    i = 0
    for _ in range(n3):
        pts.append((1.0 / 3.0, 1.0 / 3.0))
        wts.append(params[i])
        i += 1
    for _ in range(n21):
        a, w = params[i], params[i + 1]
        i += 2
        for lam in ((a, a, 1 - 2 * a), (a, 1 - 2 * a, a), (1 - 2 * a, a, a)):
            pts.append((lam[1], lam[2]))
            wts.append(w)
    for _ in range(n111):
        a, b, w = params[i], params[i + 1], params[i + 2]
        i += 3
        c = 1 - a - b
        for lam in ((a, b, c), (a, c, b), (b, a, c), (b, c, a), (c, a, b), (c, b, a)):
            pts.append((lam[1], lam[2]))
            wts.append(w)
    return np.array(pts), np.array(wts)


def _moments(struct, params, deg):
    """Residuals of the moment equations sum_k w_k psi(r_k) = int psi over
    the reference triangle, for psi running over the orthogonal polynomials
    psi_ab = (1-s)^a P_a(2r/(1-s)-1) P_b^{(2a+1,0)}(2s-1), a+b <= deg.
    Their integrals vanish except int psi_00 = 1/2; in this basis the system
    is well conditioned (monomial moments are not: at degree 10 they span
    eight orders of magnitude)."""
    P, W = _expand(struct, params)
    r, s = P[:, 0], P[:, 1]
    t = r + s - 1.0
    res = []
    for d in range(deg + 1):
        for b in range(d + 1):
            a = d - b
            g = sum(math.comb(a, i) ** 2 * t**i * r ** (a - i) for i in range(a + 1))
            h = eval_jacobi(b, 2 * a + 1, 0, 2.0 * s - 1.0)
            res.append(np.sum(W * g * h) - (0.5 if d == 0 else 0.0))
    return np.array(res)


@lru_cache(maxsize=None)
def triangle_rule(p: int):
    """(r, s, w) arrays of the degree-2p symmetric rule described above."""
    struct, orbits, weights = _ORBITS[p]
    x = []
    # parameter vector order: S3 weights, then (a, w) per S21, then (a, b, w) per S111
    k = 0
    wi = 0
    for _ in range(struct[0]):
        x.append(weights[wi])
        wi += 1
    for _ in range(struct[1]):
        x += [orbits[k][0], weights[wi]]
        k += 1
        wi += 1
    for _ in range(struct[2]):
        x += [orbits[k][0], orbits[k][1], weights[wi]]
        k += 1
        wi += 1
    x = np.array(x, dtype=np.float64)
    deg = 2 * p
    for _ in range(60):
        r = _moments(struct, x, deg)
        J = np.empty((r.size, x.size))
        for c in range(x.size):
            h = 1e-7 * max(1.0, abs(x[c]))
            xp = x.copy()
            xm = x.copy()
            xp[c] += h
            xm[c] -= h
            J[:, c] = (_moments(struct, xp, deg) - _moments(struct, xm, deg)) / (2 * h)
        dx = np.linalg.lstsq(J, -r, rcond=None)[0]
        x = x + dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    P, W = _expand(struct, x)
    return P[:, 0].copy(), P[:, 1].copy(), W.copy()


@lru_cache(maxsize=None)
def gauss_legendre(n: int):
    """n-point Gauss-Legendre nodes (ascending) and weights on [-1, 1],
    symmetrised bitwise: x[n-1-k] == -x[k], w[n-1-k] == w[k]."""
    x, w = np.polynomial.legendre.leggauss(n)
    xs = 0.5 * (x - x[::-1])
    ws = 0.5 * (w + w[::-1])
    if n % 2 == 1:
        xs[n // 2] = 0.0
    return xs.copy(), ws.copy()
