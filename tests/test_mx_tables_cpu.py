"""Host-side checks of the matrix-core stage kernels' table operands
(dg_matrix_core_tables), no GPU needed.

1. Every block equals the layout written out independently here from the
   library's reference tables (exact: the same products of the same values).
2. An emulation of the 16 x 16 x 4 products with those operands, in the two
   result orders of the FP64 and FP32 instructions (register r of lane group
   g holds row 4r+g and 4g+r; both measured on the GPU), reproduces the plain
   contractions of eq. (2ddg0): the modes evaluated at the volume and side
   points, and the volume and surface lifts, landing in each lane on the
   modes 4s+g that the lane holds (which the stage update needs).
"""
import numpy as np
import pytest

from paper_1601_07944_amd import binding as B

NQ = {1: 3, 2: 6, 3: 12, 4: 16, 5: 25}


def sizes(p):
    np_ = (p + 1) * (p + 2) // 2
    nq, ne = NQ[p], p + 1
    ns = 3 * ne
    kp = -(-np_ // 4)
    return np_, nq, ne, ns, kp, -(-nq // 16), -(-ns // 16), -(-kp // 4)


def row(fp64, g, r):
    return 4 * r + g if fp64 else 4 * g + r


def mode(fp64, tm, i):
    return 16 * tm + i if fp64 else 4 * (4 * tm + i % 4) + i // 4


def expected_blocks(p, fp64):
    t = B.reference_tables(p)
    np_, nq, ne, ns, kp, tq, ts, tm = sizes(p)
    phi, w = t["phi"], t["w"]
    drw, dsw = w[:, None] * t["dphidr"], w[:, None] * t["dphids"]
    ps = t["phi_side"].reshape(ns, np_)
    gw = np.tile(t["gw"], 3)
    out = []

    def block(f):
        return np.array([f(lane % 16, lane // 16) for lane in range(64)])

    for a in range(tq):
        for s in range(kp):
            out.append(block(lambda i, k: phi[min(16 * a + i, nq - 1), 4 * s + k] if 4 * s + k < np_ else 0.0))
    for tab in (drw, dsw):
        for b in range(tm):
            for a in range(tq):
                for s in range(4):
                    def f(i, k):
                        m, pt = mode(fp64, b, i), 16 * a + row(fp64, k, s)
                        return tab[pt, m] if (m < np_ and pt < nq) else 0.0
                    out.append(block(f))
    for a in range(ts):
        for s in range(kp):
            out.append(block(lambda i, k: ps[min(16 * a + i, ns - 1), 4 * s + k] if 4 * s + k < np_ else 0.0))
    for b in range(tm):
        for a in range(ts):
            for s in range(4):
                def f(i, k):
                    m, sp = mode(fp64, b, i), 16 * a + row(fp64, k, s)
                    return gw[sp] * ps[sp, m] if (m < np_ and sp < ns) else 0.0
                out.append(block(f))
    # the adjoint's transposed contractions
    for tab in (drw, dsw):
        for a in range(tq):
            for s in range(kp):
                out.append(block(lambda i, k: tab[min(16 * a + i, nq - 1), 4 * s + k] if 4 * s + k < np_ else 0.0))
    for b in range(tm):
        for a in range(tq):
            for s in range(4):
                def f(i, k):
                    m, pt = mode(fp64, b, i), 16 * a + row(fp64, k, s)
                    return phi[pt, m] if (m < np_ and pt < nq) else 0.0
                out.append(block(f))
    for b in range(tm):
        for a in range(ts):
            for s in range(4):
                def f(i, k):
                    m, sp = mode(fp64, b, i), 16 * a + row(fp64, k, s)
                    return ps[sp, m] if (m < np_ and sp < ns) else 0.0
                out.append(block(f))
    # side points past the first tile, evaluated per lane (lane 16g + j: mode 4s + g)
    nt = ns - 16 if 16 < ns <= 20 else 0
    for scale in (np.ones(ns), gw):
        for pt in range(nt):
            for s in range(kp):
                sp = 16 + pt
                out.append(block(lambda i, k: scale[sp] * ps[sp, 4 * s + k] if 4 * s + k < np_ else 0.0))
    return np.array(out)


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_table_operands_match_layout(p, fp64):
    got = B.matrix_core_tables(p, fp64)
    ref = expected_blocks(p, fp64)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


def mfma(A, Bop, fp64):
    """One 16 x 16 x 4 product from lane-ordered operands: returns the
    result as [lane][register]."""
    a = A.reshape(4, 16).T        # a[i, k] = lane 16k + i
    b = Bop.reshape(4, 16)        # b[k, j] = lane 16k + j
    d = a @ b                     # d[i, j]
    out = np.empty((64, 4))
    for lane in range(64):
        j, g = lane % 16, lane // 16
        for r in range(4):
            out[lane, r] = d[row(fp64, g, r), j]
    return out


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("p", [1, 3, 4, 5])
def test_emulated_products_reproduce_the_contractions(p, fp64):
    rng = np.random.default_rng(p + 10 * fp64)
    t = B.reference_tables(p)
    np_, nq, ne, ns, kp, tq, ts, tm = sizes(p)
    T = B.matrix_core_tables(p, fp64)
    o_phi, o_dr = 0, tq * kp
    o_ds = o_dr + tm * tq * 4
    o_pe = o_ds + tm * tq * 4
    o_le = o_pe + ts * kp
    c = rng.normal(size=(np_, 16))  # one variable of a 16-element block: c[mode, element]
    lanes = np.arange(64)
    jj, gg = lanes % 16, lanes // 16

    # evaluation at the volume points: register r of lane (j, g) is point 16t + row(g, r)
    for a in range(tq):
        acc = np.zeros((64, 4))
        for s in range(kp):
            Bop = c[np.minimum(4 * s + gg, np_ - 1), jj]  # padded modes load the last one
            acc += mfma(T[o_phi + a * kp + s], Bop, fp64)
        for r in range(4):
            pt = np.minimum(16 * a + row(fp64, gg, r), nq - 1)
            ref = np.einsum("lm,ml->l", t["phi"][pt], c[:, jj])
            assert np.allclose(acc[:, r], ref, rtol=0, atol=1e-12)

    # volume lift of fluxes F (point x element): the lane's register s' is
    # its point 16t + row(g, s'); results land on the lane's modes 4(4tm+r)+g
    F = rng.normal(size=(16 * tq, 16))
    for b in range(tm):
        acc = np.zeros((64, 4))
        for a in range(tq):
            for s in range(4):
                Bop = F[16 * a + row(fp64, gg, s), jj]
                acc += mfma(T[o_dr + (b * tq + a) * 4 + s], Bop, fp64)
        w = t["w"][:, None] * t["dphidr"]
        for r in range(4):
            m = 4 * (4 * b + r) + gg
            ok = m < np_
            ref = np.einsum("pl,pl->l", w[:, np.minimum(m, np_ - 1)], F[:nq, jj])
            assert np.allclose(acc[ok, r], ref[ok], rtol=0, atol=1e-12)
            assert np.all(acc[~ok, r] == 0.0)

    # traces at the side points and the surface lift with Gauss weights
    ps = t["phi_side"].reshape(ns, np_)
    gw = np.tile(t["gw"], 3)
    for a in range(ts):
        acc = np.zeros((64, 4))
        for s in range(kp):
            acc += mfma(T[o_pe + a * kp + s], c[np.minimum(4 * s + gg, np_ - 1), jj], fp64)
        for r in range(4):
            sp = np.minimum(16 * a + row(fp64, gg, r), ns - 1)
            assert np.allclose(acc[:, r], np.einsum("lm,ml->l", ps[sp], c[:, jj]), rtol=0, atol=1e-12)
    G = rng.normal(size=(16 * ts, 16))
    for b in range(tm):
        acc = np.zeros((64, 4))
        for a in range(ts):
            for s in range(4):
                acc += mfma(T[o_le + (b * ts + a) * 4 + s], G[16 * a + row(fp64, gg, s), jj], fp64)
        for r in range(4):
            m = 4 * (4 * b + r) + gg
            ok = m < np_
            ref = np.einsum("pl,pl->l", (gw[:, None] * ps)[:, np.minimum(m, np_ - 1)], G[:ns, jj])
            assert np.allclose(acc[ok, r], ref[ok], rtol=0, atol=1e-12)
