// Host-side construction of the reference-element tables: quadrature rules
// and the orthonormal modal basis with its gradients.
//
// Basis.  The paper expands each element's solution in an orthonormal basis
// of the polynomials of degree <= p on the reference triangle
// {(0,0),(1,0),(0,1)} so that the mass matrix is the identity (eq. (np) and
// the text after eq. (2ddg0)).  We use the Dubiner (Koornwinder) basis in
// collapsed coordinates,
//     phi_ab(r,s) = sqrt(2(2a+1)(a+b+1)) (1-s)^a P_a(2r/(1-s)-1) P_b^(2a+1,0)(2s-1),
// ordered by total degree a+b and then by b, evaluated here with three-term
// recurrences: (1-s)^a P_a(...) through the homogeneous Legendre recurrence
// (no division by 1-s), P_b^(alpha,0) through the Jacobi recurrence, and the
// gradients by differentiating both recurrences.
//
// Volume rule.  Symmetric rule of degree 2p (Section "Volume Integration
// Kernel"; 3 points at p=1 and 16 at p=4 per the Kernel Runtime
// Distribution section), with the orbit structure of the classical minimal
// rules; the approximate orbit parameters below name the rule (at p=3 two
// rules share the structure) and Gauss-Newton on the moment equations
// sum_k w_k phi_j(r_k) = int phi_j  (j over the orthonormal basis of degree
// 2p, well conditioned) fixes it to rounding.
//
// Edge rule.  (p+1)-point Gauss-Legendre on [-1,1] (Section "Surface
// Integration Kernel") by Newton on the Legendre polynomial, symmetrised so
// that node p-k is exactly -node k with an identical weight: the two
// elements sharing an edge then evaluate bitwise the same physical points.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dg_internal.h"

namespace dgh {

namespace {

// Jacobi P_n^(alpha,0)(y) and its derivative for n = 0..nmax.
void jacobi_alpha0(int nmax, double alpha, double y, double* P, double* dP)
{
    P[0] = 1.0;
    dP[0] = 0.0;
    if (nmax == 0) return;
    const double beta = 0.0;
    P[1] = 0.5 * (alpha - beta + (alpha + beta + 2.0) * y);
    dP[1] = 0.5 * (alpha + beta + 2.0);
    for (int n = 2; n <= nmax; ++n) {
        double ab = alpha + beta;
        double c0 = 2.0 * n * (n + ab) * (2.0 * n + ab - 2.0);
        double c1 = (2.0 * n + ab - 1.0) * (2.0 * n + ab) * (2.0 * n + ab - 2.0);
        double c2 = (2.0 * n + ab - 1.0) * (alpha * alpha - beta * beta);
        double c3 = 2.0 * (n + alpha - 1.0) * (n + beta - 1.0) * (2.0 * n + ab);
        P[n] = ((c1 * y + c2) * P[n - 1] - c3 * P[n - 2]) / c0;
        dP[n] = (c1 * P[n - 1] + (c1 * y + c2) * dP[n - 1] - c3 * dP[n - 2]) / c0;
    }
}

}  // namespace

int n_modes(int p) { return (p + 1) * (p + 2) / 2; }

void basis_eval(int p, double r, double s, double* phi, double* dr, double* ds)
{
    // L_a = (1-s)^a P_a(2r/(1-s) - 1), homogeneous Legendre recurrence:
    // (a+1) L_{a+1} = (2a+1)(2r+s-1) L_a - a (1-s)^2 L_{a-1}
    double L[16], Lr[16], Ls[16];
    const double x = 2.0 * r + s - 1.0, w = 1.0 - s;
    L[0] = 1.0;
    Lr[0] = 0.0;
    Ls[0] = 0.0;
    if (p >= 1) {
        L[1] = x;
        Lr[1] = 2.0;
        Ls[1] = 1.0;
    }
    for (int a = 1; a < p; ++a) {
        double k1 = (2.0 * a + 1.0), k2 = (double)a, inv = 1.0 / (a + 1.0);
        L[a + 1] = (k1 * x * L[a] - k2 * w * w * L[a - 1]) * inv;
        Lr[a + 1] = (k1 * (2.0 * L[a] + x * Lr[a]) - k2 * w * w * Lr[a - 1]) * inv;
        Ls[a + 1] = (k1 * (L[a] + x * Ls[a]) - k2 * (-2.0 * w * L[a - 1] + w * w * Ls[a - 1])) * inv;
    }
    int j = 0;
    double P[16], dP[16];
    for (int d = 0; d <= p; ++d) {
        for (int b = 0; b <= d; ++b, ++j) {
            int a = d - b;
            jacobi_alpha0(b, 2.0 * a + 1.0, 2.0 * s - 1.0, P, dP);
            double K = std::sqrt(2.0 * (2.0 * a + 1.0) * (a + b + 1.0));
            double h = P[b], hs = 2.0 * dP[b];
            if (phi) phi[j] = K * L[a] * h;
            if (dr) dr[j] = K * Lr[a] * h;
            if (ds) ds[j] = K * (Ls[a] * h + L[a] * hs);
        }
    }
}

namespace {

struct OrbitSpec {
    int n3, n21, n111;
    std::vector<double> guess;  // S3 weights, (a, w) per S21, (a, b, w) per S111
};

OrbitSpec orbit_spec(int p)
{
    switch (p) {
    case 1: return {0, 1, 0, {0.167, 0.1667}};
    case 2: return {0, 2, 0, {0.0916, 0.055, 0.446, 0.112}};
    case 3: return {0, 2, 1, {0.0631, 0.0254, 0.249, 0.0584, 0.636, 0.310, 0.0414}};
    case 4: return {1, 3, 1, {0.0722, 0.459, 0.0475, 0.171, 0.0516, 0.0505, 0.0162, 0.00839, 0.263, 0.0136}};
    default:
        return {1, 2, 3, {0.0454, 0.486, 0.0184, 0.109, 0.0227, 0.142, 0.308, 0.0364, 0.0250, 0.247, 0.0142, 0.00954, 0.0668, 0.0047}};
    }
}

// Points, weights and their derivatives with respect to the parameters.
// Barycentric (l1, l2, l3) maps to (r, s) = (l2, l3).
void expand_rule(const OrbitSpec& o, const std::vector<double>& x, std::vector<double>& r, std::vector<double>& s,
                 std::vector<double>& w, std::vector<double>& dr, std::vector<double>& ds, std::vector<double>& dw)
{
    const int npar = (int)x.size();
    r.clear();
    s.clear();
    w.clear();
    dr.clear();
    ds.clear();
    dw.clear();
    auto push = [&](double rr, double ss, double ww, int ip, const double* drr, const double* dss, int iw) {
        r.push_back(rr);
        s.push_back(ss);
        w.push_back(ww);
        for (int c = 0; c < npar; ++c) {
            double a = 0, b = 0;
            if (drr && c >= ip && c < ip + 2) {
                a = drr[c - ip];
                b = dss[c - ip];
            }
            dr.push_back(a);
            ds.push_back(b);
            dw.push_back(c == iw ? 1.0 : 0.0);
        }
    };
    int i = 0;
    for (int t = 0; t < o.n3; ++t, ++i) push(1.0 / 3.0, 1.0 / 3.0, x[i], -1, nullptr, nullptr, i);
    for (int t = 0; t < o.n21; ++t, i += 2) {
        double a = x[i], wt = x[i + 1];
        // barycentric (a,a,1-2a), (a,1-2a,a), (1-2a,a,a); d/da of (r, s)
        double d1[2] = {1.0, 0.0}, e1[2] = {-2.0, 0.0};
        double d2[2] = {-2.0, 0.0}, e2[2] = {1.0, 0.0};
        double d3[2] = {1.0, 0.0}, e3[2] = {1.0, 0.0};
        push(a, 1.0 - 2.0 * a, wt, i, d1, e1, i + 1);
        push(1.0 - 2.0 * a, a, wt, i, d2, e2, i + 1);
        push(a, a, wt, i, d3, e3, i + 1);
    }
    for (int t = 0; t < o.n111; ++t, i += 3) {
        double a = x[i], b = x[i + 1], c = 1.0 - a - b, wt = x[i + 2];
        // six permutations of (a, b, c); (r, s) are the 2nd and 3rd entries;
        // d/d(a, b) with dc = -(da + db)
        struct Perm {
            double r, s, ra, rb, sa, sb;
        } P[6] = {
            {b, c, 0, 1, -1, -1}, {c, b, -1, -1, 0, 1}, {a, c, 1, 0, -1, -1},
            {c, a, -1, -1, 1, 0}, {a, b, 1, 0, 0, 1},   {b, a, 0, 1, 1, 0},
        };
        for (auto& q : P) {
            double drr[2] = {q.ra, q.rb}, dss[2] = {q.sa, q.sb};
            push(q.r, q.s, wt, i, drr, dss, i + 2);
        }
    }
}

// Solve min ||J dx + f|| by Householder QR (rows >= cols).
std::vector<double> lstsq(std::vector<double> J, std::vector<double> f, int rows, int cols)
{
    for (int k = 0; k < cols; ++k) {
        double nrm = 0;
        for (int i = k; i < rows; ++i) nrm += J[i * cols + k] * J[i * cols + k];
        nrm = std::sqrt(nrm);
        double alpha = J[k * cols + k] > 0 ? -nrm : nrm;
        std::vector<double> v(rows, 0.0);
        for (int i = k; i < rows; ++i) v[i] = J[i * cols + k];
        v[k] -= alpha;
        double vv = 0;
        for (int i = k; i < rows; ++i) vv += v[i] * v[i];
        if (vv == 0) continue;
        for (int c = k; c < cols; ++c) {
            double d = 0;
            for (int i = k; i < rows; ++i) d += v[i] * J[i * cols + c];
            d = 2.0 * d / vv;
            for (int i = k; i < rows; ++i) J[i * cols + c] -= d * v[i];
        }
        double d = 0;
        for (int i = k; i < rows; ++i) d += v[i] * f[i];
        d = 2.0 * d / vv;
        for (int i = k; i < rows; ++i) f[i] -= d * v[i];
    }
    std::vector<double> x(cols);
    for (int k = cols - 1; k >= 0; --k) {
        double acc = -f[k];
        for (int c = k + 1; c < cols; ++c) acc -= J[k * cols + c] * x[c];
        x[k] = acc / J[k * cols + k];
    }
    return x;
}

}  // namespace

void volume_rule(int p, std::vector<double>& r, std::vector<double>& s, std::vector<double>& w)
{
    OrbitSpec o = orbit_spec(p);
    std::vector<double> x = o.guess;
    const int deg = 2 * p, nm = n_modes(deg), npar = (int)x.size();
    const double mean0 = std::sqrt(2.0) * 0.5;  // int phi_1 = sqrt(2) * area
    std::vector<double> dr, ds, dw, phi(nm), gr(nm), gs(nm);
    for (int it = 0; it < 60; ++it) {
        expand_rule(o, x, r, s, w, dr, ds, dw);
        const int npts = (int)r.size();
        std::vector<double> f(nm, 0.0), J((size_t)nm * npar, 0.0);
        f[0] = -mean0;
        for (int k = 0; k < npts; ++k) {
            basis_eval(deg, r[k], s[k], phi.data(), gr.data(), gs.data());
            for (int j = 0; j < nm; ++j) {
                f[j] += w[k] * phi[j];
                for (int c = 0; c < npar; ++c)
                    J[j * npar + c] += dw[k * npar + c] * phi[j] +
                                       w[k] * (gr[j] * dr[k * npar + c] + gs[j] * ds[k * npar + c]);
            }
        }
        std::vector<double> dx = lstsq(J, f, nm, npar);
        double mx = 0;
        for (int c = 0; c < npar; ++c) {
            x[c] += dx[c];
            mx = std::fmax(mx, std::fabs(dx[c]));
        }
        if (mx < 1e-16) break;
    }
    expand_rule(o, x, r, s, w, dr, ds, dw);
}

void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        // Newton on P_n from the Chebyshev-like initial guess, ascending order
        double z = -std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pn = (n == 1) ? z : p1, pm = (n == 1) ? 1.0 : p0;
            dp = n * (z * pn - pm) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    std::vector<double> xs(n), ws(n);
    for (int i = 0; i < n; ++i) {
        xs[i] = 0.5 * (x[i] - x[n - 1 - i]);
        ws[i] = 0.5 * (w[i] + w[n - 1 - i]);
    }
    if (n % 2 == 1) xs[n / 2] = 0.0;
    x = xs;
    w = ws;
}

// Side points of the reference triangle; side q runs from vertex q to q+1.
void side_point(int q, double xi, double* r, double* s)
{
    switch (q) {
    case 0: *r = 0.5 * (1.0 + xi); *s = 0.0; break;
    case 1: *r = 0.5 * (1.0 - xi); *s = 0.5 * (1.0 + xi); break;
    default: *r = 0.0; *s = 0.5 * (1.0 - xi); break;
    }
}

// Table layout shared with the kernels (all doubles):
//   PHI [NQ][NP]        phi_j at volume point k
//   DRW [NQ][NP]        w_k dphi_j/dr at volume point k
//   DSW [NQ][NP]        w_k dphi_j/ds at volume point k
//   PHS [3][NE][NP]     phi_j at edge point k of side q
//   GW  [NE]            Gauss-Legendre weights
//   QW  [NQ]            volume weights (projection)
//   QR  [NQ], QS [NQ]   volume points (reference coordinates)
std::vector<double> build_tables(int p, TableLayout* lay)
{
    std::vector<double> r, s, w, gx, gw;
    volume_rule(p, r, s, w);
    gauss_rule(p + 1, gx, gw);
    const int np = n_modes(p), nq = (int)r.size(), ne = p + 1;
    TableLayout L;
    L.np = np;
    L.nq = nq;
    L.ne = ne;
    L.phi = 0;
    L.drw = L.phi + nq * np;
    L.dsw = L.drw + nq * np;
    L.phs = L.dsw + nq * np;
    L.gw = L.phs + 3 * ne * np;
    L.qw = L.gw + ne;
    L.qr = L.qw + nq;
    L.qs = L.qr + nq;
    L.size = L.qs + nq;
    std::vector<double> t(L.size, 0.0);
    std::vector<double> phi(np), dr(np), ds(np);
    for (int k = 0; k < nq; ++k) {
        basis_eval(p, r[k], s[k], phi.data(), dr.data(), ds.data());
        for (int j = 0; j < np; ++j) {
            t[L.phi + k * np + j] = phi[j];
            t[L.drw + k * np + j] = w[k] * dr[j];
            t[L.dsw + k * np + j] = w[k] * ds[j];
        }
        t[L.qw + k] = w[k];
        t[L.qr + k] = r[k];
        t[L.qs + k] = s[k];
    }
    for (int q = 0; q < 3; ++q)
        for (int k = 0; k < ne; ++k) {
            double rr, ss;
            side_point(q, gx[k], &rr, &ss);
            basis_eval(p, rr, ss, phi.data(), nullptr, nullptr);
            for (int j = 0; j < np; ++j) t[L.phs + (q * ne + k) * np + j] = phi[j];
        }
    for (int k = 0; k < ne; ++k) t[L.gw + k] = gw[k];
    if (lay) *lay = L;
    return t;
}

std::vector<double> build_mx_tables(int p, const std::vector<double>& t, const TableLayout& L, bool f64)
{
    auto row = [&](int g, int r) { return f64 ? dgk::mx_row<true>(g, r) : dgk::mx_row<false>(g, r); };
    auto mode = [&](int tm, int i) { return f64 ? dgk::mx_mode<true>(tm, i) : dgk::mx_mode<false>(tm, i); };
    const dgk::MxLayout x = dgk::mx_layout(p);
    std::vector<double> o((size_t)x.blocks * 64, 0.0);
    auto put = [&](int blk, int lane, double v) { o[(size_t)blk * 64 + lane] = v; };
    for (int lane = 0; lane < 64; ++lane) {
        const int i = lane % 16, k = lane / 16;
        for (int tq = 0; tq < x.tq; ++tq)
            for (int s = 0; s < x.kp; ++s) {
                const int pt = std::min(16 * tq + i, x.nq - 1), j = 4 * s + k;
                put(x.phi + tq * x.kp + s, lane, j < x.np ? t[L.phi + pt * x.np + j] : 0.0);
            }
        for (int tm = 0; tm < x.tm; ++tm)
            for (int tq = 0; tq < x.tq; ++tq)
                for (int s = 0; s < 4; ++s) {
                    const int j = mode(tm, i), pt = 16 * tq + row(k, s), b = (tm * x.tq + tq) * 4 + s;
                    const bool in = j < x.np && pt < x.nq;
                    put(x.dr + b, lane, in ? t[L.drw + pt * x.np + j] : 0.0);
                    put(x.ds + b, lane, in ? t[L.dsw + pt * x.np + j] : 0.0);
                }
        for (int ts = 0; ts < x.ts; ++ts)
            for (int s = 0; s < x.kp; ++s) {
                const int sp = std::min(16 * ts + i, x.ns - 1), j = 4 * s + k;
                put(x.pe + ts * x.kp + s, lane, j < x.np ? t[L.phs + sp * x.np + j] : 0.0);
            }
        for (int tm = 0; tm < x.tm; ++tm)
            for (int ts = 0; ts < x.ts; ++ts)
                for (int s = 0; s < 4; ++s) {
                    const int j = mode(tm, i), sp = 16 * ts + row(k, s);
                    const bool in = j < x.np && sp < x.ns;
                    put(x.le + (tm * x.ts + ts) * 4 + s, lane, in ? t[L.gw + sp % x.ne] * t[L.phs + sp * x.np + j] : 0.0);
                    put(x.pel + (tm * x.ts + ts) * 4 + s, lane, in ? t[L.phs + sp * x.np + j] : 0.0);
                }
        for (int tq = 0; tq < x.tq; ++tq)
            for (int s = 0; s < x.kp; ++s) {
                const int pt = std::min(16 * tq + i, x.nq - 1), j = 4 * s + k;
                put(x.dre + tq * x.kp + s, lane, j < x.np ? t[L.drw + pt * x.np + j] : 0.0);
                put(x.dse + tq * x.kp + s, lane, j < x.np ? t[L.dsw + pt * x.np + j] : 0.0);
            }
        for (int tm = 0; tm < x.tm; ++tm)
            for (int tq = 0; tq < x.tq; ++tq)
                for (int s = 0; s < 4; ++s) {
                    const int j = mode(tm, i), pt = 16 * tq + row(k, s);
                    put(x.phl + (tm * x.tq + tq) * 4 + s, lane, j < x.np && pt < x.nq ? t[L.phi + pt * x.np + j] : 0.0);
                }
        // lane 16g + j: k = g here
        for (int pt = 0; pt < x.nt; ++pt)
            for (int s = 0; s < x.kp; ++s) {
                const int sp = 16 + pt, j = 4 * s + k;
                put(x.tpe + pt * x.kp + s, lane, j < x.np ? t[L.phs + sp * x.np + j] : 0.0);
                put(x.tle + pt * x.kp + s, lane, j < x.np ? t[L.gw + sp % x.ne] * t[L.phs + sp * x.np + j] : 0.0);
            }
    }
    return o;
}

}  // namespace dgh
