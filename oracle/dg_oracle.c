/*
 * dg_oracle.c -- plain, serial FP64 CPU reference of the modal DG method.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.  It shares no code with
 * the HIP library: basis, geometry, flux, numerical flux and time stepping
 * are written out here again from their definitions.
 *
 * What it computes (Fuhry, Giuliani, Krivodonova, "Discontinuous Galerkin
 * methods on graphics processing units for nonlinear hyperbolic conservation
 * laws"):
 *   - the semi-discrete right-hand side of eq. (2ddg0): for every element i,
 *     mode j and equation m
 *       R = (1/det J_i) [ sum_k w_k grad_r phi_j(r_k) . (adj(J_i) F(U_i(r_k)))
 *                         - sum_q l_q sum_k omega_k phi_j(r_qk) Fn_k ]
 *     with the volume term of eq. (volume) after the element map eq. (2dmap)
 *     and the surface term eq. (surface) after the edge map eq. (1dmap);
 *   - the element loop visits one element at a time and evaluates the
 *     numerical flux of each of its three sides itself, so every interior
 *     edge flux is computed twice (once from each side);
 *   - the neighbour's trace is taken at the reversed edge point (Section
 *     "Surface Integration Kernel": the two elements traverse a shared edge
 *     in opposite directions);
 *   - L2 projection onto the orthonormal basis (mass matrix = det J * I);
 *   - three-stage SSP Runge-Kutta in Shu-Osher form and a CFL time step;
 *   - the paper's classic second- and fourth-order Runge-Kutta steps;
 *   - the Barth-Jespersen slope limiter for p = 1 (Section "Limiting
 *     Kernel"), optionally applied after every RK stage.
 *
 * Conventions (readings of points the paper leaves open):
 *   - J = d(x,y)/d(r,s) = [[x2-x1, x3-x1], [y2-y1, y3-y1]];
 *     grad_x phi = J^{-T} grad_r phi, so the volume integrand is
 *     grad_r phi . (adj(J) F) with adj(J) = det(J) J^{-1}.
 *   - Basis: orthonormal Dubiner polynomials on {(0,0),(1,0),(0,1)}:
 *       phi_ab = sqrt(2(2a+1)(a+b+1)) g_a(r,s) P_b^{(2a+1,0)}(2s-1),
 *       g_a = (1-s)^a P_a(2r/(1-s)-1) = sum_i C(a,i)^2 (r+s-1)^i r^(a-i),
 *     ordered by total degree a+b, then by b.
 *   - Local side q runs from vertex q to vertex q+1 (counter-clockwise);
 *     side points: q=0 ((1+x)/2, 0), q=1 ((1-x)/2, (1+x)/2), q=2 (0, (1-x)/2)
 *     for Gauss node x in [-1,1]; the neighbour's point for node k is p-k.
 *   - Numerical flux: local Lax-Friedrichs,
 *       Fn = (F(U_L).n + F(U_R).n)/2 - lambda (U_R - U_L)/2,
 *       lambda = max(|v_L.n| + c_L, |v_R.n| + c_R),  c = sqrt(gamma p / rho).
 *   - Edge scale l = |edge|/2 (eq. (len)); Gauss weights sum to 2.
 *   - Time step: dt = CFL min_i r_i / (|v_i| + c_i) with the inscribed radius
 *     r_i = det J_i / perimeter_i and the state at the cell average
 *     sqrt(2) c_{i,0}.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define M 4
#define NP_MAX 21
#define NQ_MAX 25
#define NE_MAX 6

typedef struct {
    int p, np, nq, ne;
    int64_t n;
    double gamma;
    double *vxy;     /* [n][3][2] */
    int64_t *nbr;    /* [n][3] */
    int8_t *nbs;     /* [n][3] */
    double *qr, *qs, *qw; /* volume rule [nq] */
    double *gx, *gw;      /* Gauss-Legendre [ne] */
    /* basis values at the fixed reference points */
    double *phi_v; /* [nq][np] */
    double *dr_v;  /* [nq][np] */
    double *ds_v;  /* [nq][np] */
    double *phi_s; /* [3][ne][np] */
    double bc_state[M]; /* state of boundary code -3 */
    int has_bc;         /* some side is a domain boundary (negative code) */
} orc_ctx;

/* ---------------------------------------------------------------- basis */
static double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

static double ipow(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

/* Jacobi polynomial by its explicit sum:
 * P_n^{(a,b)}(x) = sum_s C(n+a, n-s) C(n+b, s) ((x-1)/2)^s ((x+1)/2)^(n-s) */
static double jacobi(int n, int a, int b, double x)
{
    double xm = 0.5 * (x - 1.0), xp = 0.5 * (x + 1.0), sum = 0.0;
    for (int s = 0; s <= n; ++s) sum += binom(n + a, n - s) * binom(n + b, s) * ipow(xm, s) * ipow(xp, n - s);
    return sum;
}

/* d/dx P_n^{(a,b)}(x) = (n+a+b+1)/2 P_{n-1}^{(a+1,b+1)}(x) */
static double djacobi(int n, int a, int b, double x)
{
    if (n == 0) return 0.0;
    return 0.5 * (double)(n + a + b + 1) * jacobi(n - 1, a + 1, b + 1, x);
}

/* All np basis functions and their r, s derivatives at (r, s). */
void orc_basis(int p, double r, double s, double *phi, double *dphidr, double *dphids)
{
    int j = 0;
    double t = r + s - 1.0;
    for (int d = 0; d <= p; ++d) {
        for (int b = 0; b <= d; ++b, ++j) {
            int a = d - b;
            double g = 0.0, gr = 0.0, gs = 0.0;
            for (int i = 0; i <= a; ++i) {
                double c2 = binom(a, i) * binom(a, i);
                g += c2 * ipow(t, i) * ipow(r, a - i);
                if (i >= 1) {
                    gr += c2 * (double)i * ipow(t, i - 1) * ipow(r, a - i);
                    gs += c2 * (double)i * ipow(t, i - 1) * ipow(r, a - i);
                }
                if (a - i >= 1) gr += c2 * (double)(a - i) * ipow(t, i) * ipow(r, a - i - 1);
            }
            double h = jacobi(b, 2 * a + 1, 0, 2.0 * s - 1.0);
            double hs = 2.0 * djacobi(b, 2 * a + 1, 0, 2.0 * s - 1.0);
            double K = sqrt(2.0 * (2 * a + 1) * (a + b + 1));
            if (phi) phi[j] = K * g * h;
            if (dphidr) dphidr[j] = K * gr * h;
            if (dphids) dphids[j] = K * (gs * h + g * hs);
        }
    }
}

static void side_point(int q, double x, double *r, double *s)
{
    if (q == 0) {
        *r = 0.5 * (1.0 + x);
        *s = 0.0;
    } else if (q == 1) {
        *r = 0.5 * (1.0 - x);
        *s = 0.5 * (1.0 + x);
    } else {
        *r = 0.0;
        *s = 0.5 * (1.0 - x);
    }
}

/* -------------------------------------------------------------- context */
orc_ctx *orc_create(int p, int64_t n, const double *vxy, const int64_t *nbr, const int8_t *nbs, double gamma, int nq,
                    const double *qr, const double *qs, const double *qw, int ne, const double *gx, const double *gw)
{
    if (p < 1 || p > 5 || nq > NQ_MAX || ne > NE_MAX) return NULL;
    orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    c->p = p;
    c->np = (p + 1) * (p + 2) / 2;
    c->nq = nq;
    c->ne = ne;
    c->n = n;
    c->gamma = gamma;
    c->vxy = (double *)malloc(sizeof(double) * 6 * n);
    memcpy(c->vxy, vxy, sizeof(double) * 6 * n);
    c->nbr = (int64_t *)malloc(sizeof(int64_t) * 3 * n);
    memcpy(c->nbr, nbr, sizeof(int64_t) * 3 * n);
    c->nbs = (int8_t *)malloc(3 * n);
    memcpy(c->nbs, nbs, 3 * n);
    for (int64_t x = 0; x < 3 * n; ++x)
        if (nbr[x] < 0) c->has_bc = 1;
    /* prescribed boundary state until orc_set_bc_state: a gas at rest, rho = 1, p = 1 */
    c->bc_state[0] = 1.0;
    c->bc_state[1] = c->bc_state[2] = 0.0;
    c->bc_state[3] = 1.0 / (gamma - 1.0);
    c->qr = (double *)malloc(sizeof(double) * nq);
    c->qs = (double *)malloc(sizeof(double) * nq);
    c->qw = (double *)malloc(sizeof(double) * nq);
    memcpy(c->qr, qr, sizeof(double) * nq);
    memcpy(c->qs, qs, sizeof(double) * nq);
    memcpy(c->qw, qw, sizeof(double) * nq);
    c->gx = (double *)malloc(sizeof(double) * ne);
    c->gw = (double *)malloc(sizeof(double) * ne);
    memcpy(c->gx, gx, sizeof(double) * ne);
    memcpy(c->gw, gw, sizeof(double) * ne);
    int np = c->np;
    c->phi_v = (double *)malloc(sizeof(double) * nq * np);
    c->dr_v = (double *)malloc(sizeof(double) * nq * np);
    c->ds_v = (double *)malloc(sizeof(double) * nq * np);
    c->phi_s = (double *)malloc(sizeof(double) * 3 * ne * np);
    for (int k = 0; k < nq; ++k) orc_basis(p, qr[k], qs[k], c->phi_v + k * np, c->dr_v + k * np, c->ds_v + k * np);
    for (int q = 0; q < 3; ++q)
        for (int k = 0; k < ne; ++k) {
            double r, s;
            side_point(q, gx[k], &r, &s);
            orc_basis(p, r, s, c->phi_s + (q * ne + k) * np, NULL, NULL);
        }
    return c;
}

/* state of boundary code -3 (conserved variables) */
void orc_set_bc_state(orc_ctx *c, const double *U)
{
    for (int m = 0; m < M; ++m) c->bc_state[m] = U[m];
}

void orc_destroy(orc_ctx *c)
{
    if (!c) return;
    free(c->vxy);
    free(c->nbr);
    free(c->nbs);
    free(c->qr);
    free(c->qs);
    free(c->qw);
    free(c->gx);
    free(c->gw);
    free(c->phi_v);
    free(c->dr_v);
    free(c->ds_v);
    free(c->phi_s);
    free(c);
}

int orc_np(const orc_ctx *c) { return c->np; }

/* ------------------------------------------------------------- geometry */
static void element_geometry(const orc_ctx *c, int64_t i, double adj[2][2], double *det)
{
    const double *v = c->vxy + 6 * i;
    double x1 = v[0], y1 = v[1], x2 = v[2], y2 = v[3], x3 = v[4], y3 = v[5];
    *det = (x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1);
    adj[0][0] = y3 - y1;
    adj[0][1] = -(x3 - x1);
    adj[1][0] = -(y2 - y1);
    adj[1][1] = x2 - x1;
}

/* outward unit normal and half length of local side q (vertex q -> q+1) */
static void side_geometry(const orc_ctx *c, int64_t i, int q, double *nx, double *ny, double *l)
{
    const double *v = c->vxy + 6 * i;
    int a = q, b = (q + 1) % 3;
    double dx = v[2 * b] - v[2 * a], dy = v[2 * b + 1] - v[2 * a + 1];
    double len = sqrt(dx * dx + dy * dy);
    *nx = dy / len;
    *ny = -dx / len;
    *l = 0.5 * len;
}

void orc_det(const orc_ctx *c, double *det)
{
    for (int64_t i = 0; i < c->n; ++i) {
        double adj[2][2];
        element_geometry(c, i, adj, det + i);
    }
}

/* physical coordinates of reference points (r, s) on every element */
void orc_map_points(const orc_ctx *c, int npts, const double *r, const double *s, double *xy /* [n][npts][2] */)
{
    for (int64_t i = 0; i < c->n; ++i) {
        const double *v = c->vxy + 6 * i;
        for (int k = 0; k < npts; ++k) {
            double l1 = 1.0 - r[k] - s[k];
            xy[(i * npts + k) * 2 + 0] = v[0] * l1 + v[2] * r[k] + v[4] * s[k];
            xy[(i * npts + k) * 2 + 1] = v[1] * l1 + v[3] * r[k] + v[5] * s[k];
        }
    }
}

void orc_quad_points(const orc_ctx *c, double *xy) { orc_map_points(c, c->nq, c->qr, c->qs, xy); }

/* U_h at reference points of every element: out[n][npts][M] */
void orc_eval(const orc_ctx *c, const double *C, int npts, const double *r, const double *s, double *out)
{
    int np = c->np;
    double *phi = (double *)malloc(sizeof(double) * npts * np);
    for (int k = 0; k < npts; ++k) orc_basis(c->p, r[k], s[k], phi + k * np, NULL, NULL);
    for (int64_t i = 0; i < c->n; ++i)
        for (int k = 0; k < npts; ++k)
            for (int m = 0; m < M; ++m) {
                double u = 0.0;
                for (int j = 0; j < np; ++j) u += C[(i * M + m) * np + j] * phi[k * np + j];
                out[(i * npts + k) * M + m] = u;
            }
    free(phi);
}

/* ------------------------------------------------------- forward operator */
/* double precision: orc_euler_flux, orc_llf, orc_rhs_element, orc_rhs */
#define R_T double
#define R_ABS(x) fabs(x)
#define R_SQRT(x) sqrt(x)
#define R_GE(a, b) ((a) >= (b))
#define R_NAME(name) orc_##name
#include "dg_oracle_forward.inc"
#undef R_T
#undef R_ABS
#undef R_SQRT
#undef R_GE
#undef R_NAME

/* double complex (complex-step derivatives): orc_cs_rhs */
#define R_T double _Complex
#define R_ABS(x) (creal(x) < 0.0 ? -(x) : (x))
#define R_SQRT(x) csqrt(x)
#define R_GE(a, b) (creal(a) >= creal(b))
#define R_NAME(name) orc_cs_##name
#include "dg_oracle_forward.inc"
#undef R_T
#undef R_ABS
#undef R_SQRT
#undef R_GE
#undef R_NAME

/* L2 projection of point values u[n][nq][M] at the volume points:
 * c_j = sum_k w_k phi_j(r_k) u(x(r_k))  (mass matrix det J * I) */
void orc_project(const orc_ctx *c, const double *u, double *C)
{
    const int np = c->np, nq = c->nq;
    for (int64_t i = 0; i < c->n; ++i)
        for (int m = 0; m < M; ++m)
            for (int j = 0; j < np; ++j) {
                double s = 0.0;
                for (int k = 0; k < nq; ++k) s += c->qw[k] * c->phi_v[k * np + j] * u[(i * nq + k) * M + m];
                C[(i * M + m) * np + j] = s;
            }
}

/* CFL time step; returns 0, or -1 (and dt = NaN) for a non-physical mean */
int orc_max_dt(const orc_ctx *c, const double *C, double cfl, double *dt)
{
    const int np = c->np;
    double best = INFINITY;
    int bad = 0;
    for (int64_t i = 0; i < c->n; ++i) {
        double adj[2][2], det;
        element_geometry(c, i, adj, &det);
        double per = 0.0;
        for (int q = 0; q < 3; ++q) {
            double nx, ny, l;
            side_geometry(c, i, q, &nx, &ny, &l);
            per += 2.0 * l;
        }
        double U[M];
        for (int m = 0; m < M; ++m) U[m] = sqrt(2.0) * C[(i * M + m) * np + 0];
        double rho = U[0], u = U[1] / rho, v = U[2] / rho;
        double pr = (c->gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v));
        if (!(rho > 0.0) || !(pr > 0.0)) {
            bad = 1;
            continue;
        }
        double lam = sqrt(u * u + v * v) + sqrt(c->gamma * pr / rho);
        double d = (det / per) / lam;
        if (d < best) best = d;
    }
    if (bad) {
        *dt = NAN;
        return -1;
    }
    *dt = cfl * best;
    return 0;
}

/* One SSP-RK3 step in Shu-Osher form, in place:
 *   u1 = u + dt L(u)
 *   u2 = 3/4 u + 1/4 (u1 + dt L(u1))
 *   u  = 1/3 u + 2/3 (u2 + dt L(u2)) */
void orc_rk3_step(const orc_ctx *c, double *C, double dt)
{
    size_t len = (size_t)c->n * M * c->np;
    double *L = (double *)malloc(sizeof(double) * len);
    double *u1 = (double *)malloc(sizeof(double) * len);
    double *u2 = (double *)malloc(sizeof(double) * len);
    orc_rhs(c, C, L);
    for (size_t x = 0; x < len; ++x) u1[x] = C[x] + dt * L[x];
    orc_rhs(c, u1, L);
    for (size_t x = 0; x < len; ++x) u2[x] = 0.75 * C[x] + 0.25 * (u1[x] + dt * L[x]);
    orc_rhs(c, u2, L);
    for (size_t x = 0; x < len; ++x) C[x] = (1.0 / 3.0) * C[x] + (2.0 / 3.0) * (u2[x] + dt * L[x]);
    free(L);
    free(u1);
    free(u2);
}

/* ------------------------------------------------------------- limiter */
/* Barth-Jespersen slope limiter for p = 1 (Section "Limiting Kernel", eqs.
 * (limit), (limitmax), (limitmin)), each conserved variable separately:
 *   - centroid values: U_i at its own centroid (1/3, 1/3) and each
 *     neighbour's U at its own centroid, all from the input state (a side
 *     on the domain boundary contributes no neighbour);
 *   - Umax, Umin: the largest and smallest of the four;
 *   - at every Gauss point r_qk of the element's three sides, with
 *     d = U_i(r_qk) - U_i(centroid): alpha_k = min(1, (Umax - U_i(centroid)) / d)
 *     if d > 0, min(1, (Umin - U_i(centroid)) / d) if d < 0, and 1 if d = 0;
 *   - alpha = the smallest alpha_k multiplies the two linear coefficients
 *     (modes 1 and 2); mode 0 is left as it is.
 * Returns -1 (state untouched) unless p = 1. */
int orc_limit_bj(const orc_ctx *c, double *C)
{
    if (c->p != 1) return -1;
    const int np = c->np;
    double phic[NP_MAX];
    orc_basis(c->p, 1.0 / 3.0, 1.0 / 3.0, phic, NULL, NULL);
    double *cen = (double *)malloc(sizeof(double) * c->n * M);
    for (int64_t i = 0; i < c->n; ++i)
        for (int m = 0; m < M; ++m) {
            double u = 0.0;
            for (int j = 0; j < np; ++j) u += phic[j] * C[(i * M + m) * np + j];
            cen[i * M + m] = u;
        }
    double *alpha = (double *)malloc(sizeof(double) * c->n * M);
    for (int64_t i = 0; i < c->n; ++i)
        for (int m = 0; m < M; ++m) {
            const double ub = cen[i * M + m];
            double umax = ub, umin = ub;
            for (int q = 0; q < 3; ++q) {
                if (c->nbr[i * 3 + q] < 0) continue; /* a domain boundary: no neighbour */
                const double un = cen[c->nbr[i * 3 + q] * M + m];
                if (un > umax) umax = un;
                if (un < umin) umin = un;
            }
            double a = 1.0;
            for (int q = 0; q < 3; ++q)
                for (int k = 0; k < c->ne; ++k) {
                    double u = 0.0;
                    for (int j = 0; j < np; ++j) u += c->phi_s[(q * c->ne + k) * np + j] * C[(i * M + m) * np + j];
                    const double d = u - ub;
                    double ak = 1.0;
                    if (d > 0.0)
                        ak = (umax - ub) / d;
                    else if (d < 0.0)
                        ak = (umin - ub) / d;
                    if (ak > 1.0) ak = 1.0;
                    if (ak < a) a = ak;
                }
            alpha[i * M + m] = a;
        }
    for (int64_t i = 0; i < c->n; ++i)
        for (int m = 0; m < M; ++m)
            for (int j = 1; j < np; ++j) C[(i * M + m) * np + j] *= alpha[i * M + m];
    free(cen);
    free(alpha);
    return 0;
}

/* orc_rk3_step with the limiter applied to each stage's result and to the
 * new state (Section "Time-stepping": intermediate stages and the next time
 * level are both limited). */
int orc_rk3_step_limited(const orc_ctx *c, double *C, double dt)
{
    if (c->p != 1) return -1;
    size_t len = (size_t)c->n * M * c->np;
    double *L = (double *)malloc(sizeof(double) * len);
    double *u1 = (double *)malloc(sizeof(double) * len);
    double *u2 = (double *)malloc(sizeof(double) * len);
    orc_rhs(c, C, L);
    for (size_t x = 0; x < len; ++x) u1[x] = C[x] + dt * L[x];
    orc_limit_bj(c, u1);
    orc_rhs(c, u1, L);
    for (size_t x = 0; x < len; ++x) u2[x] = 0.75 * C[x] + 0.25 * (u1[x] + dt * L[x]);
    orc_limit_bj(c, u2);
    orc_rhs(c, u2, L);
    for (size_t x = 0; x < len; ++x) C[x] = (1.0 / 3.0) * C[x] + (2.0 / 3.0) * (u2[x] + dt * L[x]);
    orc_limit_bj(c, C);
    free(L);
    free(u1);
    free(u2);
    return 0;
}

/* The paper's classic explicit Runge-Kutta integrators (Section
 * "Time-stepping"), one step in place, optionally limited like
 * orc_rk3_step_limited (each stage's solution and the new state):
 *   scheme 1, second order (Heun):  u1 = u + dt L(u);
 *                                   u  = u/2 + (u1 + dt L(u1))/2
 *   scheme 2, fourth order:  k1 = L(u), k2 = L(u + dt/2 k1),
 *                            k3 = L(u + dt/2 k2), k4 = L(u + dt k3),
 *                            u  = u + dt (k1 + 2 k2 + 2 k3 + k4) / 6
 * Returns -1 for an unknown scheme or a limiter request at p != 1. */
int orc_rk_step(const orc_ctx *c, double *C, double dt, int scheme, int limit)
{
    if (scheme != 1 && scheme != 2) return -1;
    if (limit && c->p != 1) return -1;
    size_t len = (size_t)c->n * M * c->np;
    double *L = (double *)malloc(sizeof(double) * len);
    double *U = (double *)malloc(sizeof(double) * len);
    if (scheme == 1) {
        orc_rhs(c, C, L);
        for (size_t x = 0; x < len; ++x) U[x] = C[x] + dt * L[x];
        if (limit) orc_limit_bj(c, U);
        orc_rhs(c, U, L);
        for (size_t x = 0; x < len; ++x) C[x] = 0.5 * C[x] + 0.5 * (U[x] + dt * L[x]);
    } else {
        double *K = (double *)malloc(sizeof(double) * len); /* k1 + 2 k2 + 2 k3 so far */
        orc_rhs(c, C, L);
        for (size_t x = 0; x < len; ++x) {
            K[x] = L[x];
            U[x] = C[x] + 0.5 * dt * L[x];
        }
        if (limit) orc_limit_bj(c, U);
        orc_rhs(c, U, L);
        for (size_t x = 0; x < len; ++x) {
            K[x] += 2.0 * L[x];
            U[x] = C[x] + 0.5 * dt * L[x];
        }
        if (limit) orc_limit_bj(c, U);
        orc_rhs(c, U, L);
        for (size_t x = 0; x < len; ++x) {
            K[x] += 2.0 * L[x];
            U[x] = C[x] + dt * L[x];
        }
        if (limit) orc_limit_bj(c, U);
        orc_rhs(c, U, L);
        for (size_t x = 0; x < len; ++x) C[x] = C[x] + dt * (K[x] + L[x]) / 6.0;
        free(K);
    }
    if (limit) orc_limit_bj(c, C);
    free(L);
    free(U);
    return 0;
}

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------- adjoint */
/* Hand-written discrete adjoint (vector-Jacobian product) of orc_rhs:
 * Cbar = (dR/dC)^T Rbar.  Reverse mode through each element's arithmetic in
 * the order of rhs_element: the surface flux of side q contributes to this
 * element (left state) and to its neighbour (right state), the volume term
 * to this element only.  The scatter into the neighbour makes the loop
 * serial.  Ties of the wave-speed max take the left branch; d|x|/dx at 0 is
 * +1. */

/* reverse of euler_flux: (Fx_bar, Fy_bar) -> U_bar (accumulated) */
static void euler_flux_vjp(double gamma, const double U[M], const double Fxb[M], const double Fyb[M], double Ub[M])
{
    const double g1 = gamma - 1.0;
    double rho = U[0], u = U[1] / rho, v = U[2] / rho, E = U[3];
    double pr = g1 * (E - 0.5 * rho * (u * u + v * v));
    /* Fx = (rho u, rho u u + p, rho u v, u (E + p)), Fy = (rho v, rho u v, rho v v + p, v (E + p)) */
    double rhob = Fxb[0] * u + Fxb[1] * u * u + Fxb[2] * u * v + Fyb[0] * v + Fyb[1] * u * v + Fyb[2] * v * v;
    double ub = Fxb[0] * rho + Fxb[1] * 2.0 * rho * u + Fxb[2] * rho * v + Fxb[3] * (E + pr) + Fyb[1] * rho * v;
    double vb = Fxb[2] * rho * u + Fyb[0] * rho + Fyb[1] * rho * u + Fyb[2] * 2.0 * rho * v + Fyb[3] * (E + pr);
    double pb = Fxb[1] + Fxb[3] * u + Fyb[2] + Fyb[3] * v;
    double Eb = Fxb[3] * u + Fyb[3] * v;
    /* p = g1 (E - rho (u^2 + v^2) / 2) */
    Eb += g1 * pb;
    rhob += -0.5 * g1 * (u * u + v * v) * pb;
    ub += -g1 * rho * u * pb;
    vb += -g1 * rho * v * pb;
    /* u = U1 / rho, v = U2 / rho */
    Ub[1] += ub / rho;
    Ub[2] += vb / rho;
    rhob += -(ub * u + vb * v) / rho;
    Ub[0] += rhob;
    Ub[3] += Eb;
}

/* reverse of llf: Fn_bar -> (UL_bar, UR_bar) (accumulated) */
static void llf_vjp(double gamma, const double UL[M], const double UR[M], double nx, double ny, const double Fb[M],
                    double ULb[M], double URb[M])
{
    const double g1 = gamma - 1.0;
    const double *Us[2] = {UL, UR};
    double *Ubs[2] = {ULb, URb};
    double lam_s[2], vn_s[2], c_s[2], u_s[2], v_s[2], p_s[2];
    for (int side = 0; side < 2; ++side) {
        const double *U = Us[side];
        double u = U[1] / U[0], v = U[2] / U[0];
        double p = g1 * (U[3] - 0.5 * U[0] * (u * u + v * v));
        u_s[side] = u;
        v_s[side] = v;
        p_s[side] = p;
        vn_s[side] = u * nx + v * ny;
        c_s[side] = sqrt(gamma * p / U[0]);
        lam_s[side] = fabs(vn_s[side]) + c_s[side];
    }
    int left_max = lam_s[0] >= lam_s[1];
    double lam = left_max ? lam_s[0] : lam_s[1];
    double lamb = 0.0;
    for (int m = 0; m < M; ++m) {
        /* Fn = 0.5 (fL + fR) - 0.5 lam (UR - UL) */
        lamb += -0.5 * Fb[m] * (UR[m] - UL[m]);
        URb[m] += -0.5 * lam * Fb[m];
        ULb[m] += 0.5 * lam * Fb[m];
    }
    for (int side = 0; side < 2; ++side) {
        const double *U = Us[side];
        double *Ub = Ubs[side];
        /* f = Fx nx + Fy ny with weight 0.5 from the average */
        double Fxb[M], Fyb[M];
        for (int m = 0; m < M; ++m) {
            Fxb[m] = 0.5 * Fb[m] * nx;
            Fyb[m] = 0.5 * Fb[m] * ny;
        }
        euler_flux_vjp(gamma, U, Fxb, Fyb, Ub);
        /* lam_side = |vn| + c, c = sqrt(gamma p / rho) */
        double lsb = (side == 0) == (left_max != 0) ? lamb : 0.0;
        if (lsb == 0.0) continue;
        double vnb = lsb * (vn_s[side] >= 0.0 ? 1.0 : -1.0);
        double cb = lsb;
        double rho = U[0], u = u_s[side], v = v_s[side], p = p_s[side], c = c_s[side];
        double pb = cb * gamma / (2.0 * c * rho);
        double rhob = -cb * gamma * p / (2.0 * c * rho * rho);
        double ub = vnb * nx, vb = vnb * ny;
        /* p = g1 (E - rho (u^2 + v^2) / 2) */
        Ub[3] += g1 * pb;
        rhob += -0.5 * g1 * (u * u + v * v) * pb;
        ub += -g1 * rho * u * pb;
        vb += -g1 * rho * v * pb;
        Ub[1] += ub / rho;
        Ub[2] += vb / rho;
        rhob += -(ub * u + vb * v) / rho;
        Ub[0] += rhob;
    }
}

/* reverse of the ghost state: U_L_bar += (dU_g/dU_L)^T U_g_bar.  The wall's
 * Jacobian is the reflection diag(1, I - 2 n n^T, 1), its own transpose; the
 * outflow ghost is the identity; the prescribed state does not depend on U_L.
 * (At a wall or outflow side the two wave speeds of the flux are the same
 * function of U_L, so whichever branch of the maximum rounding selects, the
 * derivative is the same.) */
static void ghost_vjp(int64_t code, double nx, double ny, const double URb[M], double ULb[M])
{
    if (code == -1) {
        double mnb = URb[1] * nx + URb[2] * ny;
        ULb[0] += URb[0];
        ULb[1] += URb[1] - 2.0 * mnb * nx;
        ULb[2] += URb[2] - 2.0 * mnb * ny;
        ULb[3] += URb[3];
    } else if (code == -2) {
        for (int m = 0; m < M; ++m) ULb[m] += URb[m];
    }
}

void orc_rhs_vjp(const orc_ctx *c, const double *C, const double *Rb, double *Cb)
{
    const int np = c->np, nq = c->nq, ne = c->ne;
    memset(Cb, 0, sizeof(double) * (size_t)c->n * M * np);
    for (int64_t i = 0; i < c->n; ++i) {
        double adj[2][2], det;
        element_geometry(c, i, adj, &det);
        const double *ci = C + i * M * np;
        double *cbi = Cb + i * M * np;
        double Rs[M][NP_MAX]; /* Rbar / det J: cotangent of (volume - surface) */
        for (int m = 0; m < M; ++m)
            for (int j = 0; j < np; ++j) Rs[m][j] = Rb[(i * M + m) * np + j] / det;

        /* volume: vol[m][j] += w_k (dr_jk Gr_m + ds_jk Gs_m) */
        for (int k = 0; k < nq; ++k) {
            double U[M], Fxb[M], Fyb[M], Ub[M] = {0.0, 0.0, 0.0, 0.0};
            for (int m = 0; m < M; ++m) {
                U[m] = 0.0;
                for (int j = 0; j < np; ++j) U[m] += ci[m * np + j] * c->phi_v[k * np + j];
            }
            for (int m = 0; m < M; ++m) {
                double Grb = 0.0, Gsb = 0.0;
                for (int j = 0; j < np; ++j) {
                    Grb += c->qw[k] * c->dr_v[k * np + j] * Rs[m][j];
                    Gsb += c->qw[k] * c->ds_v[k * np + j] * Rs[m][j];
                }
                /* Gr = a00 Fx + a01 Fy, Gs = a10 Fx + a11 Fy */
                Fxb[m] = adj[0][0] * Grb + adj[1][0] * Gsb;
                Fyb[m] = adj[0][1] * Grb + adj[1][1] * Gsb;
            }
            euler_flux_vjp(c->gamma, U, Fxb, Fyb, Ub);
            for (int m = 0; m < M; ++m)
                for (int j = 0; j < np; ++j) cbi[m * np + j] += c->phi_v[k * np + j] * Ub[m];
        }

        /* surface: sur[m][j] += l w_k phi_j(r_qk) Fn_m; R has -sur.  On a
         * domain boundary U_R is the ghost state of U_L, and its cotangent
         * goes back to U_L through the ghost's Jacobian (ghost_vjp). */
        for (int q = 0; q < 3; ++q) {
            int64_t nb = c->nbr[i * 3 + q];
            const int boundary = nb < 0;
            int qn = boundary ? 0 : c->nbs[i * 3 + q];
            const double *cn = C + (boundary ? i : nb) * M * np;
            double *cbn = Cb + (boundary ? i : nb) * M * np;
            double nx, ny, l;
            side_geometry(c, i, q, &nx, &ny, &l);
            for (int k = 0; k < ne; ++k) {
                const double *phiL = c->phi_s + (q * ne + k) * np;
                const double *phiR = c->phi_s + (qn * ne + (ne - 1 - k)) * np;
                double UL[M], UR[M], Fb[M], ULb[M] = {0.0, 0.0, 0.0, 0.0}, URb[M] = {0.0, 0.0, 0.0, 0.0};
                for (int m = 0; m < M; ++m) {
                    UL[m] = 0.0;
                    UR[m] = 0.0;
                    for (int j = 0; j < np; ++j) {
                        UL[m] += ci[m * np + j] * phiL[j];
                        UR[m] += cn[m * np + j] * phiR[j];
                    }
                    Fb[m] = 0.0;
                    for (int j = 0; j < np; ++j) Fb[m] += -l * c->gw[k] * phiL[j] * Rs[m][j];
                }
                if (boundary) {
                    orc_ghost(c, nb, UL, nx, ny, UR);
                    llf_vjp(c->gamma, UL, UR, nx, ny, Fb, ULb, URb);
                    ghost_vjp(nb, nx, ny, URb, ULb);
                    for (int m = 0; m < M; ++m)
                        for (int j = 0; j < np; ++j) cbi[m * np + j] += phiL[j] * ULb[m];
                    continue;
                }
                llf_vjp(c->gamma, UL, UR, nx, ny, Fb, ULb, URb);
                for (int m = 0; m < M; ++m)
                    for (int j = 0; j < np; ++j) {
                        cbi[m * np + j] += phiL[j] * ULb[m];
                        cbn[m * np + j] += phiR[j] * URb[m];
                    }
            }
        }
    }
}

/* Adjoint of one SSP-RK3 step with a fixed dt (dt is not differentiated):
 * given ubar of the result, Cb = d(step)/dC ^T ubar.  Recomputes the stages:
 *   u2bar = 2/3 ubar + 2/3 dt J(u2)^T ubar
 *   u1bar = 1/4 u2bar + 1/4 dt J(u1)^T u2bar
 *   Cb    = 1/3 ubar + 3/4 u2bar + u1bar + dt J(u)^T u1bar */
void orc_rk3_step_vjp(const orc_ctx *c, const double *C, double dt, const double *ub, double *Cb)
{
    size_t len = (size_t)c->n * M * c->np;
    double *L = (double *)malloc(sizeof(double) * len);
    double *u1 = (double *)malloc(sizeof(double) * len);
    double *u2 = (double *)malloc(sizeof(double) * len);
    double *t = (double *)malloc(sizeof(double) * len);
    double *u2b = (double *)malloc(sizeof(double) * len);
    double *u1b = (double *)malloc(sizeof(double) * len);
    orc_rhs(c, C, L);
    for (size_t x = 0; x < len; ++x) u1[x] = C[x] + dt * L[x];
    orc_rhs(c, u1, L);
    for (size_t x = 0; x < len; ++x) u2[x] = 0.75 * C[x] + 0.25 * (u1[x] + dt * L[x]);
    orc_rhs_vjp(c, u2, ub, t);
    for (size_t x = 0; x < len; ++x) u2b[x] = (2.0 / 3.0) * ub[x] + (2.0 / 3.0) * dt * t[x];
    orc_rhs_vjp(c, u1, u2b, t);
    for (size_t x = 0; x < len; ++x) u1b[x] = 0.25 * u2b[x] + 0.25 * dt * t[x];
    orc_rhs_vjp(c, C, u1b, t);
    for (size_t x = 0; x < len; ++x) Cb[x] = (1.0 / 3.0) * ub[x] + 0.75 * u2b[x] + u1b[x] + dt * t[x];
    free(L);
    free(u1);
    free(u2);
    free(t);
    free(u2b);
    free(u1b);
}
