// HIP kernels (gfx950) of the modal DG right-hand side for the 2D Euler
// equations, eq. (2ddg0) with the flux of eq. (euler).
//
// Data layout.  Modal coefficients are element-blocked structure of arrays:
// C[blk][m][j][lane] with LANES = 16 elements per block, so that one (m, j)
// row of a block is one 128-byte line: a one-lane wavefront reading mode j of
// variable m touches four whole lines, and a neighbour gather touches one
// line per row it needs.  Edge traces and per-side surface fluxes use the
// same blocking: T[blk][q][k][m][lane] (side q of the element, edge point k).
//
// Kernels (one work-item per element or per edge, wave64):
//   k_traces   U at the p+1 Gauss points of the three sides of each element
//              (the side loop is uniform across the wavefront, so the basis
//              tables are read through scalar loads);
//   k_edge     per edge: gathers the two traces (the right element's at the
//              reversed point, Section "Surface Integration Kernel"),
//              evaluates the local Lax-Friedrichs flux once and stores it,
//              scaled by l*omega_k, into one slot per element side (one
//              writer per slot, no atomics: the paper's left/right
//              temporaries, kept per side);
//   k_element  per element: volume integral eq. (volume) at the degree-2p
//              points, lift of its three side slots, multiplication by the
//              inverse mass matrix 1/det J (orthonormal basis), and either a
//              plain RHS store or a fused SSP-RK3 stage update; for RK
//              stages it also writes the traces of the updated state so the
//              next stage needs no trace pass;
//   k_dt_*     deterministic two-pass min reduction of the CFL step.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dg_internal.h"

// 1: the mixed-precision four-lane kernels do their contractions with
// MFMA; 0: on the vector ALUs like the FP64 kernels
#ifndef DG_MIXED_MFMA
#define DG_MIXED_MFMA 1
#endif

namespace dgk {

template <int P>
struct Ord {
    static constexpr int NP = (P + 1) * (P + 2) / 2;
    static constexpr int NQ = P == 1 ? 3 : P == 2 ? 6 : P == 3 ? 12 : P == 4 ? 16 : 25;
    static constexpr int NE = P + 1;
    // table offsets, identical to the host layout (checked at mesh creation)
    static constexpr int PHI = 0;
    static constexpr int DRW = PHI + NQ * NP;
    static constexpr int DSW = DRW + NQ * NP;
    static constexpr int PHS = DSW + NQ * NP;
    static constexpr int GW = PHS + 3 * NE * NP;
    static constexpr int QW = GW + NE;
    static constexpr int QR = QW + NQ;
    static constexpr int QS = QR + NQ;
};

constexpr int BLOCK = 256;

__device__ __forceinline__ int state_off(int e, int nfield) { return (e / LANES) * nfield * LANES + (e % LANES); }

// Reciprocal and square root for the flux arithmetic: the hardware
// approximations (v_rcp, v_rsq) refined by one Newton step, a few
// instructions instead of the correctly rounded division / square-root
// sequences (results within a few units in the last place; the two sides of
// an edge call the same functions, so the flux stays exactly antisymmetric).
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double root(double y)
{
    const double r = __builtin_amdgcn_rsq(y);  // ~ 1/sqrt(y)
    const double s = y * r;
    const double h = 0.5 * r;
    const double d = fma(-s, s, y);
    const double s1 = fma(h, d, s);
    return fma(h, fma(-s1, s1, y), s1);
}
__device__ __forceinline__ float root(float y)
{
    const float r = __builtin_amdgcn_rsqf(y);
    const float s = y * r;
    return fmaf(0.5f * r, fmaf(-s, s, y), s);
}

// ---------------------------------------------------------------- physics
// Euler flux eq. (euler) at one point; p = (gamma-1)(E - rho |v|^2 / 2).
// T is the arithmetic type (double, or float in the mixed-precision form).
template <typename T>
__device__ __forceinline__ void euler_flux(T gm1, const T U[4], T Fx[4], T Fy[4])
{
    const T ri = recip(U[0]);
    const T u = U[1] * ri, v = U[2] * ri;
    const T p = gm1 * (U[3] - T(0.5) * (U[1] * u + U[2] * v));
    Fx[0] = U[1];
    Fx[1] = U[1] * u + p;
    Fx[2] = U[2] * u;
    Fx[3] = u * (U[3] + p);
    Fy[0] = U[2];
    Fy[1] = U[1] * v;
    Fy[2] = U[2] * v + p;
    Fy[3] = v * (U[3] + p);
}

// Local Lax-Friedrichs flux across unit normal n (from L to R):
// Fn = (F(UL).n + F(UR).n)/2 - lambda/2 (UR - UL),
// lambda = max(|vL.n| + cL, |vR.n| + cR).  Exchanging L and R and negating n
// negates Fn bitwise, which keeps the scheme exactly conservative: every
// quantity that depends on n is an odd function of it in floating point too
// (products with n, and fused multiply-adds whose addend is itself odd in n),
// and the two sides enter the final combination through a sum and a
// difference, which are exactly symmetric.  Contraction is therefore spelled
// out with fma() and the compiler's own fusing is off here: a product fused
// into the sum F(UL).n + F(UR).n from one side but not the other would break
// that symmetry at the level of the rounding unit.
template <typename T>
__device__ __forceinline__ void llf(T gamma, T gm1, const T UL[4], const T UR[4], T nx, T ny, T Fn[4])
{
#pragma clang fp contract(off)
    const T riL = recip(UL[0]), riR = recip(UR[0]);
    const T uL = UL[1] * riL, vL = UL[2] * riL, uR = UR[1] * riR, vR = UR[2] * riR;
    const T pL = gm1 * fma(T(-0.5), fma(UL[1], uL, UL[2] * vL), UL[3]);
    const T pR = gm1 * fma(T(-0.5), fma(UR[1], uR, UR[2] * vR), UR[3]);
    const T vnL = fma(uL, nx, vL * ny), vnR = fma(uR, nx, vR * ny);
    const T lam = fmax(fabs(vnL) + root((gamma * riL) * pL), fabs(vnR) + root((gamma * riR) * pR));
    const T fL[4] = {UL[0] * vnL, fma(pL, nx, UL[1] * vnL), fma(pL, ny, UL[2] * vnL), (UL[3] + pL) * vnL};
    const T fR[4] = {UR[0] * vnR, fma(pR, nx, UR[1] * vnR), fma(pR, ny, UR[2] * vnR), (UR[3] + pR) * vnR};
#pragma unroll
    for (int m = 0; m < 4; ++m) Fn[m] = T(0.5) * fma(-lam, UR[m] - UL[m], fL[m] + fR[m]);
}

// Ghost state across a domain boundary (Section "Surface Integration
// Kernel": the right-hand state of a boundary edge is a ghost state set by
// the kind of boundary), at the same point as UL, n the outward unit normal.
// bc: 0 interior side (UR kept), 1 solid wall (density and energy kept,
// momentum mirrored about the wall), 2 outflow (the interior state), 3 the
// prescribed state G.  Written as selects, without branches: the kind varies
// between the elements of a wavefront, and the stage kernels keep no
// divergent control flow around their (heavily register-allocated) surface
// loops.
template <typename T>
__device__ __forceinline__ void ghost_state(int bc, const T (&UL)[4], T nx, T ny, const T (&G)[4], T (&UR)[4])
{
    const bool keep = bc == 0, fixed = bc == 3;
    const T s = bc == 1 ? T(2) * (UL[1] * nx + UL[2] * ny) : T(0);
    UR[0] = keep ? UR[0] : (fixed ? G[0] : UL[0]);
    UR[1] = keep ? UR[1] : (fixed ? G[1] : UL[1] - s * nx);
    UR[2] = keep ? UR[2] : (fixed ? G[2] : UL[2] - s * ny);
    UR[3] = keep ? UR[3] : (fixed ? G[3] : UL[3]);
}

// ---------------------------------------------------------------- traces
template <int P>
__device__ __forceinline__ void store_traces(const double (&c)[4][Ord<P>::NP], const double* __restrict__ tab,
                                             double* __restrict__ t0)
{
    using O = Ord<P>;
#pragma unroll
    for (int qk = 0; qk < 3 * O::NE; ++qk) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            double u = 0.0;
#pragma unroll
            for (int j = 0; j < O::NP; ++j) u = fma(tab[O::PHS + qk * O::NP + j], c[m][j], u);
            t0[(qk * 4 + m) * LANES] = u;
        }
    }
}

template <int P>
__global__ __launch_bounds__(BLOCK) void k_traces(int n, const double* __restrict__ C, double* __restrict__ T,
                                                  const double* __restrict__ tab, double* __restrict__ Rz)
{
    using O = Ord<P>;
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= n) return;
    if (Rz) {
#pragma unroll
        for (int x = 0; x < 4 * O::NP; ++x) Rz[state_off(e, 4 * O::NP) + x * LANES] = 0.0;
    }
    const double* c0 = C + state_off(e, 4 * O::NP);
    double c[4][O::NP];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < O::NP; ++j) c[m][j] = c0[(m * O::NP + j) * LANES];
    store_traces<P>(c, tab, T + state_off(e, 3 * O::NE * 4));
}

// ---------------------------------------------------------------- edges
// A boundary edge (right element = the negative boundary code; these edges
// come first in the list, grouped by kind) takes the ghost state of its
// left trace at the same point as the right state and writes the left slot
// only.
template <int P>
__global__ __launch_bounds__(BLOCK) void k_edge(int nedge, const int* __restrict__ el, const int* __restrict__ er,
                                                const int* __restrict__ sd, const double* __restrict__ eg,
                                                const double* __restrict__ T, double* __restrict__ S,
                                                const double* __restrict__ tab, double gamma,
                                                const double* __restrict__ bcs)
{
    using O = Ord<P>;
    constexpr int NE = O::NE;
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= nedge) return;
    const int l = el[i], r = er[i], sides = sd[i];
    const int ql = sides & 3, qr = (sides >> 2) & 3;
    const double nx = eg[i], ny = eg[nedge + i], hl = eg[2 * nedge + i];
    const int offl = state_off(l, 3 * NE * 4) + ql * NE * 4 * LANES;
    const double gm1 = gamma - 1.0;
    if (r < 0) {
        const double G[4] = {bcs[0], bcs[1], bcs[2], bcs[3]};
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            double UL[4], UR[4], F[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) UR[m] = UL[m] = T[offl + (k * 4 + m) * LANES];
            ghost_state<double>(-r, UL, nx, ny, G, UR);
            llf<double>(gamma, gm1, UL, UR, nx, ny, F);
            const double w = hl * tab[O::GW + k];
#pragma unroll
            for (int m = 0; m < 4; ++m) S[offl + (k * 4 + m) * LANES] = -w * F[m];
        }
        return;
    }
    const int offr = state_off(r, 3 * NE * 4) + qr * NE * 4 * LANES;
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        const int kr = NE - 1 - k;
        double UL[4], UR[4], F[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            UL[m] = T[offl + (k * 4 + m) * LANES];
            UR[m] = T[offr + (kr * 4 + m) * LANES];
        }
        llf<double>(gamma, gm1, UL, UR, nx, ny, F);
        const double w = hl * tab[O::GW + k];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            S[offl + (k * 4 + m) * LANES] = -w * F[m];
            S[offr + (kr * 4 + m) * LANES] = w * F[m];
        }
    }
}

// Edge colouring (the paper's suggested alternative to per-side
// temporaries): the edges of one colour share no element, so one launch per
// colour lets every edge evaluate its flux once and add its lift straight
// into both elements' accumulators R[blk][m][j][lane] (before 1/det J),
// without atomics and without a slot buffer.  The side tables sit in LDS
// (the side differs per edge).
template <int P>
__global__ __launch_bounds__(BLOCK) void k_edge_lift(int e0, int e1, int nedge, const int* __restrict__ el,
                                                     const int* __restrict__ er, const int* __restrict__ sd,
                                                     const double* __restrict__ eg, const double* __restrict__ T,
                                                     double* __restrict__ R, const double* __restrict__ tab,
                                                     double gamma, const double* __restrict__ bcs)
{
    using O = Ord<P>;
    constexpr int NE = O::NE, NP = O::NP;
    __shared__ double phs[3 * NE * NP];
    for (int x = threadIdx.x; x < 3 * NE * NP; x += BLOCK) phs[x] = tab[O::PHS + x];
    __syncthreads();
    const int i = e0 + blockIdx.x * BLOCK + threadIdx.x;
    if (i >= e1) return;
    const int l = el[i], r = er[i], sides = sd[i];
    const int ql = sides & 3, qr = (sides >> 2) & 3;
    const double nx = eg[i], ny = eg[nedge + i], hl = eg[2 * nedge + i];
    const int offl = state_off(l, 3 * NE * 4) + ql * NE * 4 * LANES;
    const int offr = r >= 0 ? state_off(r, 3 * NE * 4) + qr * NE * 4 * LANES : 0;
    const double gm1 = gamma - 1.0;
    const double G[4] = {bcs[0], bcs[1], bcs[2], bcs[3]};
    double WF[NE][4];  // l * omega_k * Fn at the left element's points
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        double UL[4], UR[4], F[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) UR[m] = UL[m] = T[offl + (k * 4 + m) * LANES];
        if (r >= 0) {
#pragma unroll
            for (int m = 0; m < 4; ++m) UR[m] = T[offr + ((NE - 1 - k) * 4 + m) * LANES];
        } else {
            ghost_state<double>(-r, UL, nx, ny, G, UR);
        }
        llf<double>(gamma, gm1, UL, UR, nx, ny, F);
        const double w = hl * tab[O::GW + k];
#pragma unroll
        for (int m = 0; m < 4; ++m) WF[k][m] = w * F[m];
    }
    const double* tl = phs + ql * NE * NP;
    const double* tr = phs + qr * NE * NP;
    const int sl = state_off(l, 4 * NP), sr = r >= 0 ? state_off(r, 4 * NP) : 0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            double a = 0.0;
#pragma unroll
            for (int k = 0; k < NE; ++k) a = fma(tl[k * NP + j], WF[k][m], a);
            R[sl + (m * NP + j) * LANES] -= a;
        }
    if (r < 0) return;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            double a = 0.0;
#pragma unroll
            for (int k = 0; k < NE; ++k) a = fma(tr[(NE - 1 - k) * NP + j], WF[k][m], a);
            R[sr + (m * NP + j) * LANES] += a;
        }
}

// ---------------------------------------------------------------- elements
// The grid covers the padded element count: padding lanes write zeros, so
// every state this kernel produces has a defined (zero) padding.
// Volume integral eq. (volume) of one element, added to acc:
// sum_k w_k grad phi_j(r_k) . (adj(J) F(U(r_k))); the point loop stays
// rolled so only one point's table rows are live.
template <int P>
__device__ __forceinline__ void volume_integral(const double (&c)[4][Ord<P>::NP], double a00, double a01, double a10,
                                                double a11, double gm1, const double* __restrict__ tab,
                                                double (&acc)[4][Ord<P>::NP])
{
    using O = Ord<P>;
    constexpr int NP = O::NP, NQ = O::NQ;
#pragma unroll 1
    for (int k = 0; k < NQ; ++k) {
        double U[4], Fx[4], Fy[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            double u = 0.0;
#pragma unroll
            for (int j = 0; j < NP; ++j) u = fma(tab[O::PHI + k * NP + j], c[m][j], u);
            U[m] = u;
        }
        euler_flux<double>(gm1, U, Fx, Fy);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const double gr = a00 * Fx[m] + a01 * Fy[m];
            const double gs = a10 * Fx[m] + a11 * Fy[m];
#pragma unroll
            for (int j = 0; j < NP; ++j)
                acc[m][j] = fma(tab[O::DRW + k * NP + j], gr, fma(tab[O::DSW + k * NP + j], gs, acc[m][j]));
        }
    }
}

// The volume integral alone, into V (edge-wise path with the volume and
// surface work on two streams: run beside k_traces / k_edge).
template <int P>
__global__ __launch_bounds__(BLOCK) void k_volume(int n, const double* __restrict__ C, double* __restrict__ V,
                                                  const double* __restrict__ geo, const double* __restrict__ tab,
                                                  double gm1)
{
    using O = Ord<P>;
    constexpr int NP = O::NP;
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= n) return;
    const int so = state_off(e, 4 * NP);
    const double* g = geo + state_off(e, 6);
    double c[4][NP], acc[4][NP];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            c[m][j] = C[so + (m * NP + j) * LANES];
            acc[m][j] = 0.0;
        }
    volume_integral<P>(c, g[0], g[LANES], g[2 * LANES], g[3 * LANES], gm1, tab, acc);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NP; ++j) V[so + (m * NP + j) * LANES] = acc[m][j];
}

// SRC, where the accumulators start and what the kernel adds:
//   SRC_SLOTS  zero + volume integral + the side slots S (edge-wise);
//   SRC_RACC   the surface integral in Racc (coloured edges) + volume
//              integral; Racc is zeroed again when the next stage's traces
//              are written;
//   SRC_VOLUME the volume integral in Racc (k_volume on a second stream) +
//              the side slots S.
enum { SRC_SLOTS = 0, SRC_RACC = 1, SRC_VOLUME = 2 };
template <int P, int MODE, bool TRACE, int SRC>
__global__ __launch_bounds__(BLOCK) void k_element(int n, int npad, const double* __restrict__ C, const double* U0,
                                                   double* out, const double* __restrict__ S,
                                                   const double* __restrict__ geo, const double* __restrict__ tab,
                                                   double gm1, double dt, const double* __restrict__ dt_dev,
                                                   double* __restrict__ Tn, double* __restrict__ Racc)
{
    using O = Ord<P>;
    constexpr int NP = O::NP, NQ = O::NQ, NE = O::NE;
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= npad) return;
    const int so = state_off(e, 4 * NP);
    if (e >= n) {
#pragma unroll
        for (int x = 0; x < 4 * NP; ++x) out[so + x * LANES] = 0.0;
        return;
    }
    const double* g = geo + state_off(e, 6);
    const double a00 = g[0], a01 = g[LANES], a10 = g[2 * LANES], a11 = g[3 * LANES], idet = g[4 * LANES];

    double c[4][NP];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NP; ++j) c[m][j] = C[so + (m * NP + j) * LANES];

    double acc[4][NP];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NP; ++j) acc[m][j] = SRC != SRC_SLOTS ? Racc[so + (m * NP + j) * LANES] : 0.0;
    if constexpr (SRC == SRC_RACC && TRACE) {
#pragma unroll
        for (int x = 0; x < 4 * NP; ++x) Racc[so + x * LANES] = 0.0;
    }

    if constexpr (SRC != SRC_VOLUME) volume_integral<P>(c, a00, a01, a10, a11, gm1, tab, acc);

    // surface integral: lift the three side slots (already l * omega_k * Fn)
    const int to = state_off(e, 3 * NE * 4);
#pragma unroll 1
    for (int qk = 0; qk < (SRC == SRC_RACC ? 0 : 3 * NE); ++qk) {
        double sv[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) sv[m] = S[to + (qk * 4 + m) * LANES];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int j = 0; j < NP; ++j) acc[m][j] = fma(tab[O::PHS + qk * NP + j], sv[m], acc[m][j]);
    }

    if constexpr (MODE == 0) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int j = 0; j < NP; ++j) out[so + (m * NP + j) * LANES] = idet * acc[m][j];
    } else {
        const double h = dt_dev ? dt_dev[0] : dt;
        // stage-0 values are all loaded before the first store: in stage 3
        // U0 and out are the same array
        double u0[4][NP];
        if constexpr (MODE != 1) {
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int j = 0; j < NP; ++j) u0[m][j] = U0[so + (m * NP + j) * LANES];
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                const double L = idet * acc[m][j];
                double v;
                if constexpr (MODE == 1) {
                    v = c[m][j] + h * L;
                } else if constexpr (MODE == 2) {
                    v = 0.75 * u0[m][j] + 0.25 * (c[m][j] + h * L);
                } else {
                    v = (1.0 / 3.0) * u0[m][j] + (2.0 / 3.0) * (c[m][j] + h * L);
                }
                c[m][j] = v;
            }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int j = 0; j < NP; ++j) out[so + (m * NP + j) * LANES] = c[m][j];
        if constexpr (TRACE) store_traces<P>(c, tab, Tn + to);
    }
}

// ---------------------------------------------------------------- CFL step per element
// r_in / (|v| + c) at the element mean sqrt(2) c_0; -1 for a non-physical
// (or NaN) mean.  Shared by the reduction kernel and the fused stages, with
// contraction off so that both evaluate it bit for bit the same way.
__device__ __forceinline__ double dt_local(double gamma, double rin, double c0r, double c0x, double c0y, double c0e)
{
#pragma clang fp contract(off)
    const double s2 = 1.4142135623730951;
    const double rho = s2 * c0r, mx = s2 * c0x, my = s2 * c0y, E = s2 * c0e;
    const double u = mx / rho, v = my / rho;
    const double p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v));
    if (rho > 0.0 && p > 0.0) return rin / (sqrt(u * u + v * v) + sqrt(gamma * p / rho));
    return -1.0;
}

// min over a block of 256 values (every thread of the block must call it):
// within each wavefront by butterfly shuffles, then across the four
// wavefronts through LDS.  min is exact and order-independent, so the result
// does not depend on the reduction order.
__device__ __forceinline__ double block_min(double v, double* red)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < BLOCK / WAVE; ++w) r = fmin(r, red[w]);
    __syncthreads();  // red may be reused
    return r;
}

// Step length for the fused multi-step path: cfl * min of the per-block
// minima of the previous stage 3 (or of the reduction kernel), NaN if any
// mean is non-physical.  Every block computes the same value.
__device__ __forceinline__ double dt_from_min(double v, double cfl, double* red)
{
    const double mn = block_min(v, red);
    return mn < 0.0 ? __builtin_nan("") : cfl * mn;
}
__device__ __forceinline__ double dt_from_partials(const double* __restrict__ pin, int count, double cfl, double* red)
{
    double v = INFINITY;
    for (int i = threadIdx.x; i < count; i += BLOCK) v = fmin(v, pin[i]);
    return dt_from_min(v, cfl, red);
}

// ---------------------------------------------------------------- fused stage
// Element-wise surface integration: each work-item evaluates the numerical
// flux of its own three sides (so every edge flux is computed twice, once
// from each side; LLF is written so the two evaluations are exact
// negatives and conservation is kept bitwise), gathering the neighbour's
// trace from the neighbour's coefficients.  One kernel then does the whole
// right-hand side of eq. (2ddg0) and the SSP-RK3 stage update, with no edge
// temporaries in memory.  The neighbour's side differs per lane, so the side
// tables it needs are read from LDS (odd stride between sides: the three
// possible side addresses fall in different banks); tables indexed by the
// element's own side or volume point are uniform and go through scalar loads.

// the stage combination of MODE 4 (StageGen) for one coefficient (x: its
// index)
__device__ __forceinline__ double stage_general(const StageGen& gs, double cs, double h, double L, int x,
                                                const double* out)
{
    const double xv = gs.a == 0.0 ? 0.0 : (gs.X ? gs.X[x] : out[x]);
    if (gs.S) gs.S[x] = (gs.s_init ? cs : gs.S[x]) + (gs.d * h) * L;
    return gs.a * xv + gs.b * cs + (gs.g * h) * L;
}

// Workgroups are dealt round-robin to the 8 XCDs; remap them so that each
// XCD works on one contiguous range of the space-filling-curve order and
// neighbour gathers stay in that XCD's L2.
__device__ __forceinline__ int xcd_block(int bid, int nblk_grid)
{
    const int chunk = nblk_grid >> 3;  // grid is padded to a multiple of 8
    return (bid & 7) * chunk + (bid >> 3);
}

// T = double: everything in FP64.  T = float (mixed precision): the
// contractions, traces, fluxes and the lift of modes j >= 1 in FP32; the
// mean mode (j = 0, whose only contribution is the surface flux: grad phi_0 =
// 0) is accumulated in FP64 from the FP32 fluxes, and 1/det J and the stage
// update are FP64.  The two sides of an edge see bitwise equal traces and
// exactly opposite normals, so the FP32 fluxes cancel exactly and the means
// stay conservative to FP64 rounding.
// MODE 3 updates the stage-0 state in place: U0 is then unused and the
// stage-0 values are read through `out` itself, so every pointer can be
// __restrict__ and the epilogue can stream (different (m, j) are provably
// different addresses of one base).
// BC: the mesh has domain-boundary sides (sbc, bcs read); periodic meshes
// run the variant without them.
template <int P, int MODE, typename T, bool BC>
__global__ __launch_bounds__(BLOCK) void k_stage(int n, int npad, const double* __restrict__ C,
                                                 const double* __restrict__ U0, double* __restrict__ out,
                                                 const double* __restrict__ geo,
                                                 const int* __restrict__ snb, const int* __restrict__ sside,
                                                 const double* __restrict__ sgeo, const T* __restrict__ tab,
                                                 const double* __restrict__ tab64, double gamma, double dt,
                                                 const double* __restrict__ dt_dev, StageGen gs,
                                                 const int* __restrict__ sbc, const double* __restrict__ bcs)
{
    using O = Ord<P>;
    constexpr int NP = O::NP, NQ = O::NQ, NE = O::NE;
    constexpr int SS = (NE * NP) | 1;
    __shared__ T phs[3 * SS];
    __shared__ T urs[2 * NE * 4 * BLOCK];  // neighbours' traces of sides 1 and 2, [side-1][k][m][lane]
    for (int i = threadIdx.x; i < 3 * NE * NP; i += BLOCK) phs[(i / (NE * NP)) * SS + i % (NE * NP)] = tab[O::PHS + i];
    __syncthreads();

    const int e = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    if (e >= npad) return;
    const int so = state_off(e, 4 * NP);
    if (e >= n) {
#pragma unroll
        for (int x = 0; x < 4 * NP; ++x) out[so + x * LANES] = 0.0;
        return;
    }
    const T gam = T(gamma), gm1 = T(gamma - 1.0);
    const double* g = geo + state_off(e, 6);
    const T a00 = T(g[0]), a01 = T(g[LANES]), a10 = T(g[2 * LANES]), a11 = T(g[3 * LANES]);
    const double idet = g[4 * LANES];

    // FP32 compute keeps only the rounded state live; the stage update
    // re-reads the FP64 state at the end
    constexpr bool F64 = sizeof(T) == sizeof(double);
    T c[4][NP];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NP; ++j) c[m][j] = T(C[so + (m * NP + j) * LANES]);

    double acc0[4] = {0.0, 0.0, 0.0, 0.0};  // mean mode, FP64
    T acc[4][NP];                          // acc[m][0] unused
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NP; ++j) acc[m][j] = T(0);

    // surface integral, eq. (surface), over the element's three sides.  The
    // neighbours' traces of all three sides are evaluated first, right after
    // the element's own coefficients are read: the elements of a workgroup
    // are mostly each other's neighbours, and their coefficients are then
    // still in the caches (a side gathered later in the kernel's life finds
    // them evicted on large meshes).  Sides 1 and 2 wait in LDS rows private
    // to the lane, side 0 (gathered last) stays in registers.
    const int sides = sside[state_off(e, 1)];
    const int bcv = BC ? sbc[state_off(e, 1)] : 0;
    T G[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) G[m] = BC ? T(bcs[m]) : T(0);

    // the neighbour's trace at its side qn, at the reversed edge points
    auto gather = [&](int q, T (&UR)[NE][4]) {
        const int nb = snb[state_off(e, 3) + q * LANES];
        const int qn = (sides >> (2 * q)) & 3;
#pragma unroll
        for (int k = 0; k < NE; ++k)
#pragma unroll
            for (int m = 0; m < 4; ++m) UR[k][m] = T(0);
        const int nbo = state_off(nb, 4 * NP);
        const T* tq = phs + qn * SS;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            T cv[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) cv[m] = T(C[nbo + (m * NP + j) * LANES]);
#pragma unroll
            for (int k = 0; k < NE; ++k) {
                const T t = tq[(NE - 1 - k) * NP + j];
#pragma unroll
                for (int m = 0; m < 4; ++m) UR[k][m] = fma(t, cv[m], UR[k][m]);
            }
        }
    };
    // one side: own trace, numerical flux, lift
    auto side = [&](int q, T (&UR)[NE][4]) {
        const int bc = (bcv >> (4 * q)) & 15;
        const int go = state_off(e, 9) + 3 * q * LANES;
        const T nx = T(sgeo[go]), ny = T(sgeo[go + LANES]);
        const double hl = sgeo[go + 2 * LANES];
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            const T* tl = tab + O::PHS + (q * NE + k) * NP;
            T UL[4], F[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                T u = T(0);
#pragma unroll
                for (int j = 0; j < NP; ++j) u = fma(tl[j], c[m][j], u);
                UL[m] = u;
            }
            if constexpr (BC) ghost_state<T>(bc, UL, nx, ny, G, UR[k]);
            llf<T>(gam, gm1, UL, UR[k], nx, ny, F);
            const double w = -hl * tab64[O::GW + k];
            const double w0 = w * tab64[O::PHS + (q * NE + k) * NP];  // phi_0 is constant
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                acc0[m] = fma(w0, double(F[m]), acc0[m]);
                F[m] *= T(w);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int j = 1; j < NP; ++j) acc[m][j] = fma(tl[j], F[m], acc[m][j]);
        }
    };

    // (sides 1 and 2 first: gathering side 0 last keeps the fewest values
    // live across the gathers)
#pragma unroll
    for (int q = 1; q < 3; ++q) {
        T URq[NE][4];
        gather(q, URq);
#pragma unroll
        for (int k = 0; k < NE; ++k)
#pragma unroll
            for (int m = 0; m < 4; ++m) urs[(((q - 1) * NE + k) * 4 + m) * BLOCK + threadIdx.x] = URq[k][m];
    }
    T UR0[NE][4];
    gather(0, UR0);
    side(0, UR0);
#pragma unroll 1
    for (int q = 1; q < 3; ++q) {
        T UR[NE][4];
#pragma unroll
        for (int k = 0; k < NE; ++k)
#pragma unroll
            for (int m = 0; m < 4; ++m) UR[k][m] = urs[(((q - 1) * NE + k) * 4 + m) * BLOCK + threadIdx.x];
        side(q, UR);
    }

    // volume integral, eq. (volume); grad phi_0 = 0, so modes j >= 1 only
#pragma unroll 1
    for (int k = 0; k < NQ; ++k) {
        T U[4], Fx[4], Fy[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            T u = T(0);
#pragma unroll
            for (int j = 0; j < NP; ++j) u = fma(tab[O::PHI + k * NP + j], c[m][j], u);
            U[m] = u;
        }
        euler_flux<T>(gm1, U, Fx, Fy);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const T gr = a00 * Fx[m] + a01 * Fy[m];
            const T gs = a10 * Fx[m] + a11 * Fy[m];
#pragma unroll
            for (int j = 1; j < NP; ++j)
                acc[m][j] = fma(tab[O::DRW + k * NP + j], gr, fma(tab[O::DSW + k * NP + j], gs, acc[m][j]));
        }
    }

    // inverse mass matrix 1/det J (FP64), then the RHS or the SSP-RK3 stage.
    // The output and the stage-0 state are touched once here: non-temporal
    // accesses leave the caches to the neighbours' coefficients (4% faster
    // at 4M triangles, p=3)
    const double h = MODE == 0 ? 0.0 : (dt_dev ? dt_dev[0] : dt);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const int x = so + (m * NP + j) * LANES;
            const double L = idet * (j == 0 ? acc0[m] : double(acc[m][j]));
            if constexpr (MODE == 0) {
                __builtin_nontemporal_store(L, &out[x]);
            } else {
                const double cs = F64 ? double(c[m][j]) : C[x];
                if constexpr (MODE == 1) {
                    __builtin_nontemporal_store(cs + h * L, &out[x]);
                } else if constexpr (MODE == 2) {
                    __builtin_nontemporal_store(0.75 * __builtin_nontemporal_load(&U0[x]) + 0.25 * (cs + h * L),
                                                &out[x]);
                } else if constexpr (MODE == 3) {
                    __builtin_nontemporal_store(
                        (1.0 / 3.0) * __builtin_nontemporal_load(&out[x]) + (2.0 / 3.0) * (cs + h * L), &out[x]);
                } else {
                    out[x] = stage_general(gs, cs, h, L, x, out);
                }
            }
        }
}

// ---------------------------------------------------------------- fused stage, 4 lanes per element
// The same right-hand side and stage update as k_stage, with the element's
// work spread over a quad of lanes.  The contractions are split by variable:
// lane m of the quad owns variable m (its N_p coefficients, accumulators and
// gathered neighbour coefficients), and all lanes of a wavefront walk the
// same volume point or side point, so every table read is uniform (scalar
// loads).  The nonlinear flux is split by point: points are taken four at a
// time, each lane evaluates its variable at the four points, a 4 x 4
// transpose through LDS hands lane i the four variables at point i, lane i
// evaluates the flux there once, and a second transpose returns flux
// component m at the four points to lane m for the lift.  The transposes
// stay inside one wavefront (the quad's lanes), so they need no workgroup
// barrier, only ordering of the LDS accesses.

// broadcast lane S of each quad to the whole quad
template <int S>
__device__ __forceinline__ double quad_bcast(double x)
{
    constexpr int ctrl = S * 0x55;  // quad_perm(S, S, S, S)
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int S>
__device__ __forceinline__ float quad_bcast(float x)
{
    constexpr int ctrl = S * 0x55;
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, 0xF, 0xF, false));
}

// sum_j t[j] x[j] with two interleaved accumulators (shorter dependency
// chain); both sides of an edge evaluate a shared trace with this same
// order, so they get bitwise equal values
template <int NP, typename T, typename Ptr>
__device__ __forceinline__ T dot2(Ptr t, const T (&x)[NP])
{
    T a = T(0), b = T(0);
#pragma unroll
    for (int j = 0; j + 1 < NP; j += 2) {
        a = fma(t[j], x[j], a);
        b = fma(t[j + 1], x[j + 1], b);
    }
    if constexpr (NP % 2) a = fma(t[NP - 1], x[NP - 1], a);
    return a + b;
}

// Orders the LDS accesses of the lanes of one wavefront around an exchange:
// accesses before it stay before, accesses after it stay after.  The
// hardware executes one wavefront's LDS instructions in order, so this is
// all an exchange between lanes of one wavefront needs.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same pointer, opaque to the optimiser: table rows read twice (trace
// evaluation, then lift) are loaded again instead of being kept in scalar
// registers across the exchange, which would exceed the scalar register file.
__device__ __forceinline__ int reload(int off)
{
    asm volatile("" : "+s"(off));
    return off;
}

// p + off for a per-lane offset into an LDS array, formed once (the
// optimiser would otherwise recompute the full address for every constant
// displacement instead of using the instruction's offset field)
template <typename T>
using lds_ptr = const __attribute__((address_space(3))) T*;
template <typename T>
__device__ __forceinline__ lds_ptr<T> lds_row(const T* p, int off)
{
    lds_ptr<T> r = (lds_ptr<T>)(p + off);
    asm volatile("" : "+v"(r));
    return r;
}

// Exchange slots of one quad: entry (i, v) holds a pair of values for point
// i of the current group and variable v, at pair slot 20 * quad + 5 * i + v.
// In both access directions (lane m of a quad writing entries (i, m) for a
// fixed i, or reading entries (m, v) for a fixed v) the 16 lanes of four
// consecutive quads then hit 16 distinct slots modulo 16, i.e. all LDS
// banks once.
template <typename T>
struct alignas(2 * sizeof(T)) Pair {
    T a, b;
};
constexpr int XROW = 5;
constexpr int XQUAD = 4 * XROW;

// Per-lane context of the four-lane kernels: element e, variable m, the
// element's geometry, and its quad's exchange slots.
template <int P, typename T>
struct Quad4 {
    int e, m, bcv;  // bcv: the element's boundary kinds, 4 bits per side
    T gam, gm1, a00, a01, a10, a11;
    T G[4];  // the prescribed boundary state
    double idet;
    Pair<T>* xr;
};

template <int P, typename T, bool BC>
__device__ __forceinline__ Quad4<P, T> quad4_setup(int e, int m, double gamma, const double* __restrict__ geo,
                                                 const int* __restrict__ sbc, const double* __restrict__ bcs,
                                                 Pair<T>* xq)
{
    Quad4<P, T> z;
    z.e = e;
    z.m = m;
    z.bcv = BC ? sbc[state_off(e, 1)] : 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) z.G[v] = BC ? T(bcs[v]) : T(0);
    z.gam = T(gamma);
    z.gm1 = T(gamma - 1.0);
    const double* g = geo + state_off(e, 6);
    z.a00 = T(g[0]);
    z.a01 = T(g[LANES]);
    z.a10 = T(g[2 * LANES]);
    z.a11 = T(g[3 * LANES]);
    z.idet = g[4 * LANES];
    z.xr = xq + (threadIdx.x >> 2) * XQUAD;
    return z;
}

// The lift of lane m's variable for the element's right-hand side, eq.
// (2ddg0) before the inverse mass matrix: volume integral, eq. (volume),
// and surface integral, eq. (surface), with the neighbours' coefficients
// gathered from Cn.  acc[j] (j >= 1) in T, the mean mode acc0 in FP64.
// phs: the side tables in LDS, sides' points reversed, rows of stride SS.
template <int P, typename T, bool BC>
__device__ __forceinline__ void rhs_quad(const Quad4<P, T>& z, const T (&c)[Ord<P>::NP], const double* Cn,
                                         const int* __restrict__ snb, const int* __restrict__ sside,
                                         const double* __restrict__ sgeo, const T* __restrict__ tab,
                                         const double* __restrict__ tab64, const T* phs, T (&acc)[Ord<P>::NP],
                                         double& acc0)
{
    using O = Ord<P>;
    constexpr int NP = O::NP, NQ = O::NQ, NE = O::NE;
    constexpr int SS = (NE * NP) | 1;
    const int e = z.e, m = z.m;
    Pair<T>* const xr = z.xr;
#pragma unroll
    for (int j = 0; j < NP; ++j) acc[j] = T(0);
    acc0 = 0.0;

    // the neighbours' coefficients of this lane's variable, one side in
    // flight: side 0's before the volume integral, each next side's once the
    // previous side is done, so the gathers' latency overlaps arithmetic.
    // (Two sides in flight hold N_p more values per lane: at p = 4 that
    // costs a wavefront per SIMD and 16% of the time, at p = 5 3%; one side
    // is no slower at p = 1..3.)
    constexpr int PF = 1;
    const int sides = sside[state_off(e, 1)];
    const int* const nb = snb + state_off(e, 3);
    T cn[PF][NP];
#pragma unroll
    for (int r = 0; r < PF; ++r) {
        const int o = state_off(nb[r * LANES], 4 * NP) + m * NP * LANES;
#pragma unroll
        for (int j = 0; j < NP; ++j) cn[r][j] = T(Cn[o + j * LANES]);
    }

    // volume integral, eq. (volume), four points at a time; the last group
    // repeats point NQ-1 where NQ is not a multiple of 4 (the repeats are
    // evaluated and dropped)
#pragma unroll 1
    for (int k0 = 0; k0 < NQ; k0 += 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) xr[i * XROW + m].a = dot2<NP>(tab + O::PHI + min(k0 + i, NQ - 1) * NP, c);
        wave_sync();
        T U[4], Fx[4], Fy[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) U[v] = xr[m * XROW + v].a;
        euler_flux<T>(z.gm1, U, Fx, Fy);
        wave_sync();
#pragma unroll
        for (int v = 0; v < 4; ++v)
            xr[m * XROW + v] = Pair<T>{z.a00 * Fx[v] + z.a01 * Fy[v], z.a10 * Fx[v] + z.a11 * Fy[v]};
        wave_sync();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = k0 + i;
            if (k < NQ) {
                const Pair<T> G = xr[i * XROW + m];
#pragma unroll
                for (int j = 1; j < NP; ++j)
                    acc[j] = fma(tab[O::DRW + k * NP + j], G.a, fma(tab[O::DSW + k * NP + j], G.b, acc[j]));
            }
        }
        wave_sync();
    }

    // surface integral, eq. (surface): per side, its p+1 Gauss points four
    // at a time (repeating point p where p+1 is not a multiple of 4)
#pragma unroll 1
    for (int q = 0; q < 3; ++q) {
        const int qn = (sides >> (2 * q)) & 3;
        const int go = state_off(e, 9) + 3 * q * LANES;
        const T nx = T(sgeo[go]), ny = T(sgeo[go + LANES]);
        const double hl = sgeo[go + 2 * LANES];
        const lds_ptr<T> tq = lds_row(phs, qn * SS);
#pragma unroll 1
        for (int k0 = 0; k0 < NE; k0 += 4) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = min(k0 + i, NE - 1);
                xr[i * XROW + m] = Pair<T>{dot2<NP>(tab + O::PHS + (q * NE + k) * NP, c), dot2<NP>(tq + k * NP, cn[0])};
            }
            wave_sync();
            T UL[4], UR[4], F[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const Pair<T> t = xr[m * XROW + v];
                UL[v] = t.a;
                UR[v] = t.b;
            }
            if constexpr (BC) ghost_state<T>((z.bcv >> (4 * q)) & 15, UL, nx, ny, z.G, UR);
            llf<T>(z.gam, z.gm1, UL, UR, nx, ny, F);
            wave_sync();
#pragma unroll
            for (int v = 0; v < 4; ++v) xr[m * XROW + v].a = F[v];
            wave_sync();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = k0 + i;
                if (k < NE) {
                    const T Fk = xr[i * XROW + m].a;
                    const double w = -hl * tab64[O::GW + k];
                    acc0 = fma(w * tab64[O::PHS + (q * NE + k) * NP], double(Fk), acc0);
                    const T wf = T(w) * Fk;
                    const T* tl = tab + reload(O::PHS + (q * NE + k) * NP);
#pragma unroll
                    for (int j = 1; j < NP; ++j) acc[j] = fma(tl[j], wf, acc[j]);
                }
            }
            wave_sync();
        }
        // the next side's neighbour moves to the front (a rolled loop
        // cannot index registers by q)
#pragma unroll
        for (int r = 0; r + 1 < PF; ++r)
#pragma unroll
            for (int j = 0; j < NP; ++j) cn[r][j] = cn[r + 1][j];
        if (q + PF < 3) {
            const int nbo = state_off(nb[(q + PF) * LANES], 4 * NP) + m * NP * LANES;
#pragma unroll
            for (int j = 0; j < NP; ++j) cn[PF - 1][j] = T(Cn[nbo + j * LANES]);
        }
    }
}

// ---------------------------------------------------------------- mixed precision on the matrix cores
// The FP32 contractions of rhs_quad on v_mfma_f32_4x4x1f32.  That
// instruction treats every quad of lanes as one 4 x 4 block: register i of
// lane 4b+j gains A(lane 4b+i) * B(lane 4b+j).  A quad is one element and
// lane j holds variable j, so with B = a coefficient of the lane's variable
// and A = a table entry chosen by the lane's position i in the quad, one
// instruction adds a rank-one term to a 4 x 4 block of every element of the
// wavefront:
//   evaluation: A = phi_j(point k0+i), B = c_j: after j = 0..N_p-1, register
//     i of lane m is variable m at point k0+i (what the scalar path writes
//     into the exchange slots before its first transpose);
//   lift: A = w grad phi_{4g+i}(point k) (or the side trace table), B = the
//     lane's flux component at point k: register i of the accumulator group
//     g of lane m is mode 4g+i of variable m.
// The table operands (one value per quad position) come from a copy of the
// FP32 tables in LDS with the rows padded to multiples of four.
template <int P>
struct MTab {
    using O = Ord<P>;
    static constexpr int NP = O::NP, NQ = O::NQ, NE = O::NE;
    static constexpr int NQ4 = (NQ + 3) / 4 * 4, NE4 = (NE + 3) / 4 * 4, NPP = (NP + 3) / 4 * 4, NG = NPP / 4;
    // PHI rows k < NQ4 (k >= NQ repeats NQ-1), N_p columns
    static constexpr int PHI = 0;
    // w dphi/dr and w dphi/ds rows k < NQ, NPP columns (zero padded)
    static constexpr int DR = PHI + NQ4 * NP, DS = DR + NQ * NPP;
    // side traces for evaluation: [q][k < NE4 (k >= NE repeats NE-1)][N_p]
    static constexpr int PSE = DS + NQ * NPP;
    // side traces for the lift: [q * NE + k][NPP] (zero padded)
    static constexpr int PSL = PSE + 3 * NE4 * NP;
    static constexpr int SIZE = PSL + 3 * NE * NPP;
};

typedef float v4f __attribute__((ext_vector_type(4)));

// sum_j A_j B_j over a quad block (A = t[j] of the lane's quad position, B =
// b[j] of the lane's variable) in two independent MFMA chains, even and odd
// j, added at the end
template <int NP>
__device__ __forceinline__ v4f mfma_dot(const float* t, const float (&b)[NP])
{
    v4f u0 = {0.f, 0.f, 0.f, 0.f}, u1 = u0;
#pragma unroll
    for (int j = 0; j + 1 < NP; j += 2) {
        u0 = __builtin_amdgcn_mfma_f32_4x4x1f32(t[j], b[j], u0, 0, 0, 0);
        u1 = __builtin_amdgcn_mfma_f32_4x4x1f32(t[j + 1], b[j + 1], u1, 0, 0, 0);
    }
    if constexpr (NP % 2) u0 = __builtin_amdgcn_mfma_f32_4x4x1f32(t[NP - 1], b[NP - 1], u0, 0, 0, 0);
    return u0 + u1;
}

template <int P>
__device__ __forceinline__ void load_mfma_tables(const float* __restrict__ tab, float* t)
{
    using O = Ord<P>;
    using M = MTab<P>;
    constexpr int NP = O::NP, NQ = O::NQ, NE = O::NE, NPP = M::NPP;
    for (int x = threadIdx.x; x < M::SIZE; x += BLOCK) {
        float v;
        if (x < M::DR) {
            const int k = x / NP, j = x % NP;
            v = tab[O::PHI + min(k, NQ - 1) * NP + j];
        } else if (x < M::PSE) {
            const int y = x - M::DR, w = y / (NQ * NPP), r = y % (NQ * NPP), k = r / NPP, j = r % NPP;
            v = j < NP ? tab[(w ? O::DSW : O::DRW) + k * NP + j] : 0.f;
        } else if (x < M::PSL) {
            const int y = x - M::PSE, q = y / (M::NE4 * NP), r = y % (M::NE4 * NP), k = r / NP, j = r % NP;
            v = tab[O::PHS + (q * NE + min(k, NE - 1)) * NP + j];
        } else {
            const int y = x - M::PSL, row = y / NPP, j = y % NPP;
            v = j < NP ? tab[O::PHS + row * NP + j] : 0.f;
        }
        t[x] = v;
    }
}

// rhs_quad for T = float with the contractions on the matrix cores (same
// arguments, plus the LDS tables of load_mfma_tables); the fluxes, the
// exchanges and the FP64 mean mode are those of rhs_quad.
template <int P, bool BC>
__device__ __forceinline__ void rhs_quad_mfma(const Quad4<P, float>& z, const float (&c)[Ord<P>::NP],
                                              const double* Cn, const int* __restrict__ snb,
                                              const int* __restrict__ sside, const double* __restrict__ sgeo,
                                              const double* __restrict__ tab64, const float* phs, const float* mt,
                                              float (&acc)[Ord<P>::NP], double& acc0)
{
    using O = Ord<P>;
    using M = MTab<P>;
    constexpr int NP = O::NP, NQ = O::NQ, NE = O::NE, NPP = M::NPP, NG = M::NG;
    constexpr int SS = (NE * NP) | 1;
    const int e = z.e, m = z.m;
    Pair<float>* const xr = z.xr;
    const v4f zero = {0.f, 0.f, 0.f, 0.f};
    // two accumulator sets (independent MFMA chains): r-derivative and
    // surface terms in av, s-derivative terms in as
    v4f av[NG], as[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) av[g] = as[g] = zero;
    acc0 = 0.0;

    // one neighbour side in flight, as in rhs_quad (two sides cost 12% at p=5)
    constexpr int PF = 1;
    const int sides = sside[state_off(e, 1)];
    const int* const nb = snb + state_off(e, 3);
    float cn[PF][NP];
#pragma unroll
    for (int r = 0; r < PF; ++r) {
        const int o = state_off(nb[r * LANES], 4 * NP) + m * NP * LANES;
#pragma unroll
        for (int j = 0; j < NP; ++j) cn[r][j] = float(Cn[o + j * LANES]);
    }

    // volume integral, four points at a time (point NQ-1 repeated in the
    // last group where NQ is not a multiple of 4)
#pragma unroll 1
    for (int k0 = 0; k0 < NQ; k0 += 4) {
        const float* tp = mt + M::PHI + (k0 + m) * NP;  // A: this lane's quad position is its point
        const v4f u = mfma_dot<NP>(tp, c);
#pragma unroll
        for (int i = 0; i < 4; ++i) xr[i * XROW + m].a = u[i];
        wave_sync();
        float U[4], Fx[4], Fy[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) U[v] = xr[m * XROW + v].a;
        euler_flux<float>(z.gm1, U, Fx, Fy);
        wave_sync();
#pragma unroll
        for (int v = 0; v < 4; ++v)
            xr[m * XROW + v] = Pair<float>{z.a00 * Fx[v] + z.a01 * Fy[v], z.a10 * Fx[v] + z.a11 * Fy[v]};
        wave_sync();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = k0 + i;
            if (k < NQ) {
                const Pair<float> G = xr[i * XROW + m];
                const float* tr = mt + M::DR + k * NPP + m;  // A: mode 4g + (quad position)
                const float* ts = mt + M::DS + k * NPP + m;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    av[g] = __builtin_amdgcn_mfma_f32_4x4x1f32(tr[4 * g], G.a, av[g], 0, 0, 0);
                    as[g] = __builtin_amdgcn_mfma_f32_4x4x1f32(ts[4 * g], G.b, as[g], 0, 0, 0);
                }
            }
        }
        wave_sync();
    }

    // surface integral, per side, its p+1 Gauss points four at a time
#pragma unroll 1
    for (int q = 0; q < 3; ++q) {
        const int qn = (sides >> (2 * q)) & 3;
        const int go = state_off(e, 9) + 3 * q * LANES;
        const float nx = float(sgeo[go]), ny = float(sgeo[go + LANES]);
        const double hl = sgeo[go + 2 * LANES];
#pragma unroll 1
        for (int k0 = 0; k0 < NE; k0 += 4) {
            // own trace: the side table; neighbour trace: its side's table
            // with the points reversed (rows past p repeat point p)
            const float* tl = mt + M::PSE + (q * M::NE4 + k0 + m) * NP;
            const float* tn = phs + qn * SS + min(k0 + m, NE - 1) * NP;
            const v4f ul = mfma_dot<NP>(tl, c), ur = mfma_dot<NP>(tn, cn[0]);
#pragma unroll
            for (int i = 0; i < 4; ++i) xr[i * XROW + m] = Pair<float>{ul[i], ur[i]};
            wave_sync();
            float UL[4], UR[4], F[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const Pair<float> t = xr[m * XROW + v];
                UL[v] = t.a;
                UR[v] = t.b;
            }
            if constexpr (BC) ghost_state<float>((z.bcv >> (4 * q)) & 15, UL, nx, ny, z.G, UR);
            llf<float>(z.gam, z.gm1, UL, UR, nx, ny, F);
            wave_sync();
#pragma unroll
            for (int v = 0; v < 4; ++v) xr[m * XROW + v].a = F[v];
            wave_sync();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = k0 + i;
                if (k < NE) {
                    const float Fk = xr[i * XROW + m].a;
                    const double w = -hl * tab64[O::GW + k];
                    acc0 = fma(w * tab64[O::PHS + (q * NE + k) * NP], double(Fk), acc0);
                    const float wf = float(w) * Fk;
                    const float* ta = mt + M::PSL + (q * NE + k) * NPP + m;
#pragma unroll
                    for (int g = 0; g < NG; ++g) av[g] = __builtin_amdgcn_mfma_f32_4x4x1f32(ta[4 * g], wf, av[g], 0, 0, 0);
                }
            }
            wave_sync();
        }
#pragma unroll
        for (int r = 0; r + 1 < PF; ++r)
#pragma unroll
            for (int j = 0; j < NP; ++j) cn[r][j] = cn[r + 1][j];
        if (q + PF < 3) {
            const int nbo = state_off(nb[(q + PF) * LANES], 4 * NP) + m * NP * LANES;
#pragma unroll
            for (int j = 0; j < NP; ++j) cn[PF - 1][j] = float(Cn[nbo + j * LANES]);
        }
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) acc[j] = av[j / 4][j % 4] + as[j / 4][j % 4];
}

// side tables into LDS with the points of each side in reverse order: row k
// of side q is the trace of mode j at the point that the neighbour across
// side q sees as its point k (every thread of the block calls it)
template <int P, typename T>
__device__ __forceinline__ void load_side_tables(const T* __restrict__ tab, T* phs)
{
    using O = Ord<P>;
    constexpr int NP = O::NP, NE = O::NE, SS = (NE * NP) | 1;
    for (int i = threadIdx.x; i < 3 * NE * NP; i += BLOCK) {
        const int q = i / (NE * NP), r = i % (NE * NP), k = r / NP, j = r % NP;
        phs[q * SS + (NE - 1 - k) * NP + j] = tab[O::PHS + i];
    }
    __syncthreads();
}

// Fused step length (multi-step path): MODE 1 with pin != nullptr computes
// the step length itself from the previous per-block minima pin[0..pin_count)
// and logical block 0 stores it to dt_store (and dt_hist); MODE 3 with
// pout != nullptr writes the minimum over its 64 elements of the new
// state's r_in / (|v| + c) to pout[logical block].
template <int P, int MODE, typename T, bool BC>
__global__ __launch_bounds__(BLOCK) void k_stage4(int n, int npad, const double* __restrict__ C,
                                                  const double* __restrict__ U0, double* __restrict__ out,
                                                  const double* __restrict__ geo, const int* __restrict__ snb,
                                                  const int* __restrict__ sside, const double* __restrict__ sgeo,
                                                  const T* __restrict__ tab, const double* __restrict__ tab64,
                                                  double gamma, double dt, const double* __restrict__ dt_dev,
                                                  const double* __restrict__ pin, int pin_count, double cfl,
                                                  double* __restrict__ dt_store, double* __restrict__ dt_hist,
                                                  double* __restrict__ pout, StageGen gs,
                                                  const int* __restrict__ sbc, const double* __restrict__ bcs)
{
    using O = Ord<P>;
    constexpr int NP = O::NP, NE = O::NE;
    constexpr int SS = (NE * NP) | 1;
    constexpr bool F64 = sizeof(T) == sizeof(double);
    // the FP32 form runs its contractions on the matrix cores (MFMA)
    constexpr bool MF = !F64 && DG_MIXED_MFMA;
    __shared__ T phs[3 * SS];
    __shared__ double red[BLOCK / WAVE];
    __shared__ Pair<T> xq[(BLOCK / 4) * XQUAD];
    __shared__ float mt[MF ? MTab<P>::SIZE : 1];
    if constexpr (MF) load_mfma_tables<P>((const float*)tab, mt);
    load_side_tables<P, T>(tab, phs);

    const int lb = xcd_block(blockIdx.x, gridDim.x);
    double hfused = 0.0;
    if constexpr (MODE == 1) {
        if (pin) hfused = dt_from_partials(pin, pin_count, cfl, red);
    }

    // 64 elements per workgroup; every lane stays active until the stores
    // (the exchanges read the neighbouring lanes)
    const int e = lb * (BLOCK / 4) + (threadIdx.x >> 2);
    const int m = threadIdx.x & 3;
    if (e >= npad) return;  // whole workgroups leave together (npad % 64 == 0)
    const bool real = e < n;
    const int so = state_off(e, 4 * NP) + m * NP * LANES;
    const Quad4<P, T> z = quad4_setup<P, T, BC>(e, m, gamma, geo, sbc, bcs, xq);

    T c[NP], acc[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) c[j] = T(C[so + j * LANES]);
    double acc0;
    if constexpr (MF)
        rhs_quad_mfma<P, BC>(z, c, C, snb, sside, sgeo, tab64, phs, mt, acc, acc0);
    else
        rhs_quad<P, T, BC>(z, c, C, snb, sside, sgeo, tab, tab64, phs, acc, acc0);

    double h = MODE == 0 ? 0.0 : (dt_dev ? dt_dev[0] : dt);
    if constexpr (MODE == 1) {
        if (pin) {
            h = hfused;
            if (lb == 0 && threadIdx.x == 0) {
                dt_store[0] = h;
                if (dt_hist) dt_hist[0] = h;
            }
        }
    }
    double mean = 0.0;  // new value of mode 0 of this lane's variable
    if (!real) {
#pragma unroll
        for (int j = 0; j < NP; ++j) out[so + j * LANES] = 0.0;
    } else {
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const int x = so + j * LANES;
            const double L = z.idet * (j == 0 ? acc0 : double(acc[j]));
            double v;
            if constexpr (MODE == 0) {
                v = L;
            } else {
                const double cs = F64 ? double(c[j]) : C[x];
                if constexpr (MODE == 1) {
                    v = cs + h * L;
                } else if constexpr (MODE == 2) {
                    v = 0.75 * U0[x] + 0.25 * (cs + h * L);
                } else if constexpr (MODE == 3) {
                    v = (1.0 / 3.0) * out[x] + (2.0 / 3.0) * (cs + h * L);
                } else {
                    v = stage_general(gs, cs, h, L, x, out);
                }
            }
            out[x] = v;
            if (j == 0) mean = v;
        }
    }
    if constexpr (MODE == 3) {
        if (pout) {
            const double r0 = quad_bcast<0>(mean), r1 = quad_bcast<1>(mean), r2 = quad_bcast<2>(mean),
                         r3 = quad_bcast<3>(mean);
            double val = INFINITY;
            if (real && m == 0) val = dt_local(gamma, geo[state_off(e, 6) + 5 * LANES], r0, r1, r2, r3);
            const double mn = block_min(val, red);
            if (threadIdx.x == 0) pout[lb] = mn;
        }
    }
}

// ---------------------------------------------------------------- stage on the matrix cores, 16 elements per wavefront
// The fused stage of k_stage4 with every contraction of eq. (2ddg0) on the
// 16 x 16 x 4 matrix products (v_mfma_f64_16x16x4f64 in FP64,
// v_mfma_f32_16x16x4f32 in the mixed form): one wavefront per block of 16
// elements, the elements are the 16 columns of each product.  Operand layout:
// the 16 x 4 table operand A has row i, column k in lane 16k+i; the 4 x 16
// operand B has row k, column j in lane 16k+j; register r of the 16 x 16
// result in lane 16g+j is column j, row mx_row(g, r) = 4r+g for the FP64
// instruction and 4g+r for the FP32 one.
// Lane 16g+j holds modes 4s+g (s < KP) of the four variables of element j:
// the B operands of every contraction over modes (k-step s).
//   evaluation at 16 points (volume, eq. (volume), or the three sides' Gauss
//     points, eq. (surface)): register r of lane group g is point
//     mx_row(g, r) of the tile, all four variables at four points per lane,
//     which is what the fluxes need: no exchange between lanes;
//   lift back to modes: the lane's fluxes at its points are the B operands,
//     k-step s' pairing lane group g with point mx_row(g, s') (the table
//     operand is ordered to match), and the result rows are ordered so that
//     register r of lane group g of mode tile tm is mode 4(4tm+r)+g: the
//     lane's own modes, so the stage update needs no exchange either.
// The neighbour's trace across side q is the neighbour's side q' at the
// reversed point; q' differs between the columns, so the neighbour's traces
// on all three sides are evaluated (one product per side) and each column
// keeps the points facing it in LDS.  Padded points repeat a real one (finite
// fluxes) and carry zero weights; padded modes have zero table entries.
// Mixed form (T = float): as in k_stage4, FP32 contractions, traces and
// fluxes; the mean mode accumulated in FP64 from the FP32 fluxes (the lanes
// of a column add their side points' terms and then each other's); 1/det J
// and the stage update in FP64 from the FP64 state kept in registers.
typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));
template <typename T>
using mxv = std::conditional_t<sizeof(T) == sizeof(double), dx4, fx4>;
__device__ __forceinline__ dx4 mfma16(double a, double b, dx4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ fx4 mfma16(float a, float b, fx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// at p = 4 the FP64 kernel fits three wavefronts per SIMD without spilling
// (at most 168 registers) when asked to, except the boundary variant of the
// third stage (fused step-length partials), which would spill and keeps two;
// p = 5 would spill, p <= 3 fits three by itself
template <int P, int MODE, typename T, bool BC>
constexpr int mx_waves = P == 4 && sizeof(T) == sizeof(double) && !(BC && MODE == 3) ? 3 : 1;
template <int P, int MODE, typename T, bool BC>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(mx_waves<P, MODE, T, BC>))) void k_stage_mx(
    int n, int npad, const double* __restrict__ C, const double* __restrict__ U0, double* __restrict__ out,
    const double* __restrict__ geo, const int* __restrict__ snb, const int* __restrict__ sside,
    const double* __restrict__ sgeo, const T* __restrict__ tmx, const double* __restrict__ tab64, double gamma,
    double dt, const double* __restrict__ dt_dev, const double* __restrict__ pin, int pin_count, double cfl,
    double* __restrict__ dt_store, double* __restrict__ dt_hist, double* __restrict__ pout, StageGen gs,
    const int* __restrict__ sbc, const double* __restrict__ bcs)
{
    using O = Ord<P>;
    using V = mxv<T>;
    constexpr bool F64 = sizeof(T) == sizeof(double);
    constexpr MxLayout X = mx_layout(P);
    constexpr int NP = X.np, NE = X.ne, NS = X.ns, KP = X.kp, TQ = X.tq, TS = X.ts, TM = X.tm;
    // side points past the first tile (p = 5: 2 of 18) are evaluated per
    // lane, a dot product over the lane's modes added up over the column's
    // four lanes, instead of a second tile of products that is mostly
    // padding; in the mixed form only (the FP64 kernel would need more than
    // 256 registers for it at p = 5 and lose its second wavefront per SIMD)
    constexpr int NTL = F64 ? 0 : X.nt, TSP = NTL ? 1 : TS;
    constexpr int NW = BLOCK / WAVE;
    constexpr int NVH = 2;  // neighbour variables gathered together (half the registers of four)
    __shared__ T xs[NW][3][4][NE][LANES];  // neighbour traces facing each side, per wavefront
    __shared__ double red[NW];

    const int lb = xcd_block(blockIdx.x, gridDim.x);
    double hfused = 0.0;
    if constexpr (MODE == 1) {
        if (pin) hfused = dt_from_partials(pin, pin_count, cfl, red);
    }

    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE, j = lane % 16, g = lane / 16;
    const int blk = lb * NW + w;  // 16-element block of this wavefront
    if (lb * NW * LANES >= npad) return;  // whole workgroups leave together (npad % 64 == 0)
    const int e = blk * LANES + j;
    const bool real = e < n;
    auto row = [&](int r) { return mx_row<F64>(g, r); };
    const double* gp = geo + state_off(e, 6);
    const T a00 = T(gp[0]), a01 = T(gp[LANES]), a10 = T(gp[2 * LANES]), a11 = T(gp[3 * LANES]);
    const double idet = gp[4 * LANES];
    const T gam = T(gamma), gm1 = T(gamma - 1.0);
    const int base = blk * 4 * NP * LANES + j;
    const T* tl = tmx + lane;
    auto A = [&](int b) { return tl[b * WAVE]; };

    // own coefficients: c[v][s] = mode 4s+g of variable v (a padded mode
    // loads the last mode; its table entries are zero)
    double c[4][KP];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int s = 0; s < KP; ++s) c[v][s] = C[base + (v * NP + min(4 * s + g, NP - 1)) * LANES];

    V acc[4][TM];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int t = 0; t < TM; ++t) acc[v][t] = V{0, 0, 0, 0};

    // the neighbours' coefficients, two variables of one side at a time:
    // where registers allow (mixed form, FP64 up to p = 3), each pair is
    // gathered one step ahead of its use and the first before the volume
    // integral (FP64 at p = 4, 5 would lose a wavefront per SIMD to it)
    constexpr bool PIPE = !F64 || P <= 3;
    constexpr int NT = 3 * (4 / NVH);  // (side, variable pair) steps
    const int sides = sside[state_off(e, 1)];
    const int* const nb = snb + state_off(e, 3);
    auto gather = [&](int t, T (&dst)[NVH][KP]) {
        const int q = t / (4 / NVH), v0 = (t % (4 / NVH)) * NVH;
        const int nbase = state_off(nb[q * LANES], 4 * NP);
#pragma unroll
        for (int v = 0; v < NVH; ++v)
#pragma unroll
            for (int s = 0; s < KP; ++s) dst[v][s] = T(C[nbase + ((v0 + v) * NP + min(4 * s + g, NP - 1)) * LANES]);
    };
    T cnx[NVH][KP];
    if constexpr (PIPE) gather(0, cnx);

    // volume integral, eq. (volume)
#pragma unroll
    for (int tq = 0; tq < TQ; ++tq) {
        V u[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) u[v] = V{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KP; ++s) {
            const T a = A(X.phi + tq * KP + s);
#pragma unroll
            for (int v = 0; v < 4; ++v) u[v] = mfma16(a, T(c[v][s]), u[v]);
        }
        // the flux at the lane's point r is k-step r of the lift
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const T U[4] = {u[0][r], u[1][r], u[2][r], u[3][r]};
            T Fx[4], Fy[4];
            euler_flux<T>(gm1, U, Fx, Fy);
#pragma unroll
            for (int tm = 0; tm < TM; ++tm) {
                const T ar = A(X.dr + (tm * TQ + tq) * 4 + r), as = A(X.ds + (tm * TQ + tq) * 4 + r);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    acc[v][tm] = mfma16(ar, a00 * Fx[v] + a01 * Fy[v], acc[v][tm]);
                    acc[v][tm] = mfma16(as, a10 * Fx[v] + a11 * Fy[v], acc[v][tm]);
                }
            }
        }
    }

    // surface integral, eq. (surface): the neighbours' traces first, side
    // by side; each column keeps, in LDS, the p+1 points of its neighbour's
    // side that face it, in its own order (reversed), so no lane holds
    // neighbour values across the sides (register r of tile ts is side point
    // 16ts+row(r), side-major)
    // the neighbour's traces at all its side points for step t, and the
    // points facing this column into LDS
    auto traces = [&](int t, const T (&cn)[NVH][KP]) {
        const int q = t / (4 / NVH), v0 = (t % (4 / NVH)) * NVH;
        const int qn = (sides >> (2 * q)) & 3;
#pragma unroll
        for (int pt = 0; pt < NTL; ++pt) {
            const int k = 16 + pt - qn * NE;  // point of the neighbour's side qn
#pragma unroll
            for (int v = 0; v < NVH; ++v) {
                T d = T(0);
#pragma unroll
                for (int s = 0; s < KP; ++s) d = fma(A(X.tpe + pt * KP + s), cn[v][s], d);
                d += __shfl_xor(d, 16);
                d += __shfl_xor(d, 32);
                if (g == 0 && k >= 0 && k < NE) xs[w][q][v0 + v][NE - 1 - k][j] = d;
            }
        }
#pragma unroll
        for (int ts = 0; ts < TSP; ++ts) {
            V tn[NVH];
#pragma unroll
            for (int v = 0; v < NVH; ++v) tn[v] = V{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KP; ++s) {
                const T a = A(X.pe + ts * KP + s);
#pragma unroll
                for (int v = 0; v < NVH; ++v) tn[v] = mfma16(a, cn[v][s], tn[v]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = 16 * ts + row(r) - qn * NE;  // point of the neighbour's side qn
                if (k >= 0 && k < NE) {
#pragma unroll
                    for (int v = 0; v < NVH; ++v) xs[w][q][v0 + v][NE - 1 - k][j] = tn[v][r];
                }
            }
        }
    };
    if constexpr (PIPE) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            T cn[NVH][KP];
#pragma unroll
            for (int v = 0; v < NVH; ++v)
#pragma unroll
                for (int s = 0; s < KP; ++s) cn[v][s] = cnx[v][s];
            if (t + 1 < NT) gather(t + 1, cnx);
            traces(t, cn);
        }
    } else {
#pragma unroll 1
        for (int t = 0; t < NT; ++t) {
            gather(t, cnx);
            traces(t, cnx);
        }
    }
    wave_sync();

    // own traces, the numerical flux of eq. (surface) (local Lax-Friedrichs)
    // at each side point, scaled by minus the half side length (the Gauss
    // weights are in the table), and the lift
    // boundary codes of the three sides; the ghost state (and the fixed
    // boundary state it may take) only where a lane's side is a boundary,
    // which keeps the boundary variant within the registers of three
    // wavefronts per SIMD at p = 4
    const int bcv = BC ? sbc[state_off(e, 1)] : 0;
    double acc0[4] = {0.0, 0.0, 0.0, 0.0};  // mixed form: the mean mode in FP64
#pragma unroll
    for (int ts = 0; ts < TSP; ++ts) {
        V ul[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) ul[v] = V{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KP; ++s) {
            const T a = A(X.pe + ts * KP + s);
#pragma unroll
            for (int v = 0; v < 4; ++v) ul[v] = mfma16(a, T(c[v][s]), ul[v]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int sp = 16 * ts + row(r);
            const int q = min(sp / NE, 2);
            const bool pad = sp >= NS;
            const int go = state_off(e, 9) + 3 * q * LANES;
            const T nx = T(sgeo[go]), ny = T(sgeo[go + LANES]);
            const double hl = sgeo[go + 2 * LANES];
            const int k = min(sp - q * NE, NE - 1);
            T UL[4], UR[4], F[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                UL[v] = ul[v][r];
                UR[v] = pad ? UL[v] : xs[w][q][v][k][j];
            }
            if constexpr (BC) {
                const int code = (bcv >> (4 * q)) & 15;
                if (code) {
                    T G[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) G[v] = T(bcs[v]);
                    ghost_state<T>(code, UL, nx, ny, G, UR);
                }
            }
            llf<T>(gam, gm1, UL, UR, nx, ny, F);
            if constexpr (!F64) {
                const double w0 = pad ? 0.0 : -hl * tab64[O::GW + k] * tab64[O::PHS + (q * NE + k) * NP];
#pragma unroll
                for (int v = 0; v < 4; ++v) acc0[v] = fma(w0, double(F[v]), acc0[v]);
            }
#pragma unroll
            for (int tm = 0; tm < TM; ++tm) {
                const T a = A(X.le + (tm * TS + ts) * 4 + r);
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v][tm] = mfma16(a, T(-hl) * F[v], acc[v][tm]);
            }
        }
    }
    if constexpr (NTL > 0) {
        // the side points past the first tile: lane group g < NTL takes point
        // 16+g (its traces summed over the column's lanes), and every lane
        // lifts all of them onto its own modes
        T ut[NTL][4];
#pragma unroll
        for (int pt = 0; pt < NTL; ++pt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                T d = T(0);
#pragma unroll
                for (int s = 0; s < KP; ++s) d = fma(A(X.tpe + pt * KP + s), T(c[v][s]), d);
                d += __shfl_xor(d, 16);
                d += __shfl_xor(d, 32);
                ut[pt][v] = d;
            }
        const bool pad = g >= NTL;
        const int sp = 16 + min(g, NTL - 1);
        const int q = min(sp / NE, 2);
        const int go = state_off(e, 9) + 3 * q * LANES;
        const T nx = T(sgeo[go]), ny = T(sgeo[go + LANES]);
        const double hl = sgeo[go + 2 * LANES];
        const int k = min(sp - q * NE, NE - 1);
        T UL[4], UR[4], F[4], wf[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            T u = ut[0][v];
#pragma unroll
            for (int pt = 1; pt < NTL; ++pt) u = g == pt ? ut[pt][v] : u;
            UL[v] = u;
            UR[v] = pad ? UL[v] : xs[w][q][v][k][j];
        }
        if constexpr (BC) {
            const int code = (bcv >> (4 * q)) & 15;
            if (code) {
                T G[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) G[v] = T(bcs[v]);
                ghost_state<T>(code, UL, nx, ny, G, UR);
            }
        }
        llf<T>(gam, gm1, UL, UR, nx, ny, F);
#pragma unroll
        for (int v = 0; v < 4; ++v) wf[v] = pad ? T(0) : T(-hl) * F[v];
        if constexpr (!F64) {
            const double w0 = pad ? 0.0 : -hl * tab64[O::GW + k] * tab64[O::PHS + (q * NE + k) * NP];
#pragma unroll
            for (int v = 0; v < 4; ++v) acc0[v] = fma(w0, double(F[v]), acc0[v]);
        }
#pragma unroll
        for (int pt = 0; pt < NTL; ++pt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const T f = __shfl(wf[v], j + 16 * pt);
#pragma unroll
                for (int s = 0; s < KP; ++s) acc[v][s / 4][s % 4] = fma(A(X.tle + pt * KP + s), f, acc[v][s / 4][s % 4]);
            }
    }
    if constexpr (!F64) {
        // the column's four lanes add their terms of the mean mode
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            acc0[v] += __shfl_xor(acc0[v], 16);
            acc0[v] += __shfl_xor(acc0[v], 32);
        }
    }

    // 1/det J (orthonormal basis) and the stage update
    double h = MODE == 0 ? 0.0 : (dt_dev ? dt_dev[0] : dt);
    if constexpr (MODE == 1) {
        if (pin) {
            h = hfused;
            if (lb == 0 && threadIdx.x == 0) {
                dt_store[0] = h;
                if (dt_hist) dt_hist[0] = h;
            }
        }
    }
    double mean[4] = {0.0, 0.0, 0.0, 0.0};  // new mode 0 (lane group 0)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int s = 0; s < KP; ++s) {
            const int jm = 4 * s + g;
            if (jm < NP) {
                const int x = base + (v * NP + jm) * LANES;
                const double a = (!F64 && s == 0 && g == 0) ? acc0[v] : double(acc[v][s / 4][s % 4]);
                const double L = idet * a;
                double val;
                if (!real) {
                    val = 0.0;
                } else if constexpr (MODE == 0) {
                    val = L;
                } else {
                    const double cs = c[v][s];
                    if constexpr (MODE == 1)
                        val = cs + h * L;
                    else if constexpr (MODE == 2)
                        val = 0.75 * __builtin_nontemporal_load(&U0[x]) + 0.25 * (cs + h * L);
                    else if constexpr (MODE == 3)
                        val = (1.0 / 3.0) * __builtin_nontemporal_load(&out[x]) + (2.0 / 3.0) * (cs + h * L);
                    else
                        val = stage_general(gs, cs, h, L, x, out);
                }
                __builtin_nontemporal_store(val, &out[x]);
                if (s == 0) mean[v] = val;
            }
        }
    if constexpr (MODE == 3) {
        if (pout) {
            double val = INFINITY;
            if (real && g == 0) val = dt_local(gamma, gp[5 * LANES], mean[0], mean[1], mean[2], mean[3]);
            const double mn = block_min(val, red);
            if (threadIdx.x == 0) pout[lb] = mn;
        }
    }
}

// ---------------------------------------------------------------- limiter
// Barth-Jespersen slope limiter for p = 1 (Section "Limiting Kernel", eqs.
// (limit), (limitmax), (limitmin)), in place, one work-item per element and
// each conserved variable separately.  The centroid value of a linear
// function is its mean, sqrt(2) c_0 in the orthonormal basis (modes 1 and 2
// vanish at the centroid); Umax / Umin are the extremes of the element's and
// its three neighbours' centroid values; at each Gauss point of the three
// sides, with d = U(r_qk) - Ubar, the admissible factor is (Umax - Ubar) / d
// for d > 0, (Umin - Ubar) / d for d < 0, and 1 for d = 0; the smallest
// factor, at most 1, scales modes 1 and 2.  Only those modes are written, so
// reading the neighbours' means while other work-items limit is race-free.
// The neighbours' indices are read once per element, the own coefficients
// and the neighbours' means of the four variables are all in flight
// together, and the slopes are written with non-temporal stores.  BC: the
// mesh has domain-boundary sides (periodic meshes skip the boundary kinds).
template <int P, bool BC>
__global__ __launch_bounds__(BLOCK) void k_limit_bj(int n, double* __restrict__ C, const int* __restrict__ snb,
                                                     const int* __restrict__ sbc, const double* __restrict__ tab)
{
    using O = Ord<P>;
    constexpr int NP = O::NP, NE = O::NE;
    const double s2 = 1.4142135623730951;
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= n) return;
    const int so = state_off(e, 4 * NP);
    int nbo[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) nbo[q] = state_off(snb[state_off(e, 3) + q * LANES], 4 * NP);
    const int bcv = BC ? sbc[state_off(e, 1)] : 0;
    double c[4][NP], un[3][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int j = 0; j < NP; ++j) c[m][j] = C[so + (m * NP + j) * LANES];
#pragma unroll
        for (int q = 0; q < 3; ++q) un[q][m] = s2 * C[nbo[q] + m * NP * LANES];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const double ub = s2 * c[m][0];
        double umax = ub, umin = ub;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            // a domain-boundary side has no neighbour
            if (!BC || ((bcv >> (4 * q)) & 15) == 0) {
                umax = fmax(umax, un[q][m]);
                umin = fmin(umin, un[q][m]);
            }
        }
        double a = 1.0;
#pragma unroll
        for (int qk = 0; qk < 3 * NE; ++qk) {
            double u = 0.0;
#pragma unroll
            for (int j = 0; j < NP; ++j) u = fma(tab[O::PHS + qk * NP + j], c[m][j], u);
            const double d = u - ub;
            const double ak = d > 0.0 ? (umax - ub) / d : d < 0.0 ? (umin - ub) / d : 1.0;
            a = fmin(a, ak);
        }
#pragma unroll
        for (int j = 1; j < NP; ++j) __builtin_nontemporal_store(a * c[m][j], &C[so + (m * NP + j) * LANES]);
    }
}



// ---------------------------------------------------------------- adjoint
// Cotangent of s = Fx(U).X + Fy(U).Y with respect to U (X, Y: cotangents of
// the x and y fluxes).  With Ku = X0 rho + X1 mx + X2 my + X3 (E+p), Kv the
// same with Y, and Pp = X1 + Y2 + u X3 + v Y3:
//   d/d rho = -(Ku u + Kv v)/rho + u X0 + v Y0 + Pp (gamma-1) |v|^2/2
//   d/d mx  = Ku/rho + u X1 + v Y1 - Pp (gamma-1) u
//   d/d my  = Kv/rho + u X2 + v Y2 - Pp (gamma-1) v
//   d/d E   = u X3 + v Y3 + Pp (gamma-1)
// The normal flux F.n is the case X = n_x Fb, Y = n_y Fb.
__device__ __forceinline__ void flux_vjp(double gm1, const double U[4], const double X[4], const double Y[4], double Ub[4])
{
    const double ri = recip(U[0]);
    const double u = U[1] * ri, v = U[2] * ri;
    const double p = gm1 * (U[3] - 0.5 * (U[1] * u + U[2] * v));
    const double H = U[3] + p;
    const double Ku = X[0] * U[0] + X[1] * U[1] + X[2] * U[2] + X[3] * H;
    const double Kv = Y[0] * U[0] + Y[1] * U[1] + Y[2] * U[2] + Y[3] * H;
    const double Pp = X[1] + Y[2] + u * X[3] + v * Y[3];
    Ub[0] += -(Ku * u + Kv * v) * ri + u * X[0] + v * Y[0] + Pp * gm1 * 0.5 * (u * u + v * v);
    Ub[1] += Ku * ri + u * X[1] + v * Y[1] - Pp * gm1 * u;
    Ub[2] += Kv * ri + u * X[2] + v * Y[2] - Pp * gm1 * v;
    Ub[3] += u * X[3] + v * Y[3] + Pp * gm1;
}

// Cotangent of the local Lax-Friedrichs flux with respect to its left
// state: 1/2 A_n(UL)^T Fb + lambda/2 Fb - (sum_m Fb_m (UR_m - UL_m))/2
// d lambda_L/d UL, the last term only when lambda_L >= lambda_R (ties take
// the left branch); d lambda_L = sign(vn) d vn + d c, sign(0) = +1, and
// d c = c/(2p) d p - c/(2 rho) d rho.
__device__ __forceinline__ void llf_vjp_left(double gamma, double gm1, const double UL[4], const double UR[4], double nx,
                                             double ny, const double Fb[4], double Ub[4])
{
    const double riL = recip(UL[0]), riR = recip(UR[0]);
    const double uL = UL[1] * riL, vL = UL[2] * riL, uR = UR[1] * riR, vR = UR[2] * riR;
    const double pL = gm1 * (UL[3] - 0.5 * (UL[1] * uL + UL[2] * vL));
    const double pR = gm1 * (UR[3] - 0.5 * (UR[1] * uR + UR[2] * vR));
    const double vnL = uL * nx + vL * ny, vnR = uR * nx + vR * ny;
    const double cL = root(gamma * pL * riL), cR = root(gamma * pR * riR);
    const double lamL = fabs(vnL) + cL, lamR = fabs(vnR) + cR;
    const double lam = fmax(lamL, lamR);
    double X[4], Y[4], jump = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        X[m] = 0.5 * nx * Fb[m];
        Y[m] = 0.5 * ny * Fb[m];
        Ub[m] += 0.5 * lam * Fb[m];
        jump += Fb[m] * (UR[m] - UL[m]);
    }
    flux_vjp(gm1, UL, X, Y, Ub);
    if (lamL >= lamR) {
        const double lb = -0.5 * jump;
        const double sv = vnL >= 0.0 ? lb : -lb;  // cotangent of vn
        const double pb = lb * cL / (2.0 * pL);   // cotangent of p through c
        Ub[0] += -sv * vnL * riL - lb * cL * riL * 0.5 + pb * gm1 * 0.5 * (uL * uL + vL * vL);
        Ub[1] += sv * nx * riL - pb * gm1 * uL;
        Ub[2] += sv * ny * riL - pb * gm1 * vL;
        Ub[3] += pb * gm1;
    }
}

// Cotangent of the local Lax-Friedrichs flux with respect to its right
// state: 1/2 A_n(UR)^T Fb - lambda/2 Fb - (sum_m Fb_m (UR_m - UL_m))/2
// d lambda_R/d UR, the last term only when lambda_R > lambda_L (ties take
// the left branch, as in llf_vjp_left).
__device__ __forceinline__ void llf_vjp_right(double gamma, double gm1, const double UL[4], const double UR[4],
                                              double nx, double ny, const double Fb[4], double Ub[4])
{
    const double riL = recip(UL[0]), riR = recip(UR[0]);
    const double uL = UL[1] * riL, vL = UL[2] * riL, uR = UR[1] * riR, vR = UR[2] * riR;
    const double pL = gm1 * (UL[3] - 0.5 * (UL[1] * uL + UL[2] * vL));
    const double pR = gm1 * (UR[3] - 0.5 * (UR[1] * uR + UR[2] * vR));
    const double vnL = uL * nx + vL * ny, vnR = uR * nx + vR * ny;
    const double cL = root(gamma * pL * riL), cR = root(gamma * pR * riR);
    const double lamL = fabs(vnL) + cL, lamR = fabs(vnR) + cR;
    const double lam = fmax(lamL, lamR);
    double X[4], Y[4], jump = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        X[m] = 0.5 * nx * Fb[m];
        Y[m] = 0.5 * ny * Fb[m];
        Ub[m] += -0.5 * lam * Fb[m];
        jump += Fb[m] * (UR[m] - UL[m]);
    }
    flux_vjp(gm1, UR, X, Y, Ub);
    const double lb = lamL >= lamR ? 0.0 : -0.5 * jump;  // cotangent of lambda_R
    const double sv = vnR >= 0.0 ? lb : -lb;
    const double pb = lb * cR / (2.0 * pR);
    Ub[0] += -sv * vnR * riR - lb * cR * riR * 0.5 + pb * gm1 * 0.5 * (uR * uR + vR * vR);
    Ub[1] += sv * nx * riR - pb * gm1 * uR;
    Ub[2] += sv * ny * riR - pb * gm1 * vR;
    Ub[3] += pb * gm1;
}

// Cotangent of the flux on a side of kind bc (0 interior: llf_vjp_left
// alone; the neighbour adds its own part in gather form) with U_R the ghost
// state of U_L: the left cotangent plus the right one taken back through the
// ghost's Jacobian, the wall's reflection (its own transpose), the outflow's
// identity, or nothing for a prescribed state.  Selects, not branches.
__device__ __forceinline__ void llf_vjp_side(int bc, double gamma, double gm1, const double UL[4], const double UR[4],
                                             double nx, double ny, const double Fb[4], double Ub[4])
{
    llf_vjp_left(gamma, gm1, UL, UR, nx, ny, Fb, Ub);
    double Vb[4] = {0.0, 0.0, 0.0, 0.0};
    llf_vjp_right(gamma, gm1, UL, UR, nx, ny, Fb, Vb);
    const double s = bc == 1 ? 2.0 * (Vb[1] * nx + Vb[2] * ny) : 0.0;
    const bool back = bc == 1 || bc == 2;
    Ub[0] += back ? Vb[0] : 0.0;
    Ub[1] += back ? Vb[1] - s * nx : 0.0;
    Ub[2] += back ? Vb[2] - s * ny : 0.0;
    Ub[3] += back ? Vb[3] : 0.0;
}

// Vector-Jacobian product of the fused right-hand side, element-wise in
// gather form.  For element i the cotangent of its side trace at point k is
//   J_L(U_i, U_nb, n_i)^T (Fb_i(q, k) - Fb_nb(qn, p-k)),
// because the neighbour's flux on the shared edge is F(U_nb, U_i, -n_i) =
// -F(U_i, U_nb, n_i); Fb = -l omega_k (trace of Rbar/det J) on each side.
// So no cotangent is scattered into another element.  A domain-boundary
// side (BC variant) has no neighbour flux: Fb is the element's own, U_R is
// the ghost of U_L, and the ghost's cotangent returns to U_L (llf_vjp_side).
//   MODE 0: out = J(C)^T Rb
//   MODE 1: out = 2/3 Rb + 2/3 dt J(C)^T Rb          (adjoint of RK stage 3)
//   MODE 2: out = 1/4 Rb + 1/4 dt J(C)^T Rb          (adjoint of RK stage 2)
//   MODE 3: out = 1/3 X + 3/4 Y + Rb + dt J(C)^T Rb  (adjoint of RK stage 1)
template <int P, int MODE, bool BC>
__global__ __launch_bounds__(BLOCK) void k_stage_vjp(int n, int npad, const double* __restrict__ C,
                                                     const double* __restrict__ Rb, const double* __restrict__ X,
                                                     const double* __restrict__ Y, double* __restrict__ out,
                                                     const double* __restrict__ geo, const int* __restrict__ snb,
                                                     const int* __restrict__ sside, const double* __restrict__ sgeo,
                                                     const double* __restrict__ tab, double gamma, double dt,
                                                     const double* __restrict__ dt_dev, const int* __restrict__ sbc,
                                                     const double* __restrict__ bcs)
{
    using O = Ord<P>;
    constexpr int NP = O::NP, NQ = O::NQ, NE = O::NE;
    constexpr int SS = (NE * NP) | 1;
    __shared__ double phs[3 * SS];
    for (int i = threadIdx.x; i < 3 * NE * NP; i += BLOCK) phs[(i / (NE * NP)) * SS + i % (NE * NP)] = tab[O::PHS + i];
    __syncthreads();

    const int e = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    if (e >= npad) return;
    const int so = state_off(e, 4 * NP);
    if (e >= n) {
#pragma unroll
        for (int x = 0; x < 4 * NP; ++x) out[so + x * LANES] = 0.0;
        return;
    }
    const double gm1 = gamma - 1.0;
    const double* g = geo + state_off(e, 6);
    const double a00 = g[0], a01 = g[LANES], a10 = g[2 * LANES], a11 = g[3 * LANES], idet = g[4 * LANES];

    double c[4][NP], rs[4][NP], cb[4][NP];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            c[m][j] = C[so + (m * NP + j) * LANES];
            rs[m][j] = idet * Rb[so + (m * NP + j) * LANES];
            cb[m][j] = 0.0;
        }

    // volume: Grb = sum_j w dphi/dr Rs, Gsb likewise; Fxb = adj^T (Grb, Gsb)
#pragma unroll 1
    for (int k = 0; k < NQ; ++k) {
        double U[4], Xb[4], Yb[4], Ub[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            double u = 0.0, gr = 0.0, gs = 0.0;
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                u = fma(tab[O::PHI + k * NP + j], c[m][j], u);
                gr = fma(tab[O::DRW + k * NP + j], rs[m][j], gr);
                gs = fma(tab[O::DSW + k * NP + j], rs[m][j], gs);
            }
            U[m] = u;
            Xb[m] = a00 * gr + a10 * gs;
            Yb[m] = a01 * gr + a11 * gs;
        }
        flux_vjp(gm1, U, Xb, Yb, Ub);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int j = 0; j < NP; ++j) cb[m][j] = fma(tab[O::PHI + k * NP + j], Ub[m], cb[m][j]);
    }

    // surface
    const int sides = sside[state_off(e, 1)];
    const int bcv = BC ? sbc[state_off(e, 1)] : 0;
    double G[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) G[m] = BC ? bcs[m] : 0.0;
#pragma unroll 1
    for (int q = 0; q < 3; ++q) {
        const int nb = snb[state_off(e, 3) + q * LANES];
        const int qn = (sides >> (2 * q)) & 3;
        const int bc = (bcv >> (4 * q)) & 15;
        const int go = state_off(e, 9) + 3 * q * LANES;
        const double nx = sgeo[go], ny = sgeo[go + LANES], hl = sgeo[go + 2 * LANES];
        const double idn = geo[state_off(nb, 6) + 4 * LANES];
        double UR[NE][4], RR[NE][4];
#pragma unroll
        for (int k = 0; k < NE; ++k)
#pragma unroll
            for (int m = 0; m < 4; ++m) UR[k][m] = RR[k][m] = 0.0;
        const int nbo = state_off(nb, 4 * NP);
        const double* tq = phs + qn * SS;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            double cv[4], rv[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                cv[m] = C[nbo + (m * NP + j) * LANES];
                rv[m] = idn * Rb[nbo + (m * NP + j) * LANES];
            }
#pragma unroll
            for (int k = 0; k < NE; ++k) {
                const double t = tq[(NE - 1 - k) * NP + j];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    UR[k][m] = fma(t, cv[m], UR[k][m]);
                    RR[k][m] = fma(t, rv[m], RR[k][m]);
                }
            }
        }
#pragma unroll 1
        for (int k = 0; k < NE; ++k) {
            const double* tl = tab + O::PHS + (q * NE + k) * NP;
            double UL[4], Fb[4], Ub[4] = {0.0, 0.0, 0.0, 0.0};
            const double w = -hl * tab[O::GW + k];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                double u = 0.0, r = 0.0;
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    u = fma(tl[j], c[m][j], u);
                    r = fma(tl[j], rs[m][j], r);
                }
                UL[m] = u;
                Fb[m] = w * (r - (bc ? 0.0 : RR[k][m]));
            }
            if constexpr (BC) {
                ghost_state<double>(bc, UL, nx, ny, G, UR[k]);
                llf_vjp_side(bc, gamma, gm1, UL, UR[k], nx, ny, Fb, Ub);
            } else {
                llf_vjp_left(gamma, gm1, UL, UR[k], nx, ny, Fb, Ub);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int j = 0; j < NP; ++j) cb[m][j] = fma(tl[j], Ub[m], cb[m][j]);
        }
    }

    const double h = MODE == 0 ? 1.0 : (dt_dev ? dt_dev[0] : dt);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const int x = so + (m * NP + j) * LANES;
            if constexpr (MODE == 0) {
                out[x] = cb[m][j];
            } else if constexpr (MODE == 1) {
                out[x] = (2.0 / 3.0) * Rb[x] + (2.0 / 3.0) * (h * cb[m][j]);
            } else if constexpr (MODE == 2) {
                out[x] = 0.25 * Rb[x] + 0.25 * (h * cb[m][j]);
            } else {
                out[x] = (1.0 / 3.0) * X[x] + 0.75 * Y[x] + Rb[x] + h * cb[m][j];
            }
        }
}

// The adjoint with 4 lanes per element, organised as k_stage4: lane m owns
// variable m for the contractions (state, right-hand-side cotangent and the
// neighbours' ones), points are taken four at a time, and two transposes
// through LDS let lane i evaluate the full closed-form cotangent (flux_vjp,
// llf_vjp_left) at point i once and hand component m back to lane m.
// Modes as k_stage_vjp.
template <int P, int MODE, bool BC>
__global__ __launch_bounds__(BLOCK) void k_stage_vjp4(int n, int npad, const double* __restrict__ C,
                                                      const double* __restrict__ Rb, const double* __restrict__ X,
                                                      const double* __restrict__ Y, double* __restrict__ out,
                                                      const double* __restrict__ geo, const int* __restrict__ snb,
                                                      const int* __restrict__ sside, const double* __restrict__ sgeo,
                                                      const double* __restrict__ tab, double gamma, double dt,
                                                      const double* __restrict__ dt_dev, const int* __restrict__ sbc,
                                                      const double* __restrict__ bcs)
{
    using O = Ord<P>;
    constexpr int NP = O::NP, NQ = O::NQ, NE = O::NE;
    constexpr int SS = (NE * NP) | 1;
    __shared__ double phs[3 * SS];
    __shared__ Pair<double> xa[(BLOCK / 4) * XQUAD];
    __shared__ Pair<double> xb[(BLOCK / 4) * XQUAD];
    load_side_tables<P, double>(tab, phs);

    const int e = xcd_block(blockIdx.x, gridDim.x) * (BLOCK / 4) + (threadIdx.x >> 2);
    const int m = threadIdx.x & 3;
    if (e >= npad) return;  // whole workgroups leave together (npad % 64 == 0)
    const bool real = e < n;
    const int so = state_off(e, 4 * NP) + m * NP * LANES;
    const double gm1 = gamma - 1.0;
    const double* g = geo + state_off(e, 6);
    const double a00 = g[0], a01 = g[LANES], a10 = g[2 * LANES], a11 = g[3 * LANES], idet = g[4 * LANES];
    Pair<double>* const ra = xa + (threadIdx.x >> 2) * XQUAD;
    Pair<double>* const rb = xb + (threadIdx.x >> 2) * XQUAD;

    double c[NP], rs[NP], cb[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        c[j] = C[so + j * LANES];
        rs[j] = idet * Rb[so + j * LANES];
        cb[j] = 0.0;
    }

    // the neighbours' coefficients and right-hand-side cotangents of this
    // lane's variable; up to p = 3 the next side's are requested while a
    // side is computed
    constexpr int PF = P <= 3 ? 2 : 1;
    const int sides = sside[state_off(e, 1)];
    const int* const nbp = snb + state_off(e, 3);
    double cn[PF][NP], rn[PF][NP];
#pragma unroll
    for (int r = 0; r < PF; ++r) {
        const int nb = nbp[r * LANES];
        const double idn = geo[state_off(nb, 6) + 4 * LANES];
        const int o = state_off(nb, 4 * NP) + m * NP * LANES;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            cn[r][j] = C[o + j * LANES];
            rn[r][j] = idn * Rb[o + j * LANES];
        }
    }

    // volume: U, and the cotangents X, Y of the x and y fluxes, at four points
#pragma unroll 1
    for (int k0 = 0; k0 < NQ; k0 += 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = min(k0 + i, NQ - 1);
            const double um = dot2<NP>(tab + O::PHI + k * NP, c);
            const double gr = dot2<NP>(tab + O::DRW + k * NP, rs);
            const double gs = dot2<NP>(tab + O::DSW + k * NP, rs);
            ra[i * XROW + m] = Pair<double>{um, a00 * gr + a10 * gs};
            rb[i * XROW + m].a = a01 * gr + a11 * gs;
        }
        wave_sync();
        double U[4], Xv[4], Yv[4], Ub[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const Pair<double> t = ra[m * XROW + v];
            U[v] = t.a;
            Xv[v] = t.b;
            Yv[v] = rb[m * XROW + v].a;
        }
        flux_vjp(gm1, U, Xv, Yv, Ub);
        wave_sync();
#pragma unroll
        for (int v = 0; v < 4; ++v) ra[m * XROW + v].a = Ub[v];
        wave_sync();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = k0 + i;
            if (k < NQ) {
                const double ub = ra[i * XROW + m].a;
                const double* tp = tab + reload(O::PHI + k * NP);
#pragma unroll
                for (int j = 0; j < NP; ++j) cb[j] = fma(tp[j], ub, cb[j]);
            }
        }
        wave_sync();
    }

    // surface: traces of both sides and the flux cotangent Fb at four points
    const int bcv = BC ? sbc[state_off(e, 1)] : 0;
    double G[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) G[v] = BC ? bcs[v] : 0.0;
#pragma unroll 1
    for (int q = 0; q < 3; ++q) {
        const int qn = (sides >> (2 * q)) & 3;
        const int bc = (bcv >> (4 * q)) & 15;
        const int go = state_off(e, 9) + 3 * q * LANES;
        const double nx = sgeo[go], ny = sgeo[go + LANES], hl = sgeo[go + 2 * LANES];
        const lds_ptr<double> tq = lds_row(phs, qn * SS);
#pragma unroll 1
        for (int k0 = 0; k0 < NE; k0 += 4) {
            // (one point at a time: the neighbour's side table comes from LDS
            // into vector registers, four rows at once would not fit at p = 5)
#pragma unroll 1
            for (int i = 0; i < 4; ++i) {
                const int k = min(k0 + i, NE - 1);
                const double* tl = tab + O::PHS + (q * NE + k) * NP;
                const double ul = dot2<NP>(tl, c), rl = dot2<NP>(tl, rs);
                const double ur = dot2<NP>(tq + k * NP, cn[0]), rr = dot2<NP>(tq + k * NP, rn[0]);
                ra[i * XROW + m] = Pair<double>{ul, ur};
                rb[i * XROW + m].a = -hl * tab[O::GW + k] * (rl - (bc ? 0.0 : rr));
            }
            wave_sync();
            double UL[4], UR[4], Fb[4], Ub[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const Pair<double> t = ra[m * XROW + v];
                UL[v] = t.a;
                UR[v] = t.b;
                Fb[v] = rb[m * XROW + v].a;
            }
            if constexpr (BC) {
                ghost_state<double>(bc, UL, nx, ny, G, UR);
                llf_vjp_side(bc, gamma, gm1, UL, UR, nx, ny, Fb, Ub);
            } else {
                llf_vjp_left(gamma, gm1, UL, UR, nx, ny, Fb, Ub);
            }
            wave_sync();
#pragma unroll
            for (int v = 0; v < 4; ++v) ra[m * XROW + v].a = Ub[v];
            wave_sync();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = k0 + i;
                if (k < NE) {
                    const double ub = ra[i * XROW + m].a;
                    const double* tl = tab + reload(O::PHS + (q * NE + k) * NP);
#pragma unroll
                    for (int j = 0; j < NP; ++j) cb[j] = fma(tl[j], ub, cb[j]);
                }
            }
            wave_sync();
        }
        // the next side's neighbour moves to the front
#pragma unroll
        for (int r = 0; r + 1 < PF; ++r)
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                cn[r][j] = cn[r + 1][j];
                rn[r][j] = rn[r + 1][j];
            }
        if (q + PF < 3) {
            const int nb = nbp[(q + PF) * LANES];
            const double idn = geo[state_off(nb, 6) + 4 * LANES];
            const int o = state_off(nb, 4 * NP) + m * NP * LANES;
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                cn[PF - 1][j] = C[o + j * LANES];
                rn[PF - 1][j] = idn * Rb[o + j * LANES];
            }
        }
    }

    const double h = MODE == 0 ? 1.0 : (dt_dev ? dt_dev[0] : dt);
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const int x = so + j * LANES;
        if (!real) {
            out[x] = 0.0;
        } else if constexpr (MODE == 0) {
            out[x] = cb[j];
        } else if constexpr (MODE == 1) {
            out[x] = (2.0 / 3.0) * Rb[x] + (2.0 / 3.0) * (h * cb[j]);
        } else if constexpr (MODE == 2) {
            out[x] = 0.25 * Rb[x] + 0.25 * (h * cb[j]);
        } else {
            out[x] = (1.0 / 3.0) * X[x] + 0.75 * Y[x] + Rb[x] + h * cb[j];
        }
    }
}

// The adjoint of k_stage_mx (modes as k_stage_vjp), FP64, one wavefront per
// 16-element block with every contraction a 16 x 16 x 4 product: at the
// volume points the state (phi) and the scaled cotangent's flux cotangents
// (w grad phi, transposed tables) are evaluated, flux_vjp gives the
// point's state cotangent and phi lifts it back (transposed layout); at the
// side points the traces of the state and of the scaled cotangent, own and
// the neighbour's (through LDS as in k_stage_mx), give the numerical flux's
// cotangent, llf_vjp_left (llf_vjp_side on boundary sides) the state
// cotangent, and the side table lifts it.  Lane layout and result order as
// in k_stage_mx.
template <int P, int MODE, bool BC>
__global__ __launch_bounds__(BLOCK) void k_stage_vjp_mx(int n, int npad, const double* __restrict__ C,
                                                        const double* __restrict__ Rb, const double* __restrict__ X,
                                                        const double* __restrict__ Y, double* __restrict__ out,
                                                        const double* __restrict__ geo, const int* __restrict__ snb,
                                                        const int* __restrict__ sside,
                                                        const double* __restrict__ sgeo,
                                                        const double* __restrict__ tmx,
                                                        const double* __restrict__ tab, double gamma, double dt,
                                                        const double* __restrict__ dt_dev,
                                                        const int* __restrict__ sbc, const double* __restrict__ bcs)
{
    using O = Ord<P>;
    constexpr MxLayout L = mx_layout(P);
    constexpr int NP = L.np, NE = L.ne, NS = L.ns, KP = L.kp, TQ = L.tq, TS = L.ts, TM = L.tm;
    constexpr int NW = BLOCK / WAVE;
    constexpr int NVH = 2;
    __shared__ double xc[NW][3][4][NE][LANES];  // the neighbours' state traces facing each side
    __shared__ double xr[NW][3][4][NE][LANES];  // and their scaled cotangents' traces

    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE, j = lane % 16, g = lane / 16;
    const int blk = lb * NW + w;
    if (lb * NW * LANES >= npad) return;  // whole workgroups leave together (npad % 64 == 0)
    const int e = blk * LANES + j;
    const bool real = e < n;
    auto row = [&](int r) { return mx_row<true>(g, r); };
    const double* gp = geo + state_off(e, 6);
    const double a00 = gp[0], a01 = gp[LANES], a10 = gp[2 * LANES], a11 = gp[3 * LANES], idet = gp[4 * LANES];
    const double gm1 = gamma - 1.0;
    const int base = blk * 4 * NP * LANES + j;
    const double* tl = tmx + lane;
    auto A = [&](int b) { return tl[b * WAVE]; };

    // own state and right-hand-side cotangent, modes 4s+g; up to p = 3 the
    // cotangent is kept as read, for the stage combination, and scaled by
    // 1/det J where it enters a contraction; from p = 4 on it is kept
    // scaled and read again for the combination (the registers it would
    // hold cost more there)
    constexpr bool KEEP = P <= 3;
    double c[4][KP], rv[4][KP];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int s = 0; s < KP; ++s) {
            const int x = base + (v * NP + min(4 * s + g, NP - 1)) * LANES;
            c[v][s] = C[x];
            rv[v][s] = KEEP ? Rb[x] : idet * Rb[x];
        }
    auto rs = [&](int v, int s) { return KEEP ? idet * rv[v][s] : rv[v][s]; };
    dx4 acc[4][TM];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int t = 0; t < TM; ++t) acc[v][t] = dx4{0.0, 0.0, 0.0, 0.0};

    // volume: U and the flux cotangents at the lane's four points per tile
#pragma unroll
    for (int tq = 0; tq < TQ; ++tq) {
        dx4 u[4], gr[4], gs[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) u[v] = gr[v] = gs[v] = dx4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KP; ++s) {
            const double a = A(L.phi + tq * KP + s), ar = A(L.dre + tq * KP + s), as = A(L.dse + tq * KP + s);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                u[v] = mfma16(a, c[v][s], u[v]);
                gr[v] = mfma16(ar, rs(v, s), gr[v]);
                gs[v] = mfma16(as, rs(v, s), gs[v]);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double U[4], Xv[4], Yv[4], Ub[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                U[v] = u[v][r];
                Xv[v] = a00 * gr[v][r] + a10 * gs[v][r];
                Yv[v] = a01 * gr[v][r] + a11 * gs[v][r];
            }
            flux_vjp(gm1, U, Xv, Yv, Ub);
#pragma unroll
            for (int tm = 0; tm < TM; ++tm) {
                const double a = A(L.phl + (tm * TQ + tq) * 4 + r);
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v][tm] = mfma16(a, Ub[v], acc[v][tm]);
            }
        }
    }

    // the neighbours' traces of state and scaled cotangent, the points
    // facing each side kept in LDS (reversed)
    const int sides = sside[state_off(e, 1)];
    const int* const nb = snb + state_off(e, 3);
#pragma unroll 1
    for (int q = 0; q < 3; ++q) {
        const int ne_ = nb[q * LANES];
        const int nbase = state_off(ne_, 4 * NP);
        const double idn = geo[state_off(ne_, 6) + 4 * LANES];
        const int qn = (sides >> (2 * q)) & 3;
#pragma unroll
        for (int v0 = 0; v0 < 4; v0 += NVH) {
            double cn[NVH][KP], rn[NVH][KP];
#pragma unroll
            for (int v = 0; v < NVH; ++v)
#pragma unroll
                for (int s = 0; s < KP; ++s) {
                    const int x = nbase + ((v0 + v) * NP + min(4 * s + g, NP - 1)) * LANES;
                    cn[v][s] = C[x];
                    rn[v][s] = idn * Rb[x];
                }
#pragma unroll
            for (int ts = 0; ts < TS; ++ts) {
                dx4 tc[NVH], tr[NVH];
#pragma unroll
                for (int v = 0; v < NVH; ++v) tc[v] = tr[v] = dx4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < KP; ++s) {
                    const double a = A(L.pe + ts * KP + s);
#pragma unroll
                    for (int v = 0; v < NVH; ++v) {
                        tc[v] = mfma16(a, cn[v][s], tc[v]);
                        tr[v] = mfma16(a, rn[v][s], tr[v]);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = 16 * ts + row(r) - qn * NE;  // point of the neighbour's side qn
                    if (k >= 0 && k < NE) {
#pragma unroll
                        for (int v = 0; v < NVH; ++v) {
                            xc[w][q][v0 + v][NE - 1 - k][j] = tc[v][r];
                            xr[w][q][v0 + v][NE - 1 - k][j] = tr[v][r];
                        }
                    }
                }
            }
        }
    }
    wave_sync();

    // stage 3 combines two more cotangents: requested here, used at the end
    double xv[MODE == 3 ? 4 : 1][MODE == 3 ? KP : 1], yv[MODE == 3 ? 4 : 1][MODE == 3 ? KP : 1];
    if constexpr (MODE == 3) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int s = 0; s < KP; ++s) {
                const int x = base + (v * NP + min(4 * s + g, NP - 1)) * LANES;
                xv[v][s] = __builtin_nontemporal_load(&X[x]);
                yv[v][s] = __builtin_nontemporal_load(&Y[x]);
            }
    }

    // own traces, the numerical flux's cotangent and its state cotangent at
    // each side point, lifted with the side table
    const int bcv = BC ? sbc[state_off(e, 1)] : 0;
    double G[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) G[v] = BC ? bcs[v] : 0.0;
#pragma unroll
    for (int ts = 0; ts < TS; ++ts) {
        dx4 ul[4], rl[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) ul[v] = rl[v] = dx4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KP; ++s) {
            const double a = A(L.pe + ts * KP + s);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                ul[v] = mfma16(a, c[v][s], ul[v]);
                rl[v] = mfma16(a, rs(v, s), rl[v]);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int sp = 16 * ts + row(r);
            const int q = min(sp / NE, 2);
            const bool pad = sp >= NS;
            const int k = min(sp - q * NE, NE - 1);
            const int go = state_off(e, 9) + 3 * q * LANES;
            const double nx = sgeo[go], ny = sgeo[go + LANES], hl = sgeo[go + 2 * LANES];
            const int bc = BC ? (bcv >> (4 * q)) & 15 : 0;
            const double wk = -hl * tab[O::GW + k];
            double UL[4], UR[4], Fb[4], Ub[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                UL[v] = ul[v][r];
                UR[v] = pad ? UL[v] : xc[w][q][v][k][j];
                const double rr = (pad || bc) ? 0.0 : xr[w][q][v][k][j];
                Fb[v] = wk * (rl[v][r] - rr);
            }
            if constexpr (BC) {
                ghost_state<double>(bc, UL, nx, ny, G, UR);
                llf_vjp_side(bc, gamma, gm1, UL, UR, nx, ny, Fb, Ub);
            } else {
                llf_vjp_left(gamma, gm1, UL, UR, nx, ny, Fb, Ub);
            }
#pragma unroll
            for (int tm = 0; tm < TM; ++tm) {
                const double a = A(L.pel + (tm * TS + ts) * 4 + r);
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v][tm] = mfma16(a, Ub[v], acc[v][tm]);
            }
        }
    }

    const double h = MODE == 0 ? 1.0 : (dt_dev ? dt_dev[0] : dt);
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int s = 0; s < KP; ++s) {
            const int jm = 4 * s + g;
            if (jm < NP) {
                const int x = base + (v * NP + jm) * LANES;
                const double cb = acc[v][s / 4][s % 4];
                const double rb = KEEP ? rv[v][s] : Rb[x];
                double val;
                if (!real) {
                    val = 0.0;
                } else if constexpr (MODE == 0) {
                    val = cb;
                } else if constexpr (MODE == 1) {
                    val = (2.0 / 3.0) * rb + (2.0 / 3.0) * (h * cb);
                } else if constexpr (MODE == 2) {
                    val = 0.25 * rb + 0.25 * (h * cb);
                } else {
                    val = (1.0 / 3.0) * xv[v][s] + 0.75 * yv[v][s] + rb + h * cb;
                }
                __builtin_nontemporal_store(val, &out[x]);
            }
        }
}

// U_h at the volume points, user order [N][NQ][4] (a1 on its own, for
// functionals of the solution)
template <int P>
__global__ __launch_bounds__(BLOCK) void k_eval_points(int n, const int* __restrict__ perm, const double* __restrict__ C,
                                                       double* __restrict__ u, const double* __restrict__ tab)
{
    using O = Ord<P>;
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= n) return;
    const int so = state_off(e, 4 * O::NP);
    double* o = u + (size_t)perm[e] * O::NQ * 4;
    for (int k = 0; k < O::NQ; ++k)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < O::NP; ++j) s = fma(tab[O::PHI + k * O::NP + j], C[so + (m * O::NP + j) * LANES], s);
            o[k * 4 + m] = s;
        }
}

// physical quadrature weights det J_i * w_k, user order [N][NQ]
template <int P>
__global__ __launch_bounds__(BLOCK) void k_quad_weights(int n, const int* __restrict__ perm,
                                                        const double* __restrict__ vtx, double* __restrict__ wq,
                                                        const double* __restrict__ tab)
{
    using O = Ord<P>;
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= n) return;
    const double* v = vtx + (size_t)e * 6;
    const double det = (v[2] - v[0]) * (v[5] - v[1]) - (v[4] - v[0]) * (v[3] - v[1]);
    double* o = wq + (size_t)perm[e] * O::NQ;
    for (int k = 0; k < O::NQ; ++k) o[k] = det * tab[O::QW + k];
}

// ---------------------------------------------------------------- CFL step
// dt = cfl * min_i r_i / (|v_i| + c_i) over cell averages sqrt(2) c_{i,0};
// a non-physical or NaN mean makes the result NaN.  min is exact, so the
// two-pass reduction is bitwise reproducible.
template <int P>
__global__ __launch_bounds__(BLOCK) void k_dt_partial(int n, const double* __restrict__ C, const double* __restrict__ geo,
                                                      double gamma, double* __restrict__ partial)
{
    using O = Ord<P>;
    __shared__ double red[BLOCK];
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    double val = INFINITY;
    if (e < n) {
        const int so = state_off(e, 4 * O::NP);
        val = dt_local(gamma, geo[state_off(e, 6) + 5 * LANES], C[so], C[so + O::NP * LANES], C[so + 2 * O::NP * LANES],
                       C[so + 3 * O::NP * LANES]);
    }
    const double mn = block_min(val, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = mn;
}

// L2 projection of point values (user order [N][NQ][4]) onto the
// orthonormal basis: c_j = sum_k w_k phi_j(r_k) u_k (mass = det J * I).
template <int P>
__global__ __launch_bounds__(BLOCK) void k_project(int n, int npad, const int* __restrict__ perm,
                                                   const double* __restrict__ uq, double* __restrict__ C,
                                                   const double* __restrict__ tab)
{
    using O = Ord<P>;
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= npad) return;
    const int so = state_off(e, 4 * O::NP);
    if (e >= n) {
        for (int x = 0; x < 4 * O::NP; ++x) C[so + x * LANES] = 0.0;
        return;
    }
    const double* u = uq + (size_t)perm[e] * O::NQ * 4;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < O::NP; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < O::NQ; ++k) s = fma(tab[O::QW + k] * tab[O::PHI + k * O::NP + j], u[k * 4 + m], s);
            C[so + (m * O::NP + j) * LANES] = s;
        }
}

// physical volume points, user order [N][NQ][2]
template <int P>
__global__ __launch_bounds__(BLOCK) void k_quad_points(int n, const int* __restrict__ perm,
                                                       const double* __restrict__ vtx, double* __restrict__ xy,
                                                       const double* __restrict__ tab)
{
    using O = Ord<P>;
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= n) return;
    const double* v = vtx + (size_t)e * 6;
    double* o = xy + (size_t)perm[e] * O::NQ * 2;
    for (int k = 0; k < O::NQ; ++k) {
        const double r = tab[O::QR + k], s = tab[O::QS + k], l1 = 1.0 - r - s;
        o[2 * k] = v[0] * l1 + v[2] * r + v[4] * s;
        o[2 * k + 1] = v[1] * l1 + v[3] * r + v[5] * s;
    }
}

// ---------------------------------------------------------------- per-order launchers
static inline dim3 grid_for(int n) { return dim3((n + BLOCK - 1) / BLOCK); }

// Launch of k_stage<P, MODE, float, BC> (one lane per element, FP32).  The
// translation units that define DG_DEFINE_STAGE1_F32 instantiate it: p = 1
// with the other p = 1 kernels, p = 2..5 in a unit of their own compiled with
// the scheduler strategy that groups memory instructions into clauses.
// Issuing the neighbour gathers together cuts this kernel's time by a fifth
// to two fifths at p = 3; at p = 1 it costs 3%, and for the FP64 kernels it
// is neutral or slightly slower.
template <int P, int MODE, bool BC>
void stage1_f32(const MeshDev& m, const float* tab, const double* C, const double* U0, double* out, double dt,
                const double* dt_dev, const StageGen& gs, hipStream_t s)
#ifdef DG_DEFINE_STAGE1_F32
{
    const int nb = (m.npad + BLOCK - 1) / BLOCK;
    dim3 g((nb + 7) / 8 * 8);
    k_stage<P, MODE, float, BC><<<g, BLOCK, 0, s>>>(m.n, m.npad, C, U0, out, m.geo, m.side_nb, m.side_q, m.side_g,
                                                    tab, m.tab, m.gamma, dt, dt_dev, gs, m.side_bc, m.bc_state);
}
#define DG_STAGE1_F32(P, MODE, BC)                                                                               \
    template void stage1_f32<P, MODE, BC>(const MeshDev&, const float*, const double*, const double*, double*, \
                                          double, const double*, const StageGen&, hipStream_t);
#define DG_STAGE1_F32_MODES(P, BC) \
    DG_STAGE1_F32(P, 0, BC)        \
    DG_STAGE1_F32(P, 1, BC)        \
    DG_STAGE1_F32(P, 2, BC)        \
    DG_STAGE1_F32(P, 3, BC)        \
    DG_STAGE1_F32(P, 4, BC)
#define DG_STAGE1_F32_ORDER(P)    \
    DG_STAGE1_F32_MODES(P, false) \
    DG_STAGE1_F32_MODES(P, true)
#else
    ;
#endif

template <int P>
struct Launch {
    static void traces(const MeshDev& m, const double* C, double* T, hipStream_t s, double* Rz)
    {
        k_traces<P><<<grid_for(m.n), BLOCK, 0, s>>>(m.n, C, T, m.tab, Rz);
    }
    static void edge_lift(const MeshDev& m, const double* T, double* R, hipStream_t s)
    {
        for (int c = 0; c < m.ncolour; ++c) {
            const int e0 = m.colour_off[c], e1 = m.colour_off[c + 1];
            if (e1 > e0)
                k_edge_lift<P><<<grid_for(e1 - e0), BLOCK, 0, s>>>(e0, e1, m.nedge, m.ecol, m.ecol + m.nedge,
                                                                   m.ecol + 2 * m.nedge, m.edge_gc, T, R, m.tab,
                                                                   m.gamma, m.bc_state);
        }
    }
    static void edge_flux(const MeshDev& m, const double* T, double* S, hipStream_t s)
    {
        k_edge<P><<<grid_for(m.nedge), BLOCK, 0, s>>>(m.nedge, m.edge_l, m.edge_r, m.edge_sd, m.edge_g, T, S, m.tab,
                                                      m.gamma, m.bc_state);
    }
    static void element(const MeshDev& m, int mode, const double* C, const double* U0, double* out, const double* S,
                        double dt, const double* dt_dev, double* Tn, hipStream_t s, double* Racc, int src)
    {
        if (src == SRC_RACC)
            element_t<SRC_RACC>(m, mode, C, U0, out, S, dt, dt_dev, Tn, s, Racc);
        else if (src == SRC_VOLUME)
            element_t<SRC_VOLUME>(m, mode, C, U0, out, S, dt, dt_dev, Tn, s, Racc);
        else
            element_t<SRC_SLOTS>(m, mode, C, U0, out, S, dt, dt_dev, Tn, s, Racc);
    }
    static void volume(const MeshDev& m, const double* C, double* V, hipStream_t s)
    {
        k_volume<P><<<grid_for(m.n), BLOCK, 0, s>>>(m.n, C, V, m.geo, m.tab, m.gamma - 1.0);
    }
    template <int SRC>
    static void element_t(const MeshDev& m, int mode, const double* C, const double* U0, double* out,
                          const double* S, double dt, const double* dt_dev, double* Tn, hipStream_t s, double* Racc)
    {
        const double gm1 = m.gamma - 1.0;
        dim3 g = grid_for(m.npad);
#define DG_ELEM(MODE, TR)                                                                                     \
    k_element<P, MODE, TR, SRC><<<g, BLOCK, 0, s>>>(m.n, m.npad, C, U0, out, S, m.geo, m.tab, gm1, dt, dt_dev, \
                                                     Tn, Racc)
        switch (mode) {
        case 0: DG_ELEM(0, false); break;
        case 1: if (Tn) DG_ELEM(1, true); else DG_ELEM(1, false); break;
        case 2: if (Tn) DG_ELEM(2, true); else DG_ELEM(2, false); break;
        default: if (Tn) DG_ELEM(3, true); else DG_ELEM(3, false); break;
        }
#undef DG_ELEM
    }
    static void stage(const MeshDev& m, int mode, bool mixed, const double* C, const double* U0, double* out,
                      double dt, const double* dt_dev, hipStream_t s, const FusedDt& fz = FusedDt(),
                      const StageGen& gs = StageGen())
    {
        if (mixed)
            m.has_bc ? stage_t<float, true>(m, mode, m.tab32, C, U0, out, dt, dt_dev, s, fz, gs)
                     : stage_t<float, false>(m, mode, m.tab32, C, U0, out, dt, dt_dev, s, fz, gs);
        else
            m.has_bc ? stage_t<double, true>(m, mode, m.tab, C, U0, out, dt, dt_dev, s, fz, gs)
                     : stage_t<double, false>(m, mode, m.tab, C, U0, out, dt, dt_dev, s, fz, gs);
    }
    template <typename T, bool BC>
    static void stage_t(const MeshDev& m, int mode, const T* tab, const double* C, const double* U0, double* out,
                        double dt, const double* dt_dev, hipStream_t s, const FusedDt& fz, const StageGen& gs)
    {
        switch (mode) {
        case 0: stage_m<0, T, BC>(m, tab, C, U0, out, dt, dt_dev, s, fz, gs); break;
        case 1: stage_m<1, T, BC>(m, tab, C, U0, out, dt, dt_dev, s, fz, gs); break;
        case 2: stage_m<2, T, BC>(m, tab, C, U0, out, dt, dt_dev, s, fz, gs); break;
        case 3: stage_m<3, T, BC>(m, tab, C, U0, out, dt, dt_dev, s, fz, gs); break;
        default: stage_m<4, T, BC>(m, tab, C, U0, out, dt, dt_dev, s, fz, gs); break;
        }
    }
    template <int MODE, typename T, bool BC>
    static void stage_m(const MeshDev& m, const T* tab, const double* C, const double* U0, double* out, double dt,
                        const double* dt_dev, hipStream_t s, const FusedDt& fz, const StageGen& gs)
    {
        // (one lane per element only up to p = 3: from p = 4 on its values
        // exceed a lane's registers, and the library refuses it)
        constexpr bool F64 = sizeof(T) == sizeof(double);
        if (F64 ? m.mx : m.mx32) {
            dim3 g4((((m.npad + 63) / 64) + 7) / 8 * 8);
            const T* tmx = F64 ? (const T*)m.tabmx : (const T*)m.tabmx32;
            k_stage_mx<P, MODE, T, BC><<<g4, BLOCK, 0, s>>>(m.n, m.npad, C, U0, out, m.geo, m.side_nb, m.side_q,
                                                            m.side_g, tmx, m.tab, m.gamma, dt, dt_dev, fz.pin,
                                                            fz.pin_count, fz.cfl, fz.dt_store, fz.dt_hist, fz.pout,
                                                            gs, m.side_bc, m.bc_state);
            return;
        }
        if (P >= 4 || m.lanes4) {
            dim3 g4((((m.npad + 63) / 64) + 7) / 8 * 8);
            k_stage4<P, MODE, T, BC><<<g4, BLOCK, 0, s>>>(m.n, m.npad, C, U0, out, m.geo, m.side_nb, m.side_q,
                                                          m.side_g, tab, m.tab, m.gamma, dt, dt_dev, fz.pin,
                                                          fz.pin_count, fz.cfl, fz.dt_store, fz.dt_hist, fz.pout, gs,
                                                          m.side_bc, m.bc_state);
        } else if constexpr (P >= 4) {
        } else if constexpr (sizeof(T) != sizeof(double)) {
            stage1_f32<P, MODE, BC>(m, tab, C, U0, out, dt, dt_dev, gs, s);
        } else {
            const int nb = (m.npad + BLOCK - 1) / BLOCK;
            dim3 g((nb + 7) / 8 * 8);
            k_stage<P, MODE, T, BC><<<g, BLOCK, 0, s>>>(m.n, m.npad, C, U0, out, m.geo, m.side_nb, m.side_q,
                                                        m.side_g, tab, m.tab, m.gamma, dt, dt_dev, gs, m.side_bc,
                                                        m.bc_state);
        }
    }
    static void stage_vjp(const MeshDev& m, int mode, const double* C, const double* Rb, const double* X,
                          const double* Y, double* out, double dt, const double* dt_dev, hipStream_t s)
    {
        if (m.has_bc)
            stage_vjp_t<true>(m, mode, C, Rb, X, Y, out, dt, dt_dev, s);
        else
            stage_vjp_t<false>(m, mode, C, Rb, X, Y, out, dt, dt_dev, s);
    }
    template <bool BC>
    static void stage_vjp_t(const MeshDev& m, int mode, const double* C, const double* Rb, const double* X,
                            const double* Y, double* out, double dt, const double* dt_dev, hipStream_t s)
    {
        if (m.mx_vjp) {
            dim3 g4((((m.npad + 63) / 64) + 7) / 8 * 8);
#define DG_VJPMX(MODE)                                                                                          \
    k_stage_vjp_mx<P, MODE, BC><<<g4, BLOCK, 0, s>>>(m.n, m.npad, C, Rb, X, Y, out, m.geo, m.side_nb, m.side_q, \
                                                     m.side_g, m.tabmx, m.tab, m.gamma, dt, dt_dev, m.side_bc,  \
                                                     m.bc_state)
            switch (mode) {
            case 0: DG_VJPMX(0); break;
            case 1: DG_VJPMX(1); break;
            case 2: DG_VJPMX(2); break;
            default: DG_VJPMX(3); break;
            }
#undef DG_VJPMX
            return;
        }
        if (P >= 4 || m.vjp_lanes4) {
            dim3 g4((((m.npad + 63) / 64) + 7) / 8 * 8);
#define DG_VJP4(MODE)                                                                                                  \
    k_stage_vjp4<P, MODE, BC><<<g4, BLOCK, 0, s>>>(m.n, m.npad, C, Rb, X, Y, out, m.geo, m.side_nb, m.side_q, m.side_g, \
                                                   m.tab, m.gamma, dt, dt_dev, m.side_bc, m.bc_state)
            switch (mode) {
            case 0: DG_VJP4(0); break;
            case 1: DG_VJP4(1); break;
            case 2: DG_VJP4(2); break;
            default: DG_VJP4(3); break;
            }
#undef DG_VJP4
            return;
        }
        if constexpr (P <= 3) {
        const int nb = (m.npad + BLOCK - 1) / BLOCK;
        dim3 g((nb + 7) / 8 * 8);
#define DG_VJP(MODE)                                                                                                 \
    k_stage_vjp<P, MODE, BC><<<g, BLOCK, 0, s>>>(m.n, m.npad, C, Rb, X, Y, out, m.geo, m.side_nb, m.side_q, m.side_g, \
                                                 m.tab, m.gamma, dt, dt_dev, m.side_bc, m.bc_state)
        switch (mode) {
        case 0: DG_VJP(0); break;
        case 1: DG_VJP(1); break;
        case 2: DG_VJP(2); break;
        default: DG_VJP(3); break;
        }
#undef DG_VJP
        }
    }
    static void eval_points(const MeshDev& m, const double* C, double* u, hipStream_t s)
    {
        k_eval_points<P><<<grid_for(m.n), BLOCK, 0, s>>>(m.n, m.perm, C, u, m.tab);
    }
    static void quad_weights(const MeshDev& m, double* w, hipStream_t s)
    {
        k_quad_weights<P><<<grid_for(m.n), BLOCK, 0, s>>>(m.n, m.perm, m.vtx, w, m.tab);
    }
    static void dt_partial(const MeshDev& m, const double* C, double* partial, hipStream_t s)
    {
        k_dt_partial<P><<<grid_for(m.n), BLOCK, 0, s>>>(m.n, C, m.geo, m.gamma, partial);
    }
    static void project(const MeshDev& m, const double* uq, double* C, hipStream_t s)
    {
        k_project<P><<<grid_for(m.npad), BLOCK, 0, s>>>(m.n, m.npad, m.perm, uq, C, m.tab);
    }
    static void quad_points(const MeshDev& m, double* xy, hipStream_t s)
    {
        k_quad_points<P><<<grid_for(m.n), BLOCK, 0, s>>>(m.n, m.perm, m.vtx, xy, m.tab);
    }
    static int offsets_match(const dgh::TableLayout& L)
    {
        using O = Ord<P>;
        return O::NP == L.np && O::NQ == L.nq && O::NE == L.ne && O::PHI == L.phi && O::DRW == L.drw &&
               O::DSW == L.dsw && O::PHS == L.phs && O::GW == L.gw && O::QW == L.qw && O::QR == L.qr && O::QS == L.qs;
    }
};

extern template struct Launch<1>;
extern template struct Launch<2>;
extern template struct Launch<3>;
extern template struct Launch<4>;
extern template struct Launch<5>;

}  // namespace dgk
