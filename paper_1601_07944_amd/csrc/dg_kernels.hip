// Order-independent kernels and the dispatch from a runtime order p to the
// per-order instantiations (one translation unit per order).
#include "dg_kernels.h"

namespace dgk {

__global__ __launch_bounds__(BLOCK) void k_dt_final(int nb, const double* __restrict__ partial, double cfl,
                                                    double* __restrict__ dt, double* __restrict__ hist)
{
    __shared__ double red[BLOCK];
    const double h = dt_from_partials(partial, nb, cfl, red);
    if (threadIdx.x == 0) {
        dt[0] = h;
        if (hist) hist[0] = h;
    }
}

// ---------------------------------------------------------------- layout
// user layout [N][4][NP] (user element order) <-> blocked internal layout
__global__ __launch_bounds__(BLOCK) void k_pack(int n, int npad, int np, const int* __restrict__ perm,
                                                const double* __restrict__ Cu, double* __restrict__ C)
{
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= npad) return;
    const int so = state_off(e, 4 * np);
    if (e < n) {
        const double* src = Cu + (size_t)perm[e] * 4 * np;
        for (int x = 0; x < 4 * np; ++x) C[so + x * LANES] = src[x];
    } else {
        for (int x = 0; x < 4 * np; ++x) C[so + x * LANES] = 0.0;
    }
}

__global__ __launch_bounds__(BLOCK) void k_unpack(int n, int np, const int* __restrict__ perm,
                                                  const double* __restrict__ C, double* __restrict__ Cu)
{
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= n) return;
    const int so = state_off(e, 4 * np);
    double* dst = Cu + (size_t)perm[e] * 4 * np;
    for (int x = 0; x < 4 * np; ++x) dst[x] = C[so + x * LANES];
}

#define DG_DISPATCH_P(p, CALL)                     \
    switch (p) {                                   \
    case 1: Launch<1>::CALL; break;                \
    case 2: Launch<2>::CALL; break;                \
    case 3: Launch<3>::CALL; break;                \
    case 4: Launch<4>::CALL; break;                \
    default: Launch<5>::CALL; break;               \
    }

void launch_traces(const MeshDev& m, const double* C, double* T, hipStream_t s, double* Rz)
{
    DG_DISPATCH_P(m.p, traces(m, C, T, s, Rz));
}

void launch_edge_lift(const MeshDev& m, const double* T, double* R, hipStream_t s)
{
    DG_DISPATCH_P(m.p, edge_lift(m, T, R, s));
}

void launch_edge_flux(const MeshDev& m, const double* T, double* S, hipStream_t s)
{
    DG_DISPATCH_P(m.p, edge_flux(m, T, S, s));
}

void launch_element(const MeshDev& m, int mode, const double* C, const double* U0, double* out, const double* S,
                    double dt, const double* dt_dev, double* Tn, hipStream_t s, double* Racc, int src)
{
    DG_DISPATCH_P(m.p, element(m, mode, C, U0, out, S, dt, dt_dev, Tn, s, Racc, src));
}

void launch_volume(const MeshDev& m, const double* C, double* V, hipStream_t s)
{
    DG_DISPATCH_P(m.p, volume(m, C, V, s));
}

void launch_stage(const MeshDev& m, int mode, bool mixed, const double* C, const double* U0, double* out, double dt,
                  const double* dt_dev, hipStream_t s, const FusedDt& fz)
{
    DG_DISPATCH_P(m.p, stage(m, mode, mixed, C, U0, out, dt, dt_dev, s, fz));
}

void launch_stage_general(const MeshDev& m, bool mixed, const double* C, double* out, double dt,
                          const double* dt_dev, const StageGen& gs, hipStream_t s)
{
    DG_DISPATCH_P(m.p, stage(m, 4, mixed, C, nullptr, out, dt, dt_dev, s, FusedDt(), gs));
}

void launch_stage_vjp(const MeshDev& m, int mode, const double* C, const double* Rb, const double* X, const double* Y,
                      double* out, double dt, const double* dt_dev, hipStream_t s)
{
    DG_DISPATCH_P(m.p, stage_vjp(m, mode, C, Rb, X, Y, out, dt, dt_dev, s));
}

void launch_eval_points(const MeshDev& m, const double* C, double* u, hipStream_t s)
{
    DG_DISPATCH_P(m.p, eval_points(m, C, u, s));
}

void launch_quad_weights(const MeshDev& m, double* w, hipStream_t s) { DG_DISPATCH_P(m.p, quad_weights(m, w, s)); }

int dt_partials(const MeshDev& m) { return (m.n + BLOCK - 1) / BLOCK; }

void launch_dt(const MeshDev& m, const double* C, double cfl, double* partial, double* dt_dev, hipStream_t s)
{
    DG_DISPATCH_P(m.p, dt_partial(m, C, partial, s));
    k_dt_final<<<1, BLOCK, 0, s>>>(dt_partials(m), partial, cfl, dt_dev, nullptr);
}

void launch_dt_partials_only(const MeshDev& m, const double* C, double* partial, hipStream_t s)
{
    DG_DISPATCH_P(m.p, dt_partial(m, C, partial, s));
}

void launch_dt_final(const double* partial, int count, double cfl, double* dt_dev, double* dt_hist, hipStream_t s)
{
    k_dt_final<<<1, BLOCK, 0, s>>>(count, partial, cfl, dt_dev, dt_hist);
}

void launch_limit(const MeshDev& m, double* C, hipStream_t s)
{
    // the limiter is defined for p = 1 only (the caller checks)
    if (m.has_bc)
        k_limit_bj<1, true><<<grid_for(m.n), BLOCK, 0, s>>>(m.n, C, m.side_nb, m.side_bc, m.tab);
    else
        k_limit_bj<1, false><<<grid_for(m.n), BLOCK, 0, s>>>(m.n, C, m.side_nb, m.side_bc, m.tab);
}

void launch_pack(const MeshDev& m, const double* Cu, double* C, hipStream_t s)
{
    k_pack<<<grid_for(m.npad), BLOCK, 0, s>>>(m.n, m.npad, m.np, m.perm, Cu, C);
}

void launch_unpack(const MeshDev& m, const double* C, double* Cu, hipStream_t s)
{
    k_unpack<<<grid_for(m.n), BLOCK, 0, s>>>(m.n, m.np, m.perm, C, Cu);
}

void launch_project(const MeshDev& m, const double* uq, double* C, hipStream_t s) { DG_DISPATCH_P(m.p, project(m, uq, C, s)); }

void launch_quad_points(const MeshDev& m, double* xy, hipStream_t s) { DG_DISPATCH_P(m.p, quad_points(m, xy, s)); }

int table_offset_check(int p, const dgh::TableLayout& L)
{
    int ok = 0;
    DG_DISPATCH_P(p, offsets_match(L) ? (void)(ok = 1) : (void)0);
    return ok;
}

}  // namespace dgk
