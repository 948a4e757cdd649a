// Internal declarations shared by the host code and the HIP kernels of
// libdgmi.  Not part of the public ABI (that is include/dg.h).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace dgh {

// Offsets (in doubles) of the reference tables inside one device buffer.
struct TableLayout {
    int np = 0, nq = 0, ne = 0;
    int phi = 0, drw = 0, dsw = 0, phs = 0, gw = 0, qw = 0, qr = 0, qs = 0, size = 0;
};

int n_modes(int p);
void basis_eval(int p, double r, double s, double* phi, double* dr, double* ds);
void volume_rule(int p, std::vector<double>& r, std::vector<double>& s, std::vector<double>& w);
void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w);
void side_point(int q, double xi, double* r, double* s);
std::vector<double> build_tables(int p, TableLayout* lay);
// the table operands of the matrix-core stage kernel from build_tables' output
std::vector<double> build_mx_tables(int p, const std::vector<double>& tab, const TableLayout& lay, bool f64);

}  // namespace dgh

namespace dgk {

// Every per-element array is stored block-major in blocks of LANES = 16
// elements: [block][field][lane], lane = element % 16, so one field of a
// block is a 128-byte row of doubles.  (A neighbour gather touches one row
// per field; 16-element rows keep that footprint small while a wavefront of
// one-lane kernels still reads whole rows.)  WAVE is the wavefront width.
constexpr int LANES = 16;
constexpr int WAVE = 64;

// Table operands of the matrix-core stage kernels (k_stage_mx): blocks of
// 64 values, one per lane, in the operand order of the 16 x 16 x 4 matrix
// products (lane 16 k + i holds row i, column k of the 16 x 4 table operand;
// register r of lane 16 g + j of the product is row mx_row(g, r)).  Lane
// 16 g + j of that kernel holds modes 4 s + g (s < KP) of element j of a
// 16-element block; volume and side points come in tiles of 16 rows, and so
// do modes (row i of mode tile tm is mode mx_mode(tm, i)).
//   PHI [t][s]      phi_{4s+k} at volume point 16t+i (last point repeated)
//   DR, DS [tm][t][s']  w dphi/dr, w dphi/ds of mode mx_mode(tm, i) at
//                   volume point 16t+mx_row(k, s') (zero past the last point)
//   PE [ts][s]      phi_{4s+k} at side point 16ts+i (side-major: point k of
//                   side q is q(p+1)+k; last side point repeated)
//   LE [tm][ts][s'] Gauss weight times phi of mode mx_mode(tm, i) at side
//                   point 16ts+mx_row(k, s') (zero past the last side point)
// and, for the adjoint (the transposed contractions):
//   DRE, DSE [t][s] w dphi/dr, w dphi/ds of mode 4s+k at volume point
//                   16t+i (last point repeated)
//   PHL [tm][t][s'] phi of mode mx_mode(tm, i) at volume point
//                   16t+mx_row(k, s') (zero past the last point)
//   PEL [tm][ts][s'] phi of mode mx_mode(tm, i) at side point
//                   16ts+mx_row(k, s') (zero past the last side point)
// and, where the side points overrun one tile by a few (p = 5: 18 points,
// NT = 2), for the forward kernel's per-lane evaluation of those points
// (lane 16g+j holds, whatever j):
//   TPE [pt][s]     phi_{4s+g} at side point 16+pt
//   TLE [pt][s]     Gauss weight times phi_{4s+g} at side point 16+pt
// Entries of modes >= N_p are zero.
// Result rows: the FP64 product puts row 4r+g in register r of lane group
// g, the FP32 product row 4g+r; mx_mode orders the mode rows so that
// register r of lane group g of mode tile tm is mode 4(4tm+r)+g in both.
template <bool F64>
constexpr int mx_row(int g, int r) { return F64 ? 4 * r + g : 4 * g + r; }
template <bool F64>
constexpr int mx_mode(int tm, int i) { return F64 ? 16 * tm + i : 4 * (4 * tm + i % 4) + i / 4; }
struct MxLayout {
    int np, nq, ne, ns, kp, tq, ts, tm;
    int nt;  // side points past the first tile evaluated per lane (0: none)
    int phi, dr, ds, pe, le, dre, dse, phl, pel, tpe, tle, blocks;
};
constexpr MxLayout mx_layout(int p)
{
    MxLayout x{};
    x.np = (p + 1) * (p + 2) / 2;
    x.nq = p == 1 ? 3 : p == 2 ? 6 : p == 3 ? 12 : p == 4 ? 16 : 25;
    x.ne = p + 1;
    x.ns = 3 * x.ne;
    x.kp = (x.np + 3) / 4;
    x.tq = (x.nq + 15) / 16;
    x.ts = (x.ns + 15) / 16;
    x.tm = (x.kp + 3) / 4;
    x.phi = 0;
    x.dr = x.phi + x.tq * x.kp;
    x.ds = x.dr + x.tm * x.tq * 4;
    x.pe = x.ds + x.tm * x.tq * 4;
    x.le = x.pe + x.ts * x.kp;
    x.dre = x.le + x.tm * x.ts * 4;
    x.dse = x.dre + x.tq * x.kp;
    x.phl = x.dse + x.tq * x.kp;
    x.pel = x.phl + x.tm * x.tq * 4;
    x.nt = x.ns > 16 && x.ns <= 20 ? x.ns - 16 : 0;
    x.tpe = x.pel + x.tm * x.ts * 4;
    x.tle = x.tpe + x.nt * x.kp;
    x.blocks = x.tle + x.nt * x.kp;
    return x;
}

// Device view of a mesh, passed by value to the launchers.
struct MeshDev {
    int p = 0, np = 0, nq = 0, ne = 0;
    int n = 0;         // real elements
    int npad = 0;      // padded to a multiple of 64 (whole workgroups)
    int nedge = 0;
    bool lanes4 = false;  // fused kernels: 4 lanes per element instead of 1
    bool vjp_lanes4 = true;  // adjoint kernels: 4 lanes per element instead of 1
    bool mx = false;         // FP64 stages on the matrix cores (k_stage_mx)
    bool mx32 = false;       // mixed-precision stages on the matrix cores (k_stage_mx)
    bool mx_vjp = false;     // adjoint stages on the matrix cores (k_stage_vjp_mx)
    // domain boundaries: per element 4 bits per side (0 interior, 1 wall,
    // 2 outflow, 3 prescribed state), and the prescribed state (4 doubles)
    const int* side_bc = nullptr;
    double* bc_state = nullptr;
    bool has_bc = false;
    double gamma = 1.4;
    const double* tab = nullptr;      // reference tables (TableLayout)
    const float* tab32 = nullptr;     // the same tables rounded to FP32 (mixed precision)
    const double* tabmx = nullptr;    // table operands of k_stage_mx (MxLayout), FP64 result layout
    const float* tabmx32 = nullptr;   // the same for the FP32 products
    const double* geo = nullptr;      // [blk][6][LANES]: adj00 adj01 adj10 adj11 1/detJ r_in
    const double* vtx = nullptr;      // [npad][6] vertices (internal order), setup only
    const int* perm = nullptr;        // internal -> user element id
    const int* edge_l = nullptr;      // [nedge] left element (internal id)
    const int* edge_r = nullptr;      // [nedge] right element
    const int* edge_sd = nullptr;     // [nedge] side_l | side_r << 2
    const double* edge_g = nullptr;   // SoA [3][nedge]: unit normal (left -> right) x, y; half length
    // edge colouring: edges sorted by colour, colour c = [colour_off[c],
    // colour_off[c+1]); no two edges of one colour share an element
    static constexpr int MAX_COLOURS = 8;
    int ncolour = 0;
    int colour_off[MAX_COLOURS + 1] = {};
    const int* ecol = nullptr;        // [3][nedge] left, right, sides (as edge_l/r/sd) in colour order
    const double* edge_gc = nullptr;  // [3][nedge] as edge_g, in colour order
    // per element side (element-wise surface integration), block-major:
    const int* side_nb = nullptr;     // [blk][3][LANES] neighbour across side q (internal id)
    const int* side_q = nullptr;      // [blk][LANES] neighbour's sides, 2 bits per side
    const double* side_g = nullptr;   // [blk][9][LANES] outward unit normal x, y and half length per side
};

// Fused step-length bookkeeping of the multi-step path (4-lane kernels):
// stage 1 reduces pin[0..pin_count) into its step length and stores it to
// dt_store (and dt_hist); stage 3 writes per-block minima of the new state
// to pout.
struct FusedDt {
    const double* pin = nullptr;
    int pin_count = 0;
    double cfl = 0.0;
    double* dt_store = nullptr;
    double* dt_hist = nullptr;
    double* pout = nullptr;
};

// Launchers (dg_kernels.hip).  All asynchronous on `s`.
// Rz (optional): an accumulator state zeroed for the elements' own slots
void launch_traces(const MeshDev& m, const double* C, double* T, hipStream_t s, double* Rz = nullptr);
// coloured edges: one launch per colour, each edge lifting its flux
// straight into both elements' accumulators R (race-free within a colour)
void launch_edge_lift(const MeshDev& m, const double* T, double* R, hipStream_t s);
void launch_edge_flux(const MeshDev& m, const double* T, double* S, hipStream_t s);
// mode 0: R = L(C);   mode 1..3: SSP-RK3 stage (out = stage result);
// when Tnext != nullptr the traces of `out` are written to it.
// src 0: volume integral + side slots S; src 1 (coloured edges): the
// surface integral from the accumulator Racc + volume integral, Racc zeroed
// again when Tnext is set (the next stage accumulates into it); src 2: the
// volume integral from Racc (launch_volume) + side slots S
void launch_element(const MeshDev& m, int mode, const double* C, const double* U0, double* out, const double* S,
                    double dt, const double* dt_dev, double* Tnext, hipStream_t s, double* Racc = nullptr,
                    int src = 0);
// the volume integral alone, V = sum over the volume points (before 1/det J)
void launch_volume(const MeshDev& m, const double* C, double* V, hipStream_t s);
// fused right-hand side / SSP-RK3 stage (element-wise surface integral);
// mode as for launch_element, except that mode 3 updates `out` in place
// (it is the stage-0 state) and U0 must be nullptr
// A stage of a general explicit Runge-Kutta scheme (stage kernels' mode 4),
// with U the stage's input state and L = L(U):
//   out = a X + b U + g h L,  X = the array X, or `out` itself when X is null
//   (read before it is overwritten, as mode 3 reads the stage-0 state);
//   if S is set: S = (s_init ? U : S) + d h L  (an accumulator, e.g. RK4's
//   running sum of weighted stage derivatives).
struct StageGen {
    double a = 0.0, b = 0.0, g = 0.0, d = 0.0;
    const double* X = nullptr;
    double* S = nullptr;
    int s_init = 0;
};
void launch_stage(const MeshDev& m, int mode, bool mixed, const double* C, const double* U0, double* out, double dt,
                  const double* dt_dev, hipStream_t s, const FusedDt& fz = FusedDt());
void launch_stage_general(const MeshDev& m, bool mixed, const double* C, double* out, double dt,
                          const double* dt_dev, const StageGen& gs, hipStream_t s);
// number of per-block minima a 4-lane stage 3 writes (one per 64 elements)
inline int stage4_partials(const MeshDev& m) { return m.npad / 64; }
// final pass of the step-length reduction over `count` minima (also writes
// dt_hist[0] when dt_hist is not null)
void launch_dt_final(const double* partial, int count, double cfl, double* dt_dev, double* dt_hist, hipStream_t s);
// Barth-Jespersen limiter of a p = 1 state, in place
void launch_limit(const MeshDev& m, double* C, hipStream_t s);
// first pass only (dt_partials(m) minima of 256 elements each)
void launch_dt_partials_only(const MeshDev& m, const double* C, double* partial, hipStream_t s);
// adjoint of the fused right-hand side / RK stages (modes of k_stage_vjp)
void launch_stage_vjp(const MeshDev& m, int mode, const double* C, const double* Rb, const double* X, const double* Y,
                      double* out, double dt, const double* dt_dev, hipStream_t s);
void launch_eval_points(const MeshDev& m, const double* C, double* u, hipStream_t s);
void launch_quad_weights(const MeshDev& m, double* w, hipStream_t s);
void launch_dt(const MeshDev& m, const double* C, double cfl, double* partial, double* dt_dev, hipStream_t s);
int dt_partials(const MeshDev& m);
void launch_pack(const MeshDev& m, const double* Cu, double* C, hipStream_t s);
void launch_unpack(const MeshDev& m, const double* C, double* Cu, hipStream_t s);
void launch_project(const MeshDev& m, const double* uq, double* C, hipStream_t s);
void launch_quad_points(const MeshDev& m, double* xy, hipStream_t s);
int table_offset_check(int p, const dgh::TableLayout& L);

}  // namespace dgk
