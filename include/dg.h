/*
 * dg.h -- C ABI of libdgmi: the right-hand side of a modal discontinuous
 * Galerkin discretisation of the 2D Euler equations on triangle meshes, and
 * its SSP Runge-Kutta stepping, on one AMD Instinct MI355X (gfx950).
 *
 * The method is that of Fuhry, Giuliani and Krivodonova, "Discontinuous
 * Galerkin methods on graphics processing units for nonlinear hyperbolic
 * conservation laws":
 *   - conservation law d_t u + div F(u) = 0, eq. (2ddg), weak form eq.
 *     (weak2dsys), Euler flux and ideal-gas pressure eq. (euler);
 *   - each triangle mapped onto the reference triangle {(0,0),(1,0),(0,1)}
 *     by eq. (2dmap) (counter-clockwise vertices, det J > 0), each edge onto
 *     [-1,1] by eq. (1dmap) with half length l of eq. (len);
 *   - orthonormal modal basis of degree p, N_p = (p+1)(p+2)/2 (eq. (np)),
 *     so the mass matrix is det J times the identity;
 *   - semi-discrete system eq. (2ddg0): volume integral eq. (volume) with a
 *     degree-2p symmetric rule, surface integral eq. (surface) with (p+1)
 *     Gauss-Legendre points per side, numerical flux across each edge.
 *
 * Conventions fixed by this library where the paper leaves them open:
 *   - basis: orthonormal Dubiner polynomials, ordered by total degree and
 *     then by the degree in s; mode 0 is the constant sqrt(2);
 *   - local side q of an element runs from its vertex q to vertex q+1;
 *   - numerical flux: local Lax-Friedrichs at each Gauss point;
 *   - time integration: three-stage SSP Runge-Kutta (Shu-Osher form);
 *   - CFL step: dt = cfl * min_i r_i / (|v_i| + c_i), r_i = det J_i /
 *     perimeter_i (inscribed radius), state at the element mean.
 *
 * Memory and streams.  Every pointer named *_dev is device memory owned by
 * the caller (e.g. a torch tensor); the library never allocates in the calls
 * that take a stream.  Workspace sizes come from dg_mesh_info.  `stream` is
 * a hipStream_t passed as void* (NULL = the null stream).  All calls that
 * take a stream are asynchronous on it unless stated otherwise.  The mesh's
 * geometry and tables are immutable after creation, and the default
 * (element-wise) kernels keep no per-call state in the mesh, so such calls
 * on different streams with separate workspaces and outputs may overlap.
 * Three things do keep per-call state in the mesh, and with them the calls
 * on one mesh must come from one host thread at a time and, with the
 * stream concurrency on, be queued on one stream at a time: the settings
 * (dg_set_*), the two-stream edge-wise path (one side stream and one pair
 * of fork/join events per mesh) and per-launch timing (one record list per
 * mesh).  Results are deterministic: no atomics; every output is written by
 * exactly one work-item.
 * Sizes.  The kernels index per-element arrays with 32-bit offsets:
 * dg_mesh_validate refuses (DG_EUNSUPPORTED) a mesh whose padded element
 * count times max(4 N_p, 12 (p+1)) reaches 2^31, i.e. beyond about 44
 * million triangles at p = 3 and 25 million at p = 5.
 *
 * Layouts.
 *   user layout     C[N][4][N_p], element order of dg_mesh_create, variables
 *                   (rho, rho u, rho v, E), modes in basis order;
 *   internal layout the library's own element-blocked order (elements
 *                   reordered along a Hilbert curve of the centroids,
 *                   blocks of 16 elements [block][variable][mode][16],
 *                   padded to a multiple of 64); state_len doubles.
 *   dg_pack / dg_unpack convert; dg_rhs, dg_max_dt and dg_rk_step work on
 *   the internal layout.
 *
 * Errors.  Every call returns a dg_status; DG_OK is 0.  dg_last_error()
 * returns a message for the last failing call of the calling thread.  The
 * hot calls (dg_rhs, dg_rk_step) do not check the state they are given.
 */
#ifndef DGMI_DG_H
#define DGMI_DG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_mesh_s* dg_mesh;

typedef enum {
    DG_OK = 0,
    DG_EINVAL = -1,        /* null pointer, bad size or bad enum value */
    DG_EMESH = -2,         /* invalid mesh (orientation, connectivity, edges) */
    DG_EORDER = -3,        /* polynomial order outside 1..5 */
    DG_EUNSUPPORTED = -4,  /* valid input the library does not handle */
    DG_ENOMEM = -5,        /* device allocation failed */
    DG_EHIP = -6,          /* a HIP runtime call or kernel launch failed */
    DG_ENONPHYS = -7       /* non-physical element mean (rho <= 0, p <= 0, NaN) */
} dg_status;

typedef enum {
    DG_FP64 = 0,  /* every step in double precision */
    DG_MIXED = 1  /* contractions, traces, fluxes and the lift of modes >= 2 in
                     FP32; the mean mode, 1/det J, the stage update, the state
                     and the CFL reduction in FP64 (element-wise mode only) */
} dg_precision;

typedef struct {
    int p;              /* polynomial order */
    int n_modes;        /* N_p = (p+1)(p+2)/2 */
    int n_vol_points;   /* volume rule size: 3, 6, 12, 16, 25 for p = 1..5 */
    int n_edge_points;  /* p + 1 */
    int64_t n_elem;     /* elements */
    int64_t n_elem_pad; /* elements incl. padding (multiple of 64) */
    int64_t n_edges;    /* edges: element pairs plus boundary sides (1.5 n_elem on a periodic mesh) */
    int64_t state_len;  /* doubles in one internal-layout state */
    int64_t ws_rhs;     /* workspace bytes for dg_rhs and dg_max_dt */
    int64_t ws_step;    /* workspace bytes for dg_rk_step and dg_rk_step_stages */
    int64_t ws_vjp;     /* workspace bytes for dg_rk_step_vjp */
    int64_t n_colours;  /* colours of the edge colouring (DG_SURFACE_COLOURED) */
    int stage_fp64;     /* element-wise stage kernel of the current choice in FP64: 1 or 4 lanes
                           per element or 16 (16 x 16 x 4 matrix products, 16 elements per wavefront) */
    int stage_mixed;    /* the same for DG_MIXED */
    int adjoint;        /* adjoint stage kernel (dg_rhs_vjp, dg_rk_step_vjp): 1, 4 or 16, as above */
} dg_info;

/* Checks a mesh without touching the GPU (no HIP call).  Arguments as for
 * dg_mesh_create.  Returns DG_OK, DG_EINVAL, DG_EORDER, DG_EUNSUPPORTED or
 * DG_EMESH (the message names the element and side). */
int dg_mesh_validate(int p, int64_t n_elem, const double* vxy, const int64_t* nbr_elem, const int8_t* nbr_side);

/* Creates a mesh on the current HIP device (Section "Mesh Connectivity"):
 *   p         polynomial order, 1..5;
 *   n_elem    number of triangles, >= 1;
 *   vxy       host [n_elem][3][2] vertex coordinates, counter-clockwise so
 *             that det J of eq. (2dmap) is positive; periodic meshes give
 *             every element its own unwrapped coordinates;
 *   nbr_elem  host [n_elem][3]: element across local side q, or a
 *             negative boundary code for a side on the domain boundary
 *             (DG_BC_WALL, DG_BC_OUTFLOW or DG_BC_STATE, see
 *             dg_set_boundary_state; other negative values give
 *             DG_EUNSUPPORTED);
 *   nbr_side  host [n_elem][3]: that neighbour's local side index (ignored
 *             on boundary sides);
 *   gamma     ratio of specific heats (1.4 for air);
 *   out       receives the handle.
 * Validation: det J > 0; interior neighbours point back; the two copies of every
 * interior edge are the same segment in opposite directions to within 1e-12 times
 * the larger of its length and its vertices' coordinate magnitude (periodic
 * copies carry the rounding of shifted coordinates).
 * Validates first (see dg_mesh_validate), then builds the edge list (one
 * entry per edge, left = lower internal id, normal from left to right),
 * geometry (adj(J), 1/det J, inscribed radius; per-edge unit normal and
 * half length), the element order and the reference tables, and copies
 * them to the device.  Synchronous.  The host arrays are not retained. */
int dg_mesh_create(int p, int64_t n_elem, const double* vxy, const int64_t* nbr_elem, const int8_t* nbr_side,
                   double gamma, dg_mesh* out);

/* Releases the mesh's device memory.  NULL is accepted. */
int dg_mesh_destroy(dg_mesh m);

/* Sizes of the mesh's arrays and workspaces. */
int dg_mesh_info(dg_mesh m, dg_info* out);

/* Physical coordinates of the volume quadrature points, xy_dev [N][n_vol_points][2]
 * (user element order): the reference points of the degree-2p volume rule
 * (Section "Volume Integration Kernel") mapped by eq. (2dmap), for
 * evaluating initial data at them. */
int dg_quad_points(dg_mesh m, double* xy_dev, void* stream);

/* L2 projection of initial data onto the orthonormal basis (Section
 * "Outline of Algorithm" starts from projected initial coefficients; with the
 * orthonormal basis of eq. (np) the mass matrix is det J * I):
 * c_j = sum_k w_k phi_j(r_k) u(x_k) with the degree-2p volume rule.  u_dev [N][n_vol_points][4] holds the
 * conserved variables at dg_quad_points (user order); C_dev receives the
 * internal-layout state (padding zeroed). */
int dg_project(dg_mesh m, const double* u_dev, double* C_dev, void* stream);

/* User layout [N][4][N_p] -> internal layout (padding zeroed), and back. */
int dg_pack(dg_mesh m, const double* C_user_dev, double* C_dev, void* stream);
int dg_unpack(dg_mesh m, const double* C_dev, double* C_user_dev, void* stream);

/* Right-hand side of eq. (2ddg0): R = M^{-1} (volume - surface), internal
 * layout in and out (C_dev and R_dev must not overlap).  ws_dev: ws_rhs
 * bytes.  prec: DG_FP64 or DG_MIXED (DG_MIXED needs the element-wise
 * surface mode, else DG_EUNSUPPORTED). */
int dg_rhs(dg_mesh m, const double* C_dev, double* R_dev, dg_precision prec, void* ws_dev, void* stream);

/* Stable time step (Section "Outline of Algorithm": a stable step length is
 * computed on the device before every time step; the paper gives no formula,
 * the library's is the CFL bound below with the element's inscribed radius
 * and its mean wave speed |v| + c, cfl = 0.3/(2p+1) by convention): writes
 * dt = cfl * min_i r_i / (|v_i| + c_i) to dt_dev[0], or NaN when an element
 * mean is non-physical.  If dt_host is not NULL the call also copies the
 * value to *dt_host, waits for the stream, and returns DG_ENONPHYS for NaN.
 * ws_dev: ws_rhs bytes. */
int dg_max_dt(dg_mesh m, const double* C_dev, double cfl, double* dt_dev, double* dt_host, void* ws_dev,
              void* stream);

/* One explicit Runge-Kutta time step (Section "Time-stepping": every stage
 * evaluates the right-hand side of eq. (2ddg0) once) in place on the
 * internal-layout state C_dev; by default the three-stage SSP scheme:
 *   u1 = u + dt L(u);  u2 = 3/4 u + 1/4 (u1 + dt L(u1));
 *   u  = 1/3 u + 2/3 (u2 + dt L(u2)).
 * The step length is dt_dev[0] when dt_dev is not NULL (e.g. the output of
 * dg_max_dt, so a whole step stays on the device), else dt.  ws_dev:
 * ws_step bytes.  prec as for dg_rhs. */
int dg_rk_step(dg_mesh m, double* C_dev, double dt, const double* dt_dev, dg_precision prec, void* ws_dev,
               void* stream);

/* Bytes of the library's static device scratch used by dg_rk_step_noalloc
 * (64 MiB; every GPU the library runs on holds one copy until the process
 * ends). */
#define DG_NOALLOC_SCRATCH_BYTES (64LL << 20)

/* dg_rk_step without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same launches and results, bit for bit, as
 * dg_rk_step with the element-wise surface mode, with the stage states kept
 * in the library's static scratch of the mesh's device instead of ws_dev.
 * The call allocates nothing (no hipMalloc, no events, no per-launch
 * timing).  C_dev, dt, dt_dev, prec and stream as for dg_rk_step.
 * Limits and errors:
 *   - the stage states, 2 x state_len x 8 bytes (3 x with the RK4
 *     integrator), must fit DG_NOALLOC_SCRATCH_BYTES, else DG_EUNSUPPORTED
 *     (e.g. up to 104,832 triangles at p = 3 with SSP-RK3);
 *   - the surface mode must be the element-wise one (DG_EUNSUPPORTED);
 *   - the mesh's device must be the current device (DG_EINVAL).
 * Concurrency: every call on one GPU shares that GPU's scratch, and the
 * scratch keeps the last call's stage states; calls that overlap on one GPU
 * (different streams or host threads without ordering between them) race.
 * Every value a call reads from the scratch it has written itself first, so
 * nothing needs clearing between calls. */
int dg_rk_step_noalloc(dg_mesh m, double* C_dev, double dt, const double* dt_dev, dg_precision prec, void* stream);

/* nsteps SSP-RK3 steps in place, each with its own CFL step length taken
 * from the state at the start of the step (the paper's host-directed time
 * loop, Section "Time-stepping", kept on the device): the same results, bit
 * for bit, as nsteps x { dg_max_dt(C, cfl, dt_dev); dg_rk_step(C, dt_dev) }.
 * With the element-wise surface mode and 4 lanes per element the reduction
 * is fused into the stage kernels (three launches per step).  dt_dev
 * receives the last step's length; dt_hist_dev (may be NULL) receives all
 * nsteps lengths.  A non-physical mean turns the step length into NaN (and
 * the state into NaN); the call itself does not wait to check.
 * ws: ws_step bytes. */
int dg_advance(dg_mesh m, double* C_dev, int64_t nsteps, double cfl, double* dt_dev, double* dt_hist_dev,
               dg_precision prec, void* ws_dev, void* stream);

/* Adjoint (vector-Jacobian product) of dg_rhs, the derivative of the
 * discrete operator of eq. (2ddg0) transposed: Cbar = (dR/dC)^T Rbar, all
 * FP64, internal layout.  Element-wise gather form: no cotangent is
 * scattered across elements (no atomics; deterministic).  At exact ties of
 * the Lax-Friedrichs wave-speed max the left state's branch is taken, and
 * d|x|/dx = +1 at 0.  Cbar must not overlap C or Rbar.  ws: ws_rhs bytes. */
int dg_rhs_vjp(dg_mesh m, const double* C_dev, const double* Rbar_dev, double* Cbar_dev, void* ws_dev, void* stream);

/* Adjoint of one dg_rk_step (SSP-RK3) at state C_dev with the step length
 * held fixed (dt_dev[0] if dt_dev is not NULL, else dt; the step length is
 * not differentiated):
 *   u2bar = 2/3 ubar + 2/3 dt J(u2)^T ubar
 *   u1bar = 1/4 u2bar + 1/4 dt J(u1)^T u2bar
 *   Cbar  = 1/3 ubar + 3/4 u2bar + u1bar + dt J(C)^T u1bar
 * with J = dR/dC.  The stage states u1, u2 are recomputed unless the caller
 * passes them (u1_dev, u2_dev from dg_rk_step_stages, NULL otherwise).
 * Cbar must not overlap the other arrays.  ws: ws_vjp bytes of dg_info. */
int dg_rk_step_vjp(dg_mesh m, const double* C_dev, double dt, const double* dt_dev, const double* u1_dev,
                   const double* u2_dev, const double* ubar_dev, double* Cbar_dev, void* ws_dev, void* stream);

/* dg_rk_step that also keeps its two stage states (for dg_rk_step_vjp):
 * u1_dev, u2_dev receive u1 and u2 of the step (state_len doubles each,
 * caller-owned); C_dev is advanced in place.  Element-wise surface mode,
 * FP64.  ws: ws_step bytes. */
int dg_rk_step_stages(dg_mesh m, double* C_dev, double dt, const double* dt_dev, double* u1_dev, double* u2_dev,
                      void* ws_dev, void* stream);

/* dg_rk_step_stages with the new state written to Cnext_dev instead of over
 * C_dev (C_dev unchanged; Cnext_dev must not overlap C_dev, u1_dev or
 * u2_dev): a reverse sweep that recomputes a segment of steps and keeps
 * every step's input state then needs no copies.  The last stage is the
 * general form (1/3 C + 2/3 u2 + 2/3 dt L(u2)), so Cnext equals dg_rk_step's
 * result to rounding, not bit for bit; u1 and u2 are bitwise those of
 * dg_rk_step_stages. */
int dg_rk_step_stages_to(dg_mesh m, const double* C_dev, double* Cnext_dev, double dt, const double* dt_dev,
                         double* u1_dev, double* u2_dev, void* ws_dev, void* stream);

/* U_h at the volume quadrature points, u_dev [N][n_vol_points][4] (user
 * order): the modes-to-points contraction on its own, for functionals of
 * the solution. */
int dg_eval_points(dg_mesh m, const double* C_dev, double* u_dev, void* stream);

/* Physical quadrature weights det J_i * w_k, w_dev [N][n_vol_points] (user
 * order): sum_k w_ik f(x_ik) integrates f over element i exactly for
 * polynomials of degree <= 2p. */
int dg_quad_weights(dg_mesh m, double* w_dev, void* stream);

/* Organisation of the surface integral (Section "Surface Integration
 * Kernel" discusses both):
 *   DG_SURFACE_ELEMENTWISE (default): one fused kernel per right-hand side
 *     or RK stage; every element evaluates the numerical flux on its own
 *     three sides (each edge flux twice, as exact negatives of each other),
 *     gathering the neighbour's coefficients; no edge temporaries;
 *   DG_SURFACE_EDGEWISE: the paper's organisation: one work-item per edge
 *     evaluates the flux once and stores it for both elements (per-side
 *     slots, no atomics), then an element kernel combines; three kernels
 *     per right-hand side;
 *   DG_SURFACE_COLOURED: the alternative the paper proposes for its
 *     edge-wise kernel (Section "Conclusion"): the edges are coloured so
 *     that no two edges of one colour share an element (greedy, at most
 *     five colours, dg_info.n_colours), and one launch per colour lets each
 *     edge add its lifted flux straight into both elements' accumulators,
 *     with no slots and no atomics; then the element kernel adds the
 *     volume integral and finishes the stage.
 * All give the same discrete operator (equal up to rounding).  The two
 * edge-based modes run in FP64 only, without the limiter and with SSP-RK3
 * only (DG_EUNSUPPORTED otherwise). */
enum { DG_SURFACE_ELEMENTWISE = 0, DG_SURFACE_EDGEWISE = 1, DG_SURFACE_COLOURED = 2 };
int dg_set_surface_mode(dg_mesh m, int mode);

/* Volume and surface work on two streams in the edge-wise surface mode
 * (Section "Results" notes that the volume and surface contributions are
 * independent, so on meshes too small to fill the device the two kernels
 * can run side by side on separate streams).  With on = 1, every RHS or
 * RK stage of DG_SURFACE_EDGEWISE runs the volume integral on a library-
 * owned stream (default priority, created by the first call with on = 1,
 * destroyed with the mesh) beside the traces and edge fluxes on the
 * caller's stream; events order it after the work already queued on the
 * caller's stream, and the element kernel that combines both waits for it,
 * so the call stays ordered on the caller's stream.  The results equal
 * those of on = 0 bit for bit.  Other surface modes ignore the setting.
 * Returns DG_EINVAL for on outside {0, 1}, DG_EHIP if the stream or its
 * events cannot be created. */
int dg_set_stream_concurrency(dg_mesh m, int on);

/* Domain boundaries (Section "Surface Integration Kernel": on a boundary
 * edge the right-hand state is a ghost state that depends on the kind of
 * boundary; Section "Mesh Connectivity": boundary sides carry a negative
 * code in place of a neighbour).  At every Gauss point of a boundary side,
 * with U the element's own trace and n the outward unit normal:
 *   DG_BC_WALL (-1)     solid wall: density and energy kept, momentum
 *                       mirrored, m_g = m - 2 (m . n) n;
 *   DG_BC_OUTFLOW (-2)  the interior state itself (outflow / transmissive);
 *   DG_BC_STATE (-3)    a constant prescribed state (inflow, far field,
 *                       Dirichlet), set with dg_set_boundary_state from the
 *                       host array U[4] = (rho, rho u, rho v, E); until then
 *                       a gas at rest with rho = 1, p = 1.
 * The local Lax-Friedrichs flux then takes the ghost as its right state.
 * Boundaries are supported by dg_rhs, dg_rk_step and dg_advance in both
 * surface modes and both precisions, and by the limiter (which counts no
 * neighbour on a boundary side).  In the edge-wise mode the boundary edges
 * come first in the edge list, grouped by kind, so that whole wavefronts
 * take the same branch.  The adjoint entry points (dg_rhs_vjp,
 * dg_rk_step_vjp) take a boundary side's cotangent back through its ghost
 * state: the wall's reflection (its own transpose), the outflow's identity;
 * a prescribed state has none.  dg_set_boundary_state waits for all work
 * on the device, then copies the state (the next calls on any stream see
 * it); it returns DG_EINVAL for a non-physical state. */
enum { DG_BC_WALL = -1, DG_BC_OUTFLOW = -2, DG_BC_STATE = -3 };
int dg_set_boundary_state(dg_mesh m, const double* U);

/* Time integrator of dg_rk_step and dg_advance: DG_RK_SSP3 (default; the
 * three-stage SSP scheme of dg_rk_step's comment), or the paper's classic
 * explicit Runge-Kutta schemes of order two and four (Section
 * "Time-stepping"): DG_RK2, Heun's method, u1 = u + dt L(u),
 * u = u/2 + (u1 + dt L(u1))/2; DG_RK4, the classic four-stage scheme,
 * u = u + dt (k1 + 2 k2 + 2 k3 + k4)/6 with k1 = L(u), k2 = L(u + dt/2 k1),
 * k3 = L(u + dt/2 k2), k4 = L(u + dt k3).  Every stage is one fused kernel
 * (RK4 keeps its running sum in the step workspace).  With RK2 / RK4,
 * dg_advance computes each step's length with a separate reduction, and
 * dg_rk_step_stages and dg_rk_step_vjp return DG_EUNSUPPORTED (their stage
 * states and adjoint are SSP-RK3's), as does the edge-wise surface mode.
 * DG_EINVAL for an unknown scheme. */
enum { DG_RK_SSP3 = 0, DG_RK2 = 1, DG_RK4 = 2 };
int dg_set_integrator(dg_mesh m, int scheme);

/* Slope limiting (Section "Limiting Kernel"): the Barth-Jespersen limiter
 * for p = 1, each conserved variable separately.  With the centroid values
 * of the element and of its three neighbours (for a linear function, its
 * mean), Umax and Umin their extremes, and d = U(r_qk) - Ubar at each Gauss
 * point of the element's sides, the factor alpha = min(1, min_k alpha_k)
 * with alpha_k = (Umax - Ubar)/d (d > 0), (Umin - Ubar)/d (d < 0), 1 (d = 0)
 * scales the two linear coefficients; the mean is unchanged.
 *
 * dg_limit applies it once, in place, to the internal-layout state C_dev
 * (asynchronous on stream).  dg_set_limiter(m, DG_LIMITER_BJ) makes
 * dg_rk_step, dg_rk_step_stages and dg_advance limit every RK stage's
 * result and the new state, as the paper's time loop does;
 * DG_LIMITER_NONE (the default) switches it off.  Errors: DG_EUNSUPPORTED
 * for p != 1; with the limiter on, the edge-wise surface mode and
 * dg_rk_step_vjp (the limited step is not differentiable) return
 * DG_EUNSUPPORTED; DG_EINVAL for an unknown limiter. */
enum { DG_LIMITER_NONE = 0, DG_LIMITER_BJ = 1 };
int dg_set_limiter(dg_mesh m, int limiter);
int dg_limit(dg_mesh m, double* C_dev, void* stream);

/* Work-items per element in the element-wise kernels (forward right-hand
 * side and RK stages): 1 or 4.  With 4, lane m of a quad owns conserved
 * variable m for the modal contractions (all lanes walk the same points, so
 * the tables are read uniformly), and the flux at each point is evaluated
 * once, by one lane of the quad, after a transpose of the point values
 * through LDS; a second transpose returns the flux components for the lift.
 * Four lanes give four times as many wavefronts and fewer registers per
 * lane, at the price of more instructions per element: they pay off on
 * meshes too small to fill the GPU, and at p >= 4, where one lane's
 * registers cannot hold an element.  0 = automatic (4 lanes up to
 * DG_LANES4_MAX_ELEMENTS elements or for p >= 4, else 1; the adjoint
 * kernels of dg_rhs_vjp and dg_rk_step_vjp take 4 lanes from p = 3 on at
 * any size, where the one-lane adjoint holds too many values).  1 and 4
 * apply to both.  Both give the same result to rounding.  1 is refused
 * (DG_EUNSUPPORTED) from p = 4 on, where an element's values exceed a
 * lane's registers.  Returns DG_EINVAL for any value other than 0, 1, 4.
 * The FP64 stages may instead run on the matrix cores (dg_set_matrix_cores):
 * automatically only while this setting is 0. */
#define DG_LANES4_MAX_ELEMENTS 1048576
int dg_set_lanes_per_element(dg_mesh m, int lanes);

/* Right-hand side and RK stages with their contractions (eq. (2ddg0):
 * evaluation of the modes at the volume and side points, the volume and
 * surface lifts) as 16 x 16 x 4 matrix products on the matrix cores (FP64
 * products in FP64, FP32 products in DG_MIXED), the 16 elements of a block
 * as the columns, one wavefront per block, four lanes per element.  on: 1
 * uses that kernel for every stage, whatever the lane count; 0 the
 * vector-ALU kernels chosen by dg_set_lanes_per_element; -1 (the default)
 * automatic: the matrix cores at p = 4 at every size and at p = 3 and 5 up
 * to DG_LANES4_MAX_ELEMENTS elements (DG_MIXED: at p = 5 at every size), as
 * long as the lane count is automatic too (an explicit 1 or 4 keeps the
 * vector-ALU kernels).  The adjoint
 * (dg_rhs_vjp, dg_rk_step_vjp) has a matrix-core kernel of the same layout:
 * used with on = 1, and automatically at p = 3 and 4 when the lane count is
 * automatic.  Same result to rounding.  Returns DG_EINVAL for other values
 * of on. */
int dg_set_matrix_cores(dg_mesh m, int on);

/* Per-kernel timing (the paper's kernel runtime distribution, measured with
 * events around every launch).  dg_timing_enable(m, 1) makes every later
 * launch for this mesh record a pair of HIP events on its stream;
 * dg_timing_read waits for the recorded events, writes for each kernel kind
 * k the summed duration in milliseconds ms[k] and the number of launches
 * count[k] (k = DG_KERNEL_*; arrays of n >= DG_KERNEL_KINDS entries), and
 * clears the record.  Timing is off by default and adds two event records
 * per launch when on.  Not thread-safe for one mesh used from several
 * threads. */
enum {
    DG_KERNEL_TRACES = 0,   /* edge-wise path: edge traces of a state */
    DG_KERNEL_EDGE = 1,     /* edge-wise path: numerical flux per edge into side slots */
    DG_KERNEL_ELEMENT = 2,  /* edge-wise path: volume + lift + inverse mass (+ RK stage) */
    DG_KERNEL_DT = 3,       /* CFL reduction (both passes) */
    DG_KERNEL_STAGE = 4,    /* element-wise path: whole RHS (+ RK stage) in one kernel */
    DG_KERNEL_VJP = 5,      /* adjoint of the element-wise RHS (+ RK stage adjoint) */
    DG_KERNEL_LIMIT = 6,    /* slope limiter (p = 1) */
    DG_KERNEL_VOLUME = 7,   /* edge-wise path on two streams: volume integral alone */
    DG_KERNEL_KINDS = 8
};
int dg_timing_enable(dg_mesh m, int on);
int dg_timing_read(dg_mesh m, double* ms, int64_t* count, int n);

/* Host-only: the reference tables the kernels use, for checking them on a
 * machine without a GPU.  Writes into out (capacity cap doubles, in this
 * order): volume points r[nq], s[nq], weights w[nq]; Gauss nodes x[ne],
 * weights[ne]; phi[nq][np], dphi/dr[nq][np], dphi/ds[nq][np] at the volume
 * points; phi at side points [3][ne][np].  Returns the number of doubles
 * written (> 0), or a negative dg_status. */
int64_t dg_reference_tables(int p, double* out, int64_t cap);

/* Host-only: the table operands of the matrix-core stage kernels
 * (dg_set_matrix_cores), for checking them on a machine without a GPU: the
 * 16 x 4 operands of the 16 x 16 x 4 products as blocks of 64 values in lane
 * order (lane 16k+i holds row i, column k).  fp64 != 0: the FP64 kernel's
 * order (register r of lane group g of a product is row 4r+g), 0: the FP32
 * kernel's (row 4g+r; the kernel uses these values rounded to FP32).  With
 * N_p modes, N_q volume points, p+1 Gauss points per side, KP = ceil(N_p/4),
 * TQ = ceil(N_q/16), TS = ceil(3(p+1)/16), TM = ceil(KP/4), row(g, r) as
 * above and mode(tm, i) = 16tm+i (FP64) or 4(4tm+i%4)+i/4 (FP32), the
 * blocks are, in this order (entries of modes >= N_p zero):
 *   [t][s] (TQ x KP): phi_{4s+k} at volume point min(16t+i, N_q-1);
 *   [tm][t][s'] (TM x TQ x 4), twice: w dphi/dr, then w dphi/ds, of mode
 *     mode(tm, i) at volume point 16t+row(k, s') (zero past N_q);
 *   [ts][s] (TS x KP): phi_{4s+k} at side point min(16ts+i, 3(p+1)-1), side
 *     points side-major (point k of side q is q(p+1)+k);
 *   [tm][ts][s'] (TM x TS x 4): Gauss weight times phi of mode mode(tm, i) at
 *     side point 16ts+row(k, s') (zero past the last side point);
 * and for the adjoint kernel:
 *   [t][s] (TQ x KP), twice: w dphi/dr, then w dphi/ds, of mode 4s+k at
 *     volume point min(16t+i, N_q-1);
 *   [tm][t][s'] (TM x TQ x 4): phi of mode mode(tm, i) at volume point
 *     16t+row(k, s') (zero past N_q);
 *   [tm][ts][s'] (TM x TS x 4): phi of mode mode(tm, i) at side point
 *     16ts+row(k, s') (zero past the last side point);
 * and where 3(p+1) exceeds 16 by NT <= 4 (p = 5: NT = 2), for the forward
 * kernel's per-lane evaluation of side points 16.. (lane 16g+j, any j):
 *   [pt][s] (NT x KP): phi_{4s+g} at side point 16+pt;
 *   [pt][s] (NT x KP): Gauss weight times phi_{4s+g} at side point 16+pt.
 * Returns the number of doubles written (> 0), or a negative dg_status. */
int64_t dg_matrix_core_tables(int p, int fp64, double* out, int64_t cap);

/* Message of the last failing call on this thread ("" if none). */
const char* dg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DGMI_DG_H */
