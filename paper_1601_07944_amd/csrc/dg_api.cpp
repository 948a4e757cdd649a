// C ABI of libdgmi (declared in include/dg.h): mesh preprocessing on the
// host and orchestration of the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/dg.h"
#include "dg_internal.h"

struct dg_mesh_s {
    dgk::MeshDev dev;
    int device = 0;  // the HIP device the mesh was created on
    dgh::TableLayout lay;
    int64_t ws_rhs = 0, ws_step = 0, ws_vjp = 0;
    // workspace offsets (bytes)
    size_t off_T0 = 0, off_T1 = 0, off_S = 0, off_part = 0, off_u1 = 0, off_u2 = 0, off_part4 = 0;
    size_t state_bytes = 0;
    std::vector<void*> allocs;
    // per-launch event timing (dg_timing_*)
    int surface = DG_SURFACE_ELEMENTWISE;
    int limiter = DG_LIMITER_NONE;
    int integrator = DG_RK_SSP3;
    // kernel choice as requested: lanes per element (0 automatic, 1, 4) and
    // matrix cores (-1 automatic, 0 off, 1 on); apply_kernel_choice sets dev
    int lanes_req = 0, mx_req = -1;
    size_t off_acc = 0;  // RK4 accumulator state in the step workspace
    size_t off_V = 0;    // volume integral of the two-stream edge-wise path
    // edge-wise path: volume integral on a second stream beside the traces
    // and edge fluxes (created by dg_set_stream_concurrency)
    bool concurrent = false;
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool timing = false;
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};

namespace {

// The automatic kernel choice (measured on MI355X, FP64 stages; mixed
// precision and the adjoint follow the lane choice only):
//   lanes: four per element up to DG_LANES4_MAX_ELEMENTS elements or from
//     p = 4 on, else one; the adjoint four from p = 3 on;
//   matrix cores: at p = 4 at every size, at p = 3 and 5 up to
//     DG_LANES4_MAX_ELEMENTS elements (beyond that the one-lane kernel at
//     p = 3 and the four-lane kernel at p = 5 are faster), never at p <= 2
//     (the 16 x 4 products would be mostly padding); the mixed form also
//     at p = 5 at every size (its FP32 kernel evaluates the two side points
//     past the first tile per lane, which the FP64 one cannot afford in
//     registers: 4.08 against 4.32 ms per stage at 4M triangles); the adjoint on the
//     matrix cores at p = 3, 4 at every size (8-13% faster than four lanes
//     at 4M triangles; slower at p = 2, and at p = 5 it holds too many
//     registers).
// An explicit lane count keeps the vector-ALU kernels unless the matrix
// cores are switched on explicitly.
void apply_kernel_choice(dg_mesh m)
{
    dgk::MeshDev& d = m->dev;
    const bool small = d.n <= DG_LANES4_MAX_ELEMENTS;
    d.lanes4 = m->lanes_req == 4 || (m->lanes_req == 0 && (small || d.p >= 4));
    d.vjp_lanes4 = m->lanes_req == 4 || (m->lanes_req == 0 && (d.lanes4 || d.p >= 3));
    const bool mx_auto = m->lanes_req == 0 && (d.p == 4 || ((d.p == 3 || d.p == 5) && small));
    d.mx = m->mx_req == 1 || (m->mx_req == -1 && mx_auto);
    d.mx32 = m->mx_req == 1 || (m->mx_req == -1 && m->lanes_req == 0 && (mx_auto || d.p == 5));
    d.mx_vjp = m->mx_req == 1 || (m->mx_req == -1 && m->lanes_req == 0 && (d.p == 3 || d.p == 4));
}

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok()
{
    g_err.clear();
    return DG_OK;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(DG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

int n_vol_points(int p)
{
    static const int nq[6] = {0, 3, 6, 12, 16, 25};
    return nq[p];
}

// Position of grid cell (x, y), 0 <= x, y < 2^21, along the Hilbert curve
// that fills the 2^21 x 2^21 grid: quadrant by quadrant from the coarsest
// level, each quadrant's frame rotated / reflected so that consecutive cells
// are always edge neighbours (unlike a Morton curve, which jumps).
uint64_t hilbert_key(uint64_t x, uint64_t y)
{
    const uint64_t n = 1ULL << 21;
    uint64_t d = 0;
    for (uint64_t s = n >> 1; s > 0; s >>= 1) {
        const uint64_t rx = (x & s) ? 1 : 0, ry = (y & s) ? 1 : 0;
        d += s * s * ((3 * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = (n - 1) - x;
                y = (n - 1) - y;
            }
            const uint64_t t = x;
            x = y;
            y = t;
        }
    }
    return d;
}

}  // namespace

// Scratch memory of dg_rk_step_noalloc: the stage states of one step, in a
// device array that every GPU the library runs on holds until the process
// ends (one copy per device, at its own address).  In host code `scratch`
// only names the symbol; its device address comes from hipGetSymbolAddress,
// taken once per device with that device current (at the first
// dg_mesh_create on it) and kept in g_scratch_ptr.
static __device__ __align__(256) char scratch[DG_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Looks up (once) the device address of `scratch` on device `dev`, which
// must be the current device.
int scratch_setup(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(DG_EUNSUPPORTED, "device %d: at most %d devices", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return DG_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(DG_EHIP, "hipGetSymbolAddress(scratch) gave a null address");
    g_scratch_ptr[dev] = ptr;
    return DG_OK;
}

void* scratch_ptr(int dev)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return dev >= 0 && dev < MAX_DEVICES ? g_scratch_ptr[dev] : nullptr;
}

}  // namespace

extern "C" {

const char* dg_last_error(void) { return g_err.c_str(); }

int dg_mesh_validate(int p, int64_t n, const double* vxy, const int64_t* nbr, const int8_t* nbs)
{
    if (p < 1 || p > 5) return fail(DG_EORDER, "order p=%d outside 1..5", p);
    if (n < 1 || !vxy || !nbr || !nbs) return fail(DG_EINVAL, "n_elem must be >= 1 and all arrays non-null");
    const int64_t npad = (n + 63) / 64 * 64;
    const int np = dgh::n_modes(p);
    if (npad * std::max(4 * np, 12 * (p + 1)) >= (int64_t(1) << 31))
        return fail(DG_EUNSUPPORTED, "mesh too large for 32-bit element indexing (%lld elements at p=%d)",
                    (long long)n, p);
    for (int64_t i = 0; i < n; ++i) {
        const double* v = vxy + 6 * i;
        for (int c = 0; c < 6; ++c)
            if (!std::isfinite(v[c])) return fail(DG_EMESH, "element %lld: non-finite vertex coordinate", (long long)i);
        double det = (v[2] - v[0]) * (v[5] - v[1]) - (v[4] - v[0]) * (v[3] - v[1]);
        if (!(det > 0.0))
            return fail(DG_EMESH, "element %lld: det J = %g <= 0 (vertices must be counter-clockwise)", (long long)i,
                        det);
        for (int q = 0; q < 3; ++q) {
            int64_t j = nbr[3 * i + q];
            if (j < 0) {
                if (j < DG_BC_STATE)
                    return fail(DG_EUNSUPPORTED, "element %lld side %d: unknown boundary code %lld", (long long)i, q,
                                (long long)j);
                continue;  // a domain boundary: nothing to match
            }
            if (j >= n) return fail(DG_EMESH, "element %lld side %d: neighbour %lld out of range", (long long)i, q,
                                    (long long)j);
            int qn = nbs[3 * i + q];
            if (qn < 0 || qn > 2)
                return fail(DG_EMESH, "element %lld side %d: neighbour side %d outside 0..2", (long long)i, q, qn);
            if (nbr[3 * j + qn] != i || nbs[3 * j + qn] != q)
                return fail(DG_EMESH, "element %lld side %d: neighbour %lld side %d does not point back", (long long)i,
                            q, (long long)j, qn);
            if (j == i && qn == q) return fail(DG_EMESH, "element %lld side %d is its own neighbour", (long long)i, q);
            // the two copies of the edge must be the same segment traversed in
            // opposite directions (up to a periodic shift)
            const double* w = vxy + 6 * j;
            double ex = v[2 * ((q + 1) % 3)] - v[2 * q], ey = v[2 * ((q + 1) % 3) + 1] - v[2 * q + 1];
            double fx = w[2 * ((qn + 1) % 3)] - w[2 * qn], fy = w[2 * ((qn + 1) % 3) + 1] - w[2 * qn + 1];
            // tolerance: a periodic copy carries the rounding of the shifted
            // coordinates, which scales with their magnitude, not the length
            double len = std::sqrt(ex * ex + ey * ey);
            double mag = 0.0;
            for (int c = 0; c < 6; ++c) mag = std::fmax(mag, std::fmax(std::fabs(v[c]), std::fabs(w[c])));
            const double tol = 1e-12 * std::fmax(len, mag);
            if (std::fabs(ex + fx) > tol || std::fabs(ey + fy) > tol)
                return fail(DG_EMESH, "element %lld side %d and element %lld side %d are not the same edge",
                            (long long)i, q, (long long)j, qn);
        }
    }
    return ok();
}

int dg_mesh_create(int p, int64_t n, const double* vxy, const int64_t* nbr, const int8_t* nbs, double gamma,
                   dg_mesh* out)
{
    if (!out) return fail(DG_EINVAL, "out is null");
    *out = nullptr;
    int rc = dg_mesh_validate(p, n, vxy, nbr, nbs);
    if (rc != DG_OK) return rc;
    if (!(gamma > 1.0)) return fail(DG_EINVAL, "gamma must be > 1");

    const int np = dgh::n_modes(p), ne = p + 1, nq = n_vol_points(p);
    const int N = (int)n, npad = (N + 63) / 64 * 64;

    // element order along a Hilbert curve of the centroids
    std::vector<double> cx(N), cy(N);
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int i = 0; i < N; ++i) {
        const double* v = vxy + 6 * i;
        cx[i] = (v[0] + v[2] + v[4]) / 3.0;
        cy[i] = (v[1] + v[3] + v[5]) / 3.0;
        xmin = std::min(xmin, cx[i]);
        xmax = std::max(xmax, cx[i]);
        ymin = std::min(ymin, cy[i]);
        ymax = std::max(ymax, cy[i]);
    }
    const double span = std::max(std::max(xmax - xmin, ymax - ymin), 1e-300);
    std::vector<uint64_t> key(N);
    for (int i = 0; i < N; ++i) {
        uint64_t qx = (uint64_t)std::min(2097151.0, std::floor((cx[i] - xmin) / span * 2097151.0));
        uint64_t qy = (uint64_t)std::min(2097151.0, std::floor((cy[i] - ymin) / span * 2097151.0));
        key[i] = hilbert_key(qx, qy);
    }
    std::vector<int> perm(N), inv(N);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return key[a] < key[b]; });
    for (int i = 0; i < N; ++i) inv[perm[i]] = i;

    // geometry [blk][6][LANES] and vertices (internal order)
    std::vector<double> geo((size_t)npad * 6, 0.0), vtx((size_t)npad * 6, 0.0);
    for (int i = 0; i < N; ++i) {
        const double* v = vxy + 6 * perm[i];
        const double x1 = v[0], y1 = v[1], x2 = v[2], y2 = v[3], x3 = v[4], y3 = v[5];
        const double det = (x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1);
        double per = 0.0;
        for (int q = 0; q < 3; ++q) {
            double dx = v[2 * ((q + 1) % 3)] - v[2 * q], dy = v[2 * ((q + 1) % 3) + 1] - v[2 * q + 1];
            per += std::sqrt(dx * dx + dy * dy);
        }
        const size_t b = (size_t)(i / dgk::LANES) * 6 * dgk::LANES + (i % dgk::LANES);
        geo[b + 0 * dgk::LANES] = y3 - y1;     // adj(J) = det J * J^{-1}
        geo[b + 1 * dgk::LANES] = -(x3 - x1);
        geo[b + 2 * dgk::LANES] = -(y2 - y1);
        geo[b + 3 * dgk::LANES] = x2 - x1;
        geo[b + 4 * dgk::LANES] = 1.0 / det;
        geo[b + 5 * dgk::LANES] = det / per;   // inscribed radius
        std::memcpy(&vtx[(size_t)i * 6], v, 6 * sizeof(double));
    }

    // edges: boundary edges first, grouped by kind (Section "Surface
    // Integration Kernel": whole wavefronts then take the same branch), with
    // the boundary code in place of the right element; then one edge per
    // element pair, left = lower internal id, sorted by left
    std::vector<int> el, er, sd;
    std::vector<double> egx, egy, egl;
    el.reserve(3 * N / 2 + 1);
    auto add_edge = [&](int i, int j, int q, int qn) {
        const double* v = vxy + 6 * perm[i];
        double dx = v[2 * ((q + 1) % 3)] - v[2 * q], dy = v[2 * ((q + 1) % 3) + 1] - v[2 * q + 1];
        double len = std::sqrt(dx * dx + dy * dy);
        el.push_back(i);
        er.push_back(j);
        sd.push_back(q | (qn << 2));
        egx.push_back(dy / len);
        egy.push_back(-dx / len);
        egl.push_back(0.5 * len);
    };
    for (int code = DG_BC_WALL; code >= DG_BC_STATE; --code)
        for (int i = 0; i < N; ++i)
            for (int q = 0; q < 3; ++q)
                if (nbr[3 * perm[i] + q] == code) add_edge(i, code, q, 0);
    for (int i = 0; i < N; ++i) {
        const int u = perm[i];
        for (int q = 0; q < 3; ++q) {
            if (nbr[3 * u + q] < 0) continue;
            const int j = inv[nbr[3 * u + q]];
            const int qn = nbs[3 * u + q];
            if (j < i || (j == i && qn < q)) continue;
            add_edge(i, j, q, qn);
        }
    }
    const int nedge = (int)el.size();

    // greedy edge colouring in list order (lowest colour free at both
    // elements; at most 5 colours since an edge meets at most 4 others),
    // and a second copy of the edge arrays stably sorted by colour (within a
    // colour the boundary edges stay first, grouped by kind, and the
    // interior edges sorted by left element); the slot path keeps the list
    // order
    std::vector<unsigned char> used((size_t)N, 0), colour((size_t)nedge);
    int ncolour = 0;
    for (int i = 0; i < nedge; ++i) {
        const unsigned busy = used[el[i]] | (er[i] >= 0 ? used[er[i]] : 0u);
        int c = 0;
        while (busy & (1u << c)) ++c;
        colour[i] = (unsigned char)c;
        used[el[i]] |= (unsigned char)(1u << c);
        if (er[i] >= 0) used[er[i]] |= (unsigned char)(1u << c);
        ncolour = std::max(ncolour, c + 1);
    }
    if (ncolour > dgk::MeshDev::MAX_COLOURS) return fail(DG_EMESH, "edge colouring needs %d colours", ncolour);
    std::vector<int> order(nedge);
    for (int i = 0; i < nedge; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return colour[a] < colour[b]; });
    int colour_off[dgk::MeshDev::MAX_COLOURS + 1] = {};
    for (int i = 0; i < nedge; ++i) ++colour_off[colour[i] + 1];
    for (int c = 0; c < ncolour; ++c) colour_off[c + 1] += colour_off[c];
    std::vector<int> ecol((size_t)3 * nedge);  // [3][nedge]: left, right, sides in colour order
    std::vector<double> eg(3 * (size_t)nedge), egc(3 * (size_t)nedge);
    for (int i = 0; i < nedge; ++i) {
        eg[i] = egx[i];
        eg[nedge + i] = egy[i];
        eg[2 * (size_t)nedge + i] = egl[i];
        const int o = order[i];
        ecol[i] = el[o];
        ecol[nedge + i] = er[o];
        ecol[2 * (size_t)nedge + i] = sd[o];
        egc[i] = egx[o];
        egc[nedge + i] = egy[o];
        egc[2 * (size_t)nedge + i] = egl[o];
    }

    // per element side: neighbour (internal id), neighbour's side, own
    // outward unit normal and half length (from the element's own vertices)
    // A domain-boundary side gets the element itself as its "neighbour" (a
    // harmless gather) and its kind in side_bc (4 bits per side: 0 interior,
    // 1 wall, 2 outflow, 3 prescribed state).
    std::vector<int> snb((size_t)npad * 3, 0), sside((size_t)npad, 0), sbc((size_t)npad, 0);
    std::vector<double> sg((size_t)npad * 9, 0.0);
    bool has_bc = false;
    for (int i = 0; i < N; ++i) {
        const int u = perm[i];
        const double* v = vxy + 6 * u;
        const size_t b = (size_t)(i / dgk::LANES) * dgk::LANES;
        int packed = 0, bcs = 0;
        for (int q = 0; q < 3; ++q) {
            double dx = v[2 * ((q + 1) % 3)] - v[2 * q], dy = v[2 * ((q + 1) % 3) + 1] - v[2 * q + 1];
            double len = std::sqrt(dx * dx + dy * dy);
            const int64_t nq = nbr[3 * u + q];
            if (nq < 0) {
                has_bc = true;
                bcs |= (int)(-nq) << (4 * q);
                snb[b * 3 + q * dgk::LANES + i % dgk::LANES] = i;
            } else {
                snb[b * 3 + q * dgk::LANES + i % dgk::LANES] = inv[nq];
                packed |= nbs[3 * u + q] << (2 * q);
            }
            sg[b * 9 + (3 * q + 0) * dgk::LANES + i % dgk::LANES] = dy / len;
            sg[b * 9 + (3 * q + 1) * dgk::LANES + i % dgk::LANES] = -dx / len;
            sg[b * 9 + (3 * q + 2) * dgk::LANES + i % dgk::LANES] = 0.5 * len;
        }
        sside[b + i % dgk::LANES] = packed;
        sbc[b + i % dgk::LANES] = bcs;
    }

    dgh::TableLayout lay;
    std::vector<double> tab = dgh::build_tables(p, &lay);
    if (!dgk::table_offset_check(p, lay) || lay.nq != nq)
        return fail(DG_EUNSUPPORTED, "internal error: table layout mismatch at p=%d", p);

    int device = 0;
    if (hipError_t e = hipGetDevice(&device); e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if ((rc = scratch_setup(device)) != DG_OK) return rc;
    dg_mesh m = new dg_mesh_s();
    m->device = device;
    auto upload = [&](const void* src, size_t bytes, void** dst) -> int {
        void* d = nullptr;
        hipError_t e = hipMalloc(&d, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? DG_ENOMEM : DG_EHIP, "hipMalloc(%zu): %s", bytes,
                                         hipGetErrorString(e));
        m->allocs.push_back(d);
        if (bytes) {
            e = hipMemcpy(d, src, bytes, hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
        }
        *dst = d;
        return DG_OK;
    };
    std::vector<float> tab32(tab.begin(), tab.end());
    std::vector<double> tabmx = dgh::build_mx_tables(p, tab, lay, true);
    const std::vector<double> tabmx32d = dgh::build_mx_tables(p, tab, lay, false);
    std::vector<float> tabmx32(tabmx32d.begin(), tabmx32d.end());
    void *d_tab32, *d_tabmx, *d_tabmx32;
    void *d_tab, *d_geo, *d_vtx, *d_perm, *d_el, *d_er, *d_sd, *d_eg, *d_snb, *d_sside, *d_sg, *d_sbc, *d_bcs;
    void *d_ecol, *d_egc;
    const double bc_state0[4] = {1.0, 0.0, 0.0, 1.0 / (gamma - 1.0)};  // until dg_set_boundary_state: at rest, p = 1
    if ((rc = upload(tab.data(), tab.size() * 8, &d_tab)) || (rc = upload(tab32.data(), tab32.size() * 4, &d_tab32)) ||
        (rc = upload(tabmx.data(), tabmx.size() * 8, &d_tabmx)) ||
        (rc = upload(tabmx32.data(), tabmx32.size() * 4, &d_tabmx32)) || (rc = upload(geo.data(), geo.size() * 8, &d_geo)) ||
        (rc = upload(vtx.data(), vtx.size() * 8, &d_vtx)) || (rc = upload(perm.data(), perm.size() * 4, &d_perm)) ||
        (rc = upload(el.data(), el.size() * 4, &d_el)) || (rc = upload(er.data(), er.size() * 4, &d_er)) ||
        (rc = upload(sd.data(), sd.size() * 4, &d_sd)) || (rc = upload(eg.data(), eg.size() * 8, &d_eg)) ||
        (rc = upload(snb.data(), snb.size() * 4, &d_snb)) || (rc = upload(sside.data(), sside.size() * 4, &d_sside)) ||
        (rc = upload(sg.data(), sg.size() * 8, &d_sg)) || (rc = upload(sbc.data(), sbc.size() * 4, &d_sbc)) ||
        (rc = upload(bc_state0, sizeof(bc_state0), &d_bcs)) || (rc = upload(ecol.data(), ecol.size() * 4, &d_ecol)) ||
        (rc = upload(egc.data(), egc.size() * 8, &d_egc))) {
        std::string msg = g_err;
        dg_mesh_destroy(m);
        return fail(rc, "%s", msg.c_str());
    }
    dgk::MeshDev& d = m->dev;
    d.p = p;
    d.np = np;
    d.nq = nq;
    d.ne = ne;
    d.n = N;
    d.npad = npad;
    d.nedge = nedge;
    d.ncolour = ncolour;
    d.ecol = (const int*)d_ecol;
    d.edge_gc = (const double*)d_egc;
    for (int c = 0; c <= ncolour; ++c) d.colour_off[c] = colour_off[c];
    d.gamma = gamma;
    d.tab = (const double*)d_tab;
    d.tab32 = (const float*)d_tab32;
    d.tabmx = (const double*)d_tabmx;
    d.tabmx32 = (const float*)d_tabmx32;
    d.geo = (const double*)d_geo;
    d.vtx = (const double*)d_vtx;
    d.perm = (const int*)d_perm;
    d.edge_l = (const int*)d_el;
    d.edge_r = (const int*)d_er;
    d.edge_sd = (const int*)d_sd;
    d.edge_g = (const double*)d_eg;
    d.side_nb = (const int*)d_snb;
    d.side_q = (const int*)d_sside;
    d.side_g = (const double*)d_sg;
    d.side_bc = (const int*)d_sbc;
    d.bc_state = (double*)d_bcs;
    d.has_bc = has_bc;
    m->lay = lay;
    apply_kernel_choice(m);

    const size_t state = align256((size_t)npad * 4 * np * 8);
    const size_t trace = align256((size_t)npad * 3 * ne * 4 * 8);
    const size_t part = align256((size_t)dgk::dt_partials(d) * 8);
    // S: the side slots of the edge-wise mode, or the accumulator state of
    // the coloured mode
    // V: the volume integral of the two-stream edge-wise path
    const size_t slot = std::max(trace, state);
    const size_t part4 = align256((size_t)dgk::stage4_partials(d) * 8);
    m->off_T0 = 0;
    m->off_S = trace;
    m->off_part = trace + slot;
    m->off_V = trace + slot + part;
    m->ws_rhs = (int64_t)(m->off_V + state);
    m->off_T1 = m->off_V + state;
    m->off_u1 = m->off_T1 + trace;
    m->off_u2 = m->off_u1 + state;
    m->off_part4 = m->off_u2 + state;
    m->off_acc = m->off_part4 + part4;
    m->ws_step = (int64_t)(m->off_acc + state);
    m->state_bytes = state;
    m->ws_vjp = (int64_t)(4 * state);
    *out = m;
    return ok();
}

int dg_mesh_destroy(dg_mesh m)
{
    if (!m) return ok();
    for (auto& r : m->recs) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : m->pool) (void)hipEventDestroy(e);
    if (m->side) {
        (void)hipStreamSynchronize(m->side);
        (void)hipStreamDestroy(m->side);
    }
    if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
    if (m->ev_join) (void)hipEventDestroy(m->ev_join);
    for (void* p : m->allocs) (void)hipFree(p);
    delete m;
    return ok();
}

int dg_mesh_info(dg_mesh m, dg_info* out)
{
    if (!m || !out) return fail(DG_EINVAL, "null argument");
    out->p = m->dev.p;
    out->n_modes = m->dev.np;
    out->n_vol_points = m->dev.nq;
    out->n_edge_points = m->dev.ne;
    out->n_elem = m->dev.n;
    out->n_elem_pad = m->dev.npad;
    out->n_edges = m->dev.nedge;
    out->n_colours = m->dev.ncolour;
    out->state_len = (int64_t)m->dev.npad * 4 * m->dev.np;
    out->ws_rhs = m->ws_rhs;
    out->ws_step = m->ws_step;
    out->ws_vjp = m->ws_vjp;
    const int lanes = m->dev.lanes4 ? 4 : 1;
    out->stage_fp64 = m->dev.mx ? 16 : lanes;
    out->stage_mixed = m->dev.mx32 ? 16 : lanes;
    out->adjoint = m->dev.mx_vjp ? 16 : (m->dev.vjp_lanes4 || m->dev.p >= 4 ? 4 : 1);
    return ok();
}

}  // extern "C"

namespace {

hipEvent_t take_event(dg_mesh m)
{
    if (!m->pool.empty()) {
        hipEvent_t e = m->pool.back();
        m->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Runs `launch` on stream s, bracketed by events when timing is on.
template <class F>
void timed(dg_mesh m, int kind, hipStream_t s, F&& launch)
{
    if (!m->timing) {
        launch();
        return;
    }
    dg_mesh_s::Rec r{kind, take_event(m), take_event(m)};
    (void)hipEventRecord(r.a, s);
    launch();
    (void)hipEventRecord(r.b, s);
    m->recs.push_back(r);
}

// Two-stream section of the edge-wise path: fork() makes the side stream
// wait for the work queued so far on s; join() makes s wait for what was
// queued on the side stream.
hipError_t fork(dg_mesh m, hipStream_t s)
{
    hipError_t e = hipEventRecord(m->ev_fork, s);
    return e == hipSuccess ? hipStreamWaitEvent(m->side, m->ev_fork, 0) : e;
}
hipError_t join(dg_mesh m, hipStream_t s)
{
    hipError_t e = hipEventRecord(m->ev_join, m->side);
    return e == hipSuccess ? hipStreamWaitEvent(s, m->ev_join, 0) : e;
}

}  // namespace

extern "C" {

static int check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return ok();
}

int dg_quad_points(dg_mesh m, double* xy, void* stream)
{
    if (!m || !xy) return fail(DG_EINVAL, "null argument");
    dgk::launch_quad_points(m->dev, xy, (hipStream_t)stream);
    return check_launch("dg_quad_points");
}

int dg_project(dg_mesh m, const double* u, double* C, void* stream)
{
    if (!m || !u || !C) return fail(DG_EINVAL, "null argument");
    dgk::launch_project(m->dev, u, C, (hipStream_t)stream);
    return check_launch("dg_project");
}

int dg_pack(dg_mesh m, const double* Cu, double* C, void* stream)
{
    if (!m || !Cu || !C) return fail(DG_EINVAL, "null argument");
    dgk::launch_pack(m->dev, Cu, C, (hipStream_t)stream);
    return check_launch("dg_pack");
}

int dg_unpack(dg_mesh m, const double* C, double* Cu, void* stream)
{
    if (!m || !C || !Cu) return fail(DG_EINVAL, "null argument");
    dgk::launch_unpack(m->dev, C, Cu, (hipStream_t)stream);
    return check_launch("dg_unpack");
}

int dg_rhs(dg_mesh m, const double* C, double* R, dg_precision prec, void* ws, void* stream)
{
    if (!m || !C || !R || !ws) return fail(DG_EINVAL, "null argument");
    if (prec != DG_FP64 && prec != DG_MIXED) return fail(DG_EINVAL, "unknown precision %d", prec);
    if (prec == DG_MIXED && m->surface != DG_SURFACE_ELEMENTWISE)
        return fail(DG_EUNSUPPORTED, "DG_MIXED needs the element-wise surface mode");
    char* w = (char*)ws;
    double* T = (double*)(w + m->off_T0);
    double* S = (double*)(w + m->off_S);
    hipStream_t s = (hipStream_t)stream;
    if (m->surface == DG_SURFACE_ELEMENTWISE) {
        const bool mixed = prec == DG_MIXED;
        timed(m, DG_KERNEL_STAGE, s, [&] { dgk::launch_stage(m->dev, 0, mixed, C, nullptr, R, 0.0, nullptr, s); });
        return check_launch("dg_rhs");
    }
    if (m->surface == DG_SURFACE_COLOURED) {
        timed(m, DG_KERNEL_TRACES, s, [&] { dgk::launch_traces(m->dev, C, T, s, S); });
        timed(m, DG_KERNEL_EDGE, s, [&] { dgk::launch_edge_lift(m->dev, T, S, s); });
        timed(m, DG_KERNEL_ELEMENT, s,
              [&] { dgk::launch_element(m->dev, 0, C, nullptr, R, nullptr, 0.0, nullptr, nullptr, s, S, 1); });
        return check_launch("dg_rhs");
    }
    if (m->concurrent) {
        double* V = (double*)(w + m->off_V);
        hipError_t e = fork(m, s);
        if (e != hipSuccess) return hip_fail(e, "dg_rhs (stream fork)");
        timed(m, DG_KERNEL_VOLUME, m->side, [&] { dgk::launch_volume(m->dev, C, V, m->side); });
        timed(m, DG_KERNEL_TRACES, s, [&] { dgk::launch_traces(m->dev, C, T, s); });
        timed(m, DG_KERNEL_EDGE, s, [&] { dgk::launch_edge_flux(m->dev, T, S, s); });
        if ((e = join(m, s)) != hipSuccess) return hip_fail(e, "dg_rhs (stream join)");
        timed(m, DG_KERNEL_ELEMENT, s,
              [&] { dgk::launch_element(m->dev, 0, C, nullptr, R, S, 0.0, nullptr, nullptr, s, V, 2); });
        return check_launch("dg_rhs");
    }
    timed(m, DG_KERNEL_TRACES, s, [&] { dgk::launch_traces(m->dev, C, T, s); });
    timed(m, DG_KERNEL_EDGE, s, [&] { dgk::launch_edge_flux(m->dev, T, S, s); });
    timed(m, DG_KERNEL_ELEMENT, s, [&] { dgk::launch_element(m->dev, 0, C, nullptr, R, S, 0.0, nullptr, nullptr, s); });
    return check_launch("dg_rhs");
}

int dg_max_dt(dg_mesh m, const double* C, double cfl, double* dt_dev, double* dt_host, void* ws, void* stream)
{
    if (!m || !C || !dt_dev || !ws) return fail(DG_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    timed(m, DG_KERNEL_DT, s, [&] { dgk::launch_dt(m->dev, C, cfl, (double*)((char*)ws + m->off_part), dt_dev, s); });
    int rc = check_launch("dg_max_dt");
    if (rc != DG_OK || !dt_host) return rc;
    hipError_t e = hipMemcpyAsync(dt_host, dt_dev, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "dg_max_dt copy");
    if (std::isnan(*dt_host)) return fail(DG_ENONPHYS, "non-physical element mean (rho <= 0, p <= 0 or NaN)");
    return ok();
}

// the limiter after an RK stage, when the mesh has it switched on (the
// paper limits every intermediate stage and the new time level)
static void limit_stage(dg_mesh m, double* U, hipStream_t s)
{
    if (m->limiter == DG_LIMITER_BJ) timed(m, DG_KERNEL_LIMIT, s, [&] { dgk::launch_limit(m->dev, U, s); });
}

// The element-wise step (SSP-RK3, or the classic RK2 / RK4) with its stage
// states at u1, u2 and, for RK4, the running sum at acc.  With `timing`
// false no launch is bracketed by events (the allocation-free entry point
// creates none).
static void rk_step_elementwise(dg_mesh m, double* C, double dt, const double* dt_dev, bool mx, double* u1,
                                double* u2, double* acc, hipStream_t s, bool timing)
{
    const dgk::MeshDev& d = m->dev;
    auto run = [&](int kind, auto&& launch) {
        if (timing)
            timed(m, kind, s, launch);
        else
            launch();
    };
    auto limit = [&](double* U) {
        if (m->limiter == DG_LIMITER_BJ) run(DG_KERNEL_LIMIT, [&] { dgk::launch_limit(d, U, s); });
    };
    if (m->integrator == DG_RK2) {
        // Heun: u1 = u + dt L(u);  u = 1/2 u + 1/2 (u1 + dt L(u1))
        dgk::StageGen g2;
        g2.a = 0.5;
        g2.b = 0.5;
        g2.g = 0.5;  // X = the output (stage-0) state itself
        run(DG_KERNEL_STAGE, [&] { dgk::launch_stage(d, 1, mx, C, nullptr, u1, dt, dt_dev, s); });
        limit(u1);
        run(DG_KERNEL_STAGE, [&] { dgk::launch_stage_general(d, mx, u1, C, dt, dt_dev, g2, s); });
        limit(C);
        return;
    }
    if (m->integrator == DG_RK4) {
        // classic RK4 with the running sum S = u + dt (k1 + 2 k2 + 2 k3) / 6
        dgk::StageGen g;
        g.b = 1.0;
        g.g = 0.5;
        g.S = acc;
        g.d = 1.0 / 6.0;
        g.s_init = 1;  // u1 = u + dt/2 k1, S = u + dt/6 k1
        run(DG_KERNEL_STAGE, [&] { dgk::launch_stage_general(d, mx, C, u1, dt, dt_dev, g, s); });
        limit(u1);
        g = dgk::StageGen();
        g.a = 1.0;
        g.X = C;
        g.g = 0.5;
        g.S = acc;
        g.d = 1.0 / 3.0;  // u2 = u + dt/2 k2, S += dt/3 k2
        run(DG_KERNEL_STAGE, [&] { dgk::launch_stage_general(d, mx, u1, u2, dt, dt_dev, g, s); });
        limit(u2);
        g.g = 1.0;  // u3 = u + dt k3, S += dt/3 k3 (u3 reuses u1)
        run(DG_KERNEL_STAGE, [&] { dgk::launch_stage_general(d, mx, u2, u1, dt, dt_dev, g, s); });
        limit(u1);
        g = dgk::StageGen();
        g.a = 1.0;
        g.X = acc;
        g.g = 1.0 / 6.0;  // u = S + dt/6 k4
        run(DG_KERNEL_STAGE, [&] { dgk::launch_stage_general(d, mx, u1, C, dt, dt_dev, g, s); });
        limit(C);
        return;
    }
    run(DG_KERNEL_STAGE, [&] { dgk::launch_stage(d, 1, mx, C, nullptr, u1, dt, dt_dev, s); });
    limit(u1);
    run(DG_KERNEL_STAGE, [&] { dgk::launch_stage(d, 2, mx, u1, C, u2, dt, dt_dev, s); });
    limit(u2);
    run(DG_KERNEL_STAGE, [&] { dgk::launch_stage(d, 3, mx, u2, nullptr, C, dt, dt_dev, s); });
    limit(C);
}

int dg_rk_step(dg_mesh m, double* C, double dt, const double* dt_dev, dg_precision prec, void* ws, void* stream)
{
    if (!m || !C || !ws) return fail(DG_EINVAL, "null argument");
    if (prec != DG_FP64 && prec != DG_MIXED) return fail(DG_EINVAL, "unknown precision %d", prec);
    if (prec == DG_MIXED && m->surface != DG_SURFACE_ELEMENTWISE)
        return fail(DG_EUNSUPPORTED, "DG_MIXED needs the element-wise surface mode");
    char* w = (char*)ws;
    double* T0 = (double*)(w + m->off_T0);
    double* T1 = (double*)(w + m->off_T1);
    double* S = (double*)(w + m->off_S);
    double* u1 = (double*)(w + m->off_u1);
    double* u2 = (double*)(w + m->off_u2);
    hipStream_t s = (hipStream_t)stream;
    const dgk::MeshDev& d = m->dev;
    if (m->limiter != DG_LIMITER_NONE && m->surface != DG_SURFACE_ELEMENTWISE)
        return fail(DG_EUNSUPPORTED, "the limiter needs the element-wise surface mode");
    if (m->integrator != DG_RK_SSP3 && m->surface != DG_SURFACE_ELEMENTWISE)
        return fail(DG_EUNSUPPORTED, "RK2 / RK4 need the element-wise surface mode");
    if (m->surface == DG_SURFACE_ELEMENTWISE) {
        rk_step_elementwise(m, C, dt, dt_dev, prec == DG_MIXED, u1, u2, (double*)(w + m->off_acc), s, true);
        return check_launch("dg_rk_step");
    }
    if (m->surface == DG_SURFACE_COLOURED) {
        timed(m, DG_KERNEL_TRACES, s, [&] { dgk::launch_traces(d, C, T0, s, S); });
        timed(m, DG_KERNEL_EDGE, s, [&] { dgk::launch_edge_lift(d, T0, S, s); });
        timed(m, DG_KERNEL_ELEMENT, s, [&] { dgk::launch_element(d, 1, C, nullptr, u1, nullptr, dt, dt_dev, T1, s, S, 1); });
        timed(m, DG_KERNEL_EDGE, s, [&] { dgk::launch_edge_lift(d, T1, S, s); });
        timed(m, DG_KERNEL_ELEMENT, s, [&] { dgk::launch_element(d, 2, u1, C, u2, nullptr, dt, dt_dev, T0, s, S, 1); });
        timed(m, DG_KERNEL_EDGE, s, [&] { dgk::launch_edge_lift(d, T0, S, s); });
        timed(m, DG_KERNEL_ELEMENT, s, [&] { dgk::launch_element(d, 3, u2, C, C, nullptr, dt, dt_dev, nullptr, s, S, 1); });
        return check_launch("dg_rk_step");
    }
    if (m->concurrent) {
        // per stage: the volume integral of the stage input on the side
        // stream, beside the traces (stage 1) and edge fluxes on s
        double* V = (double*)(w + m->off_V);
        auto stage = [&](int mode, const double* X, const double* U0, double* out, const double* Tin,
                         double* Tn) -> hipError_t {
            hipError_t e = fork(m, s);
            if (e != hipSuccess) return e;
            timed(m, DG_KERNEL_VOLUME, m->side, [&] { dgk::launch_volume(d, X, V, m->side); });
            if (mode == 1) timed(m, DG_KERNEL_TRACES, s, [&] { dgk::launch_traces(d, X, T0, s); });
            timed(m, DG_KERNEL_EDGE, s, [&] { dgk::launch_edge_flux(d, Tin, S, s); });
            if ((e = join(m, s)) != hipSuccess) return e;
            timed(m, DG_KERNEL_ELEMENT, s,
                  [&] { dgk::launch_element(d, mode, X, U0, out, S, dt, dt_dev, Tn, s, V, 2); });
            return hipSuccess;
        };
        hipError_t e = stage(1, C, nullptr, u1, T0, T1);
        if (e == hipSuccess) e = stage(2, u1, C, u2, T1, T0);
        if (e == hipSuccess) e = stage(3, u2, C, C, T0, nullptr);
        if (e != hipSuccess) return hip_fail(e, "dg_rk_step (stream fork / join)");
        return check_launch("dg_rk_step");
    }
    timed(m, DG_KERNEL_TRACES, s, [&] { dgk::launch_traces(d, C, T0, s); });
    timed(m, DG_KERNEL_EDGE, s, [&] { dgk::launch_edge_flux(d, T0, S, s); });
    timed(m, DG_KERNEL_ELEMENT, s, [&] { dgk::launch_element(d, 1, C, nullptr, u1, S, dt, dt_dev, T1, s); });
    timed(m, DG_KERNEL_EDGE, s, [&] { dgk::launch_edge_flux(d, T1, S, s); });
    timed(m, DG_KERNEL_ELEMENT, s, [&] { dgk::launch_element(d, 2, u1, C, u2, S, dt, dt_dev, T0, s); });
    timed(m, DG_KERNEL_EDGE, s, [&] { dgk::launch_edge_flux(d, T0, S, s); });
    timed(m, DG_KERNEL_ELEMENT, s, [&] { dgk::launch_element(d, 3, u2, C, C, S, dt, dt_dev, nullptr, s); });
    return check_launch("dg_rk_step");
}

int dg_rk_step_noalloc(dg_mesh m, double* C, double dt, const double* dt_dev, dg_precision prec, void* stream)
{
    if (!m || !C) return fail(DG_EINVAL, "null argument");
    if (prec != DG_FP64 && prec != DG_MIXED) return fail(DG_EINVAL, "unknown precision %d", prec);
    if (m->surface != DG_SURFACE_ELEMENTWISE)
        return fail(DG_EUNSUPPORTED, "dg_rk_step_noalloc runs the element-wise surface mode only");
    // scratch layout: u1, u2 and, for RK4, the running sum
    const size_t need = (m->integrator == DG_RK4 ? 3 : 2) * m->state_bytes;
    if (need > (size_t)DG_NOALLOC_SCRATCH_BYTES)
        return fail(DG_EUNSUPPORTED,
                    "dg_rk_step_noalloc: this mesh needs %zu bytes of stage states, the static scratch holds %zu "
                    "(use dg_rk_step with a workspace)",
                    need, (size_t)DG_NOALLOC_SCRATCH_BYTES);
    int dev = -1;
    if (hipError_t e = hipGetDevice(&dev); e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != m->device)
        return fail(DG_EINVAL, "the mesh lives on device %d but device %d is current", m->device, dev);
    char* w = (char*)scratch_ptr(dev);
    if (!w) return fail(DG_EHIP, "no scratch address for device %d", dev);
    rk_step_elementwise(m, C, dt, dt_dev, prec == DG_MIXED, (double*)w, (double*)(w + m->state_bytes),
                        (double*)(w + 2 * m->state_bytes), (hipStream_t)stream, false);
    return check_launch("dg_rk_step_noalloc");
}

int dg_rhs_vjp(dg_mesh m, const double* C, const double* Rb, double* Cb, void* ws, void* stream)
{
    if (!m || !C || !Rb || !Cb) return fail(DG_EINVAL, "null argument");
    (void)ws;
    hipStream_t s = (hipStream_t)stream;
    timed(m, DG_KERNEL_VJP, s,
          [&] { dgk::launch_stage_vjp(m->dev, 0, C, Rb, nullptr, nullptr, Cb, 1.0, nullptr, s); });
    return check_launch("dg_rhs_vjp");
}

int dg_advance(dg_mesh m, double* C, int64_t nsteps, double cfl, double* dt_dev, double* dt_hist,
               dg_precision prec, void* ws, void* stream)
{
    if (!m || !C || !dt_dev || !ws) return fail(DG_EINVAL, "null argument");
    if (nsteps < 0) return fail(DG_EINVAL, "nsteps < 0");
    if (prec != DG_FP64 && prec != DG_MIXED) return fail(DG_EINVAL, "unknown precision %d", prec);
    if (prec == DG_MIXED && m->surface != DG_SURFACE_ELEMENTWISE)
        return fail(DG_EUNSUPPORTED, "DG_MIXED needs the element-wise surface mode");
    if (m->limiter != DG_LIMITER_NONE && m->surface != DG_SURFACE_ELEMENTWISE)
        return fail(DG_EUNSUPPORTED, "the limiter needs the element-wise surface mode");
    hipStream_t s = (hipStream_t)stream;
    const dgk::MeshDev& d = m->dev;
    char* w = (char*)ws;
    double* part = (double*)(w + m->off_part);
    double* part4 = (double*)(w + m->off_part4);
    // the per-64-element minima of the fused step length come from the
    // four-lane and matrix-core stage kernels
    const bool fused_dt = d.lanes4 || (prec == DG_FP64 ? d.mx : d.mx32);
    if (m->surface != DG_SURFACE_ELEMENTWISE || !fused_dt || m->integrator != DG_RK_SSP3) {
        // separate reduction each step
        for (int64_t k = 0; k < nsteps; ++k) {
            timed(m, DG_KERNEL_DT, s, [&] {
                dgk::launch_dt(d, C, cfl, part, dt_dev, s);
                if (dt_hist) (void)hipMemcpyAsync(dt_hist + k, dt_dev, 8, hipMemcpyDeviceToDevice, s);
            });
            int rc = dg_rk_step(m, C, 0.0, dt_dev, prec, ws, stream);
            if (rc != DG_OK) return rc;
        }
        return check_launch("dg_advance");
    }
    const bool mx = prec == DG_MIXED;
    double* u1 = (double*)(w + m->off_u1);
    double* u2 = (double*)(w + m->off_u2);
    // fused: stage 3 leaves per-block minima, stage 1 of the next step turns
    // them into its step length (a separate final pass when they are many)
    const int cnt4 = dgk::stage4_partials(d);
    constexpr int FUSE_MAX = 4096;
    if (nsteps > 0) timed(m, DG_KERNEL_DT, s, [&] { dgk::launch_dt_partials_only(d, C, part, s); });
    for (int64_t k = 0; k < nsteps; ++k) {
        const double* pin = k == 0 ? part : part4;
        const int cnt = k == 0 ? dgk::dt_partials(d) : cnt4;
        dgk::FusedDt f1;
        if (cnt <= FUSE_MAX) {
            f1.pin = pin;
            f1.pin_count = cnt;
            f1.cfl = cfl;
            f1.dt_store = dt_dev;
            f1.dt_hist = dt_hist ? dt_hist + k : nullptr;
        } else {
            timed(m, DG_KERNEL_DT, s,
                  [&] { dgk::launch_dt_final(pin, cnt, cfl, dt_dev, dt_hist ? dt_hist + k : nullptr, s); });
        }
        dgk::FusedDt f3;
        f3.pout = part4;
        timed(m, DG_KERNEL_STAGE, s, [&] { dgk::launch_stage(d, 1, mx, C, nullptr, u1, 0.0, dt_dev, s, f1); });
        limit_stage(m, u1, s);
        timed(m, DG_KERNEL_STAGE, s, [&] { dgk::launch_stage(d, 2, mx, u1, C, u2, 0.0, dt_dev, s); });
        limit_stage(m, u2, s);
        timed(m, DG_KERNEL_STAGE, s, [&] { dgk::launch_stage(d, 3, mx, u2, nullptr, C, 0.0, dt_dev, s, f3); });
        limit_stage(m, C, s);
    }
    return check_launch("dg_advance");
}

int dg_rk_step_stages(dg_mesh m, double* C, double dt, const double* dt_dev, double* u1, double* u2, void* ws,
                      void* stream)
{
    if (!m || !C || !u1 || !u2) return fail(DG_EINVAL, "null argument");
    if (m->integrator != DG_RK_SSP3) return fail(DG_EUNSUPPORTED, "the stage states are those of SSP-RK3");
    (void)ws;
    hipStream_t s = (hipStream_t)stream;
    const dgk::MeshDev& d = m->dev;
    timed(m, DG_KERNEL_STAGE, s, [&] { dgk::launch_stage(d, 1, false, C, nullptr, u1, dt, dt_dev, s); });
    limit_stage(m, u1, s);
    timed(m, DG_KERNEL_STAGE, s, [&] { dgk::launch_stage(d, 2, false, u1, C, u2, dt, dt_dev, s); });
    limit_stage(m, u2, s);
    timed(m, DG_KERNEL_STAGE, s, [&] { dgk::launch_stage(d, 3, false, u2, nullptr, C, dt, dt_dev, s); });
    limit_stage(m, C, s);
    return check_launch("dg_rk_step_stages");
}

int dg_rk_step_stages_to(dg_mesh m, const double* C, double* Cn, double dt, const double* dt_dev, double* u1,
                         double* u2, void* ws, void* stream)
{
    if (!m || !C || !Cn || !u1 || !u2) return fail(DG_EINVAL, "null argument");
    if (Cn == C || Cn == u1 || Cn == u2) return fail(DG_EINVAL, "Cnext must not overlap C, u1 or u2");
    if (m->integrator != DG_RK_SSP3) return fail(DG_EUNSUPPORTED, "the stage states are those of SSP-RK3");
    (void)ws;
    hipStream_t s = (hipStream_t)stream;
    const dgk::MeshDev& d = m->dev;
    timed(m, DG_KERNEL_STAGE, s, [&] { dgk::launch_stage(d, 1, false, C, nullptr, u1, dt, dt_dev, s); });
    limit_stage(m, u1, s);
    timed(m, DG_KERNEL_STAGE, s, [&] { dgk::launch_stage(d, 2, false, u1, C, u2, dt, dt_dev, s); });
    limit_stage(m, u2, s);
    dgk::StageGen gs;
    gs.a = 1.0 / 3.0;
    gs.X = C;
    gs.b = 2.0 / 3.0;
    gs.g = 2.0 / 3.0;
    timed(m, DG_KERNEL_STAGE, s, [&] { dgk::launch_stage_general(d, false, u2, Cn, dt, dt_dev, gs, s); });
    limit_stage(m, Cn, s);
    return check_launch("dg_rk_step_stages_to");
}

int dg_rk_step_vjp(dg_mesh m, const double* C, double dt, const double* dt_dev, const double* u1_in,
                   const double* u2_in, const double* ub, double* Cb, void* ws, void* stream)
{
    if (!m || !C || !ub || !Cb || !ws) return fail(DG_EINVAL, "null argument");
    if ((u1_in == nullptr) != (u2_in == nullptr)) return fail(DG_EINVAL, "pass both stage states or neither");
    if (m->limiter != DG_LIMITER_NONE)
        return fail(DG_EUNSUPPORTED, "the limited step is not differentiable; switch the limiter off");
    if (m->integrator != DG_RK_SSP3) return fail(DG_EUNSUPPORTED, "the step adjoint is that of SSP-RK3");
    hipStream_t s = (hipStream_t)stream;
    const dgk::MeshDev& d = m->dev;
    char* w = (char*)ws;
    double* u1 = (double*)(w);
    double* u2 = (double*)(w + m->state_bytes);
    double* u2b = (double*)(w + 2 * m->state_bytes);
    double* u1b = (double*)(w + 3 * m->state_bytes);
    if (u1_in) {
        u1 = const_cast<double*>(u1_in);
        u2 = const_cast<double*>(u2_in);
    } else {
        timed(m, DG_KERNEL_STAGE, s, [&] { dgk::launch_stage(d, 1, false, C, nullptr, u1, dt, dt_dev, s); });
        timed(m, DG_KERNEL_STAGE, s, [&] { dgk::launch_stage(d, 2, false, u1, C, u2, dt, dt_dev, s); });
    }
    timed(m, DG_KERNEL_VJP, s, [&] { dgk::launch_stage_vjp(d, 1, u2, ub, nullptr, nullptr, u2b, dt, dt_dev, s); });
    timed(m, DG_KERNEL_VJP, s, [&] { dgk::launch_stage_vjp(d, 2, u1, u2b, nullptr, nullptr, u1b, dt, dt_dev, s); });
    timed(m, DG_KERNEL_VJP, s, [&] { dgk::launch_stage_vjp(d, 3, C, u1b, ub, u2b, Cb, dt, dt_dev, s); });
    return check_launch("dg_rk_step_vjp");
}

int dg_eval_points(dg_mesh m, const double* C, double* u, void* stream)
{
    if (!m || !C || !u) return fail(DG_EINVAL, "null argument");
    dgk::launch_eval_points(m->dev, C, u, (hipStream_t)stream);
    return check_launch("dg_eval_points");
}

int dg_quad_weights(dg_mesh m, double* w, void* stream)
{
    if (!m || !w) return fail(DG_EINVAL, "null argument");
    dgk::launch_quad_weights(m->dev, w, (hipStream_t)stream);
    return check_launch("dg_quad_weights");
}

int dg_set_lanes_per_element(dg_mesh m, int lanes)
{
    if (!m) return fail(DG_EINVAL, "null mesh");
    if (lanes != 0 && lanes != 1 && lanes != 4) return fail(DG_EINVAL, "lanes per element must be 0, 1 or 4");
    if (lanes == 1 && m->dev.p >= 4)
        return fail(DG_EUNSUPPORTED, "one lane per element holds more values than a lane has registers from p = 4 on "
                                     "(p = %d): use 4 lanes (or 0, automatic)", m->dev.p);
    m->lanes_req = lanes;
    apply_kernel_choice(m);
    return ok();
}

int dg_set_matrix_cores(dg_mesh m, int on)
{
    if (!m) return fail(DG_EINVAL, "null mesh");
    if (on != 0 && on != 1 && on != -1)
        return fail(DG_EINVAL, "matrix cores: -1 (automatic), 0 (off) or 1 (on), not %d", on);
    m->mx_req = on;
    apply_kernel_choice(m);
    return ok();
}

int dg_set_boundary_state(dg_mesh m, const double* U)
{
    if (!m || !U) return fail(DG_EINVAL, "null argument");
    const double rho = U[0], p = (m->dev.gamma - 1.0) * (U[3] - 0.5 * (U[1] * U[1] + U[2] * U[2]) / rho);
    if (!(rho > 0.0) || !(p > 0.0)) return fail(DG_EINVAL, "boundary state is not physical (rho = %g, p = %g)", rho, p);
    // the state is read by kernels that may still be running on any stream:
    // let them finish before it changes
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(m->dev.bc_state, U, 4 * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "dg_set_boundary_state");
    return ok();
}

int dg_set_integrator(dg_mesh m, int scheme)
{
    if (!m) return fail(DG_EINVAL, "null mesh");
    if (scheme != DG_RK_SSP3 && scheme != DG_RK2 && scheme != DG_RK4)
        return fail(DG_EINVAL, "unknown integrator %d", scheme);
    m->integrator = scheme;
    return ok();
}

int dg_set_limiter(dg_mesh m, int limiter)
{
    if (!m) return fail(DG_EINVAL, "null mesh");
    if (limiter != DG_LIMITER_NONE && limiter != DG_LIMITER_BJ) return fail(DG_EINVAL, "unknown limiter %d", limiter);
    if (limiter == DG_LIMITER_BJ && m->dev.p != 1)
        return fail(DG_EUNSUPPORTED, "the Barth-Jespersen limiter is defined for p = 1 (this mesh has p = %d)", m->dev.p);
    m->limiter = limiter;
    return ok();
}

int dg_limit(dg_mesh m, double* C, void* stream)
{
    if (!m || !C) return fail(DG_EINVAL, "null argument");
    if (m->dev.p != 1)
        return fail(DG_EUNSUPPORTED, "the Barth-Jespersen limiter is defined for p = 1 (this mesh has p = %d)", m->dev.p);
    hipStream_t s = (hipStream_t)stream;
    timed(m, DG_KERNEL_LIMIT, s, [&] { dgk::launch_limit(m->dev, C, s); });
    return check_launch("dg_limit");
}

int dg_set_surface_mode(dg_mesh m, int mode)
{
    if (!m) return fail(DG_EINVAL, "null mesh");
    if (mode != DG_SURFACE_ELEMENTWISE && mode != DG_SURFACE_EDGEWISE && mode != DG_SURFACE_COLOURED)
        return fail(DG_EINVAL, "unknown surface mode %d", mode);
    m->surface = mode;
    return ok();
}

int dg_set_stream_concurrency(dg_mesh m, int on)
{
    if (!m) return fail(DG_EINVAL, "null mesh");
    if (on != 0 && on != 1) return fail(DG_EINVAL, "stream concurrency is 0 or 1, not %d", on);
    if (on && !m->side) {
        hipError_t e = hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "dg_set_stream_concurrency");
    }
    m->concurrent = on != 0;
    return ok();
}

int dg_timing_enable(dg_mesh m, int on)
{
    if (!m) return fail(DG_EINVAL, "null mesh");
    m->timing = on != 0;
    return ok();
}

int dg_timing_read(dg_mesh m, double* ms, int64_t* count, int n)
{
    if (!m || !ms || !count || n < DG_KERNEL_KINDS) return fail(DG_EINVAL, "bad arguments");
    for (int k = 0; k < n; ++k) {
        ms[k] = 0.0;
        count[k] = 0;
    }
    int rc = DG_OK;
    for (auto& r : m->recs) {
        float t = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess && rc == DG_OK) rc = hip_fail(e, "dg_timing_read");
        ms[r.kind] += t;
        count[r.kind] += 1;
        m->pool.push_back(r.a);
        m->pool.push_back(r.b);
    }
    m->recs.clear();
    return rc == DG_OK ? ok() : rc;
}

int64_t dg_matrix_core_tables(int p, int fp64, double* out, int64_t cap)
{
    if (p < 1 || p > 5) return fail(DG_EORDER, "order p=%d outside 1..5", p);
    if (!out) return fail(DG_EINVAL, "null argument");
    dgh::TableLayout lay;
    const std::vector<double> tab = dgh::build_tables(p, &lay);
    const std::vector<double> mx = dgh::build_mx_tables(p, tab, lay, fp64 != 0);
    if (cap < (int64_t)mx.size()) return fail(DG_EINVAL, "capacity %lld < %lld", (long long)cap, (long long)mx.size());
    std::copy(mx.begin(), mx.end(), out);
    return (int64_t)mx.size();
}

int64_t dg_reference_tables(int p, double* out, int64_t cap)
{
    if (p < 1 || p > 5) return fail(DG_EORDER, "order p=%d outside 1..5", p);
    if (!out) return fail(DG_EINVAL, "null argument");
    std::vector<double> r, s, w, gx, gw;
    dgh::volume_rule(p, r, s, w);
    dgh::gauss_rule(p + 1, gx, gw);
    const int np = dgh::n_modes(p), nq = (int)r.size(), ne = p + 1;
    const int64_t need = 3 * nq + 2 * ne + 3 * nq * np + 3 * ne * np;
    if (cap < need) return fail(DG_EINVAL, "capacity %lld < %lld", (long long)cap, (long long)need);
    double* o = out;
    for (int k = 0; k < nq; ++k) *o++ = r[k];
    for (int k = 0; k < nq; ++k) *o++ = s[k];
    for (int k = 0; k < nq; ++k) *o++ = w[k];
    for (int k = 0; k < ne; ++k) *o++ = gx[k];
    for (int k = 0; k < ne; ++k) *o++ = gw[k];
    std::vector<double> phi(np), dr(np), ds(np);
    double* P = o;
    double* DR = o + nq * np;
    double* DS = o + 2 * nq * np;
    for (int k = 0; k < nq; ++k) {
        dgh::basis_eval(p, r[k], s[k], P + k * np, DR + k * np, DS + k * np);
    }
    o += 3 * nq * np;
    for (int q = 0; q < 3; ++q)
        for (int k = 0; k < ne; ++k) {
            double rr, ss;
            dgh::side_point(q, gx[k], &rr, &ss);
            dgh::basis_eval(p, rr, ss, o + (q * ne + k) * np, nullptr, nullptr);
        }
    ok();
    return need;
}

}  // extern "C"
