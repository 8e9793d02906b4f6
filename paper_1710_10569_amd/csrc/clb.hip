// clb.hip -- single-lattice entry points of libclb (include/clb.h); the kernels they launch live in
// the headers below.
//
// Kernels (all one thread per node):
//   step_tile_kernel the fused time step (clb_step.h): pull, wall step, macroscopic, D2Q9 + D2Q5
//                    collision, store (Sec. 2.1 Eq. 8, Sec. 2.2 Eq. 19, Eq. 3, Eq. 13, Eq. 23,
//                    Sec. 3 walls), in row tiles of several shapes.
//   step_T_kernel    the temperature-only step with a prescribed velocity (clb_step.h, Sec. 3.1).
//   step_aa_kernel   the in-place step (clb_inplace.h), even and odd forms.
//   init_kernel / init_aa_kernel  equilibrium populations from FP64 fields, scattered to where
//                    the next step reads them (Eqs. 9 and 20 through the generalised equilibria).
//   moments_kernel / moments_aa_kernel  pull + wall step + macroscopic quantities -> FP64 rho, u, T.
//   populations_kernel / populations_aa_kernel  post-streaming populations in FP64, NaN where unknown.
//   diag_reduce_kernel / diag_final_kernel  FP64 sums and maxima of the moment fields, with a
//                    fixed reduction order (64-lane wavefront shuffles, then block, then a single
//                    block over the per-block partials), so repeated runs agree bitwise.
#include "clb_internal.h"
#include "clb_aux.h"
#include "clb_step.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>

namespace clb {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

int validate_desc(const clb_desc* d)
{
    if (!d) { set_error("desc is NULL"); return CLB_EINVAL; }
    if (d->precision != CLB_FP64 && d->precision != CLB_FP32_DEV && d->precision != CLB_FP64_DEV &&
        d->precision != CLB_FP32_SR) {
        set_error("unknown precision %d", d->precision);
        return CLB_EINVAL;
    }
    const clb_edge* e[4] = {&d->west, &d->east, &d->south, &d->north};
    for (int i = 0; i < 4; ++i) {
        if (e[i]->kind < CLB_PERIODIC || e[i]->kind > CLB_WALL_ADIABATIC) {
            set_error("edge %d: unknown kind %d", i, e[i]->kind);
            return CLB_EINVAL;
        }
        if (!std::isfinite(e[i]->ux) || !std::isfinite(e[i]->uy) || !std::isfinite(e[i]->T)) {
            set_error("edge %d: non-finite wall data", i);
            return CLB_EINVAL;
        }
        if (e[i]->kind != CLB_PERIODIC && (std::fabs(e[i]->ux) >= 0.5 || std::fabs(e[i]->uy) >= 0.5)) {
            set_error("edge %d: wall speed must be below 0.5 lattice units", i);
            return CLB_EINVAL;
        }
    }
    if ((d->west.kind == CLB_PERIODIC) != (d->east.kind == CLB_PERIODIC) ||
        (d->south.kind == CLB_PERIODIC) != (d->north.kind == CLB_PERIODIC)) {
        set_error("west/east and south/north must each be both periodic or both walls");
        return CLB_EINVAL;
    }
    const int minx = (d->west.kind == CLB_WALL_ADIABATIC || d->east.kind == CLB_WALL_ADIABATIC) ? 4 : 3;
    const int miny = (d->south.kind == CLB_WALL_ADIABATIC || d->north.kind == CLB_WALL_ADIABATIC) ? 4 : 3;
    if (d->nx < minx || d->ny < miny) {
        set_error("lattice %dx%d too small (need at least %dx%d)", d->nx, d->ny, minx, miny);
        return CLB_EINVAL;
    }
    // ny: the initialisation, moment and export kernels take 4 rows per workgroup along the
    // grid's y dimension, which holds at most 65536 workgroups
    if ((long long)d->nx * d->ny > (1LL << 30) || d->nx > (1 << 20) || d->ny > (1 << 18)) {
        set_error("lattice %dx%d too large", d->nx, d->ny);
        return CLB_EINVAL;
    }
    if (!std::isfinite(d->T0)) { set_error("T0 not finite"); return CLB_EINVAL; }
    if (d->prescribed_u != 0 && d->prescribed_u != 1) { set_error("prescribed_u must be 0 or 1"); return CLB_EINVAL; }
    if (d->in_place != 0 && d->in_place != 1) { set_error("in_place must be 0 or 1"); return CLB_EINVAL; }
    if (d->in_place && d->prescribed_u) { set_error("in-place streaming is not available for temperature-only lattices"); return CLB_EINVAL; }
    if (d->in_place && ((d->west.kind != CLB_PERIODIC && d->nx < 4) || (d->south.kind != CLB_PERIODIC && d->ny < 4))) {
        set_error("in-place streaming needs at least 4 nodes across a walled direction");
        return CLB_EINVAL;
    }
    return CLB_OK;
}

Geo make_geo(const clb_desc& d)
{
    Geo G;
    G.nx = d.nx;
    G.ny = d.ny;
    G.row = row_elems(d.nx);
    G.perx = d.west.kind == CLB_PERIODIC;
    G.pery = d.south.kind == CLB_PERIODIC;
    G.kind[0] = d.west.kind;
    G.kind[1] = d.east.kind;
    G.kind[2] = d.south.kind;
    G.kind[3] = d.north.kind;
    // a wall is permeable when its velocity has a component along its normal
    G.perm = (d.west.kind != CLB_PERIODIC && d.west.ux != 0.0 ? 1 : 0) | (d.east.kind != CLB_PERIODIC && d.east.ux != 0.0 ? 2 : 0) |
             (d.south.kind != CLB_PERIODIC && d.south.uy != 0.0 ? 4 : 0) | (d.north.kind != CLB_PERIODIC && d.north.uy != 0.0 ? 8 : 0);
    return G;
}

// ---------------------------------------------------------------------------------------------
// Launch helpers.


static hipError_t launch_one_step(clb_lattice* h, int shape, const void* src, void* dst, long long step)
{
    const clb_desc& d = h->desc;
    const Geo G = make_geo(d);
    const uint32_t key = step_key(uint32_t(step));
    if (d.in_place) {
        // src is the buffer, dst the snapshot pair; the parity of the step picks the form and the copies
        const bool odd = (step & 1) != 0;
        // the in-place kernel takes the store form and the workgroup width (64 or 256) of the shape
        const bool nt = tile_shape(shape).nt != 0;
        const int txw = tile_shape(shape).tx == 64 ? 64 : 256;
        const size_t sb = size_t(snap_elems(d.nx, d.ny)) * elem_bytes(d.precision);
        void* A = const_cast<void*>(src);
        const void* snow = (const char*)dst + (odd ? sb : 0);
        void* snext = (char*)dst + (odd ? 0 : sb);
        switch (d.precision) {
        case CLB_FP64: return launch_step_aa<double, double, false>(odd, nt, txw, A, snow, snext, G, make_par<double>(d, h->par), key, h->stream);
        case CLB_FP64_DEV: return launch_step_aa<double, double, true>(odd, nt, txw, A, snow, snext, G, make_par<double>(d, h->par), key, h->stream);
        case CLB_FP32_SR: return launch_step_aa<float, double, true>(odd, nt, txw, A, snow, snext, G, make_par<double>(d, h->par), key, h->stream);
        default: return launch_step_aa<float, float, true>(odd, nt, txw, A, snow, snext, G, make_par<float>(d, h->par), key, h->stream);
        }
    }
    if (d.prescribed_u) {
        switch (d.precision) {
        case CLB_FP64: return launch_step_T<double, double, false>(src, dst, G, make_par<double>(d, h->par), key, h->stream);
        case CLB_FP64_DEV: return launch_step_T<double, double, true>(src, dst, G, make_par<double>(d, h->par), key, h->stream);
        case CLB_FP32_SR: return launch_step_T<float, double, true>(src, dst, G, make_par<double>(d, h->par), key, h->stream);
        default: return launch_step_T<float, float, true>(src, dst, G, make_par<float>(d, h->par), key, h->stream);
        }
    }
    switch (d.precision) {
    case CLB_FP64: return launch_step_any<double, double, false>(shape, src, dst, G, make_par<double>(d, h->par), key, h->stream);
    case CLB_FP64_DEV: return launch_step_any<double, double, true>(shape, src, dst, G, make_par<double>(d, h->par), key, h->stream);
    case CLB_FP32_SR: return launch_step_any<float, double, true>(shape, src, dst, G, make_par<double>(d, h->par), key, h->stream);
    default: return launch_step_any<float, float, true>(shape, src, dst, G, make_par<float>(d, h->par), key, h->stream);
    }
}

static int launch_step(clb_lattice* h, long long n)
{
    if (h->desc.in_place) {
        for (long long s = 0; s < n; ++s) {
            CLB_HIP(launch_one_step(h, h->shape, h->buf[0], h->snap, h->steps));
            h->steps += 1;
        }
        return CLB_OK;
    }
    for (long long s = 0; s < n; ++s) {
        CLB_HIP(launch_one_step(h, h->shape, h->buf[h->cur], h->buf[h->cur ^ 1], h->steps));
        h->cur ^= 1;
        h->steps += 1;
    }
    return CLB_OK;
}

// Autotuner cache: (precision, ceil(log2 nx), ceil(log2 ny)) -> fastest tile shape measured.
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, int> g_tune_cache;

static int log2_class(int n) { int c = 0; while ((1 << c) < n) ++c; return c; }
static std::tuple<int, int, int> tune_key(const clb_desc& d)
{
    return std::make_tuple(d.precision, log2_class(d.nx), log2_class(d.ny));
}

// Without an autotuner result for the size class.  Two-buffer streaming: one-wavefront workgroups
// (64 x 1 tiles, one storage chunk each); when the two buffers fit the 256 MiB Infinity Cache
// (MALL) and the populations are FP32, ordinary stores, which leave the next step's input there;
// in FP64, and beyond the cache, non-temporal stores, with an occupancy-8 register budget in FP32.
// In real ping-pong stepping on MI355X these beat the 256-thread shapes by 0.5-3 % at 2048 x 1024
// and 8192 x 4096 in every precision.  In-place streaming: 256-node workgroups (1 % faster than
// one wavefront at 8192 x 4096), ordinary stores for FP32 populations that fit the cache,
// non-temporal ones otherwise.
int default_shape(const clb_desc& d)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(tune_key(d));
    if (it != g_tune_cache.end()) return it->second;
    const double footprint = (d.in_place ? 1.0 : 2.0) * double(buffer_elems(d.nx, d.ny)) * double(elem_bytes(d.precision));
    const bool fp32 = d.precision == CLB_FP32_DEV || d.precision == CLB_FP32_SR;
    const bool in_cache = footprint <= double(256 << 20);
    if (d.in_place) return in_cache && fp32 ? 2 : 6;
    if (!in_cache) return d.precision == CLB_FP32_DEV ? 13 : 11;
    return fp32 ? 12 : 11;
}

static int launch_moments(clb_lattice* h)
{
    const Geo G = make_geo(h->desc);
    if (h->desc.in_place) {
        CLB_HIP(enqueue_moments_aa(h->desc, h->par, (h->steps & 1) != 0, h->buf[0], G, h->d_fields, h->stream));
        return CLB_OK;
    }
    CLB_HIP(enqueue_moments(h->desc, h->par, h->buf[h->cur], G, h->d_fields, h->stream));
    return CLB_OK;
}

int check_params(double tau_nu, double tau_alpha, double g_beta, double Ma)
{
    if (!std::isfinite(tau_nu) || !std::isfinite(tau_alpha) || !std::isfinite(g_beta) || !std::isfinite(Ma)) {
        set_error("parameters must be finite");
        return CLB_EINVAL;
    }
    if (tau_nu <= 0.5 || tau_alpha <= 0.5) {
        set_error("relaxation times must exceed 1/2 (tau_nu=%g, tau_alpha=%g)", tau_nu, tau_alpha);
        return CLB_EINVAL;
    }
    return CLB_OK;
}

}  // namespace clb

using namespace clb;

// ---------------------------------------------------------------------------------------------
// C ABI.

extern "C" const char* clb_last_error(void) { return g_err; }

extern "C" int clb_params_from_physics(double Ra, double Pr, double Ma, double H, double dT, double* tau_nu,
                                       double* tau_alpha, double* g_beta)
{
    clear_error();
    if (!tau_nu || !tau_alpha || !g_beta) { set_error("NULL output"); return CLB_EINVAL; }
    const double in[5] = {Ra, Pr, Ma, H, dT};
    for (double v : in)
        if (!std::isfinite(v) || v <= 0.0) { set_error("physical parameters must be positive and finite"); return CLB_EINVAL; }
    const double cs = 1.0 / std::sqrt(3.0);
    const double nu = Ma * cs * H * std::sqrt(Pr / Ra);
    const double alpha = nu / Pr;
    *tau_nu = 3.0 * nu + 0.5;
    *tau_alpha = alpha / 0.25 + 0.5;
    *g_beta = Ra * nu * alpha / (dT * H * H * H);
    return CLB_OK;
}

extern "C" void clb_destroy(clb_lattice* h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    (void)hipFree(h->buf[0]);
    (void)hipFree(h->buf[1]);
    (void)hipFree(h->snap);
    (void)hipFree(h->d_fields);
    (void)hipFree(h->d_snap);
    (void)hipFree(h->d_partials);
    (void)hipFree(h->d_diag);
    if (h->ev[0]) (void)hipEventDestroy(h->ev[0]);
    if (h->ev[1]) (void)hipEventDestroy(h->ev[1]);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

static int create_impl(const clb_desc* desc, void* hip_stream, clb_lattice** out)
{
    int rc = validate_desc(desc);
    if (rc) return rc;
    clb_lattice* h = new (std::nothrow) clb_lattice;
    if (!h) { set_error("host allocation failed"); return CLB_ENOMEM; }
    *out = h;
    h->desc = *desc;
    h->shape = default_shape(*desc);
    CLB_HIP(hipGetDevice(&h->device));
    if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
    } else {
        CLB_HIP(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
        h->own_stream = true;
    }
    const size_t eb = elem_bytes(desc->precision);
    h->buf_bytes = size_t(buffer_elems(desc->nx, desc->ny)) * eb;
    const size_t n = size_t(desc->nx) * desc->ny;
    if (desc->in_place) {
        const size_t sb = 2 * size_t(snap_elems(desc->nx, desc->ny)) * eb;
        if (hipMalloc(&h->buf[0], h->buf_bytes) != hipSuccess || hipMalloc(&h->snap, sb) != hipSuccess ||
            hipMalloc((void**)&h->d_fields, 4 * n * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            set_error("device allocation of %zu bytes failed", h->buf_bytes + sb + 4 * n * sizeof(double));
            return CLB_ENOMEM;
        }
        CLB_HIP(hipMemsetAsync(h->buf[0], 0, h->buf_bytes, h->stream));
        CLB_HIP(hipMemsetAsync(h->snap, 0, sb, h->stream));
    } else {
        if (hipMalloc(&h->buf[0], h->buf_bytes) != hipSuccess || hipMalloc(&h->buf[1], h->buf_bytes) != hipSuccess ||
            hipMalloc((void**)&h->d_fields, 4 * n * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            set_error("device allocation of %zu bytes failed", 2 * h->buf_bytes + 4 * n * sizeof(double));
            return CLB_ENOMEM;
        }
        CLB_HIP(hipMemsetAsync(h->buf[0], 0, h->buf_bytes, h->stream));
        CLB_HIP(hipMemsetAsync(h->buf[1], 0, h->buf_bytes, h->stream));
    }
    CLB_HIP(hipEventCreate(&h->ev[0]));
    CLB_HIP(hipEventCreate(&h->ev[1]));
    return clb_init(h, nullptr, nullptr, nullptr);
}

extern "C" int clb_create(const clb_desc* desc, void* hip_stream, clb_lattice** out)
{
    clear_error();
    if (!out) { set_error("out is NULL"); return CLB_EINVAL; }
    *out = nullptr;
    clb_lattice* h = nullptr;
    const int rc = create_impl(desc, hip_stream, &h);
    if (rc) {
        clb_destroy(h);
        return rc;
    }
    *out = h;
    return CLB_OK;
}

extern "C" int clb_set_params(clb_lattice* h, double tau_nu, double tau_alpha, double g_beta, double Ma)
{
    clear_error();
    if (!h) { set_error("handle is NULL"); return CLB_EINVAL; }
    const int rc = check_params(tau_nu, tau_alpha, g_beta, Ma);
    if (rc) return rc;
    h->par.tau_nu = tau_nu;
    h->par.tau_alpha = tau_alpha;
    h->par.g_beta = g_beta;
    h->par.Ma = Ma;
    if (h->desc.prescribed_u && !h->par.pu_set) {
        // the moving frame of Sec. 3.1: u = (0, A) with A = Ma c_s
        h->par.pux = 0.0;
        h->par.puy = Ma / std::sqrt(3.0);
    }
    return CLB_OK;
}

extern "C" int clb_set_prescribed_velocity(clb_lattice* h, double ux, double uy)
{
    clear_error();
    if (!h) { set_error("handle is NULL"); return CLB_EINVAL; }
    if (!h->desc.prescribed_u) { set_error("the lattice was not created with prescribed_u = 1"); return CLB_ESTATE; }
    if (!std::isfinite(ux) || !std::isfinite(uy) || ux * ux + uy * uy >= 0.5) {
        set_error("prescribed velocity must be finite with |u|^2 < 1/2");
        return CLB_EINVAL;
    }
    h->par.pux = ux;
    h->par.puy = uy;
    h->par.pu_set = true;
    return CLB_OK;
}

extern "C" int clb_set_relaxation(clb_lattice* h, double s_b, double s3, double s4, double lambda2)
{
    clear_error();
    if (!h) { set_error("handle is NULL"); return CLB_EINVAL; }
    const double v[4] = {s_b, s3, s4, lambda2};
    for (double r : v)
        if (!std::isfinite(r) || r <= 0.0 || r >= 2.0) { set_error("relaxation rates must lie in (0, 2)"); return CLB_EINVAL; }
    h->par.s_b = s_b;
    h->par.s3 = s3;
    h->par.s4 = s4;
    h->par.lam2 = lambda2;
    return CLB_OK;
}

extern "C" int clb_set_body_force(clb_lattice* h, double Fvx, double Fvy)
{
    clear_error();
    if (!h) { set_error("handle is NULL"); return CLB_EINVAL; }
    if (!std::isfinite(Fvx) || !std::isfinite(Fvy)) { set_error("body force must be finite"); return CLB_EINVAL; }
    h->par.Fvx = Fvx;
    h->par.Fvy = Fvy;
    return CLB_OK;
}

extern "C" int clb_init(clb_lattice* h, const double* rho, const double* u, const double* T)
{
    clear_error();
    if (!h) { set_error("handle is NULL"); return CLB_EINVAL; }
    const clb_desc& d = h->desc;
    const size_t n = size_t(d.nx) * d.ny;
    // Stage the fields in pinned-free host memory, then one upload.
    double* host = (double*)malloc(4 * n * sizeof(double));
    if (!host) { set_error("host allocation failed"); return CLB_ENOMEM; }
    for (size_t k = 0; k < n; ++k) {
        host[k] = rho ? rho[k] : 1.0;
        host[n + k] = u ? u[k] : 0.0;
        host[2 * n + k] = u ? u[n + k] : 0.0;
        host[3 * n + k] = T ? T[k] : d.T0;
        if (d.prescribed_u) {   // the velocity is the prescribed one everywhere
            host[n + k] = h->par.pux;
            host[2 * n + k] = h->par.puy;
        }
    }
    for (size_t k = 0; k < 4 * n; ++k)
        if (!std::isfinite(host[k]) || (k < n && host[k] <= 0.0)) {
            free(host);
            set_error("initial fields must be finite with rho > 0");
            return CLB_EINVAL;
        }
    hipError_t e = hipMemcpyAsync(h->d_fields, host, 4 * n * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    free(host);
    if (e != hipSuccess) { set_error("upload of initial fields failed: %s", hipGetErrorString(e)); return CLB_EDEVICE; }
    const Geo G = make_geo(d);
    h->cur = 0;
    if (d.in_place) CLB_HIP(enqueue_init_aa(d, h->par, h->buf[0], h->snap, G, h->d_fields, h->stream));
    else CLB_HIP(enqueue_init(d, h->par, h->buf[0], G, h->d_fields, h->stream));
    h->steps = 0;
    h->has_snap = false;
    return CLB_OK;
}

extern "C" int clb_step(clb_lattice* h, long long n)
{
    clear_error();
    if (!h) { set_error("handle is NULL"); return CLB_EINVAL; }
    if (n < 0) { set_error("negative step count"); return CLB_EINVAL; }
    return launch_step(h, n);
}

extern "C" int clb_time_steps(clb_lattice* h, long long n, double* ms)
{
    clear_error();
    if (!h || !ms) { set_error("NULL argument"); return CLB_EINVAL; }
    if (n <= 0) { set_error("step count must be positive"); return CLB_EINVAL; }
    CLB_HIP(hipEventRecord(h->ev[0], h->stream));
    const int rc = launch_step(h, n);
    if (rc) return rc;
    CLB_HIP(hipEventRecord(h->ev[1], h->stream));
    CLB_HIP(hipEventSynchronize(h->ev[1]));
    float t = 0.0f;
    CLB_HIP(hipEventElapsedTime(&t, h->ev[0], h->ev[1]));
    *ms = t;
    return CLB_OK;
}

extern "C" int clb_tile_shape_count(void) { return kNumShapes; }

extern "C" int clb_tile_shape_info(int shape, int* tx, int* ty, int* spt, int* nontemporal)
{
    clear_error();
    if (shape < 0 || shape >= kNumShapes) { set_error("tile shape %d out of range", shape); return CLB_EINVAL; }
    const TileShape sh = tile_shape(shape);
    if (tx) *tx = sh.tx;
    if (ty) *ty = sh.ty;
    if (spt) *spt = sh.spt;
    if (nontemporal) *nontemporal = sh.nt;
    return CLB_OK;
}

extern "C" int clb_set_tile_shape(clb_lattice* h, int shape)
{
    clear_error();
    if (!h) { set_error("handle is NULL"); return CLB_EINVAL; }
    if (shape < 0 || shape >= kNumShapes) { set_error("tile shape %d out of range", shape); return CLB_EINVAL; }
    h->shape = shape;
    return CLB_OK;
}

extern "C" int clb_get_tile_shape(clb_lattice* h, int* shape)
{
    clear_error();
    if (!h || !shape) { set_error("NULL argument"); return CLB_EINVAL; }
    *shape = h->shape;
    return CLB_OK;
}

// Average launch time of `launches` steps with shape `shape`, ping-ponging between two scratch
// buffers that start as a copy of the current state: the same access pattern and cache behaviour
// as real stepping, and the lattice itself is not touched.  Falls back to repeated one-direction
// launches on the lattice's own buffers (reading the state, writing the spare buffer) if the scratch
// pair cannot be allocated.
static int time_shape_impl(clb_lattice* h, int shape, int launches, void* const scratch[2], double* us)
{
    void* src = scratch[0] ? scratch[0] : h->buf[h->cur];
    void* dst = scratch[0] ? scratch[1] : h->buf[h->cur ^ 1];
    for (int w = 0; w < 2; ++w) {
        CLB_HIP(launch_one_step(h, shape, src, dst, w));
        if (scratch[0]) std::swap(src, dst);
    }
    CLB_HIP(hipEventRecord(h->ev[0], h->stream));
    for (int r = 0; r < launches; ++r) {
        CLB_HIP(launch_one_step(h, shape, src, dst, 2 + r));
        if (scratch[0]) std::swap(src, dst);
    }
    CLB_HIP(hipEventRecord(h->ev[1], h->stream));
    CLB_HIP(hipEventSynchronize(h->ev[1]));
    float ms = 0.0f;
    CLB_HIP(hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
    *us = 1e3 * ms / launches;
    return CLB_OK;
}

static void scratch_pair(clb_lattice* h, void* scratch[2])
{
    scratch[0] = scratch[1] = nullptr;
    if (hipMalloc(&scratch[0], h->buf_bytes) != hipSuccess || hipMalloc(&scratch[1], h->buf_bytes) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(scratch[0]);
        (void)hipFree(scratch[1]);
        scratch[0] = scratch[1] = nullptr;
        return;
    }
    if (hipMemcpyAsync(scratch[0], h->buf[h->cur], h->buf_bytes, hipMemcpyDeviceToDevice, h->stream) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(scratch[0]);
        (void)hipFree(scratch[1]);
        scratch[0] = scratch[1] = nullptr;
    }
}

static void free_scratch(clb_lattice* h, void* scratch[2])
{
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(scratch[0]);
    (void)hipFree(scratch[1]);
}

extern "C" int clb_autotune(clb_lattice* h, int launches_per_shape, int* best_shape, double* best_us)
{
    clear_error();
    if (!h) { set_error("handle is NULL"); return CLB_EINVAL; }
    if (launches_per_shape <= 0) { set_error("launches_per_shape must be positive"); return CLB_EINVAL; }
    if (h->desc.in_place) { set_error("in-place lattices have one step kernel; tile shapes apply to two-buffer streaming"); return CLB_ESTATE; }
    void* scratch[2];
    scratch_pair(h, scratch);
    int best = -1;
    double best_t = 0.0;
    for (int s = 0; s < kNumShapes; ++s) {
        double us = 0.0;
        const int rc = time_shape_impl(h, s, launches_per_shape, scratch, &us);
        if (rc) { free_scratch(h, scratch); return rc; }
        if (best < 0 || us < best_t) { best = s; best_t = us; }
    }
    free_scratch(h, scratch);
    h->shape = best;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[tune_key(h->desc)] = best;
    }
    if (best_shape) *best_shape = best;
    if (best_us) *best_us = best_t;
    return CLB_OK;
}

extern "C" int clb_time_shape(clb_lattice* h, int shape, int launches, double* us)
{
    clear_error();
    if (!h || !us) { set_error("NULL argument"); return CLB_EINVAL; }
    if (shape < 0 || shape >= kNumShapes || launches <= 0) { set_error("bad shape or launch count"); return CLB_EINVAL; }
    if (h->desc.in_place) { set_error("in-place lattices have one step kernel; tile shapes apply to two-buffer streaming"); return CLB_ESTATE; }
    void* scratch[2];
    scratch_pair(h, scratch);
    const int rc = time_shape_impl(h, shape, launches, scratch, us);
    free_scratch(h, scratch);
    return rc;
}

extern "C" int clb_synchronize(clb_lattice* h)
{
    clear_error();
    if (!h) { set_error("handle is NULL"); return CLB_EINVAL; }
    CLB_HIP(hipStreamSynchronize(h->stream));
    return CLB_OK;
}

extern "C" int clb_moments(clb_lattice* h, double* rho, double* u, double* T)
{
    clear_error();
    if (!h) { set_error("handle is NULL"); return CLB_EINVAL; }
    int rc = launch_moments(h);
    if (rc) return rc;
    const size_t n = size_t(h->desc.nx) * h->desc.ny;
    if (rho) CLB_HIP(hipMemcpyAsync(rho, h->d_fields, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    if (u) CLB_HIP(hipMemcpyAsync(u, h->d_fields + n, 2 * n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    if (T) CLB_HIP(hipMemcpyAsync(T, h->d_fields + 3 * n, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    CLB_HIP(hipStreamSynchronize(h->stream));
    return CLB_OK;
}

extern "C" int clb_get_populations(clb_lattice* h, double* f, double* g)
{
    clear_error();
    if (!h) { set_error("handle is NULL"); return CLB_EINVAL; }
    const clb_desc& d = h->desc;
    const size_t n = size_t(d.nx) * d.ny;
    double* dev = nullptr;
    CLB_HIP(hipMalloc((void**)&dev, 14 * n * sizeof(double)));
    const Geo G = make_geo(d);
    hipError_t e = d.in_place ? enqueue_populations_aa(d, (h->steps & 1) != 0, h->buf[0], G, dev, h->stream)
                              : enqueue_populations(d, h->buf[h->cur], G, dev, h->stream);
    if (e == hipSuccess && f) e = hipMemcpyAsync(f, dev, 9 * n * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && g) e = hipMemcpyAsync(g, dev + 9 * n, 5 * n * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(dev);
    if (e != hipSuccess) { set_error("population export failed: %s", hipGetErrorString(e)); return CLB_EDEVICE; }
    return CLB_OK;
}

extern "C" int clb_diagnostics(clb_lattice* h, int snapshot, clb_diag* out)
{
    clear_error();
    if (!h || !out) { set_error("NULL argument"); return CLB_EINVAL; }
    const clb_desc& d = h->desc;
    const size_t n = size_t(d.nx) * d.ny;
    const Geo G = make_geo(d);
    const int nblocks = diag_blocks(G);
    if (!h->d_snap) CLB_HIP(hipMalloc((void**)&h->d_snap, 3 * n * sizeof(double)));
    if (!h->d_diag) CLB_HIP(hipMalloc((void**)&h->d_diag, DIAG_SLOTS * sizeof(double)));
    if (h->partials_cap < nblocks) {
        (void)hipFree(h->d_partials);
        h->d_partials = nullptr;
        CLB_HIP(hipMalloc((void**)&h->d_partials, size_t(nblocks) * DIAG_SLOTS * sizeof(double)));
        h->partials_cap = nblocks;
    }
    int rc = launch_moments(h);
    if (rc) return rc;
    CLB_HIP(enqueue_diag(h->d_fields, h->d_snap, h->has_snap ? 1 : 0, G, h->d_partials, h->d_diag, h->stream));
    double r[DIAG_SLOTS];
    CLB_HIP(hipMemcpyAsync(r, h->d_diag, sizeof r, hipMemcpyDeviceToHost, h->stream));
    if (snapshot) {
        CLB_HIP(hipMemcpyAsync(h->d_snap, h->d_fields + n, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    }
    CLB_HIP(hipStreamSynchronize(h->stream));
    if (snapshot) h->has_snap = true;
    unpack_diag(r, h->steps, out);
    if (out->nonfinite) {
        set_error("non-finite density, velocity or temperature at step %lld", h->steps);
        return CLB_EDIVERGED;
    }
    return CLB_OK;
}

// ---------------------------------------------------------------------------------------------
// Allocation-free diagnostics (clb_diagnostics_noalloc).
//
// Its scratch -- the per-block partial records of the diagnostics reduction after the final
// record -- is a file-scope device array; each GPU the library runs on holds one copy until the
// process ends.  In host code the array's name is not a device address: the address of a GPU's
// copy is looked up once, with that GPU current, and kept in g_noalloc_ptr.  Every call on a GPU
// shares its copy, so calls that overlap on one GPU race.  Nothing in it needs clearing: each
// call's reduction writes every partial record it reads and the whole final record.
namespace clb {
constexpr int NOALLOC_MAX_BLOCKS = 32768;   // one partial record per 256 nodes: 8,388,608 nodes
constexpr int NOALLOC_DEVICES = 64;
}  // namespace clb

static __device__ __align__(256) double scratch[(clb::NOALLOC_MAX_BLOCKS + 1) * clb::DIAG_SLOTS];
static std::mutex g_noalloc_mu;
static double* g_noalloc_ptr[clb::NOALLOC_DEVICES];

// Device address of `scratch` on GPU `device` (looked up on the first call for that GPU).
static double* noalloc_scratch(int device)
{
    if (device < 0 || device >= NOALLOC_DEVICES) {
        set_error("device %d is beyond the %d the allocation-free diagnostics support", device, NOALLOC_DEVICES);
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e == hipSuccess && prev != device) e = hipSetDevice(device);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != device) (void)hipSetDevice(prev);
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress of the diagnostics scratch failed on device %d: %s", device, hipGetErrorString(e));
            return nullptr;
        }
        g_noalloc_ptr[device] = static_cast<double*>(p);
    }
    return g_noalloc_ptr[device];
}

extern "C" int clb_diagnostics_noalloc(clb_lattice* h, clb_diag* out)
{
    clear_error();
    if (!h || !out) { set_error("NULL argument"); return CLB_EINVAL; }
    const Geo G = make_geo(h->desc);
    const int nblocks = diag_blocks(G);
    if (nblocks > NOALLOC_MAX_BLOCKS) {
        set_error("lattice of %lld nodes exceeds the allocation-free diagnostics' scratch (at most %lld nodes); use clb_diagnostics",
                  (long long)G.nx * G.ny, (long long)NOALLOC_MAX_BLOCKS * RED_NT);
        return CLB_EINVAL;
    }
    double* s = noalloc_scratch(h->device);
    if (!s) return CLB_EDEVICE;
    int rc = launch_moments(h);
    if (rc) return rc;
    CLB_HIP(enqueue_diag(h->d_fields, h->d_snap, h->has_snap ? 1 : 0, G, s + DIAG_SLOTS, s, h->stream));
    double r[DIAG_SLOTS];
    CLB_HIP(hipMemcpyAsync(r, s, sizeof r, hipMemcpyDeviceToHost, h->stream));
    CLB_HIP(hipStreamSynchronize(h->stream));
    unpack_diag(r, h->steps, out);
    if (out->nonfinite) {
        set_error("non-finite density, velocity or temperature at step %lld", h->steps);
        return CLB_EDIVERGED;
    }
    return CLB_OK;
}

// ---------------------------------------------------------------------------------------------
// Checkpoint / resume: a host blob holding a header (description, parameters, step count, which
// buffer is current, whether a residual snapshot exists) followed by the raw device state -- the
// current population buffer (in place: the single buffer and its two snapshot copies) and the FP64
// residual snapshot.  Restoring it into a lattice of the same description and stepping on gives
// bitwise the run that was not interrupted (the stochastic rounding is keyed by the step count,
// which the blob carries).

namespace {

constexpr char kCkptMagic[8] = {'C', 'L', 'B', '2', 'D', 'C', 'K', 'P'};
constexpr uint32_t kCkptVersion = 1;

struct CkptHeader {
    char magic[8];
    uint32_t version, header_bytes;
    clb_desc desc;
    clb::Params par;
    long long steps;
    int cur, has_snap;
    uint64_t pop_bytes, band_bytes, rsnap_bytes;
};

bool same_edge(const clb_edge& a, const clb_edge& b) { return a.kind == b.kind && a.ux == b.ux && a.uy == b.uy && a.T == b.T; }
bool same_desc(const clb_desc& a, const clb_desc& b)
{
    return a.nx == b.nx && a.ny == b.ny && a.precision == b.precision && a.T0 == b.T0 && a.prescribed_u == b.prescribed_u &&
           a.in_place == b.in_place && same_edge(a.west, b.west) && same_edge(a.east, b.east) && same_edge(a.south, b.south) &&
           same_edge(a.north, b.north);
}

CkptHeader ckpt_header(const clb_lattice* h)
{
    CkptHeader H;
    std::memset(&H, 0, sizeof H);
    std::memcpy(H.magic, kCkptMagic, sizeof H.magic);
    H.version = kCkptVersion;
    H.header_bytes = uint32_t(sizeof(CkptHeader));
    H.desc = h->desc;
    H.par = h->par;
    H.steps = h->steps;
    H.cur = h->cur;
    H.has_snap = h->has_snap ? 1 : 0;
    H.pop_bytes = h->buf_bytes;
    H.band_bytes = h->desc.in_place ? 2 * uint64_t(snap_elems(h->desc.nx, h->desc.ny)) * elem_bytes(h->desc.precision) : 0;
    H.rsnap_bytes = h->has_snap ? 3 * uint64_t(h->desc.nx) * h->desc.ny * sizeof(double) : 0;
    return H;
}

}  // namespace

extern "C" int clb_checkpoint_size(clb_lattice* h, size_t* bytes)
{
    clear_error();
    if (!h || !bytes) { set_error("NULL argument"); return CLB_EINVAL; }
    const CkptHeader H = ckpt_header(h);
    *bytes = sizeof(CkptHeader) + H.pop_bytes + H.band_bytes + H.rsnap_bytes;
    return CLB_OK;
}

extern "C" int clb_checkpoint_save(clb_lattice* h, void* host, size_t bytes)
{
    clear_error();
    if (!h || !host) { set_error("NULL argument"); return CLB_EINVAL; }
    const CkptHeader H = ckpt_header(h);
    const size_t need = sizeof(CkptHeader) + H.pop_bytes + H.band_bytes + H.rsnap_bytes;
    if (bytes < need) { set_error("checkpoint buffer holds %zu bytes, %zu needed", bytes, need); return CLB_EINVAL; }
    char* p = static_cast<char*>(host);
    std::memcpy(p, &H, sizeof H);
    p += sizeof H;
    CLB_HIP(hipMemcpyAsync(p, h->desc.in_place ? h->buf[0] : h->buf[h->cur], H.pop_bytes, hipMemcpyDeviceToHost, h->stream));
    p += H.pop_bytes;
    if (H.band_bytes) CLB_HIP(hipMemcpyAsync(p, h->snap, H.band_bytes, hipMemcpyDeviceToHost, h->stream));
    p += H.band_bytes;
    if (H.rsnap_bytes) CLB_HIP(hipMemcpyAsync(p, h->d_snap, H.rsnap_bytes, hipMemcpyDeviceToHost, h->stream));
    CLB_HIP(hipStreamSynchronize(h->stream));
    return CLB_OK;
}

extern "C" int clb_checkpoint_load(clb_lattice* h, const void* host, size_t bytes)
{
    clear_error();
    if (!h || !host) { set_error("NULL argument"); return CLB_EINVAL; }
    CkptHeader H;
    if (bytes < sizeof H) { set_error("checkpoint too short"); return CLB_EINVAL; }
    std::memcpy(&H, host, sizeof H);
    if (std::memcmp(H.magic, kCkptMagic, sizeof H.magic) != 0 || H.version != kCkptVersion ||
        H.header_bytes != sizeof(CkptHeader)) {
        set_error("not a checkpoint of this library's 2D lattices (magic, version or header size differ)");
        return CLB_EINVAL;
    }
    if (!same_desc(H.desc, h->desc)) { set_error("checkpoint was taken on a lattice of another description"); return CLB_EINVAL; }
    const CkptHeader mine = ckpt_header(h);
    if (H.pop_bytes != mine.pop_bytes || H.band_bytes != mine.band_bytes ||
        (H.has_snap && H.rsnap_bytes != 3 * uint64_t(h->desc.nx) * h->desc.ny * sizeof(double)) || (!H.has_snap && H.rsnap_bytes)) {
        set_error("checkpoint sizes do not match the lattice");
        return CLB_EINVAL;
    }
    if (bytes < sizeof H + H.pop_bytes + H.band_bytes + H.rsnap_bytes) { set_error("checkpoint truncated"); return CLB_EINVAL; }
    const size_t n = size_t(h->desc.nx) * h->desc.ny;
    if (H.has_snap && !h->d_snap) CLB_HIP(hipMalloc((void**)&h->d_snap, 3 * n * sizeof(double)));
    const char* p = static_cast<const char*>(host) + sizeof H;
    CLB_HIP(hipMemcpyAsync(h->buf[0], p, H.pop_bytes, hipMemcpyHostToDevice, h->stream));
    p += H.pop_bytes;
    if (H.band_bytes) CLB_HIP(hipMemcpyAsync(h->snap, p, H.band_bytes, hipMemcpyHostToDevice, h->stream));
    p += H.band_bytes;
    if (H.rsnap_bytes) CLB_HIP(hipMemcpyAsync(h->d_snap, p, H.rsnap_bytes, hipMemcpyHostToDevice, h->stream));
    CLB_HIP(hipStreamSynchronize(h->stream));
    h->par = H.par;
    h->steps = H.steps;
    h->cur = 0;                // the saved current buffer now sits in buf[0]
    h->has_snap = H.has_snap != 0;
    return CLB_OK;
}
