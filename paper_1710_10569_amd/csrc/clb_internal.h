// clb_internal.h -- host-side state shared by the translation units of libclb.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/clb.h"
#include "clb_device.h"

namespace clb {

// Thread-local message of the last error (clb_last_error).
void set_error(const char* fmt, ...);
void clear_error();

// HIP call check: records the failing call and returns CLB_EDEVICE from the enclosing function.
#define CLB_HIP(call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            ::clb::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                             __LINE__);                                                       \
            return CLB_EDEVICE;                                                               \
        }                                                                                     \
    } while (0)

// Elements per row (ceil(nx / CW) chunks of 14 * CW; every chunk starts on a 256-byte boundary)
// and per population buffer.
inline int row_elems(int nx) { return (nx + CW - 1) / CW * CHUNK; }
inline long long buffer_elems(int nx, int ny) { return (long long)row_elems(nx) * ny; }

inline size_t elem_bytes(int precision) { return (precision == CLB_FP32_DEV || precision == CLB_FP32_SR) ? 4 : 8; }
inline bool is_dev(int precision) { return precision != CLB_FP64; }

// Validate a lattice description; returns CLB_OK or CLB_EINVAL with a message.
int validate_desc(const clb_desc* d);

// Physical parameters of one lattice in FP64 (the source of Par<Real>).
struct Params {
    double tau_nu = 1.0, tau_alpha = 1.0, g_beta = 0.0, Ma = 0.0;
    double s_b = 1.0, s3 = 1.0, s4 = 1.0, lam2 = 1.0;
    double Fvx = 0.0, Fvy = 0.0;
    double pux = 0.0, puy = 0.0;   // prescribed velocity (temperature-only lattices)
    bool pu_set = false;           // set explicitly (else (0, Ma c_s) from clb_set_params)
};

Geo make_geo(const clb_desc& d);

// CLB_OK, or CLB_EINVAL with a message, for relaxation times / buoyancy / Mach number.
int check_params(double tau_nu, double tau_alpha, double g_beta, double Ma);

template <typename Real>
Par<Real> make_par(const clb_desc& d, const Params& p)
{
    Par<Real> P;
    const double s_nu = 1.0 / p.tau_nu, l1 = 1.0 / p.tau_alpha;
    const double TR = is_dev(d.precision) ? d.T0 : 0.0;
    P.om_nu = Real(1.0 - s_nu);
    P.om_b = Real(1.0 - p.s_b);
    P.om_3 = Real(1.0 - p.s3);
    P.om_4 = Real(1.0 - p.s4);
    P.c3 = Real((1.0 - 0.5 * p.s3) / 3.0);
    P.om_l1 = Real(1.0 - l1);
    P.om_l2 = Real(1.0 - p.lam2);
    P.g_beta = Real(p.g_beta);
    P.Fvx = Real(p.Fvx);
    P.Fvy = Real(p.Fvy);
    P.Toff = Real(TR - d.T0);
    P.TR = Real(TR);
    const clb_edge* e[4] = {&d.west, &d.east, &d.south, &d.north};
    for (int i = 0; i < 4; ++i) {
        P.uw[i][0] = Real(e[i]->ux);
        P.uw[i][1] = Real(e[i]->uy);
        P.dTw[i] = Real(e[i]->T - TR);
    }
    P.pux = Real(p.pux);
    P.puy = Real(p.puy);
    return P;
}

// Number of FP64 slots in a diagnostics partial record.
enum { DIAG_SUMS = 11, DIAG_MAXES = 4, DIAG_SLOTS = 16 };

}  // namespace clb

struct clb_lattice {
    clb_desc desc{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t buf_bytes = 0;     // bytes per population buffer
    void* buf[2] = {nullptr, nullptr};   // in-place lattices: buf[0] only
    void* snap = nullptr;     // in-place lattices: two copies of snap_elems(nx, ny) values
    int cur = 0;              // buffer holding the post-collision state of the last step
    int shape = 2;            // tile shape of the step kernel (clb_step.h)
    clb::Params par;
    long long steps = 0;
    double* d_fields = nullptr;     // 4 FP64 planes of nx*ny: init input, moments output
    double* d_snap = nullptr;       // 3 FP64 planes of nx*ny: residual snapshot (ux, uy, T)
    bool has_snap = false;
    double* d_partials = nullptr;   // per-block diagnostics partials
    int partials_cap = 0;
    double* d_diag = nullptr;       // final diagnostics record
    hipEvent_t ev[2] = {nullptr, nullptr};
};
