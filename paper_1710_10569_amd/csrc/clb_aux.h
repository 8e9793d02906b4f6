// clb_aux.h -- initialisation, moment, population-export and diagnostics kernels, shared by the
// single-lattice and batched front ends, with host-side enqueue helpers.
#pragma once

#include "clb_inplace.h"
#include "clb_internal.h"

namespace clb {

// ---------------------------------------------------------------------------------------------
// Kernels.

constexpr int TX = 64, TY = 4;   // init / moments / export kernels: 64 x 4 nodes per workgroup

// Lattice directions of Eq. 4 for the host-side and init/export kernels.
__device__ constexpr int EXd[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int EYd[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
__device__ constexpr double W5[5] = {0.5, 0.125, 0.125, 0.125, 0.125};

// Source node x - e_i of direction i, or false if it lies outside the domain.
__device__ __forceinline__ bool source_of(const Geo& G, int x, int y, int i, int& sx, int& sy)
{
    sx = x - EXd[i];
    sy = y - EYd[i];
    if (G.perx) sx = (sx + G.nx) % G.nx;
    if (G.pery) sy = (sy + G.ny) % G.ny;
    return sx >= 0 && sx < G.nx && sy >= 0 && sy < G.ny;
}

// Equilibria in FP64: f_i^eq = rho psi(e_ix, v_x) psi(e_iy, v_y) and
// g_i^eq = T (c_T^2 +- u + u^2)/2 on the axes, T (1 - 2 c_T^2 - |u|^2) at rest, c_T^2 = 1/4.
__device__ inline double psi(int e, double v) { return e == 0 ? 2.0 / 3.0 - v * v : 0.5 * (1.0 / 3.0 + e * v + v * v); }

template <typename S, bool DEV>
__global__ void init_kernel(S* __restrict__ buf, Geo G, const double* __restrict__ fields,
                            double g_beta, double T0, double Fvx, double Fvy, double TR)
{
    const int x = blockIdx.x * TX + threadIdx.x;
    const int y = blockIdx.y * TY + threadIdx.y;
    if (x >= G.nx || y >= G.ny) return;
    const long long n = (long long)G.nx * G.ny;
    const long long k = (long long)y * G.nx + x;
    const double rho = fields[k], ux = fields[n + k], uy = fields[2 * n + k], T = fields[3 * n + k];
    const double Fx = Fvx, Fy = Fvy + g_beta * (T - T0);
    const double vx = ux - 0.5 * Fx / rho, vy = uy - 0.5 * Fy / rho;
    for (int i = 0; i < 9; ++i) {
        // f_i(x) is read by the next pull from the node x - e_i... so store at the source of x.  An
        // unknown f_i (source beyond a wall) is stored in slot opp(i) of x itself, where the wall
        // step's mass balance reads what x sent out of the domain the step before: the initial
        // unknowns stand for it, so the balance returns rho at t = 0.
        int sx, sy;
        double v = rho * psi(EXd[i], vx) * psi(EYd[i], vy);
        if (DEV) v -= W9[i];
        if (!source_of(G, x, y, i, sx, sy)) {
            buf[pop_at(G, x, y) + opp_of(i) * CW] = S(v);
            continue;
        }
        buf[pop_at(G, sx, sy) + i * CW] = S(v);
    }
    const double gq[5] = {T * (0.5 - ux * ux - uy * uy), 0.5 * T * (0.25 + ux + ux * ux),
                          0.5 * T * (0.25 + uy + uy * uy), 0.5 * T * (0.25 - ux + ux * ux),
                          0.5 * T * (0.25 - uy + uy * uy)};
    for (int i = 0; i < 5; ++i) {
        int sx, sy;
        if (!source_of(G, x, y, i, sx, sy)) continue;
        double v = gq[i];
        if (DEV) v -= W5[i] * TR;
        buf[pop_at(G, sx, sy) + (9 + i) * CW] = S(v);
    }
}

// PRESC: temperature-only lattice (prescribed velocity): rho = 1 and u = u_p, T after the
// temperature wall step.
template <typename S, typename Real, bool DEV, bool PRESC>
__global__ __launch_bounds__(TX * TY) void moments_kernel(const S* __restrict__ src, Geo G, Par<Real> P,
                                                        double* __restrict__ fields)
{
    const int x = blockIdx.x * TX + threadIdx.x;
    const int y = blockIdx.y * TY + threadIdx.y;
    if (x >= G.nx || y >= G.ny) return;
    const long long n = (long long)G.nx * G.ny;
    const long long k = (long long)y * G.nx + x;
    if (PRESC) {
        Real g[5];
        pull_g(src, G, x, y, g);
        if (on_wall(G, x, y)) wall_step_T<S, Real, DEV>(src, G, P, x, y, g);
        fields[k] = 1.0;
        fields[n + k] = double(P.pux);
        fields[2 * n + k] = double(P.puy);
        fields[3 * n + k] = double(P.TR) + double((g[0] + g[1]) + (g[2] + g[3]) + g[4]);
        return;
    }
    Real f[9], g[5];
    pull(src, G, x, y, f, g);
    if (on_wall(G, x, y)) wall_step<S, Real, DEV>(src, G, P, x, y, f, g);
    const Macro<Real, DEV> m = macro<Real, DEV>(f, g, P);
    fields[k] = double(m.rho);
    fields[n + k] = double(m.ux);
    fields[2 * n + k] = double(m.uy);
    fields[3 * n + k] = double(P.TR) + double(m.dT);
}

template <typename S, bool DEV>
__global__ void populations_kernel(const S* __restrict__ src, Geo G, double TR, double* __restrict__ fo,
                                   double* __restrict__ go)
{
    const int x = blockIdx.x * TX + threadIdx.x;
    const int y = blockIdx.y * TY + threadIdx.y;
    if (x >= G.nx || y >= G.ny) return;
    double f[9], g[5];
    pull(src, G, x, y, f, g);
    const long long n = (long long)G.nx * G.ny;
    const long long k = (long long)y * G.nx + x;
    for (int i = 0; i < 9; ++i) {
        int sx, sy;
        const bool known = source_of(G, x, y, i, sx, sy);
        if (fo) fo[i * n + k] = known ? double(f[i]) + (DEV ? W9[i] : 0.0) : __builtin_nan("");
        if (i < 5 && go) go[i * n + k] = known ? double(g[i]) + (DEV ? W5[i] * TR : 0.0) : __builtin_nan("");
    }
}

// In-place lattices (clb_inplace.h): initial state in the even-time form (population i of node x
// in slot i of x) plus snapshot copy 0; moments and exported populations read the form of the
// current time's parity and take the wall step's neighbours from the current snapshot copy.
template <typename S, bool DEV>
__global__ void init_aa_kernel(S* __restrict__ A, S* __restrict__ snap0, Geo G, const double* __restrict__ fields,
                               double g_beta, double T0, double Fvx, double Fvy, double TR)
{
    const int x = blockIdx.x * TX + threadIdx.x;
    const int y = blockIdx.y * TY + threadIdx.y;
    if (x >= G.nx || y >= G.ny) return;
    const long long n = (long long)G.nx * G.ny;
    const long long k = (long long)y * G.nx + x;
    const double rho = fields[k], ux = fields[n + k], uy = fields[2 * n + k], T = fields[3 * n + k];
    const double Fx = Fvx, Fy = Fvy + g_beta * (T - T0);
    const double vx = ux - 0.5 * Fx / rho, vy = uy - 0.5 * Fy / rho;
    const double gq[5] = {T * (0.5 - ux * ux - uy * uy), 0.5 * T * (0.25 + ux + ux * ux),
                          0.5 * T * (0.25 + uy + uy * uy), 0.5 * T * (0.25 - ux + ux * ux),
                          0.5 * T * (0.25 - uy + uy * uy)};
    const long long o = pop_at(G, x, y);
    for (int q = 0; q < 14; ++q) {
        double v = q < 9 ? rho * psi(EXd[q], vx) * psi(EYd[q], vy) : gq[q - 9];
        if (DEV) v -= q < 9 ? W9[q] : W5[q - 9] * TR;
        A[o + q * CW] = S(v);
        snap_put(snap0, G, x, y, q, S(v));
    }
}

template <typename S, typename Real, bool DEV, bool ODD>
__global__ __launch_bounds__(TX * TY) void moments_aa_kernel(const S* __restrict__ A, Geo G, Par<Real> P,
                                                           double* __restrict__ fields)
{
    const int x = blockIdx.x * TX + threadIdx.x;
    const int y = blockIdx.y * TY + threadIdx.y;
    if (x >= G.nx || y >= G.ny) return;
    Real f[9], g[5];
    load_aa<S, Real, ODD>(A, G, x, y, f, g);
    if (on_wall(G, x, y)) wall_step_nb<Real, DEV>(DirectSource<S, ODD>{A}, G, P, x, y, f, g);
    const Macro<Real, DEV> m = macro<Real, DEV>(f, g, P);
    const long long n = (long long)G.nx * G.ny;
    const long long k = (long long)y * G.nx + x;
    fields[k] = double(m.rho);
    fields[n + k] = double(m.ux);
    fields[2 * n + k] = double(m.uy);
    fields[3 * n + k] = double(P.TR) + double(m.dT);
}

template <typename S, bool DEV, bool ODD>
__global__ void populations_aa_kernel(const S* __restrict__ A, Geo G, double TR, double* __restrict__ fo,
                                      double* __restrict__ go)
{
    const int x = blockIdx.x * TX + threadIdx.x;
    const int y = blockIdx.y * TY + threadIdx.y;
    if (x >= G.nx || y >= G.ny) return;
    double f[9], g[5];
    load_aa<S, double, ODD>(A, G, x, y, f, g);
    const long long n = (long long)G.nx * G.ny;
    const long long k = (long long)y * G.nx + x;
    for (int i = 0; i < 9; ++i) {
        int sx, sy;
        const bool known = source_of(G, x, y, i, sx, sy);
        if (fo) fo[i * n + k] = known ? f[i] + (DEV ? W9[i] : 0.0) : __builtin_nan("");
        if (i < 5 && go) go[i * n + k] = known ? g[i] + (DEV ? W5[i] * TR : 0.0) : __builtin_nan("");
    }
}

// Block-wide reductions of DIAG_SLOTS doubles: slots [0, DIAG_SUMS) are summed, the rest maxed.
__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <int NT>
__device__ inline void block_reduce(double (&v)[DIAG_SLOTS], double* out)
{
    __shared__ double red[NT / 64][DIAG_SLOTS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < DIAG_SLOTS; ++s) {
        const double r = s < DIAG_SUMS ? wave_sum(v[s]) : wave_max(v[s]);
        if (lane == 0) red[wave][s] = r;
    }
    __syncthreads();
    if (threadIdx.x < DIAG_SLOTS) {
        const int s = threadIdx.x;
        double r = red[0][s];
        for (int w = 1; w < NT / 64; ++w) r = s < DIAG_SUMS ? r + red[w][s] : fmax(r, red[w][s]);
        out[s] = r;
    }
}

constexpr int RED_NT = 256;

// Per-node contributions from the FP64 moment fields (dense [4][ny][nx]).
template <int NTH>
__global__ __launch_bounds__(NTH) void diag_reduce_kernel(const double* __restrict__ fields,
                                                            const double* __restrict__ snap, int has_snap,
                                                            Geo G, double* __restrict__ partials)
{
    const long long n = (long long)G.nx * G.ny;
    const long long k = (long long)blockIdx.x * NTH + threadIdx.x;
    double v[DIAG_SLOTS];
#pragma unroll
    for (int s = 0; s < DIAG_SLOTS; ++s) v[s] = 0.0;
    v[DIAG_SUMS + 1] = v[DIAG_SUMS + 2] = has_snap ? 0.0 : -1.0;
    if (k < n) {
        const int x = int(k % G.nx), y = int(k / G.nx);
        const double rho = fields[k], ux = fields[n + k], uy = fields[2 * n + k], T = fields[3 * n + k];
        const double wx = (!G.perx && (x == 0 || x == G.nx - 1)) ? 0.5 : 1.0;
        const double wy = (!G.pery && (y == 0 || y == G.ny - 1)) ? 0.5 : 1.0;
        const double w = wx * wy;
        v[0] = rho;
        v[1] = T;
        v[2] = rho * ux;
        v[3] = rho * uy;
        v[4] = w;
        v[5] = w * ux * T;
        v[6] = w * uy * T;
        // wall heat flux: (3 T_b - 4 T_1 + T_2)/2 along the inward normal, trapezoid weight along the wall
        const double* Tf = fields + 3 * n;
        if (!G.perx && x == 0) v[7] = wy * 0.5 * (3.0 * T - 4.0 * Tf[k + 1] + Tf[k + 2]);
        if (!G.perx && x == G.nx - 1) v[8] = wy * 0.5 * (3.0 * T - 4.0 * Tf[k - 1] + Tf[k - 2]);
        if (!G.pery && y == 0) v[9] = wx * 0.5 * (3.0 * T - 4.0 * Tf[k + G.nx] + Tf[k + 2 * G.nx]);
        if (!G.pery && y == G.ny - 1) v[10] = wx * 0.5 * (3.0 * T - 4.0 * Tf[k - G.nx] + Tf[k - 2 * G.nx]);
        v[DIAG_SUMS + 0] = sqrt(ux * ux + uy * uy);
        if (has_snap) {
            v[DIAG_SUMS + 1] = fmax(fabs(ux - snap[k]), fabs(uy - snap[n + k]));
            v[DIAG_SUMS + 2] = fabs(T - snap[2 * n + k]);
        }
        v[DIAG_SUMS + 3] = (__builtin_isfinite(rho) && __builtin_isfinite(ux) && __builtin_isfinite(uy) && __builtin_isfinite(T)) ? 0.0 : 1.0;
    }
    block_reduce<NTH>(v, partials + (long long)blockIdx.x * DIAG_SLOTS);
}

template <int NTH>
__global__ __launch_bounds__(NTH) void diag_final_kernel(const double* __restrict__ partials, int nblocks,
                                                           double* __restrict__ out)
{
    double v[DIAG_SLOTS];
#pragma unroll
    for (int s = 0; s < DIAG_SLOTS; ++s) v[s] = (s < DIAG_SUMS) ? 0.0 : -1.0;
    for (int b = threadIdx.x; b < nblocks; b += NTH) {
#pragma unroll
        for (int s = 0; s < DIAG_SLOTS; ++s)
            v[s] = s < DIAG_SUMS ? v[s] + partials[(long long)b * DIAG_SLOTS + s]
                                 : fmax(v[s], partials[(long long)b * DIAG_SLOTS + s]);
    }
    block_reduce<NTH>(v, out);
}

// ---------------------------------------------------------------------------------------------
// Host-side enqueue helpers (one lattice whose population buffer starts at `buf`).

inline dim3 node_grid(const Geo& G) { return dim3((G.nx + TX - 1) / TX, (G.ny + TY - 1) / TY); }

inline hipError_t enqueue_init(const clb_desc& d, const Params& p, void* buf, const Geo& G, const double* d_fields,
                               hipStream_t st)
{
    const double TR = is_dev(d.precision) ? d.T0 : 0.0;
    const dim3 grid = node_grid(G), block(TX, TY);
    switch (d.precision) {
    case CLB_FP64: init_kernel<double, false><<<grid, block, 0, st>>>((double*)buf, G, d_fields, p.g_beta, d.T0, p.Fvx, p.Fvy, TR); break;
    case CLB_FP64_DEV: init_kernel<double, true><<<grid, block, 0, st>>>((double*)buf, G, d_fields, p.g_beta, d.T0, p.Fvx, p.Fvy, TR); break;
    case CLB_FP32_SR:
    default: init_kernel<float, true><<<grid, block, 0, st>>>((float*)buf, G, d_fields, p.g_beta, d.T0, p.Fvx, p.Fvy, TR); break;
    }
    return hipGetLastError();
}

inline hipError_t enqueue_moments(const clb_desc& d, const Params& p, const void* buf, const Geo& G, double* d_fields,
                                  hipStream_t st)
{
    const dim3 grid = node_grid(G), block(TX, TY);
    if (d.prescribed_u) {
        switch (d.precision) {
        case CLB_FP64: moments_kernel<double, double, false, true><<<grid, block, 0, st>>>((const double*)buf, G, make_par<double>(d, p), d_fields); break;
        case CLB_FP64_DEV: moments_kernel<double, double, true, true><<<grid, block, 0, st>>>((const double*)buf, G, make_par<double>(d, p), d_fields); break;
        case CLB_FP32_SR: moments_kernel<float, double, true, true><<<grid, block, 0, st>>>((const float*)buf, G, make_par<double>(d, p), d_fields); break;
        default: moments_kernel<float, float, true, true><<<grid, block, 0, st>>>((const float*)buf, G, make_par<float>(d, p), d_fields); break;
        }
        return hipGetLastError();
    }
    switch (d.precision) {
    case CLB_FP64: moments_kernel<double, double, false, false><<<grid, block, 0, st>>>((const double*)buf, G, make_par<double>(d, p), d_fields); break;
    case CLB_FP64_DEV: moments_kernel<double, double, true, false><<<grid, block, 0, st>>>((const double*)buf, G, make_par<double>(d, p), d_fields); break;
    case CLB_FP32_SR: moments_kernel<float, double, true, false><<<grid, block, 0, st>>>((const float*)buf, G, make_par<double>(d, p), d_fields); break;
    default: moments_kernel<float, float, true, false><<<grid, block, 0, st>>>((const float*)buf, G, make_par<float>(d, p), d_fields); break;
    }
    return hipGetLastError();
}

inline hipError_t enqueue_populations(const clb_desc& d, const void* buf, const Geo& G, double* d_out, hipStream_t st)
{
    const size_t n = size_t(d.nx) * d.ny;
    const double TR = is_dev(d.precision) ? d.T0 : 0.0;
    const dim3 grid = node_grid(G), block(TX, TY);
    switch (d.precision) {
    case CLB_FP64: populations_kernel<double, false><<<grid, block, 0, st>>>((const double*)buf, G, TR, d_out, d_out + 9 * n); break;
    case CLB_FP64_DEV: populations_kernel<double, true><<<grid, block, 0, st>>>((const double*)buf, G, TR, d_out, d_out + 9 * n); break;
    case CLB_FP32_SR:
    default: populations_kernel<float, true><<<grid, block, 0, st>>>((const float*)buf, G, TR, d_out, d_out + 9 * n); break;
    }
    return hipGetLastError();
}

// In-place counterparts (snapshot copies: elements snap_elems(nx, ny) each, copy c at snap + c * that).
inline hipError_t enqueue_init_aa(const clb_desc& d, const Params& p, void* A, void* snap0, const Geo& G,
                                  const double* d_fields, hipStream_t st)
{
    const double TR = is_dev(d.precision) ? d.T0 : 0.0;
    const dim3 grid = node_grid(G), block(TX, TY);
    switch (d.precision) {
    case CLB_FP64: init_aa_kernel<double, false><<<grid, block, 0, st>>>((double*)A, (double*)snap0, G, d_fields, p.g_beta, d.T0, p.Fvx, p.Fvy, TR); break;
    case CLB_FP64_DEV: init_aa_kernel<double, true><<<grid, block, 0, st>>>((double*)A, (double*)snap0, G, d_fields, p.g_beta, d.T0, p.Fvx, p.Fvy, TR); break;
    default: init_aa_kernel<float, true><<<grid, block, 0, st>>>((float*)A, (float*)snap0, G, d_fields, p.g_beta, d.T0, p.Fvx, p.Fvy, TR); break;
    }
    return hipGetLastError();
}

template <typename S, typename Real, bool DEV>
inline void moments_aa_launch(bool odd, const void* A, const Geo& G, const Par<Real>& P, double* d_fields, hipStream_t st)
{
    const dim3 grid = node_grid(G), block(TX, TY);
    if (odd) moments_aa_kernel<S, Real, DEV, true><<<grid, block, 0, st>>>((const S*)A, G, P, d_fields);
    else moments_aa_kernel<S, Real, DEV, false><<<grid, block, 0, st>>>((const S*)A, G, P, d_fields);
}

// Moments of an in-place lattice; reads only the population buffer (the wall step's neighbours
// directly, DirectSource), not the snapshot.
inline hipError_t enqueue_moments_aa(const clb_desc& d, const Params& p, bool odd, const void* A, const Geo& G,
                                     double* d_fields, hipStream_t st)
{
    switch (d.precision) {
    case CLB_FP64: moments_aa_launch<double, double, false>(odd, A, G, make_par<double>(d, p), d_fields, st); break;
    case CLB_FP64_DEV: moments_aa_launch<double, double, true>(odd, A, G, make_par<double>(d, p), d_fields, st); break;
    case CLB_FP32_SR: moments_aa_launch<float, double, true>(odd, A, G, make_par<double>(d, p), d_fields, st); break;
    default: moments_aa_launch<float, float, true>(odd, A, G, make_par<float>(d, p), d_fields, st); break;
    }
    return hipGetLastError();
}

template <typename S, bool DEV>
inline void populations_aa_launch(bool odd, const void* A, const Geo& G, double TR, double* fo, double* go, hipStream_t st)
{
    const dim3 grid = node_grid(G), block(TX, TY);
    if (odd) populations_aa_kernel<S, DEV, true><<<grid, block, 0, st>>>((const S*)A, G, TR, fo, go);
    else populations_aa_kernel<S, DEV, false><<<grid, block, 0, st>>>((const S*)A, G, TR, fo, go);
}

inline hipError_t enqueue_populations_aa(const clb_desc& d, bool odd, const void* A, const Geo& G, double* d_out,
                                         hipStream_t st)
{
    const size_t n = size_t(d.nx) * d.ny;
    const double TR = is_dev(d.precision) ? d.T0 : 0.0;
    switch (d.precision) {
    case CLB_FP64: populations_aa_launch<double, false>(odd, A, G, TR, d_out, d_out + 9 * n, st); break;
    case CLB_FP64_DEV: populations_aa_launch<double, true>(odd, A, G, TR, d_out, d_out + 9 * n, st); break;
    default: populations_aa_launch<float, true>(odd, A, G, TR, d_out, d_out + 9 * n, st); break;
    }
    return hipGetLastError();
}

inline int diag_blocks(const Geo& G) { return int(((long long)G.nx * G.ny + RED_NT - 1) / RED_NT); }

// Reduce the FP64 moment fields (from enqueue_moments) into the DIAG_SLOTS record d_out.
inline hipError_t enqueue_diag(const double* d_fields, const double* d_snap, int has_snap, const Geo& G,
                               double* d_partials, double* d_out, hipStream_t st)
{
    const int nb = diag_blocks(G);
    diag_reduce_kernel<RED_NT><<<nb, RED_NT, 0, st>>>(d_fields, d_snap, has_snap, G, d_partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    diag_final_kernel<RED_NT><<<1, RED_NT, 0, st>>>(d_partials, nb, d_out);
    return hipGetLastError();
}

// Unpack a DIAG_SLOTS record.
inline void unpack_diag(const double* r, long long step, clb_diag* out)
{
    out->step = step;
    out->mass = r[0];
    out->heat = r[1];
    out->mom_x = r[2];
    out->mom_y = r[3];
    out->sum_w = r[4];
    out->sum_w_ux_T = r[5];
    out->sum_w_uy_T = r[6];
    for (int i = 0; i < 4; ++i) out->wall_flux[i] = r[7 + i];
    out->u_max = r[DIAG_SUMS + 0];
    out->du_max = r[DIAG_SUMS + 1];
    out->dT_max = r[DIAG_SUMS + 2];
    out->nonfinite = r[DIAG_SUMS + 3] > 0.0 ? 1 : 0;
}

}  // namespace clb
