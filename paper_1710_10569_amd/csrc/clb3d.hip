// clb3d.hip -- the three-dimensional CLB path (D3Q27 flow, D3Q7 temperature) on gfx950, behind
// include/clb3d.h.
//
// Storage: chunked structure of arrays, as in two dimensions.  A row (y, z) of the lattice is a
// run of ceil(nx / 64) chunks of 64 consecutive nodes along x; a chunk holds the 34 populations of
// its nodes (f of the 27 flow velocities, then g of the 7 temperature velocities) as 34 runs of 64
// values.  Stored are deviations from the rest state: f_i - w_i with w_i = w(e_ix) w(e_iy) w(e_iz),
// w(0) = 2/3, w(+-1) = 1/6, and g_j - w^T_j T0 with w^T = 1/4 (rest), 1/8 (axes).  Two buffers: a
// step pulls from one and stores into the other; population i of node x is stored at x after
// collision (f*_i(x)), and pulled by x + e_i.
//
// One thread per node, 256-thread workgroups of 64 x 4 nodes in one z plane, tiles handed to the
// eight XCDs in contiguous bands of the (x, y, z) tile order.  The two wall planes and the planes
// between them are separate launches of the same per-node code, so the interior kernel carries
// none of the wall step's registers (FP32: 57 VGPRs and 8 waves per SIMD instead of 112 and 4).
// Per node and step:
//   pull the 34 populations (z walls: sources beyond the wall are replaced by the wall step);
//   wall step on z = 0 and z = nz - 1: non-equilibrium extrapolation of all 34 populations from the
//     inner neighbour, at the node's mass-balance density (known populations + the ones it sent
//     out of the domain the step before, read from its own slots opp(i));
//   rho, u (Eq. 13), T (Eq. 23), F (Eq. 3, gravity along -z);
//   D3Q27 collision (Eq. 8 dimension by dimension): central moments by the factorised transform
//     (three passes of the one-dimensional transform along x, y, z over the nine lines of three
//     populations each), relaxation in deviation form -- k*_dev = (1 - s) k_dev + s (k^eq - k^w)
//     + (1 - s/2) C, with k^w the central moments of the rest weights, so every term is a small
//     deviation and FP32 keeps its relative precision -- and the inverse transform;
//   D3Q7 collision (Eq. 19) in the same deviation form;
//   store the 34 post-collision populations (FP32 with stochastic rounding in the SR form).
#include "clb_internal.h"
#include "../../include/clb3d.h"

#include <cstring>
#include <new>
#include <vector>

namespace clb3 {

using clb::fmix32;
using clb::round_stochastic;
using clb::step_key;
using clb::xorshift32;

constexpr int NQ = 27, NTQ = 7, NP = NQ + NTQ;
constexpr int CW3 = 64, CHUNK3 = NP * CW3;
constexpr int TX = 64, TY = 4, BNT3 = TX * TY;

// D3Q27 velocity of population i: i = (e_x + 1) + 3 (e_y + 1) + 9 (e_z + 1).
__host__ __device__ constexpr int qx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int qy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int qz(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int qopp(int i) { return 26 - i; }
// D3Q7 order: rest, +x, -x, +y, -y, +z, -z.
__host__ __device__ constexpr int tdx(int j) { return j == 1 ? 1 : (j == 2 ? -1 : 0); }
__host__ __device__ constexpr int tdy(int j) { return j == 3 ? 1 : (j == 4 ? -1 : 0); }
__host__ __device__ constexpr int tdz(int j) { return j == 5 ? 1 : (j == 6 ? -1 : 0); }

struct Geo3 {
    int nx, ny, nz;
    int nxc;            // chunks per row
    int walls;          // 1: walls on z = 0 and z = nz - 1
    int zk[2];          // bottom, top: CLB3D_DIRICHLET or CLB3D_ADIABATIC
    int nxt, nyt;       // tiles along x and y
};

template <typename Real>
struct Par3 {
    Real s_nu, s_b, s3, s4, s5, s6;   // flow rates
    Real l1, l2;                      // temperature rates
    Real g_beta, Fv[3];
    Real Toff;                        // T0_storage - T0 (zero: deviations are taken from T0)
    Real TR;                          // rest temperature of the storage form (T0)
    Real uw[2][2];                    // tangential wall velocities, bottom and top
    Real dTw[2];                      // wall temperatures minus TR
};

__host__ __device__ __forceinline__ long long row_base(const Geo3& G, int y, int z)
{
    return ((long long)z * G.ny + y) * G.nxc * (long long)CHUNK3;
}
__host__ __device__ __forceinline__ int col_of(int x) { return (x >> 6) * CHUNK3 + (x & (CW3 - 1)); }

// Source coordinate for velocity component e (pull from x - e).
__host__ __device__ __forceinline__ int src_periodic(int x, int e, int n) { return e == 0 ? x : (e > 0 ? (x > 0 ? x - 1 : n - 1) : (x < n - 1 ? x + 1 : 0)); }
__host__ __device__ __forceinline__ int src_z(const Geo3& G, int z, int e)
{
    if (!G.walls) return src_periodic(z, e, G.nz);
    return e == 0 ? z : (e > 0 ? (z > 0 ? z - 1 : 0) : (z < G.nz - 1 ? z + 1 : G.nz - 1));
}

// The 34 post-streaming populations of node (x, y, z); y and z are uniform over the wavefront.
template <typename S, typename Real>
__host__ __device__ __forceinline__ void pull3(const S* __restrict__ src, const Geo3& G, int x, int y, int z, Real f[NQ], Real g[NTQ])
{
    int cx[3];
#pragma unroll
    for (int e = -1; e <= 1; ++e) cx[e + 1] = col_of(src_periodic(x, e, G.nx));
#pragma unroll
    for (int ez = -1; ez <= 1; ++ez) {
        const int zs = src_z(G, z, ez);
#pragma unroll
        for (int ey = -1; ey <= 1; ++ey) {
            const long long rb = row_base(G, src_periodic(y, ey, G.ny), zs);
#pragma unroll
            for (int ex = -1; ex <= 1; ++ex) {
                const int i = (ex + 1) + 3 * (ey + 1) + 9 * (ez + 1);
                f[i] = Real(src[rb + cx[ex + 1] + i * CW3]);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NTQ; ++j) {
        const long long rb = row_base(G, src_periodic(y, tdy(j), G.ny), src_z(G, z, tdz(j)));
        g[j] = Real(src[rb + cx[tdx(j) + 1] + (NQ + j) * CW3]);
    }
}

template <typename S, typename Real>
__host__ __device__ __forceinline__ Real pull_dT(const S* __restrict__ src, const Geo3& G, int x, int y, int z)
{
    Real s = Real(0);
#pragma unroll
    for (int j = 0; j < NTQ; ++j) {
        const long long rb = row_base(G, src_periodic(y, tdy(j), G.ny), src_z(G, z, tdz(j)));
        s += Real(src[rb + col_of(src_periodic(x, tdx(j), G.nx)) + (NQ + j) * CW3]);
    }
    return s;
}

template <typename Real>
struct Macro3 {
    Real dr, rho, dT, F[3], u[3];
};

template <typename Real>
__host__ __device__ __forceinline__ Macro3<Real> macro3(const Real f[NQ], const Real g[NTQ], const Par3<Real>& P)
{
    Macro3<Real> m;
    m.dT = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + g[6]);
    Real dr = Real(0), jx = Real(0), jy = Real(0), jz = Real(0);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        dr += f[i];
        if (qx(i) != 0) jx += qx(i) > 0 ? f[i] : -f[i];
        if (qy(i) != 0) jy += qy(i) > 0 ? f[i] : -f[i];
        if (qz(i) != 0) jz += qz(i) > 0 ? f[i] : -f[i];
    }
    m.dr = dr;
    m.rho = Real(1) + dr;
    m.F[0] = P.Fv[0];
    m.F[1] = P.Fv[1];
    m.F[2] = P.Fv[2] + P.g_beta * (m.dT + P.Toff);
    const Real inv = Real(1) / m.rho;
    m.u[0] = (jx + Real(0.5) * m.F[0]) * inv;
    m.u[1] = (jy + Real(0.5) * m.F[1]) * inv;
    m.u[2] = (jz + Real(0.5) * m.F[2]) * inv;
    return m;
}

// --- one-dimensional factors ---------------------------------------------------------------
// Equilibrium central-moment factor m(a) = 1, 0, 1/3 and the deviation of the rest weights'
// central moment about u from it, d(a, u) = 0, -u, u^2 (the rest weights' central moments are
// 1, -u, 1/3 + u^2).
template <typename Real> __host__ __device__ __forceinline__ Real mfac(int a) { return a == 0 ? Real(1) : (a == 1 ? Real(0) : Real(1.0 / 3.0)); }
template <typename Real> __host__ __device__ __forceinline__ Real dfac(int a, Real u, Real u2) { return a == 0 ? Real(0) : (a == 1 ? -u : u2); }

// k^eq_abc - k^w_abc = dr m(a) m(b) m(c) - [prod (m + d) - prod m], the bracket telescoped so that
// every term carries a small factor d.
template <typename Real>
__host__ __device__ __forceinline__ Real delta_eq(int a, int b, int c, Real dr, const Real u[3], const Real u2[3])
{
    const Real m1 = mfac<Real>(a), m2 = mfac<Real>(b), m3 = mfac<Real>(c);
    const Real d1 = dfac<Real>(a, u[0], u2[0]), d2 = dfac<Real>(b, u[1], u2[1]), d3 = dfac<Real>(c, u[2], u2[2]);
    const Real t = d1 * ((m2 + d2) * (m3 + d3)) + m1 * (d2 * (m3 + d3) + m2 * d3);
    return dr * (m1 * m2 * m3) - t;
}

// f^eq_i(1 + dr, v) - w_i with f^eq_i = rho psi(e_x, v_x) psi(e_y, v_y) psi(e_z, v_z),
// psi(0, v) = 2/3 - v^2, psi(+-1, v) = (1/3 +- v + v^2)/2 = w(e) + dpsi(e, v).
template <typename Real> __host__ __device__ __forceinline__ Real wfac(int e) { return e == 0 ? Real(2.0 / 3.0) : Real(1.0 / 6.0); }
template <typename Real> __host__ __device__ __forceinline__ Real dpsi(int e, Real v, Real v2) { return e == 0 ? -v2 : Real(0.5) * (Real(e) * v + v2); }
template <typename Real>
__host__ __device__ __forceinline__ Real feq_dev(int i, Real dr, const Real v[3], const Real v2[3])
{
    const int ex = qx(i), ey = qy(i), ez = qz(i);
    const Real w1 = wfac<Real>(ex), w2 = wfac<Real>(ey), w3 = wfac<Real>(ez);
    const Real d1 = dpsi<Real>(ex, v[0], v2[0]), d2 = dpsi<Real>(ey, v[1], v2[1]), d3 = dpsi<Real>(ez, v[2], v2[2]);
    const Real p2 = w2 + d2, p3 = w3 + d3;
    const Real t = d1 * (p2 * p3) + w1 * (d2 * p3 + w2 * d3);
    return dr * ((w1 + d1) * (p2 * p3)) + t;
}

// g^eq_j(T, u) = T phi_j(u): phi_0 = 1/4 - |u|^2, phi_{+-d} = (1/4 +- u_d + u_d^2)/2.
template <typename Real>
__host__ __device__ __forceinline__ Real phi7(int j, const Real u[3])
{
    if (j == 0) return Real(0.25) - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const int d = (j - 1) >> 1;
    const Real s = (j & 1) ? Real(1) : Real(-1);
    return Real(0.5) * (Real(0.25) + s * u[d] + u[d] * u[d]);
}
// phi_j(a) - phi_j(b), formed without O(1) cancellation.
template <typename Real>
__host__ __device__ __forceinline__ Real dphi7(int j, const Real a[3], const Real b[3])
{
    if (j == 0) return (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]) - (a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const int d = (j - 1) >> 1;
    const Real s = (j & 1) ? Real(1) : Real(-1);
    return Real(0.5) * (s * (a[d] - b[d]) + (a[d] * a[d] - b[d] * b[d]));
}

// --- wall step (z walls) --------------------------------------------------------------------
// Node (x, y, z) on wall w (0: bottom, inward +z; 1: top, inward -z).  f, g: pulled populations on
// entry (the unknown ones meaningless), reconstructed on exit.  src holds the previous step's
// post-collision populations, so slot opp(i) of the node itself is what it sent out along opp(i).
template <typename S, typename Real>
__host__ __device__ __forceinline__ void wall_step3(const S* __restrict__ src, const Geo3& G, const Par3<Real>& P,
                                           int x, int y, int z, int w, Real f[NQ], Real g[NTQ])
{
    const int dz = w == 0 ? 1 : -1;
    Real ff[NQ], gf[NTQ];
    pull3(src, G, x, y, z + dz, ff, gf);
    const Macro3<Real> mf = macro3(ff, gf, P);
    Real dTb;
    if (G.zk[w] == CLB3D_DIRICHLET) {
        dTb = P.dTw[w];
    } else {
        const Real dTff = pull_dT<S, Real>(src, G, x, y, z + 2 * dz);
        dTb = (Real(4) * mf.dT - dTff) * Real(1.0 / 3.0);
    }
    const Real uw[3] = {P.uw[w][0], P.uw[w][1], Real(0)};
    // temperature: g_j = g^eq_j(T_b, u_w) + g_j(x_f) - g^eq_j(T_f, u_f)
    const Real Tf = P.TR + mf.dT;
#pragma unroll
    for (int j = 0; j < NTQ; ++j) g[j] = gf[j] + ((dTb - mf.dT) * phi7<Real>(j, uw) + Tf * dphi7<Real>(j, uw, mf.u));
    // density: the node's mass balance
    const long long own = row_base(G, y, z) + col_of(x);
    Real drb = Real(0);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const bool unknown = qz(i) * dz > 0;
        drb += unknown ? Real(src[own + qopp(i) * CW3]) : f[i];
    }
    const Real rb = Real(1) + drb;
    const Real Fbz = P.Fv[2] + P.g_beta * (dTb + P.Toff);
    const Real vb[3] = {uw[0] - Real(0.5) * P.Fv[0] / rb, uw[1] - Real(0.5) * P.Fv[1] / rb, -Real(0.5) * Fbz / rb};
    const Real vf[3] = {mf.u[0] - Real(0.5) * mf.F[0] / mf.rho, mf.u[1] - Real(0.5) * mf.F[1] / mf.rho,
                        mf.u[2] - Real(0.5) * mf.F[2] / mf.rho};
    const Real vb2[3] = {vb[0] * vb[0], vb[1] * vb[1], vb[2] * vb[2]};
    const Real vf2[3] = {vf[0] * vf[0], vf[1] * vf[1], vf[2] * vf[2]};
    // flow: f_i = f^eq_i(rho_b, v_b) + f_i(x_f) - f^eq_i(rho_f, v_f)
#pragma unroll
    for (int i = 0; i < NQ; ++i) f[i] = ff[i] + (feq_dev<Real>(i, drb, vb, vb2) - feq_dev<Real>(i, mf.dr, vf, vf2));
}

// --- collisions -----------------------------------------------------------------------------
template <int ST, typename Real>
__host__ __device__ __forceinline__ void fwd_line(Real* K, int m, Real u, Real u2)
{
    const Real a = K[m], b = K[m + ST], c = K[m + 2 * ST];   // e = -1, 0, +1
    const Real s = c + a, d = c - a, k0 = s + b;
    K[m] = k0;
    K[m + ST] = d - u * k0;
    K[m + 2 * ST] = (s - Real(2) * u * d) + u2 * k0;
}

template <int ST, typename Real>
__host__ __device__ __forceinline__ void inv_line(Real* K, int m, Real u, Real u2)
{
    const Real k0 = K[m], k1 = K[m + ST], k2 = K[m + 2 * ST];
    const Real m1 = k1 + u * k0;
    const Real m2 = (k2 + Real(2) * u * k1) + u2 * k0;
    K[m] = Real(0.5) * (m2 - m1);
    K[m + ST] = k0 - m2;
    K[m + 2 * ST] = Real(0.5) * (m2 + m1);
}

// D3Q27 collision in place: f (deviations) -> post-collision deviations.  UNIT: s_b = s3 = s4 = s5 = s6
// = 1 (the default rates), so the trace of the second-order diagonal and every moment of order 3 to 6
// relax to their equilibrium (plus half the forcing) in one step: the central moments of those orders
// are not needed, and the compiler drops the parts of the forward transform that only they use.  The
// result agrees with the general form to rounding (K - (K - K^eq) against K^eq).
template <typename Real, bool UNIT = false>
__host__ __device__ __forceinline__ void collide27(Real K[NQ], const Macro3<Real>& m, const Par3<Real>& P)
{
    const Real u2[3] = {m.u[0] * m.u[0], m.u[1] * m.u[1], m.u[2] * m.u[2]};
    // central moments of the deviations: passes along x (stride 1), y (stride 3), z (stride 9);
    // afterwards K[a + 3 b + 9 c] = k~_abc
#pragma unroll
    for (int l = 0; l < 9; ++l) fwd_line<1>(K, 3 * l, m.u[0], u2[0]);
#pragma unroll
    for (int l = 0; l < 9; ++l) fwd_line<3>(K, (l % 3) + 9 * (l / 3), m.u[1], u2[1]);
#pragma unroll
    for (int l = 0; l < 9; ++l) fwd_line<9>(K, l, m.u[2], u2[2]);

    // relaxation, all but the diagonal second-order block
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
        const int a = i % 3, b = (i / 3) % 3, c = i / 9, o = a + b + c;
        const int n1 = (a == 1) + (b == 1) + (c == 1);
        // forcing central moment (Eq. 11's pattern): nonzero only with exactly one index 1
        Real C = Real(0);
        if (n1 == 1) {
            const Real Fd = a == 1 ? m.F[0] : (b == 1 ? m.F[1] : m.F[2]);
            C = Fd * (mfac<Real>(a == 1 ? 0 : a) * mfac<Real>(b == 1 ? 0 : b) * mfac<Real>(c == 1 ? 0 : c));
        }
        if (o == 1) { K[i] += C; continue; }        // conserved: S = 0
        if (o == 2 && n1 == 0) continue;            // k~200, k~020, k~002 below
        const Real De = delta_eq<Real>(a, b, c, m.dr, m.u, u2);
        if (UNIT && o >= 3) { K[i] = De + Real(0.5) * C; continue; }
        const Real s = o == 2 ? P.s_nu : (o == 3 ? P.s3 : (o == 4 ? P.s4 : (o == 5 ? P.s5 : P.s6)));
        K[i] = (K[i] - s * (K[i] - De)) + (Real(1) - Real(0.5) * s) * C;
    }
    {
        // trace with s_b, deviatoric part with s_nu
        const Real Dx = delta_eq<Real>(2, 0, 0, m.dr, m.u, u2), Dy = delta_eq<Real>(0, 2, 0, m.dr, m.u, u2),
                   Dz = delta_eq<Real>(0, 0, 2, m.dr, m.u, u2);
        const Real kt = (K[2] + K[6]) + K[18], Dt = (Dx + Dy) + Dz;
        const Real third = Real(1.0 / 3.0);
        const Real tr = (UNIT ? Dt : kt - P.s_b * (kt - Dt)) * third;
        const Real ax = K[2] - kt * third, ay = K[6] - kt * third, az = K[18] - kt * third;
        K[2] = tr + (ax - P.s_nu * (ax - (Dx - Dt * third)));
        K[6] = tr + (ay - P.s_nu * (ay - (Dy - Dt * third)));
        K[18] = tr + (az - P.s_nu * (az - (Dz - Dt * third)));
    }

#pragma unroll
    for (int l = 0; l < 9; ++l) inv_line<9>(K, l, m.u[2], u2[2]);
#pragma unroll
    for (int l = 0; l < 9; ++l) inv_line<3>(K, (l % 3) + 9 * (l / 3), m.u[1], u2[1]);
#pragma unroll
    for (int l = 0; l < 9; ++l) inv_line<1>(K, 3 * l, m.u[0], u2[0]);
}

// D3Q7 collision in place (deviations g_j - w^T_j TR).
template <typename Real>
__host__ __device__ __forceinline__ void collide7(Real g[NTQ], const Macro3<Real>& m, const Par3<Real>& P)
{
    const Real T = P.TR + m.dT;
    Real s2 = Real(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const Real gp = g[1 + 2 * d], gm = g[2 + 2 * d], u = m.u[d];
        const Real m1 = gp - gm;
        const Real k1 = m1 - u * T;                                                     // k~_d
        const Real k2 = (((gp + gm) - Real(0.25) * m.dT) - Real(2) * u * m1) + u * u * T;   // k~_dd - T/4
        const Real m1s = (k1 - P.l1 * k1) + u * T;
        const Real m2s = ((k2 - P.l2 * k2) + Real(0.25) * m.dT) + (Real(2) * u * m1s - u * u * T);   // m2* - TR/4
        g[1 + 2 * d] = Real(0.5) * (m2s + m1s);
        g[2 + 2 * d] = Real(0.5) * (m2s - m1s);
        s2 += m2s;
    }
    g[0] = m.dT - s2;
}

// Round and store the 34 values of one node (FP32 storage of FP64 arithmetic: stochastic rounding,
// 17 words per node: fmix32(node + key), then xorshift32; each word's halves round two values).
template <typename S, typename Real>
__device__ __forceinline__ void store3(S* __restrict__ dst, long long o, const Real f[NQ], const Real g[NTQ],
                                       uint32_t key, uint32_t node)
{
    if constexpr (sizeof(S) == 4 && sizeof(Real) == 8) {
        uint32_t r = fmix32(node + key);
#pragma unroll
        for (int k = 0; k < NP / 2; ++k) {
            if (k > 0) r = xorshift32(r);
            const int i0 = 2 * k, i1 = 2 * k + 1;
            const Real a = i0 < NQ ? f[i0] : g[i0 - NQ];
            const Real c = i1 < NQ ? f[i1] : g[i1 - NQ];
            __builtin_nontemporal_store(round_stochastic(a, r), dst + o + i0 * CW3);
            __builtin_nontemporal_store(round_stochastic(c, r >> 16), dst + o + i1 * CW3);
        }
    } else {
#pragma unroll
        for (int i = 0; i < NQ; ++i) __builtin_nontemporal_store(S(f[i]), dst + o + i * CW3);
#pragma unroll
        for (int j = 0; j < NTQ; ++j) __builtin_nontemporal_store(S(g[j]), dst + o + (NQ + j) * CW3);
    }
}

// The planes one launch covers: z0 .. z0 + count - 1, or (walls_only) the two wall planes z = 0
// and z = nz - 1.
struct Planes {
    int z0, count, walls_only;
    long long ntiles;   // tiles of the launch: nxt nyt count
};

// Tile t of the band-ordered grid -> node of this thread; y and z are uniform over the wavefront.
__device__ __forceinline__ bool node_of(const Geo3& G, const Planes& Z, int& x, int& y, int& z)
{
    const unsigned q = gridDim.x >> 3;
    const long long t = (long long)(blockIdx.x & 7u) * q + (blockIdx.x >> 3);
    if (t >= Z.ntiles) return false;
    const long long txy = (long long)G.nxt * G.nyt;
    const int p = int(t / txy);
    const int r = int(t - (long long)p * txy);
    const int ty = r / G.nxt, tx = r - ty * G.nxt;
    x = tx * TX + int(threadIdx.x & (TX - 1));
    y = __builtin_amdgcn_readfirstlane(ty * TY + int(threadIdx.x >> 6));
    z = __builtin_amdgcn_readfirstlane(Z.walls_only ? (p == 0 ? 0 : G.nz - 1) : Z.z0 + p);
    return x < G.nx && y < G.ny;
}

__host__ __device__ __forceinline__ int wall_of(const Geo3& G, int z)
{
    return !G.walls ? -1 : (z == 0 ? 0 : (z == G.nz - 1 ? 1 : -1));
}

// The whole update of node (x, y, z): pull, wall step (wall planes), macroscopic, both collisions;
// the 34 post-collision populations are left in f, g.  WALL: 1 the node lies on a wall plane,
// 0 it does not, -1 test at run time.  (The step launches the wall planes and the others
// separately, so that the interior kernel carries none of the wall step's registers.)
template <int WALL, bool UNIT = false, typename S, typename Real>
__host__ __device__ __forceinline__ void update_node3(const S* __restrict__ src, const Geo3& G, const Par3<Real>& P, int x, int y,
                                                      int z, Real f[NQ], Real g[NTQ])
{
    pull3(src, G, x, y, z, f, g);
    if (WALL != 0) {
        const int w = wall_of(G, z);
        if (WALL == 1 || w >= 0) wall_step3(src, G, P, x, y, z, w, f, g);
    }
    const Macro3<Real> m = macro3(f, g, P);
    collide27<Real, UNIT>(f, m, P);
    collide7(g, m, P);
}

// rho, u, T of node (x, y, z) of the current state into FP64 planes (rho, ux, uy, uz, T).
template <typename S, typename Real>
__host__ __device__ __forceinline__ void moments_node3(const S* __restrict__ src, const Geo3& G, const Par3<Real>& P, int x, int y,
                                                       int z, double* __restrict__ out)
{
    Real f[NQ], g[NTQ];
    pull3(src, G, x, y, z, f, g);
    const int w = wall_of(G, z);
    if (w >= 0) wall_step3(src, G, P, x, y, z, w, f, g);
    const Macro3<Real> m = macro3(f, g, P);
    const long long n = (long long)G.nx * G.ny * G.nz, k = ((long long)z * G.ny + y) * G.nx + x;
    out[k] = double(m.rho);
    out[n + k] = double(m.u[0]);
    out[2 * n + k] = double(m.u[1]);
    out[3 * n + k] = double(m.u[2]);
    out[4 * n + k] = double(P.TR) + double(m.dT);
}

// One step over the planes of Z; WALL: Z is the two wall planes (1) or planes without walls (0);
// UNIT: the unit-rate collision (collide27).
template <typename S, typename Real, int WALL, bool UNIT = false>
__global__ __launch_bounds__(BNT3) void step3_kernel(const S* __restrict__ src, S* __restrict__ dst, Geo3 G, Par3<Real> P,
                                                    Planes Z, uint32_t key)
{
    int x, y, z;
    if (!node_of(G, Z, x, y, z)) return;
    Real f[NQ], g[NTQ];
    update_node3<WALL, UNIT>(src, G, P, x, y, z, f, g);
    store3<S, Real>(dst, row_base(G, y, z) + col_of(x), f, g, key, uint32_t(((long long)z * G.ny + y) * G.nx + x));
}

template <typename S, typename Real>
__global__ __launch_bounds__(BNT3) void moments3_kernel(const S* __restrict__ src, Geo3 G, Par3<Real> P, Planes Z,
                                                       double* __restrict__ out)
{
    int x, y, z;
    if (!node_of(G, Z, x, y, z)) return;
    moments_node3(src, G, P, x, y, z, out);
}

// Field index of the node x + e (periodic wrap), or of x itself (ok = 0) beyond a z wall.
__host__ __device__ __forceinline__ long long field_at(const Geo3& G, int x, int y, int z, int ex, int ey, int ez, int& ok)
{
    const int xx = (x + ex + G.nx) % G.nx, yy = (y + ey + G.ny) % G.ny;
    int zz = z + ez;
    ok = 1;
    if (G.walls) {
        if (zz < 0 || zz >= G.nz) ok = 0;
    } else {
        zz = (zz + G.nz) % G.nz;
    }
    return ok ? ((long long)zz * G.ny + yy) * G.nx + xx : ((long long)z * G.ny + y) * G.nx + x;
}

// Initial state from FP64 planes (rho, ux, uy, uz, T): slot i of node x holds the population that
// node x + e_i pulls, f_i(x + e_i) = f^eq_i(rho, u - F/(2 rho)) there; where x + e_i lies beyond a z
// wall, the slot holds what the node sent out, taken as the initial value of the unknown
// population it pairs with, f_opp(i)(x).  Temperature slots: g^eq_j(T, u) of x + e_j (of x itself
// beyond a wall, where the wall step replaces them).
template <typename S, typename Real>
__host__ __device__ __forceinline__ void init_node3(S* __restrict__ dst, const Geo3& G, const Par3<Real>& P,
                                                    const double* __restrict__ fl, int x, int y, int z)
{
    const long long n = (long long)G.nx * G.ny * G.nz;
    const long long o = row_base(G, y, z) + col_of(x);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        int ok;
        const long long k = field_at(G, x, y, z, qx(i), qy(i), qz(i), ok);
        const int q = ok ? i : qopp(i);
        const Real rho = Real(fl[k]), dT = Real(fl[4 * n + k] - double(P.TR));
        const Real Fz = P.Fv[2] + P.g_beta * (dT + P.Toff);
        const Real v[3] = {Real(fl[n + k]) - Real(0.5) * P.Fv[0] / rho, Real(fl[2 * n + k]) - Real(0.5) * P.Fv[1] / rho,
                           Real(fl[3 * n + k]) - Real(0.5) * Fz / rho};
        const Real v2[3] = {v[0] * v[0], v[1] * v[1], v[2] * v[2]};
        dst[o + i * CW3] = S(feq_dev<Real>(q, rho - Real(1), v, v2));
    }
#pragma unroll
    for (int j = 0; j < NTQ; ++j) {
        int ok;
        const long long k = field_at(G, x, y, z, tdx(j), tdy(j), tdz(j), ok);
        const Real u[3] = {Real(fl[n + k]), Real(fl[2 * n + k]), Real(fl[3 * n + k])};
        const Real dT = Real(fl[4 * n + k] - double(P.TR));
        // g^eq_j - w^T_j TR = dT phi_j(u) + TR (phi_j(u) - w^T_j)
        const Real zero[3] = {Real(0), Real(0), Real(0)};
        dst[o + (NQ + j) * CW3] = S(dT * phi7<Real>(j, u) + P.TR * dphi7<Real>(j, u, zero));
    }
}

template <typename S, typename Real>
__global__ __launch_bounds__(BNT3) void init3_kernel(S* __restrict__ dst, Geo3 G, Par3<Real> P, Planes Z, const double* __restrict__ fl)
{
    int x, y, z;
    if (!node_of(G, Z, x, y, z)) return;
    init_node3(dst, G, P, fl, x, y, z);
}

// Diagnostics: per-workgroup partial sums in a fixed order, then one workgroup sums the partials.
constexpr int DG = 7;   // mass, momentum x y z, heat, uzT, max speed
__global__ __launch_bounds__(256) void diag3_partial_kernel(const double* __restrict__ fl, long long n, int nx, int ny, int nz,
                                                           int walls, double T0, double* __restrict__ part)
{
    __shared__ double sh[DG][256];
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    double v[DG] = {0, 0, 0, 0, 0, 0, 0};
    if (k < n) {
        const double r = fl[k], ux = fl[n + k], uy = fl[2 * n + k], uz = fl[3 * n + k], T = fl[4 * n + k];
        const int z = int(k / ((long long)nx * ny));
        const double wz = (walls && (z == 0 || z == nz - 1)) ? 0.5 : 1.0;
        v[0] = r;
        v[1] = r * ux;
        v[2] = r * uy;
        v[3] = r * uz;
        v[4] = T;
        v[5] = wz * uz * (T - T0);
        v[6] = sqrt(ux * ux + uy * uy + uz * uz);
    }
    for (int q = 0; q < DG; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s)
            for (int q = 0; q < DG; ++q)
                sh[q][threadIdx.x] = q == 6 ? fmax(sh[q][threadIdx.x], sh[q][threadIdx.x + s]) : sh[q][threadIdx.x] + sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < DG) part[(long long)blockIdx.x * DG + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void diag3_final_kernel(const double* __restrict__ part, int nb, const double* __restrict__ fl,
                                                         long long n, int nx, int ny, int nz, double* __restrict__ out)
{
    __shared__ double sh[DG + 6][256];
    double v[DG + 6] = {0};
    for (int b = threadIdx.x; b < nb; b += 256)
        for (int q = 0; q < DG; ++q) v[q] = q == 6 ? fmax(v[q], part[(long long)b * DG + q]) : v[q] + part[(long long)b * DG + q];
    // plane sums of T on z = 0, 1, 2, nz - 3, nz - 2, nz - 1
    const long long plane = (long long)nx * ny;
    for (int p = 0; p < 6; ++p) {
        const int zp = p < 3 ? p : nz - 6 + p;
        if (zp < 0 || zp >= nz) continue;
        for (long long k = threadIdx.x; k < plane; k += 256) v[DG + p] += fl[4 * n + zp * plane + k];
    }
    for (int q = 0; q < DG + 6; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s)
            for (int q = 0; q < DG + 6; ++q)
                sh[q][threadIdx.x] = q == 6 ? fmax(sh[q][threadIdx.x], sh[q][threadIdx.x + s]) : sh[q][threadIdx.x] + sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < DG + 6) out[threadIdx.x] = sh[threadIdx.x][0];
}

}  // namespace clb3

using namespace clb3;

struct clb3d_lattice {
    clb3d_desc desc{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t buf_bytes = 0;
    void* buf[2] = {nullptr, nullptr};
    int cur = 0;                     // buffer holding the post-collision state of the last step
    double tau_nu = 1.0, tau_alpha = 1.0, g_beta = 0.0;
    double s_b = 1.0, s3 = 1.0, s4 = 1.0, s5 = 1.0, s6 = 1.0, lam2 = 1.0;
    double Fv[3] = {0.0, 0.0, 0.0};
    long long steps = 0;
    double* d_fields = nullptr;      // 5 FP64 planes: init input, moments output
    double* d_part = nullptr;        // diagnostics partials
    double* d_diag = nullptr;        // final diagnostics record (13 values)
    hipEvent_t ev[2] = {nullptr, nullptr};
};

namespace {

using clb::set_error;
using clb::clear_error;

bool is_fp32(int p) { return p == CLB_FP32_DEV || p == CLB_FP32_SR; }

int validate3(const clb3d_desc* d)
{
    if (!d) { set_error("NULL description"); return CLB_EINVAL; }
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) { set_error("nx, ny, nz must be >= 1"); return CLB_EINVAL; }
    if (d->precision < CLB_FP64 || d->precision > CLB_FP32_SR) { set_error("unknown precision %d", d->precision); return CLB_EINVAL; }
    const int kb = d->bottom.kind, kt = d->top.kind;
    for (int k : {kb, kt})
        if (k != CLB3D_PERIODIC && k != CLB3D_DIRICHLET && k != CLB3D_ADIABATIC) { set_error("unknown wall kind %d", k); return CLB_EINVAL; }
    if ((kb == CLB3D_PERIODIC) != (kt == CLB3D_PERIODIC)) { set_error("bottom and top must both be periodic or both walls"); return CLB_EINVAL; }
    if (kb != CLB3D_PERIODIC && d->nz < 3) { set_error("z walls need nz >= 3"); return CLB_EINVAL; }
    const double nodes = double(d->nx) * d->ny * d->nz;
    if (nodes > 2.0e9) { set_error("too many nodes (%.3g)", nodes); return CLB_EINVAL; }
    const double vals[] = {d->bottom.ux, d->bottom.uy, d->bottom.T, d->top.ux, d->top.uy, d->top.T, d->T0};
    for (double v : vals)
        if (!std::isfinite(v)) { set_error("non-finite wall data or T0"); return CLB_EINVAL; }
    return CLB_OK;
}

Geo3 make_geo3(const clb3d_desc& d)
{
    Geo3 G;
    G.nx = d.nx; G.ny = d.ny; G.nz = d.nz;
    G.nxc = (d.nx + CW3 - 1) / CW3;
    G.walls = d.bottom.kind != CLB3D_PERIODIC;
    G.zk[0] = d.bottom.kind; G.zk[1] = d.top.kind;
    G.nxt = (d.nx + TX - 1) / TX;
    G.nyt = (d.ny + TY - 1) / TY;
    return G;
}

template <typename Real>
Par3<Real> make_par3(const clb3d_lattice* h)
{
    Par3<Real> P;
    const clb3d_desc& d = h->desc;
    P.s_nu = Real(1.0 / h->tau_nu); P.s_b = Real(h->s_b);
    P.s3 = Real(h->s3); P.s4 = Real(h->s4); P.s5 = Real(h->s5); P.s6 = Real(h->s6);
    P.l1 = Real(1.0 / h->tau_alpha); P.l2 = Real(h->lam2);
    P.g_beta = Real(h->g_beta);
    for (int i = 0; i < 3; ++i) P.Fv[i] = Real(h->Fv[i]);
    P.TR = Real(d.T0);
    P.Toff = Real(0);
    P.uw[0][0] = Real(d.bottom.ux); P.uw[0][1] = Real(d.bottom.uy);
    P.uw[1][0] = Real(d.top.ux); P.uw[1][1] = Real(d.top.uy);
    P.dTw[0] = Real(d.bottom.T - d.T0);
    P.dTw[1] = Real(d.top.T - d.T0);
    return P;
}

unsigned grid_of(const Planes& Z) { return unsigned((Z.ntiles + 7) / 8 * 8); }

Planes planes(const Geo3& G, int z0, int count, int walls_only)
{
    Planes Z;
    Z.z0 = z0;
    Z.count = count;
    Z.walls_only = walls_only;
    Z.ntiles = (long long)G.nxt * G.nyt * count;
    return Z;
}
Planes all_planes(const Geo3& G) { return planes(G, 0, G.nz, 0); }

size_t buffer_bytes3(const clb3d_desc& d)
{
    const size_t eb = is_fp32(d.precision) ? 4 : 8;
    return size_t((d.nx + CW3 - 1) / CW3) * d.ny * d.nz * CHUNK3 * eb;
}

long long nodes3(const clb3d_desc& d) { return (long long)d.nx * d.ny * d.nz; }
long long diag_blocks(const clb3d_desc& d) { return (nodes3(d) + 255) / 256; }

// Occupancy of the interior launch.  FP32 storage with FP32 arithmetic needs 57 VGPRs, so 8 wavefronts
// per SIMD fit, but fewer are faster (256 x 256 x 129 layer, one MI355X: 413.7 us per step at 8, 406.4
// at 6, 404.7 at 5, against a 402 us ceiling of the access pattern): dynamic LDS the kernel does not
// use holds a CU to 5 workgroups of 256 threads.  The FP64-arithmetic forms run at 4 wavefronts by
// their registers.
template <typename S, typename Real>
constexpr size_t occupancy_lds3()
{
    return sizeof(S) == 4 && sizeof(Real) == 4 ? size_t(160 * 1024 / 5) : 0;
}

template <typename S, typename Real>
int launch_step(clb3d_lattice* h, long long n)
{
    const Geo3 G = make_geo3(h->desc);
    const Par3<Real> P = make_par3<Real>(h);
    // with walls: the two wall planes, then the planes between them (independent nodes of the same
    // step); periodic z: every plane in one launch
    const Planes Zw = planes(G, 0, 2, 1);
    const Planes Zi = G.walls ? planes(G, 1, G.nz - 2, 0) : all_planes(G);
    const bool unit = h->s_b == 1.0 && h->s3 == 1.0 && h->s4 == 1.0 && h->s5 == 1.0 && h->s6 == 1.0;
    constexpr size_t lds = occupancy_lds3<S, Real>();
    for (long long s = 0; s < n; ++s) {
        const S* src = static_cast<const S*>(h->buf[h->cur]);
        S* dst = static_cast<S*>(h->buf[h->cur ^ 1]);
        const uint32_t key = step_key(uint32_t(h->steps));
        if (G.walls) {
            if (unit) hipLaunchKernelGGL((step3_kernel<S, Real, 1, true>), dim3(grid_of(Zw)), dim3(BNT3), 0, h->stream, src, dst, G, P, Zw, key);
            else hipLaunchKernelGGL((step3_kernel<S, Real, 1>), dim3(grid_of(Zw)), dim3(BNT3), 0, h->stream, src, dst, G, P, Zw, key);
            CLB_HIP(hipGetLastError());
        }
        if (Zi.count > 0) {
            if (unit) hipLaunchKernelGGL((step3_kernel<S, Real, 0, true>), dim3(grid_of(Zi)), dim3(BNT3), lds, h->stream, src, dst, G, P, Zi, key);
            else hipLaunchKernelGGL((step3_kernel<S, Real, 0>), dim3(grid_of(Zi)), dim3(BNT3), lds, h->stream, src, dst, G, P, Zi, key);
            CLB_HIP(hipGetLastError());
        }
        h->cur ^= 1;
        ++h->steps;
    }
    return CLB_OK;
}

int step_any(clb3d_lattice* h, long long n)
{
    switch (h->desc.precision) {
    case CLB_FP32_DEV: return launch_step<float, float>(h, n);
    case CLB_FP32_SR: return launch_step<float, double>(h, n);
    default: return launch_step<double, double>(h, n);
    }
}

template <typename S, typename Real>
int launch_moments(clb3d_lattice* h)
{
    const Geo3 G = make_geo3(h->desc);
    const Planes Z = all_planes(G);
    hipLaunchKernelGGL((moments3_kernel<S, Real>), dim3(grid_of(Z)), dim3(BNT3), 0, h->stream,
                       static_cast<const S*>(h->buf[h->cur]), G, make_par3<Real>(h), Z, h->d_fields);
    CLB_HIP(hipGetLastError());
    return CLB_OK;
}

int moments_any(clb3d_lattice* h)
{
    switch (h->desc.precision) {
    case CLB_FP32_DEV: return launch_moments<float, float>(h);
    case CLB_FP32_SR: return launch_moments<float, double>(h);
    default: return launch_moments<double, double>(h);
    }
}

template <typename S, typename Real>
int launch_init(clb3d_lattice* h)
{
    const Geo3 G = make_geo3(h->desc);
    const Planes Z = all_planes(G);
    hipLaunchKernelGGL((init3_kernel<S, Real>), dim3(grid_of(Z)), dim3(BNT3), 0, h->stream,
                       static_cast<S*>(h->buf[h->cur]), G, make_par3<Real>(h), Z, h->d_fields);
    CLB_HIP(hipGetLastError());
    return CLB_OK;
}

// Initial fields: the given arrays, or rho = 1, u = 0, T = T0.
int upload_fields(clb3d_lattice* h, const double* rho, const double* u, const double* T)
{
    const long long n = nodes3(h->desc);
    std::vector<double> host;
    try {
        host.assign(size_t(5 * n), 0.0);
    } catch (const std::bad_alloc&) {
        set_error("host allocation of the initial fields failed");
        return CLB_ENOMEM;
    }
    for (long long k = 0; k < n; ++k) {
        host[k] = rho ? rho[k] : 1.0;
        host[n + k] = u ? u[k] : 0.0;
        host[2 * n + k] = u ? u[n + k] : 0.0;
        host[3 * n + k] = u ? u[2 * n + k] : 0.0;
        host[4 * n + k] = T ? T[k] : h->desc.T0;
    }
    for (long long k = 0; k < n; ++k)
        if (!(host[k] > 0.0) || !std::isfinite(host[k]) || !std::isfinite(host[n + k]) || !std::isfinite(host[2 * n + k]) ||
            !std::isfinite(host[3 * n + k]) || !std::isfinite(host[4 * n + k])) {
            set_error("initial fields must be finite with rho > 0 (node %lld)", k);
            return CLB_EINVAL;
        }
    CLB_HIP(hipMemcpyAsync(h->d_fields, host.data(), size_t(5 * n) * sizeof(double), hipMemcpyHostToDevice, h->stream));
    CLB_HIP(hipStreamSynchronize(h->stream));
    return CLB_OK;
}

int check_rate(double s, const char* name)
{
    if (!(s > 0.0 && s < 2.0)) { set_error("%s must lie in (0, 2), got %g", name, s); return CLB_EINVAL; }
    return CLB_OK;
}

}  // namespace

extern "C" size_t clb3d_footprint(const clb3d_desc* desc)
{
    clear_error();
    if (validate3(desc) != CLB_OK) return 0;
    return 2 * buffer_bytes3(*desc) + size_t(5 * nodes3(*desc)) * sizeof(double) +
           size_t(diag_blocks(*desc)) * DG * sizeof(double) + 16 * sizeof(double);
}

extern "C" void clb3d_destroy(clb3d_lattice* h)
{
    if (!h) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    (void)hipFree(h->buf[0]);
    (void)hipFree(h->buf[1]);
    (void)hipFree(h->d_fields);
    (void)hipFree(h->d_part);
    (void)hipFree(h->d_diag);
    for (hipEvent_t& e : h->ev)
        if (e) (void)hipEventDestroy(e);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    (void)hipSetDevice(prev);
    delete h;
}

extern "C" int clb3d_create(const clb3d_desc* desc, void* hip_stream, clb3d_lattice** out)
{
    clear_error();
    if (!out) { set_error("NULL output"); return CLB_EINVAL; }
    *out = nullptr;
    int rc = validate3(desc);
    if (rc) return rc;
    clb3d_lattice* h = new (std::nothrow) clb3d_lattice;
    if (!h) { set_error("host allocation failed"); return CLB_ENOMEM; }
    h->desc = *desc;
    if (hipGetDevice(&h->device) != hipSuccess) { delete h; set_error("no HIP device"); return CLB_EDEVICE; }
    auto fail = [&](int code) { clb3d_destroy(h); return code; };
    if (hip_stream) {
        h->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) { set_error("stream creation failed"); return fail(CLB_EDEVICE); }
        h->own_stream = true;
    }
    h->buf_bytes = buffer_bytes3(*desc);
    const long long n = nodes3(*desc);
    const size_t field_bytes = size_t(5 * n) * sizeof(double);
    const size_t part_bytes = size_t(diag_blocks(*desc)) * DG * sizeof(double);
    if (hipMalloc(&h->buf[0], h->buf_bytes) != hipSuccess || hipMalloc(&h->buf[1], h->buf_bytes) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&h->d_fields), field_bytes) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&h->d_part), part_bytes) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&h->d_diag), 16 * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation of %.3g GB failed", double(2 * h->buf_bytes + field_bytes) / 1e9);
        return fail(CLB_ENOMEM);
    }
    // padding lanes of partial chunks are never read as populations; clear them once
    if (hipMemsetAsync(h->buf[0], 0, h->buf_bytes, h->stream) != hipSuccess ||
        hipMemsetAsync(h->buf[1], 0, h->buf_bytes, h->stream) != hipSuccess ||
        hipEventCreate(&h->ev[0]) != hipSuccess || hipEventCreate(&h->ev[1]) != hipSuccess) {
        set_error("device initialisation failed");
        return fail(CLB_EDEVICE);
    }
    rc = clb3d_init(h, nullptr, nullptr, nullptr);
    if (rc) return fail(rc);
    *out = h;
    return CLB_OK;
}

extern "C" int clb3d_set_params(clb3d_lattice* h, double tau_nu, double tau_alpha, double g_beta)
{
    clear_error();
    if (!h) { set_error("lattice is NULL"); return CLB_EINVAL; }
    if (!(tau_nu > 0.5) || !(tau_alpha > 0.5) || !std::isfinite(tau_nu) || !std::isfinite(tau_alpha) || !std::isfinite(g_beta)) {
        set_error("need tau_nu, tau_alpha > 1/2 and a finite g_beta");
        return CLB_EINVAL;
    }
    h->tau_nu = tau_nu;
    h->tau_alpha = tau_alpha;
    h->g_beta = g_beta;
    return CLB_OK;
}

extern "C" int clb3d_set_relaxation(clb3d_lattice* h, double s_b, double s3, double s4, double s5, double s6, double lambda2)
{
    clear_error();
    if (!h) { set_error("lattice is NULL"); return CLB_EINVAL; }
    int rc;
    if ((rc = check_rate(s_b, "s_b")) || (rc = check_rate(s3, "s3")) || (rc = check_rate(s4, "s4")) ||
        (rc = check_rate(s5, "s5")) || (rc = check_rate(s6, "s6")) || (rc = check_rate(lambda2, "lambda2")))
        return rc;
    h->s_b = s_b; h->s3 = s3; h->s4 = s4; h->s5 = s5; h->s6 = s6; h->lam2 = lambda2;
    return CLB_OK;
}

extern "C" int clb3d_set_body_force(clb3d_lattice* h, double Fx, double Fy, double Fz)
{
    clear_error();
    if (!h) { set_error("lattice is NULL"); return CLB_EINVAL; }
    if (!std::isfinite(Fx) || !std::isfinite(Fy) || !std::isfinite(Fz)) { set_error("non-finite body force"); return CLB_EINVAL; }
    h->Fv[0] = Fx; h->Fv[1] = Fy; h->Fv[2] = Fz;
    return CLB_OK;
}

extern "C" int clb3d_init(clb3d_lattice* h, const double* rho, const double* u, const double* T)
{
    clear_error();
    if (!h) { set_error("lattice is NULL"); return CLB_EINVAL; }
    CLB_HIP(hipSetDevice(h->device));
    int rc = upload_fields(h, rho, u, T);
    if (rc) return rc;
    h->cur = 0;
    h->steps = 0;
    switch (h->desc.precision) {
    case CLB_FP32_DEV: rc = launch_init<float, float>(h); break;
    case CLB_FP32_SR: rc = launch_init<float, double>(h); break;
    default: rc = launch_init<double, double>(h); break;
    }
    if (rc) return rc;
    CLB_HIP(hipStreamSynchronize(h->stream));
    return CLB_OK;
}

extern "C" int clb3d_step(clb3d_lattice* h, long long n)
{
    clear_error();
    if (!h) { set_error("lattice is NULL"); return CLB_EINVAL; }
    if (n < 0) { set_error("negative step count"); return CLB_EINVAL; }
    CLB_HIP(hipSetDevice(h->device));
    return step_any(h, n);
}

extern "C" int clb3d_moments(clb3d_lattice* h, double* rho, double* u, double* T)
{
    clear_error();
    if (!h) { set_error("lattice is NULL"); return CLB_EINVAL; }
    CLB_HIP(hipSetDevice(h->device));
    int rc = moments_any(h);
    if (rc) return rc;
    const long long n = nodes3(h->desc);
    const size_t b = size_t(n) * sizeof(double);
    if (rho) CLB_HIP(hipMemcpyAsync(rho, h->d_fields, b, hipMemcpyDeviceToHost, h->stream));
    if (u) CLB_HIP(hipMemcpyAsync(u, h->d_fields + n, 3 * b, hipMemcpyDeviceToHost, h->stream));
    if (T) CLB_HIP(hipMemcpyAsync(T, h->d_fields + 4 * n, b, hipMemcpyDeviceToHost, h->stream));
    CLB_HIP(hipStreamSynchronize(h->stream));
    return CLB_OK;
}

extern "C" int clb3d_diagnostics(clb3d_lattice* h, clb3d_diag* out)
{
    clear_error();
    if (!h || !out) { set_error("NULL argument"); return CLB_EINVAL; }
    CLB_HIP(hipSetDevice(h->device));
    int rc = moments_any(h);
    if (rc) return rc;
    const clb3d_desc& d = h->desc;
    const long long n = nodes3(d), nb = diag_blocks(d);
    hipLaunchKernelGGL(diag3_partial_kernel, dim3(unsigned(nb)), dim3(256), 0, h->stream, h->d_fields, n, d.nx, d.ny, d.nz,
                       int(d.bottom.kind != CLB3D_PERIODIC), d.T0, h->d_part);
    CLB_HIP(hipGetLastError());
    hipLaunchKernelGGL(diag3_final_kernel, dim3(1), dim3(256), 0, h->stream, h->d_part, int(nb), h->d_fields, n, d.nx, d.ny,
                       d.nz, h->d_diag);
    CLB_HIP(hipGetLastError());
    double v[DG + 6];
    CLB_HIP(hipMemcpyAsync(v, h->d_diag, sizeof v, hipMemcpyDeviceToHost, h->stream));
    CLB_HIP(hipStreamSynchronize(h->stream));
    out->mass = v[0];
    out->momentum[0] = v[1];
    out->momentum[1] = v[2];
    out->momentum[2] = v[3];
    out->heat = v[4];
    out->uzT = v[5];
    out->max_speed = v[6];
    for (int p = 0; p < 6; ++p) out->plane_T[p] = v[DG + p];
    out->step = h->steps;
    return CLB_OK;
}

extern "C" int clb3d_time_steps(clb3d_lattice* h, long long n, double* ms)
{
    clear_error();
    if (!h || !ms) { set_error("NULL argument"); return CLB_EINVAL; }
    if (n <= 0) { set_error("step count must be positive"); return CLB_EINVAL; }
    CLB_HIP(hipSetDevice(h->device));
    CLB_HIP(hipEventRecord(h->ev[0], h->stream));
    const int rc = step_any(h, n);
    if (rc) return rc;
    CLB_HIP(hipEventRecord(h->ev[1], h->stream));
    CLB_HIP(hipEventSynchronize(h->ev[1]));
    float t = 0.0f;
    CLB_HIP(hipEventElapsedTime(&t, h->ev[0], h->ev[1]));
    *ms = t;
    return CLB_OK;
}

extern "C" int clb3d_synchronize(clb3d_lattice* h)
{
    clear_error();
    if (!h) { set_error("lattice is NULL"); return CLB_EINVAL; }
    CLB_HIP(hipSetDevice(h->device));
    CLB_HIP(hipStreamSynchronize(h->stream));
    CLB_HIP(hipGetLastError());
    return CLB_OK;
}

// ---------------------------------------------------------------------------------------------
// Checkpoint / resume of a 3D lattice: header (description, parameters, step count) and the
// current population buffer.  Restoring it into a lattice of the same description and stepping on
// gives bitwise the uninterrupted run.

namespace {

constexpr char kCkpt3Magic[8] = {'C', 'L', 'B', '3', 'D', 'C', 'K', 'P'};
constexpr uint32_t kCkpt3Version = 1;

struct Ckpt3Header {
    char magic[8];
    uint32_t version, header_bytes;
    clb3d_desc desc;
    double tau_nu, tau_alpha, g_beta, s_b, s3, s4, s5, s6, lam2, Fv[3];
    long long steps;
    uint64_t pop_bytes;
};

bool same_wall3(const clb3d_wall& a, const clb3d_wall& b) { return a.kind == b.kind && a.ux == b.ux && a.uy == b.uy && a.T == b.T; }
bool same_desc3(const clb3d_desc& a, const clb3d_desc& b)
{
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.precision == b.precision && a.T0 == b.T0 &&
           same_wall3(a.bottom, b.bottom) && same_wall3(a.top, b.top);
}

Ckpt3Header ckpt3_header(const clb3d_lattice* h)
{
    Ckpt3Header H;
    std::memset(&H, 0, sizeof H);
    std::memcpy(H.magic, kCkpt3Magic, sizeof H.magic);
    H.version = kCkpt3Version;
    H.header_bytes = uint32_t(sizeof(Ckpt3Header));
    H.desc = h->desc;
    H.tau_nu = h->tau_nu; H.tau_alpha = h->tau_alpha; H.g_beta = h->g_beta;
    H.s_b = h->s_b; H.s3 = h->s3; H.s4 = h->s4; H.s5 = h->s5; H.s6 = h->s6; H.lam2 = h->lam2;
    for (int i = 0; i < 3; ++i) H.Fv[i] = h->Fv[i];
    H.steps = h->steps;
    H.pop_bytes = h->buf_bytes;
    return H;
}

}  // namespace

extern "C" int clb3d_checkpoint_size(clb3d_lattice* h, size_t* bytes)
{
    clear_error();
    if (!h || !bytes) { set_error("NULL argument"); return CLB_EINVAL; }
    *bytes = sizeof(Ckpt3Header) + h->buf_bytes;
    return CLB_OK;
}

extern "C" int clb3d_checkpoint_save(clb3d_lattice* h, void* host, size_t bytes)
{
    clear_error();
    if (!h || !host) { set_error("NULL argument"); return CLB_EINVAL; }
    const Ckpt3Header H = ckpt3_header(h);
    const size_t need = sizeof H + H.pop_bytes;
    if (bytes < need) { set_error("checkpoint buffer holds %zu bytes, %zu needed", bytes, need); return CLB_EINVAL; }
    CLB_HIP(hipSetDevice(h->device));
    std::memcpy(host, &H, sizeof H);
    CLB_HIP(hipMemcpyAsync(static_cast<char*>(host) + sizeof H, h->buf[h->cur], H.pop_bytes, hipMemcpyDeviceToHost, h->stream));
    CLB_HIP(hipStreamSynchronize(h->stream));
    return CLB_OK;
}

extern "C" int clb3d_checkpoint_load(clb3d_lattice* h, const void* host, size_t bytes)
{
    clear_error();
    if (!h || !host) { set_error("NULL argument"); return CLB_EINVAL; }
    Ckpt3Header H;
    if (bytes < sizeof H) { set_error("checkpoint too short"); return CLB_EINVAL; }
    std::memcpy(&H, host, sizeof H);
    if (std::memcmp(H.magic, kCkpt3Magic, sizeof H.magic) != 0 || H.version != kCkpt3Version ||
        H.header_bytes != sizeof(Ckpt3Header)) {
        set_error("not a checkpoint of this library's 3D lattices (magic, version or header size differ)");
        return CLB_EINVAL;
    }
    if (!same_desc3(H.desc, h->desc)) { set_error("checkpoint was taken on a lattice of another description"); return CLB_EINVAL; }
    if (H.pop_bytes != h->buf_bytes) { set_error("checkpoint sizes do not match the lattice"); return CLB_EINVAL; }
    if (bytes < sizeof H + H.pop_bytes) { set_error("checkpoint truncated"); return CLB_EINVAL; }
    CLB_HIP(hipSetDevice(h->device));
    CLB_HIP(hipMemcpyAsync(h->buf[0], static_cast<const char*>(host) + sizeof H, H.pop_bytes, hipMemcpyHostToDevice, h->stream));
    CLB_HIP(hipStreamSynchronize(h->stream));
    h->tau_nu = H.tau_nu; h->tau_alpha = H.tau_alpha; h->g_beta = H.g_beta;
    h->s_b = H.s_b; h->s3 = H.s3; h->s4 = H.s4; h->s5 = H.s5; h->s6 = H.s6; h->lam2 = H.lam2;
    for (int i = 0; i < 3; ++i) h->Fv[i] = H.Fv[i];
    h->steps = H.steps;
    h->cur = 0;
    return CLB_OK;
}
