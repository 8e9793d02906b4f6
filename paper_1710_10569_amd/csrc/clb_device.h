// clb_device.h -- per-node device code of the CLB thermal lattice Boltzmann step for gfx950.
//
// One node update = pull streaming (Eqs. 12, 22 in pull form) -> wall step on wall nodes
// (Sec. 3 boundary conditions) -> macroscopic quantities (Eqs. 3, 13, 23) -> D2Q9 CLB collision
// (Sec. 2.1, Eq. 8) -> D2Q5 CLB collision (Sec. 2.2, Eq. 19) -> store at the node itself.
//
// Storage: chunked structure of arrays.  A row of the lattice is a run of chunks of CW = 64
// consecutive nodes; a chunk holds the 14 populations (f0..f8, then g0..g4) of its nodes as 14 runs
// of 64 values, so population i of node (x, y) is at pop_at(x, y) + i * CW.  A wavefront of 64
// nodes of a chunk then reads and writes one contiguous 14 * 64-value block (and its neighbours'),
// instead of 28 streams 14 planes apart.  The buffer read by a step holds post-collision values of
// the previous step at their source node, so f_i(x, t) = buf_i(x - e_i).
//
// The storage type S (what the buffers hold) and the arithmetic type Real may differ: populations
// are converted on load and rounded once on store.  FP32 storage with FP64 arithmetic rounds
// stochastically (store_node below): round-to-nearest repeats the same rounding error at every
// step once the flow is (nearly) steady, and the slow modes of the steady solve integrate that
// bias into a shift of the fixed point; rounding up or down at random, with probability set by
// the dropped fraction, makes the store unbiased.
//
// Two storage forms share this code through the template flag DEV:
//   DEV = false: buf holds f_i and g_i.
//   DEV = true : buf holds f_i - w_i and g_i - w^T_i T0 (w: D2Q9 rest weights, w^T = (1/2, 1/8 x4)).
//               All moments below are then formed as deviations from the rest state, so no value
//               of order one is ever added to a small one; this is what makes FP32 storage usable.
// The algebra is the same for both: R0 (rest density) and TR (rest temperature) are 1 and T0 for
// DEV, 0 and 0 otherwise; "dr" is rho - R0 and "dT" is T - TR.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace clb {

enum { K_PERIODIC = 0, K_DIRICHLET = 1, K_ADIABATIC = 2 };
enum { WEST = 0, EAST = 1, SOUTH = 2, NORTH = 3 };

// Geometry of one lattice (kernel argument, or an entry of the batch table).
struct Geo {
    int nx, ny;          // nodes
    int row;             // elements per row: ceil(nx / CW) chunks of 14 * CW
    int perx, pery;      // 1 if the x (resp. y) direction is periodic
    int kind[4];         // W, E, S, N
    int perm;            // bit w set: wall w is permeable (its velocity has a normal component)
};

// Chunk width (nodes) and chunk size (elements) of the storage layout.
constexpr int CW = 64, CHUNK = 14 * CW;
// Offset of node x within its row, and of population 0 of node (x, y) in a buffer.
__host__ __device__ __forceinline__ int chunk_col(int x) { return (x >> 6) * CHUNK + (x & (CW - 1)); }
__host__ __device__ __forceinline__ long long pop_at(const Geo& G, int x, int y)
{
    return (long long)y * G.row + chunk_col(x);
}

// Addressing of a buffer.  B32 = false: element offsets in 64 bits.  B32 = true (buffers of less than
// 4 GiB, as batch lattices are): byte offsets in 32 bits, so that a load or store takes the buffer's
// (workgroup-uniform) base from scalar registers and a 32-bit offset per lane, with no 64-bit address
// arithmetic per access.  Off<S, B32> is the offset type; node_off the offset of population 0 of node
// (x, y); slot(p, k, o) the element of population slot k at offset o.
template <bool B32> struct OffT { using type = long long; };
template <> struct OffT<true> { using type = uint32_t; };
template <typename S, bool B32> using Off = typename OffT<B32>::type;

template <typename S, bool B32>
__device__ __forceinline__ Off<S, B32> scale_off(long long elems)
{
    if constexpr (B32) return uint32_t(elems) * uint32_t(sizeof(S));
    else return elems;
}
template <typename S, bool B32>
__device__ __forceinline__ Off<S, B32> node_off(const Geo& G, int x, int y)
{
    if constexpr (B32) return (uint32_t(y) * uint32_t(G.row) + uint32_t(chunk_col(x))) * uint32_t(sizeof(S));
    else return pop_at(G, x, y);
}
template <bool B32, typename S, typename O>
__device__ __forceinline__ S& slot(S* p, int k, O o)
{
    if constexpr (B32) return *reinterpret_cast<S*>(reinterpret_cast<char*>(p) + k * CW * int(sizeof(S)) + o);
    else return p[o + k * CW];
}
template <bool B32, typename S, typename O>
__device__ __forceinline__ const S& slot(const S* p, int k, O o)
{
    if constexpr (B32) return *reinterpret_cast<const S*>(reinterpret_cast<const char*>(p) + k * CW * int(sizeof(S)) + o);
    else return p[o + k * CW];
}

// Per-lattice physical parameters in the arithmetic type.
template <typename Real>
struct Par {
    Real om_nu, om_b, om_3, om_4;   // 1 - s for s_nu, s_b, s3, s4
    Real c3;                        // (1 - s3/2) / 3: forcing weight of k~21, k~12 (Eq. 11)
    Real om_l1, om_l2;              // 1 - lambda1, 1 - lambda2
    Real g_beta, Fvx, Fvy;          // Eq. 3
    Real Toff;                      // TR - T0, so that T - T0 = dT + Toff
    Real TR;                        // rest temperature of the storage form
    Real uw[4][2];                  // wall velocities, W E S N
    Real dTw[4];                    // wall temperatures minus TR
    Real pux, puy;                  // prescribed velocity (temperature-only mode, Sec. 3.1)
};

template <typename Real> __device__ __forceinline__ Real R0v();
template <> __device__ __forceinline__ float R0v<float>() { return 1.0f; }
template <> __device__ __forceinline__ double R0v<double>() { return 1.0; }

// Select one of four values by a runtime index i in 0..3 without indexing a kernel-argument array
// (which would make the compiler copy the argument block to private memory).  Selecting on the two
// bits of i, rather than comparing i with 0, 1, 2, keeps the compiler from turning the chain into
// a switch, i.e. branches.
template <typename T>
__device__ __forceinline__ T sel4(T v0, T v1, T v2, T v3, int i)
{
    const T lo = (i & 1) ? v1 : v0, hi = (i & 1) ? v3 : v2;
    return (i & 2) ? hi : lo;
}

// ---------------------------------------------------------------------------------------------
// Debug build only (CLB_POISON_UNKNOWN, libclb_poison.so): every population whose streaming source
// lies outside a wall is replaced by NaN as soon as it is loaded, so that a wall step that used an
// unknown population instead of reconstructing it would turn the node's results into NaN.
template <typename Real>
__device__ __forceinline__ void poison_unknown(const Geo& G, int x, int y, Real f[9], Real g[5])
{
#ifdef CLB_POISON_UNKNOWN
    const bool wm = !G.perx && x == 0, wp = !G.perx && x == G.nx - 1;
    const bool sm = !G.pery && y == 0, sp = !G.pery && y == G.ny - 1;
    const Real nan = Real(__builtin_nan(""));
    // direction i is unknown when its source x - e_i lies beyond a wall
    constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const bool unknown = (ex[i] > 0 && wm) || (ex[i] < 0 && wp) || (ey[i] > 0 && sm) || (ey[i] < 0 && sp);
        if (f && unknown) f[i] = nan;
        if (i < 5 && unknown) g[i] = nan;
    }
#else
    (void)G; (void)x; (void)y; (void)f; (void)g;
#endif
}

// Pull: the 14 post-streaming populations of node (x, y).  Periodic directions wrap; in a
// walled direction a source outside the domain is clamped to the edge -- the value read is then
// meaningless and is replaced by the wall step.
template <typename S, typename Real, bool B32 = false>
__device__ __forceinline__ void pull(const S* __restrict__ src, const Geo& G, int x, int y,
                                     Real f[9], Real g[5])
{
    const int xm = x > 0 ? x - 1 : (G.perx ? G.nx - 1 : 0);
    const int xp = x < G.nx - 1 ? x + 1 : (G.perx ? 0 : G.nx - 1);
    const int ym = y > 0 ? y - 1 : (G.pery ? G.ny - 1 : 0);
    const int yp = y < G.ny - 1 ? y + 1 : (G.pery ? 0 : G.ny - 1);
    using O = Off<S, B32>;
    const O rc = scale_off<S, B32>((long long)y * G.row), rm = scale_off<S, B32>((long long)ym * G.row),
            rp = scale_off<S, B32>((long long)yp * G.row);
    const O cc = scale_off<S, B32>(chunk_col(x)), cm = scale_off<S, B32>(chunk_col(xm)), cp = scale_off<S, B32>(chunk_col(xp));
    f[0] = Real(slot<B32>(src, 0, rc + cc));
    f[1] = Real(slot<B32>(src, 1, rc + cm));
    f[2] = Real(slot<B32>(src, 2, rm + cc));
    f[3] = Real(slot<B32>(src, 3, rc + cp));
    f[4] = Real(slot<B32>(src, 4, rp + cc));
    f[5] = Real(slot<B32>(src, 5, rm + cm));
    f[6] = Real(slot<B32>(src, 6, rm + cp));
    f[7] = Real(slot<B32>(src, 7, rp + cp));
    f[8] = Real(slot<B32>(src, 8, rp + cm));
    g[0] = Real(slot<B32>(src, 9, rc + cc));
    g[1] = Real(slot<B32>(src, 10, rc + cm));
    g[2] = Real(slot<B32>(src, 11, rm + cc));
    g[3] = Real(slot<B32>(src, 12, rc + cp));
    g[4] = Real(slot<B32>(src, 13, rp + cc));
    poison_unknown<Real>(G, x, y, f, g);
}

template <typename S, typename Real, bool B32 = false>
__device__ __forceinline__ void pull_g(const S* __restrict__ src, const Geo& G, int x, int y, Real g[5])
{
    const int xm = x > 0 ? x - 1 : (G.perx ? G.nx - 1 : 0);
    const int xp = x < G.nx - 1 ? x + 1 : (G.perx ? 0 : G.nx - 1);
    const int ym = y > 0 ? y - 1 : (G.pery ? G.ny - 1 : 0);
    const int yp = y < G.ny - 1 ? y + 1 : (G.pery ? 0 : G.ny - 1);
    using O = Off<S, B32>;
    const O rc = scale_off<S, B32>((long long)y * G.row), rm = scale_off<S, B32>((long long)ym * G.row),
            rp = scale_off<S, B32>((long long)yp * G.row);
    const O cc = scale_off<S, B32>(chunk_col(x)), cm = scale_off<S, B32>(chunk_col(xm)), cp = scale_off<S, B32>(chunk_col(xp));
    g[0] = Real(slot<B32>(src, 9, rc + cc));
    g[1] = Real(slot<B32>(src, 10, rc + cm));
    g[2] = Real(slot<B32>(src, 11, rm + cc));
    g[3] = Real(slot<B32>(src, 12, rc + cp));
    g[4] = Real(slot<B32>(src, 13, rp + cc));
    poison_unknown<Real>(G, x, y, nullptr, g);
}

// ---------------------------------------------------------------------------------------------
// Macroscopic quantities of a node: T (Eq. 23), F (Eq. 3), rho and u (Eq. 13).
template <typename Real, bool DEV>
struct Macro {
    Real dr, rho, jx, jy, dT, Fx, Fy, ux, uy;
};

template <typename Real, bool DEV>
__device__ __forceinline__ Macro<Real, DEV> macro(const Real f[9], const Real g[5], const Par<Real>& P)
{
    Macro<Real, DEV> m;
    m.dT = (g[0] + g[1]) + (g[2] + g[3]) + g[4];
    m.Fx = P.Fvx;
    m.Fy = P.Fvy + P.g_beta * (m.dT + P.Toff);
    m.dr = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    m.rho = (DEV ? R0v<Real>() : Real(0)) + m.dr;
    m.jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    m.jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const Real inv = Real(1) / m.rho;
    m.ux = (m.jx + Real(0.5) * m.Fx) * inv;
    m.uy = (m.jy + Real(0.5) * m.Fy) * inv;
    return m;
}

// ---------------------------------------------------------------------------------------------
// Wall step.
//
// psi(e, v): the 1D factor of the D2Q9 equilibrium whose central moments are Eq. 9,
// f_i^eq = rho psi(e_ix, v_x) psi(e_iy, v_y), psi(0, v) = 2/3 - v^2, psi(+-1, v) = (1/3 +- v + v^2)/2.
template <typename Real>
__device__ __forceinline__ void psi3(Real v, Real p[3])   // p[0]: e = 0, p[1]: e = +1, p[2]: e = -1
{
    const Real v2 = v * v;
    p[0] = Real(2.0 / 3.0) - v2;
    p[1] = Real(0.5) * (Real(1.0 / 3.0) + v + v2);
    p[2] = Real(0.5) * (Real(1.0 / 3.0) - v + v2);
}

// Difference of the product-form equilibria at two velocities, per unit density, in Eq. 4 order.
template <typename Real>
__device__ __forceinline__ void feq_diff(Real ax, Real ay, Real bx, Real by, Real d[9])
{
    Real pax[3], pay[3], pbx[3], pby[3];
    psi3(ax, pax); psi3(ay, pay); psi3(bx, pbx); psi3(by, pby);
    // direction i -> (index of e_x in psi3, index of e_y in psi3)
    d[0] = pax[0] * pay[0] - pbx[0] * pby[0];
    d[1] = pax[1] * pay[0] - pbx[1] * pby[0];
    d[2] = pax[0] * pay[1] - pbx[0] * pby[1];
    d[3] = pax[2] * pay[0] - pbx[2] * pby[0];
    d[4] = pax[0] * pay[2] - pbx[0] * pby[2];
    d[5] = pax[1] * pay[1] - pbx[1] * pby[1];
    d[6] = pax[2] * pay[1] - pbx[2] * pby[1];
    d[7] = pax[2] * pay[2] - pbx[2] * pby[2];
    d[8] = pax[1] * pay[2] - pbx[1] * pby[2];
}

// Lattice directions of Eq. 4 as compile-time constants.
__host__ __device__ constexpr int ex_of(int i) { return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0); }
__host__ __device__ constexpr int ey_of(int i) { return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0); }

// Force-corrected non-equilibrium bounce-back on an edge node of a straight wall with inward
// normal n = (nx, ny) and tangent t = (ny, -nx) ((t, n) right-handed).  In the wall's frame a
// direction has components (a, b) = (e.t, e.n); the three with b = +1 are unknown and are rebuilt
// so that sum f = rho, sum f e = rho u_w - F/2 (so Eq. 13 returns u_w) and the normal population's
// non-equilibrium part is bounced back:
//   rho = (sum_{b=0} f + 2 sum_{b=-1} f - F_n/2) / (1 - u_n),  D = rho u_n (2/3 - u_t^2),
//   f(0,1) = f(0,-1) + D,
//   f(+-1,1) = f(-+1,-1) -+ (f(1,0) - f(-1,0))/2 +- (rho u_t - F_t/2)/2 + (rho u_n - F_n/2 - D)/2.
// The four normals are numbered 0: (1, 0) (west wall), 1: (-1, 0) (east), 2: (0, 1) (south),
// 3: (0, -1) (north).  zdir<K>(a, b) is the direction with wall-frame components (a, b) for normal
// K, i.e. e = a t + b n; at<A, B>(f, k) gathers f(A, B) for the runtime normal k with one 4-way
// select, so the formula is evaluated once, in the wall frame, with f in registers.
__host__ __device__ constexpr int zdir_of(int ex, int ey)
{
    return ex == 0 ? (ey == 0 ? 0 : (ey == 1 ? 2 : 4))
         : ex == 1 ? (ey == 0 ? 1 : (ey == 1 ? 5 : 8))
                   : (ey == 0 ? 3 : (ey == 1 ? 6 : 7));
}
__host__ __device__ constexpr int znx(int k) { return k == 0 ? 1 : (k == 1 ? -1 : 0); }
__host__ __device__ constexpr int zny(int k) { return k == 2 ? 1 : (k == 3 ? -1 : 0); }
__host__ __device__ constexpr int zdir(int k, int a, int b)
{
    return zdir_of(a * zny(k) + b * znx(k), -a * znx(k) + b * zny(k));
}
template <int A, int B, typename Real>
__device__ __forceinline__ Real at(const Real f[9], int k)
{
    return sel4(f[zdir(0, A, B)], f[zdir(1, A, B)], f[zdir(2, A, B)], f[zdir(3, A, B)], k);
}
// frame component b = e.n of direction i for normal k, and a = e.t
__host__ __device__ constexpr int zb(int k, int i) { return ex_of(i) * znx(k) + ey_of(i) * zny(k); }
__host__ __device__ constexpr int za(int k, int i) { return ex_of(i) * zny(k) - ey_of(i) * znx(k); }

// zou_he: the three unknowns for a given density rho (Zou-He's own density, for which also
// sum f = rho, is the one permeable walls use).
template <typename Real, bool DEV>
__device__ __forceinline__ void zou_he(Real f[9], int nx, int ny, Real uwx, Real uwy, Real Fx, Real Fy, Real rho)
{
    const int k = nx != 0 ? int(nx < 0) : 2 + int(ny < 0);
    const Real tx = Real(ny), ty = Real(-nx);
    const Real un = uwx * Real(nx) + uwy * Real(ny);
    const Real ut = uwx * tx + uwy * ty;
    const Real Fn = Fx * Real(nx) + Fy * Real(ny);
    const Real Ft = Fx * tx + Fy * ty;
    const Real fP0 = at<1, 0>(f, k), fM0 = at<-1, 0>(f, k);
    const Real fZM = at<0, -1>(f, k), fPM = at<1, -1>(f, k), fMM = at<-1, -1>(f, k);
    const Real d0 = fP0 - fM0;
    const Real D = rho * un * (Real(2.0 / 3.0) - ut * ut);
    const Real half_t = Real(0.5) * (rho * ut - Real(0.5) * Ft);
    const Real half_n = Real(0.5) * (rho * un - Real(0.5) * Fn - D);
    const Real nZP = fZM + D;
    const Real nPP = fMM - Real(0.5) * d0 + half_t + half_n;
    const Real nMP = fPM + Real(0.5) * d0 - half_t + half_n;
    // the unknowns (b = +1): per normal a compile-time choice, selected by k
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const Real v0 = zb(0, i) == 1 ? (za(0, i) == 0 ? nZP : (za(0, i) == 1 ? nPP : nMP)) : f[i];
        const Real v1 = zb(1, i) == 1 ? (za(1, i) == 0 ? nZP : (za(1, i) == 1 ? nPP : nMP)) : f[i];
        const Real v2 = zb(2, i) == 1 ? (za(2, i) == 0 ? nZP : (za(2, i) == 1 ? nPP : nMP)) : f[i];
        const Real v3 = zb(3, i) == 1 ? (za(3, i) == 0 ? nZP : (za(3, i) == 1 ? nPP : nMP)) : f[i];
        f[i] = sel4(v0, v1, v2, v3, k);
    }
}

// Corner closure terms for direction (EX, EY) of the product-form equilibrium at velocity v, per unit
// density, formed without cancellation: odd = psi psi_i - psi psi_opp(i), and dev = psi psi_i - w_i
// (w_i = psi psi_i at v = 0).  With psi(e, v) = psi(e, 0) + dpsi(e, v), dpsi(0, v) = -v^2 and
// dpsi(+-1, v) = (+-v + v^2)/2; psi(1, v) - psi(-1, v) = v and psi(1, v) + psi(-1, v) = 1/3 + v^2.
template <int EX, int EY, typename Real>
__device__ __forceinline__ Real feq_odd(Real vx, Real vy)
{
    if constexpr (EY == 0) return Real(EX) * vx * (Real(2.0 / 3.0) - vy * vy);
    else if constexpr (EX == 0) return Real(EY) * vy * (Real(2.0 / 3.0) - vx * vx);
    else return Real(0.5) * (Real(EX) * vx * (Real(1.0 / 3.0) + vy * vy) + Real(EY) * vy * (Real(1.0 / 3.0) + vx * vx));
}
template <int EX, int EY, typename Real>
__device__ __forceinline__ Real feq_dev(Real vx, Real vy)
{
    const Real ax = EX == 0 ? Real(2.0 / 3.0) : Real(1.0 / 6.0), ay = EY == 0 ? Real(2.0 / 3.0) : Real(1.0 / 6.0);
    const Real bx = EX == 0 ? -vx * vx : Real(0.5) * (Real(EX) * vx + vx * vx);
    const Real by = EY == 0 ? -vy * vy : Real(0.5) * (Real(EY) * vy + vy * vy);
    return (ax * by + bx * ay) + bx * by;
}

// Temperature non-equilibrium extrapolation: g_i = g^eq_i(T_b, a) + g_i(x_f) - g^eq_i(T_f, b) with
// a the wall velocity and b the velocity at x_f.  g^eq_i(T, u) = T phi_i(u): phi_0 = 1/2 - |u|^2,
// phi_{1,3} = (1/4 +- u_x + u_x^2)/2, phi_{2,4} = (1/4 +- u_y + u_y^2)/2.  T_b phi(a) - T_f phi(b)
// is formed as (T_b - T_f) phi(a) + T_f (phi(a) - phi(b)) so that no O(1) terms cancel.
template <typename Real>
__device__ __forceinline__ void nee_g(Real g[5], const Real gf[5], Real dTbf, Real Tf, Real ax, Real ay, Real bx, Real by)
{
    const Real pw1 = Real(0.5) * (Real(0.25) + ax + ax * ax), pw3 = Real(0.5) * (Real(0.25) - ax + ax * ax);
    const Real pw2 = Real(0.5) * (Real(0.25) + ay + ay * ay), pw4 = Real(0.5) * (Real(0.25) - ay + ay * ay);
    const Real pw0 = Real(0.5) - (ax * ax + ay * ay);
    const Real d0 = (bx * bx + by * by) - (ax * ax + ay * ay);
    const Real sx = (ax - bx) + (ax * ax - bx * bx), sxm = (bx - ax) + (ax * ax - bx * bx);
    const Real sy = (ay - by) + (ay * ay - by * by), sym = (by - ay) + (ay * ay - by * by);
    g[0] = gf[0] + dTbf * pw0 + Tf * d0;
    g[1] = gf[1] + dTbf * pw1 + Tf * Real(0.5) * sx;
    g[2] = gf[2] + dTbf * pw2 + Tf * Real(0.5) * sy;
    g[3] = gf[3] + dTbf * pw3 + Tf * Real(0.5) * sxm;
    g[4] = gf[4] + dTbf * pw4 + Tf * Real(0.5) * sym;
}

// Wall step at node (x, y), which must lie on a wall.  f, g hold the pulled populations on entry
// (unknown ones meaningless) and the reconstructed ones on exit.
//   1. g: non-equilibrium extrapolation from the inner neighbour x_f (diagonal one at corners):
//      g_i = g_i^eq(T_b, u_w) + g_i(x_f) - g_i^eq(T_f, u_f), T_b = T_w (Dirichlet) or
//      (4 T_f - T_ff)/3 (adiabatic; x_ff the second inner node).
//   2. F at the node from T_b.
//   3. Density rho_b.  On an impermeable wall (u_w.n = 0) and at every corner: the node's mass
//      balance, the known populations plus those the node sent out of the domain the step before
//      (f*_opp(i) for each unknown i), so the node exchanges no mass with the outside; on a
//      permeable wall: Zou-He's own density.
//   4. f: Zou-He's unknowns at rho_b on edges; at corners the unknowns whose opposite is known
//      bounce back its non-equilibrium part, f_i = f_opp(i) + f^eq_i - f^eq_opp(i), and the two along
//      the cut-off diagonal take f^eq_i, all at (rho_b, u_w - F_b/(2 rho_b)), so Eq. 13 returns u_w.
//   5. Impermeable: f_0 = rho_b - sum_{i>0} f_i.
// Corner data: velocity of the west/east wall; temperature of a Dirichlet wall if one meets
// there, the west/east wall's otherwise.
//
// Geometry of a wall node: the walls it lies on, its inner neighbour x_f = x + (dx, dy), the wall
// whose velocity (vw) and temperature (tw, tkind) it takes, the normal k of an edge node or the
// corner c, and the directions o[] of the populations it sent out of the domain the step before
// (o[0..2]; at corners also o[3..4]).
struct WallGeom {
    bool onW, onE, onS, onN, corner, second;   // second: x_ff is read (adiabatic temperature)
    int xw, yw, dx, dy, vw, kx, ky, tw, tkind, k, c;
    int o[5];
};

// Entry i (0..3) of four 4-bit constants: a shift and a mask (a select chain over constants is
// turned into branches by the compiler).
__host__ __device__ constexpr unsigned nib4(int v0, int v1, int v2, int v3)
{
    return unsigned(v0) | (unsigned(v1) << 4) | (unsigned(v2) << 8) | (unsigned(v3) << 12);
}
__device__ __forceinline__ int nib(unsigned table, int i) { return int((table >> (4 * i)) & 15u); }

__device__ __forceinline__ WallGeom wall_geom(const Geo& G, int x, int y)
{
    WallGeom W;
    W.onW = !G.perx && x == 0;
    W.onE = !G.perx && x == G.nx - 1;
    W.onS = !G.pery && y == 0;
    W.onN = !G.pery && y == G.ny - 1;
    W.xw = W.onW ? WEST : (W.onE ? EAST : -1);
    W.yw = W.onS ? SOUTH : (W.onN ? NORTH : -1);
    W.dx = W.onW ? 1 : (W.onE ? -1 : 0);
    W.dy = W.onS ? 1 : (W.onN ? -1 : 0);
    W.corner = W.xw >= 0 && W.yw >= 0;
    W.vw = W.xw >= 0 ? W.xw : W.yw;
    W.kx = W.xw >= 0 ? sel4(G.kind[0], G.kind[1], G.kind[2], G.kind[3], W.xw) : K_PERIODIC;
    W.ky = W.yw >= 0 ? sel4(G.kind[0], G.kind[1], G.kind[2], G.kind[3], W.yw) : K_PERIODIC;
    W.tw = (W.corner && W.kx != K_DIRICHLET && W.ky == K_DIRICHLET) ? W.yw : W.vw;
    W.tkind = W.tw == W.xw ? W.kx : W.ky;
    W.second = W.tkind != K_DIRICHLET;
    W.k = W.dx != 0 ? int(W.dx < 0) : 2 + int(W.dy < 0);   // 0: dx = 1, 1: dx = -1, 2: dy = 1, 3: dy = -1
    W.c = (W.dx > 0 ? 0 : 1) + (W.dy > 0 ? 0 : 2);   // corner: 0 SW, 1 SE, 2 NW, 3 NE
    // edge (inward normal k): the outgoing populations have e.n = -1; corner (inward (dx, dy)): the
    // five with e_x = -dx or e_y = -dy
    const int k = W.k, c = W.c;
    W.o[0] = W.corner ? (W.dx > 0 ? 3 : 1) : nib(nib4(zdir(0, 0, -1), zdir(1, 0, -1), zdir(2, 0, -1), zdir(3, 0, -1)), k);
    W.o[1] = W.corner ? (W.dy > 0 ? 4 : 2) : nib(nib4(zdir(0, 1, -1), zdir(1, 1, -1), zdir(2, 1, -1), zdir(3, 1, -1)), k);
    W.o[2] = nib(W.corner ? nib4(7, 8, 6, 5) : nib4(zdir(0, -1, -1), zdir(1, -1, -1), zdir(2, -1, -1), zdir(3, -1, -1)), W.corner ? c : k);
    W.o[3] = nib(nib4(6, 5, 7, 8), c);
    W.o[4] = nib(nib4(8, 7, 5, 6), c);
    return W;
}

// Sources of the wall step's other inputs.  PullSource: two-buffer streaming; the inner
// neighbours' post-streaming populations by pull from the previous step's buffer, and the node's
// own outgoing populations from its own slots of that buffer (f*_k(x) is stored at x, slot k).
template <typename S>
struct PullSource {
    const S* src;
    template <typename Real>
    __device__ __forceinline__ void all(const Geo& G, int x, int y, Real f[9], Real g[5]) const { pull(src, G, x, y, f, g); }
    template <typename Real>
    __device__ __forceinline__ void temp(const Geo& G, int x, int y, Real g[5]) const { pull_g(src, G, x, y, g); }
    // f*_k(x) of the previous step for the outgoing direction k = W.o[j]
    template <typename Real>
    __device__ __forceinline__ Real outgoing(const Geo& G, int x, int y, const WallGeom& W, int j) const
    {
        return Real(src[pop_at(G, x, y) + W.o[j] * CW]);
    }
};

// REST: every wall of the lattice is at rest (u_w = 0, hence impermeable); the wall velocity is then a
// compile-time zero and the terms it multiplies are not formed (the result is the general form's up
// to the sign of an exact zero).
template <typename Real, bool DEV, bool REST = false, typename NB>
__device__ __forceinline__ void wall_step_nb(const NB& nb, const Geo& G, const Par<Real>& P,
                                             int x, int y, Real f[9], Real g[5])
{
    const WallGeom W = wall_geom(G, x, y);
    const bool onW = W.onW, onE = W.onE, onS = W.onS, onN = W.onN, corner = W.corner;
    const int dx = W.dx, dy = W.dy, vw = W.vw, tw = W.tw, tkind = W.tkind;
    const Real uwx = REST ? Real(0) : sel4(P.uw[0][0], P.uw[1][0], P.uw[2][0], P.uw[3][0], vw);
    const Real uwy = REST ? Real(0) : sel4(P.uw[0][1], P.uw[1][1], P.uw[2][1], P.uw[3][1], vw);

    Real ff[9], gf[5];
    nb.all(G, x + dx, y + dy, ff, gf);
    const Macro<Real, DEV> mf = macro<Real, DEV>(ff, gf, P);

    Real dTb;
    if (tkind == K_DIRICHLET) {
        dTb = sel4(P.dTw[0], P.dTw[1], P.dTw[2], P.dTw[3], tw);
    } else {
        Real gff[5];
        nb.temp(G, x + 2 * dx, y + 2 * dy, gff);
        const Real dTff = (gff[0] + gff[1]) + (gff[2] + gff[3]) + gff[4];
        dTb = (Real(4) * mf.dT - dTff) * Real(1.0 / 3.0);
    }
    nee_g(g, gf, dTb - mf.dT, P.TR + mf.dT, uwx, uwy, mf.ux, mf.uy);
    const Real Fxb = P.Fvx;
    const Real Fyb = P.Fvy + P.g_beta * (dTb + P.Toff);

    // unknown directions: source x - e_i beyond a wall
    bool unk[9];
#pragma unroll
    for (int i = 0; i < 9; ++i)
        unk[i] = (ex_of(i) > 0 && onW) || (ex_of(i) < 0 && onE) || (ey_of(i) > 0 && onS) || (ey_of(i) < 0 && onN);
    const Real R0 = DEV ? Real(1) : Real(0);
    const bool imperm = REST || corner || ((G.perm >> vw) & 1) == 0;
    // edge (inward normal k): the known populations are those with e.n <= 0, the outgoing ones
    // have e.n = -1; corner (inward (dx, dy)): known f_0 and the three populations from inside,
    // (-dx, 0), (0, -dy), (-dx, -dy), and the five with e_x = -dx or e_y = -dy left the domain.
    // Both are formed with selects, without branches, and the node's kind picks one.
    const int k = W.k, c = W.c;
    const Real K0 = (f[0] + at<1, 0>(f, k)) + at<-1, 0>(f, k);
    const Real Km = (at<0, -1>(f, k) + at<1, -1>(f, k)) + at<-1, -1>(f, k);
    const Real un = uwx * Real(dx) + uwy * Real(dy);
    const Real Fn = Fxb * Real(dx) + Fyb * Real(dy);
    const Real dr_zh = (R0 + K0 + Real(2) * Km - Real(0.5) * Fn) / (Real(1) - un) - R0;
    Real out = (nb.template outgoing<Real>(G, x, y, W, 0) + nb.template outgoing<Real>(G, x, y, W, 1)) +
               nb.template outgoing<Real>(G, x, y, W, 2);
    if (corner) out += nb.template outgoing<Real>(G, x, y, W, 3) + nb.template outgoing<Real>(G, x, y, W, 4);
    const Real known_c = (f[0] + (dx > 0 ? f[3] : f[1])) + ((dy > 0 ? f[4] : f[2]) + sel4(f[7], f[8], f[6], f[5], c));
    const Real dr = !imperm ? dr_zh : (corner ? known_c : K0 + Km) + out;   // rho_b - R0
    const Real rho = R0 + dr;

    if (!corner) {
        zou_he<Real, DEV>(f, dx, dy, uwx, uwy, Fxb, Fyb, rho);
    } else {
        const Real ir = Real(1) / rho;
        const Real vx = uwx - Real(0.5) * Fxb * ir, vy = uwy - Real(0.5) * Fyb * ir;
        // one of each opposite pair on the axes is unknown: bounce back the other's
        // non-equilibrium part (the odd parts of directions 3, 4 are those of 1, 2 negated)
        const Real o1 = rho * feq_odd<1, 0>(vx, vy), o2 = rho * feq_odd<0, 1>(vx, vy);
        f[1] = unk[1] ? f[3] + o1 : f[1];
        f[3] = unk[3] ? f[1] - o1 : f[3];
        f[2] = unk[2] ? f[4] + o2 : f[2];
        f[4] = unk[4] ? f[2] - o2 : f[4];
        // diagonals: the cut-off one is (-1, 1)/(1, -1) at the south-west and north-east corners
        // (anti), else (1, 1)/(-1, -1); its two populations take f^eq, the other pair bounces back
        const bool anti = dx == dy;
        const Real sx = anti ? Real(-1) : Real(1);
        // cut-off diagonal (sx, 1) and (-sx, -1): equilibrium deviations from the rest weight 1/36
        const Real ax = Real(1.0 / 6.0), bpx = Real(0.5) * (sx * vx + vx * vx), bmx = Real(0.5) * (-sx * vx + vx * vx);
        const Real bpy = Real(0.5) * (vy + vy * vy), bmy = Real(0.5) * (-vy + vy * vy);
        const Real dpp = (ax * bpy + bpx * ax) + bpx * bpy, dmm = (ax * bmy + bmx * ax) + bmx * bmy;
        const Real cp = dr * (Real(1.0 / 36.0) + dpp) + R0 * dpp;   // direction (sx, 1)
        const Real cm = dr * (Real(1.0 / 36.0) + dmm) + R0 * dmm;   // direction (-sx, -1)
        // bounced diagonal (-sx, 1) and (sx, -1): odd part of (-sx, 1)
        const Real od = rho * Real(0.5) * (-sx * vx * (Real(1.0 / 3.0) + vy * vy) + vy * (Real(1.0 / 3.0) + vx * vx));
        if (anti) {   // cut-off 6 = (-1, 1), 8 = (1, -1); bounced 5 = (1, 1), 7 = (-1, -1)
            f[6] = unk[6] ? cp : f[6];
            f[8] = unk[8] ? cm : f[8];
            f[5] = unk[5] ? f[7] + od : f[5];
            f[7] = unk[7] ? f[5] - od : f[7];
        } else {      // cut-off 5 = (1, 1), 7 = (-1, -1); bounced 6 = (-1, 1), 8 = (1, -1)
            f[5] = unk[5] ? cp : f[5];
            f[7] = unk[7] ? cm : f[7];
            f[6] = unk[6] ? f[8] + od : f[6];
            f[8] = unk[8] ? f[6] - od : f[8];
        }
    }
    // 5. impermeable: f_0 = rho_b - sum_{i>0} f_i.  On an edge Zou-He's unknowns sum to K_m - F_n/2
    //    (u_n = 0), so this is f_0 + (out - K_m) + F_n/2; at a corner the sum is formed directly.
    if (imperm) {
        if (corner) f[0] = dr - ((((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]))));
        else f[0] += (out - Km) + Real(0.5) * Fn;
    }
}

template <typename S, typename Real, bool DEV>
__device__ __forceinline__ void wall_step(const S* __restrict__ src, const Geo& G, const Par<Real>& P,
                                       int x, int y, Real f[9], Real g[5])
{
    wall_step_nb<Real, DEV>(PullSource<S>{src}, G, P, x, y, f, g);
}

__device__ __forceinline__ bool on_wall(const Geo& G, int x, int y)
{
    return (!G.perx && (x == 0 || x == G.nx - 1)) || (!G.pery && (y == 0 || y == G.ny - 1));
}

// Temperature-only wall step (prescribed velocity u_p, Sec. 3.1): the g part of wall_step with
// the velocity u_p at the wall node and at x_f.
template <typename S, typename Real, bool DEV>
__device__ __forceinline__ void wall_step_T(const S* __restrict__ src, const Geo& G, const Par<Real>& P,
                                            int x, int y, Real g[5])
{
    const bool onW = !G.perx && x == 0, onE = !G.perx && x == G.nx - 1;
    const bool onS = !G.pery && y == 0, onN = !G.pery && y == G.ny - 1;
    const int xw = onW ? WEST : (onE ? EAST : -1);
    const int yw = onS ? SOUTH : (onN ? NORTH : -1);
    const int dx = onW ? 1 : (onE ? -1 : 0);
    const int dy = onS ? 1 : (onN ? -1 : 0);
    const bool corner = xw >= 0 && yw >= 0;
    const int vw = xw >= 0 ? xw : yw;
    const int kx = xw >= 0 ? sel4(G.kind[0], G.kind[1], G.kind[2], G.kind[3], xw) : K_PERIODIC;
    const int ky = yw >= 0 ? sel4(G.kind[0], G.kind[1], G.kind[2], G.kind[3], yw) : K_PERIODIC;
    const int tw = (corner && kx != K_DIRICHLET && ky == K_DIRICHLET) ? yw : vw;
    const int tkind = tw == xw ? kx : ky;
    Real gf[5];
    pull_g(src, G, x + dx, y + dy, gf);
    const Real dTf = (gf[0] + gf[1]) + (gf[2] + gf[3]) + gf[4];
    Real dTb;
    if (tkind == K_DIRICHLET) {
        dTb = sel4(P.dTw[0], P.dTw[1], P.dTw[2], P.dTw[3], tw);
    } else {
        Real gff[5];
        pull_g(src, G, x + 2 * dx, y + 2 * dy, gff);
        const Real dTff = (gff[0] + gff[1]) + (gff[2] + gff[3]) + gff[4];
        dTb = (Real(4) * dTf - dTff) * Real(1.0 / 3.0);
    }
    nee_g(g, gf, dTb - dTf, P.TR + dTf, P.pux, P.puy, P.pux, P.puy);
}

// ---------------------------------------------------------------------------------------------
// Collisions.  Inputs: the node's post-wall-step populations (storage form) and its macroscopic
// quantities; outputs overwrite f and g with the post-collision populations (storage form).
//
// D2Q9, Eq. 8.  With Gamma = M f (Eq. 7a) and Gamma~ = N(u) Gamma (Eq. 7b), only the
// non-equilibrium parts n = Gamma~ - Gamma~^eq are relaxed: n* = (I - S) n + (I - S/2) C.  S acts on
// the pair (k~20, k~02) as s_b on their sum and s_nu on their difference, and as s_nu, s3, s3,
// s4 on k~11, k~21, k~12, k~22; the first central moments go from -F/2 to +F/2.  The raw
// post-collision moments are N(-u) Gamma~* (N(u)^-1 = N(-u)), and f* = M^-1 Gamma*.
// UNIT: s_b = s3 = s4 = 1 (the paper's default rates), so the bulk, third- and fourth-order
// non-equilibrium parts relax to zero in one step and need not be formed; the result is the general
// form's (up to the sign of an exact zero).
template <typename Real, bool DEV, bool UNIT = false>
__device__ __forceinline__ void collide_f(Real f[9], const Macro<Real, DEV>& m, const Par<Real>& P)
{
    const Real R0 = DEV ? Real(1) : Real(0);
    const Real third = Real(1.0 / 3.0), ninth = Real(1.0 / 9.0);
    const Real ux = m.ux, uy = m.uy, rho = m.rho, dr = m.dr, jx = m.jx, jy = m.jy;
    // raw moments of the stored populations (Eq. 6 order), relative to the rest state
    const Real m20 = (f[1] + f[3]) + ((f[5] + f[6]) + (f[7] + f[8]));
    const Real m02 = (f[2] + f[4]) + ((f[5] + f[6]) + (f[7] + f[8]));
    const Real m11 = (f[5] - f[6]) + (f[7] - f[8]);
    const Real m21 = (f[5] + f[6]) - (f[7] + f[8]);
    const Real m12 = (f[5] - f[6]) - (f[7] - f[8]);
    const Real m22 = (f[5] + f[6]) + (f[7] + f[8]);
    const Real ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;
    const Real k20 = m20 + R0 * third, k02 = m02 + R0 * third;   // full k20, k02
    // non-equilibrium central moments
    const Real c20 = (m20 - dr * third) - Real(2) * ux * jx + ux2 * rho;
    const Real c02 = (m02 - dr * third) - Real(2) * uy * jy + uy2 * rho;
    const Real c11 = m11 - ux * jy - uy * jx + uxy * rho;
    // relaxation (Eq. 8)
    Real c20s, c02s, c21s, c12s, c22s;
    const Real c11s = P.om_nu * c11;
    if constexpr (UNIT) {
        const Real dif_s = P.om_nu * (c20 - c02);
        c20s = Real(0.5) * dif_s;
        c02s = Real(0.5) * -dif_s;
        c21s = P.c3 * m.Fy;
        c12s = P.c3 * m.Fx;
        c22s = Real(0);
        (void)m21; (void)m12; (void)m22; (void)k20; (void)k02;
    } else {
        const Real c21 = m21 - Real(2) * ux * m11 - uy * k20 + Real(2) * uxy * jx + ux2 * jy - ux2 * uy * rho;
        const Real c12 = m12 - Real(2) * uy * m11 - ux * k02 + Real(2) * uxy * jy + uy2 * jx - ux * uy2 * rho;
        const Real c22 = (m22 - dr * ninth) - Real(2) * ux * m12 - Real(2) * uy * m21 + Real(4) * uxy * m11
                       + uy2 * k20 + ux2 * k02 - Real(2) * ux * uy2 * jx - Real(2) * uy * ux2 * jy + ux2 * uy2 * rho;
        const Real sum_s = P.om_b * (c20 + c02), dif_s = P.om_nu * (c20 - c02);
        c20s = Real(0.5) * (sum_s + dif_s);
        c02s = Real(0.5) * (sum_s - dif_s);
        c21s = P.om_3 * c21 + P.c3 * m.Fy;
        c12s = P.om_3 * c12 + P.c3 * m.Fx;
        c22s = P.om_4 * c22;
    }
    const Real hx = Real(0.5) * m.Fx, hy = Real(0.5) * m.Fy;   // k~10*, k~01*
    // back to raw moments, N(-u) Gamma~* (Gamma~*_20 = rho/3 + c20s, ..., Gamma~*_22 = rho/9 + c22s)
    const Real t20 = rho * third + c20s, t02 = rho * third + c02s;
    const Real K10 = ux * rho + hx, K01 = uy * rho + hy;
    const Real D20 = dr * third + c20s + Real(2) * ux * hx + ux2 * rho;
    const Real D02 = dr * third + c02s + Real(2) * uy * hy + uy2 * rho;
    const Real K11 = c11s + ux * hy + uy * hx + uxy * rho;
    const Real K21 = c21s + Real(2) * ux * c11s + uy * t20 + Real(2) * uxy * hx + ux2 * hy + ux2 * uy * rho;
    const Real K12 = c12s + Real(2) * uy * c11s + ux * t02 + Real(2) * uxy * hy + uy2 * hx + ux * uy2 * rho;
    const Real D22 = dr * ninth + c22s + Real(2) * ux * c12s + Real(2) * uy * c21s + Real(4) * uxy * c11s
                   + uy2 * t20 + ux2 * t02 + Real(2) * ux * uy2 * hx + Real(2) * uy * ux2 * hy + ux2 * uy2 * rho;
    // f* = M^-1 Gamma* (relative to the rest state)
    f[0] = dr - D20 - D02 + D22;
    f[1] = Real(0.5) * (K10 + D20 - K12 - D22);
    f[2] = Real(0.5) * (K01 + D02 - K21 - D22);
    f[3] = Real(0.5) * (-K10 + D20 + K12 - D22);
    f[4] = Real(0.5) * (-K01 + D02 + K21 - D22);
    f[5] = Real(0.25) * (K11 + K21 + K12 + D22);
    f[6] = Real(0.25) * (-K11 + K21 - K12 + D22);
    f[7] = Real(0.25) * (K11 - K21 - K12 + D22);
    f[8] = Real(0.25) * (-K11 - K21 + K12 + D22);
}

// D2Q5, Eq. 19: the first central moments relax with lambda1, the second with lambda2, towards
// Eq. 20's [T, 0, 0, T/4, T/4]; back-transform with N_T(-u) and M_T^-1 (Eq. 21).
// UNIT: lambda2 = 1, the second-order non-equilibrium parts relax to zero and need not be formed.
template <typename Real, bool DEV, bool UNIT = false>
__device__ __forceinline__ void collide_g(Real g[5], const Macro<Real, DEV>& m, const Par<Real>& P)
{
    const Real ux = m.ux, uy = m.uy, dT = m.dT;
    const Real T = P.TR + dT;
    const Real kx = g[1] - g[3], ky = g[2] - g[4];
    const Real m20 = g[1] + g[3], m02 = g[2] + g[4];
    const Real cx = kx - ux * T, cy = ky - uy * T;
    const Real cxs = P.om_l1 * cx, cys = P.om_l1 * cy;
    Real c20s, c02s;
    if constexpr (UNIT) {
        c20s = c02s = Real(0);
        (void)m20; (void)m02;
    } else {
        const Real c20 = (m20 - Real(0.25) * dT) - Real(2) * ux * kx + ux * ux * T;
        const Real c02 = (m02 - Real(0.25) * dT) - Real(2) * uy * ky + uy * uy * T;
        c20s = P.om_l2 * c20;
        c02s = P.om_l2 * c02;
    }
    const Real Kx = cxs + ux * T, Ky = cys + uy * T;
    const Real D20 = Real(0.25) * dT + c20s + Real(2) * ux * cxs + ux * ux * T;
    const Real D02 = Real(0.25) * dT + c02s + Real(2) * uy * cys + uy * uy * T;
    g[0] = dT - D20 - D02;
    g[1] = Real(0.5) * (Kx + D20);
    g[2] = Real(0.5) * (Ky + D02);
    g[3] = Real(0.5) * (-Kx + D20);
    g[4] = Real(0.5) * (-Ky + D02);
}

// ---------------------------------------------------------------------------------------------
// Storage rounding.
// MurmurHash3's 32-bit finalizer (Appleby): a bijective mixer with full avalanche, used as a
// counter-based generator (distinct counters give distinct, well-mixed words).
__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// Marsaglia's xorshift32 with shifts (13, 17, 5): a bijection of the nonzero 32-bit words, so a
// uniform nonzero word stays uniform; full-rate shifts and xors only.
__device__ __forceinline__ uint32_t xorshift32(uint32_t x)
{
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

// Key of the random words of one time step of a lattice (step: number of steps taken before it).
__host__ __device__ __forceinline__ uint32_t step_key(uint32_t step) { return fmix32(step * 0x9e3779b9u + 0x7f4a7c15u); }

// FP64 -> FP32 with stochastic rounding, u a uniform 16-bit word: the 29 mantissa bits FP32 drops
// are offset by a uniform random amount and cut off, so |v| is rounded up with probability
// (dropped part) / (FP32 spacing) to within 2^-17, and down otherwise (carries into the exponent
// are the step to the next binade).  The truncated value has at most 24 significant bits, so the
// conversion to FP32 is exact in FP32's normal range; NaN stays NaN, +-inf stay inf.
__device__ __forceinline__ float round_stochastic(double v, uint32_t u)
{
    uint64_t b = uint64_t(__double_as_longlong(v));
    b += (uint64_t(u & 0xffffu) << 13) | (uint64_t(1) << 12);
    b &= ~((uint64_t(1) << 29) - 1);
    return float(__longlong_as_double((long long)b));
}

// Round the 14 post-collision populations of node `node` (= y * nx + x) to the storage type; for FP32
// storage of FP64 values the node draws one word fmix32(node + key) and six more by xorshift32
// from it; each word's two 16-bit halves round two populations.  The rounding of a node thus
// depends only on (node, step), never on the tile shape or the batch.
template <typename S, typename Real>
__device__ __forceinline__ void round_node(const Real f[9], const Real g[5], uint32_t key, uint32_t node, S v[14])
{
    if constexpr (sizeof(S) == 4 && sizeof(Real) == 8) {
        uint32_t r = fmix32(node + key);
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            if (k > 0) r = xorshift32(r);
            const Real a = 2 * k < 9 ? f[2 * k] : g[2 * k - 9];
            const Real c = 2 * k + 1 < 9 ? f[2 * k + 1] : g[2 * k + 1 - 9];
            v[2 * k] = round_stochastic(a, r);
            v[2 * k + 1] = round_stochastic(c, r >> 16);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) v[i] = S(f[i]);
#pragma unroll
        for (int i = 0; i < 5; ++i) v[9 + i] = S(g[i]);
    }
}

// Round and store them with population 0 at offset o (population i at o + i CW).
template <typename S, typename Real, bool NT, bool B32 = false>
__device__ __forceinline__ void store_node(S* __restrict__ dst, Off<S, B32> o, const Real f[9], const Real g[5],
                                           uint32_t key, uint32_t node)
{
    S v[14];
    round_node<S, Real>(f, g, key, node, v);
#pragma unroll
    for (int i = 0; i < 14; ++i) {
        if (NT) __builtin_nontemporal_store(v[i], &slot<B32>(dst, i, o));
        else slot<B32>(dst, i, o) = v[i];
    }
}

// ---------------------------------------------------------------------------------------------
// The whole node update: pull, wall step (wall nodes only), macroscopic, both collisions, and the
// store of the 14 post-collision populations at the node itself.  NT selects non-temporal stores.
//
// The whole update of node (x, y) of one step; key = step_key(step) (used by FP32 storage of
// FP64 arithmetic only).
template <typename S, typename Real, bool DEV, bool NT, bool UNIT = false>
__device__ __forceinline__ void node_update(const S* __restrict__ src, S* __restrict__ dst, const Geo& G,
                                            const Par<Real>& P, int x, int y, uint32_t key)
{
    Real f[9], g[5];
    pull(src, G, x, y, f, g);
    if (on_wall(G, x, y)) wall_step<S, Real, DEV>(src, G, P, x, y, f, g);
    const Macro<Real, DEV> m = macro<Real, DEV>(f, g, P);
    collide_f<Real, DEV, UNIT>(f, m, P);
    collide_g<Real, DEV, UNIT>(g, m, P);
    store_node<S, Real, NT>(dst, pop_at(G, x, y), f, g, key, uint32_t(y) * uint32_t(G.nx) + uint32_t(x));
}

// ExchangeSource: two-buffer streaming where the wall node's inner neighbour x_f = x + (dx, 0) of a
// wall in x may be held by the next or previous lane of the wavefront: its 14 post-streaming
// populations (in the storage type, exactly the values that lane pulled) come from that lane
// through a cross-lane move (`got`), else from memory as in PullSource.
template <typename S, bool B32>
struct ExchangeSource {
    const S* src;
    bool got;
    const S* nf;   // 14 values: f then g
    template <typename Real>
    __device__ __forceinline__ void all(const Geo& G, int x, int y, Real f[9], Real g[5]) const
    {
        if (got) {
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = Real(nf[i]);
#pragma unroll
            for (int i = 0; i < 5; ++i) g[i] = Real(nf[9 + i]);
        } else {
            pull<S, Real, B32>(src, G, x, y, f, g);
        }
    }
    template <typename Real>
    __device__ __forceinline__ void temp(const Geo& G, int x, int y, Real g[5]) const
    {
        pull_g<S, Real, B32>(src, G, x, y, g);
    }
    template <typename Real>
    __device__ __forceinline__ Real outgoing(const Geo& G, int x, int y, const WallGeom& W, int j) const
    {
        return Real(slot<B32>(src, W.o[j], node_off<S, B32>(G, x, y)));
    }
};

// node_update for a whole wavefront, every lane taking part (valid: the lane holds node (x, y)).
// Same arithmetic and result as node_update; a node on a wall in x whose inner neighbour is
// held by the adjacent lane takes that lane's pulled populations instead of loading them again
// (one cross-lane move per population instead of 14 loads issued for one or two lanes of the
// wavefront).  The adjacent lane's node is checked, so any node-to-lane mapping is correct.
template <typename S, typename Real, bool DEV, bool NT, bool UNIT = false, bool B32 = false, bool REST = false>
__device__ __forceinline__ void node_update_wave(const S* __restrict__ src, S* __restrict__ dst, const Geo& G,
                                                 const Par<Real>& P, int x, int y, bool valid, uint32_t key)
{
    S raw[14];
    if (valid) pull<S, S, B32>(src, G, x, y, raw, raw + 9);
    const bool xwall = valid && !G.perx && (x == 0 || x == G.nx - 1) && G.nx > 1;
    const bool ywall = !G.pery && (y == 0 || y == G.ny - 1);
    const bool want = xwall && !ywall;   // edge nodes of the x walls (corners use the diagonal)
    const int dx = x == 0 ? 1 : -1;
    bool got = false;
    S nb[14];
    if (__ballot(want) != 0) {   // wavefront-uniform
        const int lane = int(__lane_id());
        const int from = want ? lane + dx : lane;
        const int sx = __shfl(valid ? x : -1, from, 64), sy = __shfl(y, from, 64);
        got = want && sx == x + dx && sy == y;
#pragma unroll
        for (int i = 0; i < 14; ++i) nb[i] = __shfl(raw[i], from, 64);
    }
    if (!valid) return;
    Real f[9], g[5];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = Real(raw[i]);
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = Real(raw[9 + i]);
    if (on_wall(G, x, y)) wall_step_nb<Real, DEV, REST>(ExchangeSource<S, B32>{src, got, nb}, G, P, x, y, f, g);
    const Macro<Real, DEV> m = macro<Real, DEV>(f, g, P);
    collide_f<Real, DEV, UNIT>(f, m, P);
    collide_g<Real, DEV, UNIT>(g, m, P);
    store_node<S, Real, NT, B32>(dst, node_off<S, B32>(G, x, y), f, g, key, uint32_t(y) * uint32_t(G.nx) + uint32_t(x));
}

// Two nodes of one column, (x, y0) and (x, y1): both pulls are issued before either update is
// computed, so a thread has 28 loads in flight instead of 14.
template <typename S, typename Real, bool DEV, bool NT>
__device__ __forceinline__ void node_update2(const S* __restrict__ src, S* __restrict__ dst, const Geo& G,
                                             const Par<Real>& P, int x, int y0, int y1, uint32_t key)
{
    Real fa[9], ga[5], fb[9], gb[5];
    pull(src, G, x, y0, fa, ga);
    pull(src, G, x, y1, fb, gb);
    if (on_wall(G, x, y0)) wall_step<S, Real, DEV>(src, G, P, x, y0, fa, ga);
    if (on_wall(G, x, y1)) wall_step<S, Real, DEV>(src, G, P, x, y1, fb, gb);
    {
        const Macro<Real, DEV> m = macro<Real, DEV>(fa, ga, P);
        collide_f<Real, DEV>(fa, m, P);
        collide_g<Real, DEV>(ga, m, P);
        store_node<S, Real, NT>(dst, pop_at(G, x, y0), fa, ga, key, uint32_t(y0) * uint32_t(G.nx) + uint32_t(x));
    }
    {
        const Macro<Real, DEV> m = macro<Real, DEV>(fb, gb, P);
        collide_f<Real, DEV>(fb, m, P);
        collide_g<Real, DEV>(gb, m, P);
        store_node<S, Real, NT>(dst, pop_at(G, x, y1), fb, gb, key, uint32_t(y1) * uint32_t(G.nx) + uint32_t(x));
    }
}

// Temperature-only node update (prescribed velocity u_p, Sec. 3.1): only the D2Q5 equation runs,
// with u = u_p at every node; only the five g populations of a node are read and written.
template <typename S, typename Real, bool DEV, bool NT>
__device__ __forceinline__ void node_update_T(const S* __restrict__ src, S* __restrict__ dst, const Geo& G,
                                              const Par<Real>& P, int x, int y, uint32_t key)
{
    Real g[5];
    pull_g(src, G, x, y, g);
    if (on_wall(G, x, y)) wall_step_T<S, Real, DEV>(src, G, P, x, y, g);
    Macro<Real, DEV> m;
    m.dT = (g[0] + g[1]) + (g[2] + g[3]) + g[4];
    m.ux = P.pux;
    m.uy = P.puy;
    collide_g<Real, DEV>(g, m, P);
    const long long o = pop_at(G, x, y);
    S v[5];
    if constexpr (sizeof(S) == 4 && sizeof(Real) == 8) {
        uint32_t r = fmix32(uint32_t(y) * uint32_t(G.nx) + uint32_t(x) + key);
        const uint32_t r2 = xorshift32(r);
        v[0] = round_stochastic(g[0], r);
        v[1] = round_stochastic(g[1], r >> 16);
        v[2] = round_stochastic(g[2], r2);
        v[3] = round_stochastic(g[3], r2 >> 16);
        v[4] = round_stochastic(g[4], xorshift32(r2));
    } else {
#pragma unroll
        for (int i = 0; i < 5; ++i) v[i] = S(g[i]);
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        if (NT) __builtin_nontemporal_store(v[i], dst + o + (9 + i) * CW);
        else dst[o + (9 + i) * CW] = v[i];
    }
}

}  // namespace clb
