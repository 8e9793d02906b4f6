// clb_inplace.h -- in-place streaming (AA pattern): one population buffer instead of two.
//
// Time t even: the post-streaming population f_i(x, t) is at slot i of node x; the step reads the
// node's own 14 slots and writes f*_i(x) to slot opp(i) of the same node.  Time t odd: f_i(x, t)
// = f*_i(x - e_i, t - 1) is at slot opp(i) of node x - e_i; the step reads it there and writes
// f*_i(x) to slot i of node x + e_i, where the next even step expects f_i(x + e_i, t + 1).  In both
// steps a thread reads and writes the same 14 locations and no other thread touches them, so the
// update is race-free in one buffer.  Populations whose source lies outside a wall are not read
// (the wall step replaces them).  A population whose target lies outside a wall stays in slot
// opp(q) of its own node at either parity (for a flow population the wall step's mass balance
// reads it there one step later); that slot is the one the node's unknown population opp(q)
// occupies, which no other node reads or writes.
//
// The wall step needs the post-streaming state of the inner neighbours x_f and x_ff of a wall node
// at the same time step -- values the neighbours' own threads overwrite during that step.  They
// are therefore also kept in a snapshot of the wall-adjacent bands (columns 1, 2, nx-3, nx-2 when
// x has walls; rows 1, 2, ny-3, ny-2 when y has walls), two copies by time parity: while step t
// reads copy t mod 2, the threads that produce the post-collision values streaming into a band
// node write them to copy (t + 1) mod 2.  Values are the stored (rounded) ones, so every node
// update sees bitwise the same inputs as with two-buffer pull streaming.
#pragma once

#include "clb_device.h"

namespace clb {

// opposite direction of Eq. 4's numbering (D2Q5 uses directions 0..4 of the same table)
__host__ __device__ constexpr int opp_of(int i)
{
    return i == 0 ? 0 : i == 1 ? 3 : i == 2 ? 4 : i == 3 ? 1 : i == 4 ? 2 : i == 5 ? 7 : i == 6 ? 8 : i == 7 ? 5 : 6;
}

// Snapshot layout: band b (0 west, 1 east, 2 south, 3 north), depth k (0: next to the wall, 1: one
// further), population slot q (0..13), position j along the wall: ((b * 2 + k) * 14 + q) * len + j,
// len = max(nx, ny).  Population-major, so that neighbouring nodes of a band, which neighbouring
// lanes write and read, are contiguous.  Elements per copy:
// Each copy ends in SNAP_SPARE elements that nothing reads: the target of the snapshot stores of
// populations that leave the domain (a store to a fixed spare address instead of a branch per
// population).
constexpr int SNAP_SPARE = 64;
__host__ __device__ __forceinline__ long long snap_elems(int nx, int ny) { return 8LL * (nx > ny ? nx : ny) * 14 + SNAP_SPARE; }

// Snapshot offset of population 0 of node (x, y) (population q at + q * len), or -1 if the node lies
// in no band.  x-bands are tried first.  xb = false: the lattice keeps no column bands (its x-wall
// nodes take their inner neighbours from the adjacent lanes, node_update_aa_wave), only row bands.
__device__ __forceinline__ long long snap_at(const Geo& G, int x, int y, bool xb = true)
{
    const long long len = G.nx > G.ny ? G.nx : G.ny;
    int b = -1, k = 0, j = 0;
    if (xb && !G.perx && (x == 1 || x == 2)) { b = 0; k = x - 1; j = y; }
    else if (xb && !G.perx && (x == G.nx - 2 || x == G.nx - 3)) { b = 1; k = G.nx - 2 - x; j = y; }
    else if (!G.pery && (y == 1 || y == 2)) { b = 2; k = y - 1; j = x; }
    else if (!G.pery && (y == G.ny - 2 || y == G.ny - 3)) { b = 3; k = G.ny - 2 - y; j = x; }
    if (b < 0) return -1;
    return (b * 2 + k) * 14 * len + j;
}

// snap_at for the wall step's neighbours, which always lie in a band (at least 4 nodes across a
// walled direction); a node outside every band would read band 0's first entry, never out of bounds
__device__ __forceinline__ long long snap_at_checked(const Geo& G, int x, int y, bool xb = true)
{
    const long long o = snap_at(G, x, y, xb);
    return o < 0 ? 0 : o;
}

// Write population slot q of band node (x, y) into every band holding the node (a node can lie in
// an x band and a y band).
template <typename S>
__device__ __forceinline__ void snap_put(S* __restrict__ snap, const Geo& G, int x, int y, int q, S v)
{
    const long long len = G.nx > G.ny ? G.nx : G.ny;
    if (!G.perx && (x == 1 || x == 2)) snap[((0 * 2 + x - 1) * 14 + q) * len + y] = v;
    if (!G.perx && (x == G.nx - 2 || x == G.nx - 3)) snap[((1 * 2 + G.nx - 2 - x) * 14 + q) * len + y] = v;
    if (!G.pery && (y == 1 || y == 2)) snap[((2 * 2 + y - 1) * 14 + q) * len + x] = v;
    if (!G.pery && (y == G.ny - 2 || y == G.ny - 3)) snap[((3 * 2 + G.ny - 2 - y) * 14 + q) * len + x] = v;
}

// The wall step's inner neighbours, read from the snapshot copy of the current time step, and the
// node's own outgoing populations: at either parity f*_k(x) of a direction k that left the domain
// is in slot opp(k) of x itself (the even step writes every f*_k to slot opp(k); the odd step keeps
// the outgoing ones there, a slot no other node reads or writes).
template <typename S>
__device__ __forceinline__ S aa_outgoing(const S* __restrict__ A, const Geo& G, int x, int y, int k)
{
    return A[pop_at(G, x, y) + (k == 1 ? 3 : k == 2 ? 4 : k == 3 ? 1 : k == 4 ? 2 : k == 5 ? 7 : k == 6 ? 8 : k == 7 ? 5 : 6) * CW];
}

template <typename S>
struct SnapSource {
    const S* snap;
    const S* A;
    bool xb = true;   // the lattice keeps column bands
    template <typename Real>
    __device__ __forceinline__ Real outgoing(const Geo& G, int x, int y, const WallGeom& W, int j) const
    {
        return Real(aa_outgoing(A, G, x, y, W.o[j]));
    }
    template <typename Real>
    __device__ __forceinline__ void all(const Geo& G, int x, int y, Real f[9], Real g[5]) const
    {
        const long long len = G.nx > G.ny ? G.nx : G.ny;
        const long long o = snap_at_checked(G, x, y, xb);
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = Real(snap[o + i * len]);
#pragma unroll
        for (int i = 0; i < 5; ++i) g[i] = Real(snap[o + (9 + i) * len]);
    }
    template <typename Real>
    __device__ __forceinline__ void temp(const Geo& G, int x, int y, Real g[5]) const
    {
        const long long len = G.nx > G.ny ? G.nx : G.ny;
        const long long o = snap_at_checked(G, x, y, xb);
#pragma unroll
        for (int i = 0; i < 5; ++i) g[i] = Real(snap[o + (9 + i) * len]);
    }
};

// Neighbour of (x, y) along e (periodic wrap); false if it lies outside a wall.
__device__ __forceinline__ bool step_to(const Geo& G, int x, int y, int ex, int ey, int& qx, int& qy)
{
    qx = x + ex;
    qy = y + ey;
    if (qx < 0 || qx >= G.nx) {
        if (!G.perx) return false;
        qx = qx < 0 ? G.nx - 1 : 0;
    }
    if (qy < 0 || qy >= G.ny) {
        if (!G.pery) return false;
        qy = qy < 0 ? G.ny - 1 : 0;
    }
    return true;
}

// Row bases and column offsets of a node and its neighbours (neighbours beyond a wall are clamped
// onto the edge, as in pull), in the addressing of clb_device.h (B32: 32-bit byte offsets).
template <typename S, bool B32>
struct AANbr {
    Off<S, B32> rm, rc, rp, cm, cc, cp;
};
template <typename S, bool B32>
__device__ __forceinline__ AANbr<S, B32> aa_nbr(const Geo& G, int x, int y)
{
    const int xm = x > 0 ? x - 1 : (G.perx ? G.nx - 1 : 0);
    const int xp = x < G.nx - 1 ? x + 1 : (G.perx ? 0 : G.nx - 1);
    const int ym = y > 0 ? y - 1 : (G.pery ? G.ny - 1 : 0);
    const int yp = y < G.ny - 1 ? y + 1 : (G.pery ? 0 : G.ny - 1);
    return {scale_off<S, B32>((long long)ym * G.row), scale_off<S, B32>((long long)y * G.row),
            scale_off<S, B32>((long long)yp * G.row), scale_off<S, B32>(chunk_col(xm)),
            scale_off<S, B32>(chunk_col(x)), scale_off<S, B32>(chunk_col(xp))};
}
// offset of the node one step along (dx, dy) (each -1, 0 or +1, known at compile time after unrolling)
template <typename S, bool B32>
__device__ __forceinline__ Off<S, B32> aa_at(const AANbr<S, B32>& n, int dx, int dy)
{
    return (dy < 0 ? n.rm : (dy > 0 ? n.rp : n.rc)) + (dx < 0 ? n.cm : (dx > 0 ? n.cp : n.cc));
}

// Post-streaming populations of node (x, y) at a time of parity ODD.  At a wall node the unknown
// ones are read from a clamped neighbour and are meaningless: the wall step replaces them.
template <typename S, typename Real, bool ODD, bool B32 = false>
__device__ __forceinline__ void load_aa(const S* __restrict__ A, const Geo& G, int x, int y, Real f[9], Real g[5])
{
    if (!ODD) {
        const Off<S, B32> o = node_off<S, B32>(G, x, y);
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = Real(slot<B32>(A, i, o));
#pragma unroll
        for (int i = 0; i < 5; ++i) g[i] = Real(slot<B32>(A, 9 + i, o));
        poison_unknown<Real>(G, x, y, f, g);
        return;
    }
    const AANbr<S, B32> n = aa_nbr<S, B32>(G, x, y);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = Real(slot<B32>(A, opp_of(i), aa_at(n, -ex_of(i), -ey_of(i))));
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = Real(slot<B32>(A, 9 + opp_of(i), aa_at(n, -ex_of(i), -ey_of(i))));
    poison_unknown<Real>(G, x, y, f, g);
}

// Store the node's rounded post-collision values v (f* then g*) for the next time step, and copy
// those that stream into a snapshot band node into the next snapshot.
template <typename S, bool ODD, bool NT, bool B32 = false>
__device__ __forceinline__ void store_aa(S* __restrict__ A, S* __restrict__ snext, const Geo& G, int x, int y,
                                         const S v[14], bool xb = true)
{
    if (!ODD) {
        const Off<S, B32> o = node_off<S, B32>(G, x, y);
#pragma unroll
        for (int q = 0; q < 14; ++q) {
            const int k = q < 9 ? opp_of(q) : 9 + opp_of(q - 9);
            if (NT) __builtin_nontemporal_store(v[q], &slot<B32>(A, k, o));
            else slot<B32>(A, k, o) = v[q];
        }
    } else {
        const AANbr<S, B32> n = aa_nbr<S, B32>(G, x, y);
        // targets beyond a wall (wall nodes only): the population is kept in slot opp(q) of the node
        // itself, one address select instead of a branch per population.  For a flow population
        // the wall step's mass balance reads it there; a temperature one lands in the slot of the
        // node's unknown g_opp(i), which no node writes in this step and the wall step replaces.
        const bool okxm = G.perx || x > 0, okxp = G.perx || x < G.nx - 1;
        const bool okym = G.pery || y > 0, okyp = G.pery || y < G.ny - 1;
#pragma unroll
        for (int q = 0; q < 14; ++q) {
            const int i = q < 9 ? q : q - 9;
            const int dx = ex_of(i), dy = ey_of(i);
            const bool ok = (dx < 0 ? okxm : (dx > 0 ? okxp : true)) && (dy < 0 ? okym : (dy > 0 ? okyp : true));
            const int keep = q < 9 ? opp_of(q) : 9 + opp_of(q - 9);
            const Off<S, B32> a = ok ? aa_at(n, dx, dy) + scale_off<S, B32>(q * CW)
                                     : aa_at(n, 0, 0) + scale_off<S, B32>(keep * CW);
            if (NT) __builtin_nontemporal_store(v[q], &slot<B32>(A, 0, a));
            else slot<B32>(A, 0, a) = v[q];
        }
    }
    // only nodes within one step of a band can stream into it
    const bool colb = xb && !G.perx;   // the lattice has column bands
    const bool near = (colb && (x <= 3 || x >= G.nx - 4)) || (!G.pery && (y <= 3 || y >= G.ny - 4));
    if (!near) return;
    // per neighbour offset d = -1, 0, +1: the snapshot base of the column band holding column x + d
    // (or -1) and the position of row y + d along it (or -1 outside a wall), and likewise for rows
    const long long len = G.nx > G.ny ? G.nx : G.ny;
    long long cbase[3], rbase[3];
    int ypos[3], xpos[3];
#pragma unroll
    for (int d = -1; d <= 1; ++d) {
        const int tx = x + d, ty = y + d;
        cbase[d + 1] = !colb ? -1 : (tx == 1 || tx == 2) ? (0 * 2 + tx - 1) * 14 * len
                                  : (tx == G.nx - 2 || tx == G.nx - 3) ? (1 * 2 + G.nx - 2 - tx) * 14 * len : -1;
        rbase[d + 1] = G.pery ? -1 : (ty == 1 || ty == 2) ? (2 * 2 + ty - 1) * 14 * len
                                  : (ty == G.ny - 2 || ty == G.ny - 3) ? (3 * 2 + G.ny - 2 - ty) * 14 * len : -1;
        ypos[d + 1] = ty >= 0 && ty < G.ny ? ty : (G.pery ? (ty < 0 ? G.ny - 1 : 0) : -1);
        xpos[d + 1] = tx >= 0 && tx < G.nx ? tx : (G.perx ? (tx < 0 ? G.nx - 1 : 0) : -1);
    }
    // a node can lie in a column band and a row band: both copies are written.  The populations are
    // grouped by the band they stream into (e_x for column bands, e_y for row bands), one branch per
    // group; within a group a population whose target lies beyond a wall goes to the spare elements.
    const long long spare = 8LL * 14 * len;
    if (colb) {
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if (cbase[e] < 0) continue;
#pragma unroll
            for (int q = 0; q < 14; ++q) {
                const int i = q < 9 ? q : q - 9;
                if (ex_of(i) + 1 != e) continue;
                const int dy = ey_of(i) + 1;
                snext[ypos[dy] >= 0 ? cbase[e] + q * len + ypos[dy] : spare] = v[q];
            }
        }
    }
    if (!G.pery) {
        // Depth 1 of a row band (rows 2 and ny - 3) serves only the second inner neighbour x_ff, of
        // which only the temperature populations are read; with ny >= 5 no lookup of an inner
        // neighbour x_f lands there (rows 1 and ny - 2 are depth 0), so its flow populations are
        // not written.
        const bool g_only_rows = G.ny >= 5;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if (rbase[e] < 0) continue;
            const int ty = y + e - 1;
            if (!(g_only_rows && (ty == 2 || ty == G.ny - 3))) {
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    if (ey_of(q) + 1 != e) continue;
                    const int dx = ex_of(q) + 1;
                    snext[xpos[dx] >= 0 ? rbase[e] + q * len + xpos[dx] : spare] = v[q];
                }
            }
#pragma unroll
            for (int q = 9; q < 14; ++q) {
                if (ey_of(q - 9) + 1 != e) continue;
                const int dx = ex_of(q - 9) + 1;
                snext[xpos[dx] >= 0 ? rbase[e] + q * len + xpos[dx] : spare] = v[q];
            }
        }
    }
}

// The whole in-place update of node (x, y) at a time of parity ODD: the same wall step,
// macroscopic quantities, collisions and storage rounding as node_update.
template <typename S, typename Real, bool DEV, bool ODD, bool NT>
__device__ __forceinline__ void node_update_aa(S* __restrict__ A, const S* __restrict__ snow, S* __restrict__ snext,
                                               const Geo& G, const Par<Real>& P, int x, int y, uint32_t key)
{
    Real f[9], g[5];
    load_aa<S, Real, ODD>(A, G, x, y, f, g);
    if (on_wall(G, x, y)) wall_step_nb<Real, DEV>(SnapSource<S>{snow, A}, G, P, x, y, f, g);
    const Macro<Real, DEV> m = macro<Real, DEV>(f, g, P);
    collide_f<Real, DEV>(f, m, P);
    collide_g<Real, DEV>(g, m, P);
    S v[14];
    round_node<S, Real>(f, g, key, uint32_t(y) * uint32_t(G.nx) + uint32_t(x), v);
    store_aa<S, ODD, NT>(A, snext, G, x, y, v);
}

// DirectSource: the wall step's inputs read straight from the in-place buffer, for kernels that do
// not write it (moments, residual): the inner neighbours' post-streaming populations by load_aa,
// bitwise the values the snapshot holds, so these kernels need no snapshot.
template <typename S, bool ODD>
struct DirectSource {
    const S* A;
    template <typename Real>
    __device__ __forceinline__ Real outgoing(const Geo& G, int x, int y, const WallGeom& W, int j) const
    {
        return Real(aa_outgoing(A, G, x, y, W.o[j]));
    }
    template <typename Real>
    __device__ __forceinline__ void all(const Geo& G, int x, int y, Real f[9], Real g[5]) const
    {
        load_aa<S, Real, ODD>(A, G, x, y, f, g);
    }
    template <typename Real>
    __device__ __forceinline__ void temp(const Geo& G, int x, int y, Real g[5]) const
    {
        Real f[9];
        load_aa<S, Real, ODD>(A, G, x, y, f, g);
    }
};

// XchgSource: an x-wall edge node's inner neighbours x_f = x + (dx, 0) and x_ff = x + (2 dx, 0) from
// the lanes that hold them (got, got2: their post-streaming populations as those lanes loaded them),
// everything else from the snapshot.
template <typename S>
struct XchgSource {
    SnapSource<S> snap;
    bool got, got2;
    const S* nb;    // x_f: f then g
    const S* nb2;   // x_ff: g
    template <typename Real>
    __device__ __forceinline__ Real outgoing(const Geo& G, int x, int y, const WallGeom& W, int j) const
    {
        return snap.template outgoing<Real>(G, x, y, W, j);
    }
    template <typename Real>
    __device__ __forceinline__ void all(const Geo& G, int x, int y, Real f[9], Real g[5]) const
    {
        if (got) {
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = Real(nb[i]);
#pragma unroll
            for (int i = 0; i < 5; ++i) g[i] = Real(nb[9 + i]);
        } else {
            snap.all(G, x, y, f, g);
        }
    }
    template <typename Real>
    __device__ __forceinline__ void temp(const Geo& G, int x, int y, Real g[5]) const
    {
        if (got2) {
#pragma unroll
            for (int i = 0; i < 5; ++i) g[i] = Real(nb2[i]);
        } else {
            snap.temp(G, x, y, g);
        }
    }
};

// node_update_aa for a whole wavefront, every lane taking part (valid: the lane holds node (x, y)):
// same arithmetic and result, but an x-wall edge node whose inner neighbours x_f, x_ff are held by
// the lanes next to it takes their loaded populations through cross-lane moves instead of the
// snapshot.  xb = false: the lattice keeps no column bands, which is correct when every x-wall edge
// node finds both neighbours in its wavefront (the caller's node-to-lane mapping guarantees it).
template <typename S, typename Real, bool DEV, bool ODD, bool NT, bool B32 = false, bool UNIT = false, bool REST = false>
__device__ __forceinline__ void node_update_aa_wave(S* __restrict__ A, const S* __restrict__ snow, S* __restrict__ snext,
                                                    const Geo& G, const Par<Real>& P, int x, int y, bool valid,
                                                    bool xb, uint32_t key)
{
    S raw[14];
    if (valid) load_aa<S, S, ODD, B32>(A, G, x, y, raw, raw + 9);
    const bool xwall = valid && !G.perx && (x == 0 || x == G.nx - 1) && G.nx > 1;
    const bool ywall = !G.pery && (y == 0 || y == G.ny - 1);
    const bool want = xwall && !ywall;   // corners use the diagonal neighbour (row bands)
    const int dx = x == 0 ? 1 : -1;
    const int kind = sel4(G.kind[0], G.kind[1], G.kind[2], G.kind[3], x == 0 ? WEST : EAST);
    const bool want2 = want && kind != K_DIRICHLET;   // x_ff: adiabatic temperature
    bool got = false, got2 = false;
    S nb[14], nb2[5];
    if (__ballot(want) != 0) {   // wavefront-uniform
        const int lane = int(__lane_id());
        const int from = want ? lane + dx : lane;
        const int sx = __shfl(valid ? x : -1, from, 64), sy = __shfl(y, from, 64);
        got = want && sx == x + dx && sy == y;
#pragma unroll
        for (int i = 0; i < 14; ++i) nb[i] = __shfl(raw[i], from, 64);
        if (__ballot(want2) != 0) {
            const int from2 = want2 ? lane + 2 * dx : lane;
            const int sx2 = __shfl(valid ? x : -1, from2, 64), sy2 = __shfl(y, from2, 64);
            got2 = want2 && sx2 == x + 2 * dx && sy2 == y;
#pragma unroll
            for (int i = 0; i < 5; ++i) nb2[i] = __shfl(raw[9 + i], from2, 64);
        }
    }
    if (!valid) return;
    Real f[9], g[5];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = Real(raw[i]);
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = Real(raw[9 + i]);
    if (on_wall(G, x, y))
        wall_step_nb<Real, DEV, REST>(XchgSource<S>{SnapSource<S>{snow, A, xb}, got, got2, nb, nb2}, G, P, x, y, f, g);
    const Macro<Real, DEV> m = macro<Real, DEV>(f, g, P);
    collide_f<Real, DEV, UNIT>(f, m, P);
    collide_g<Real, DEV, UNIT>(g, m, P);
    S v[14];
    round_node<S, Real>(f, g, key, uint32_t(y) * uint32_t(G.nx) + uint32_t(x), v);
    store_aa<S, ODD, NT, B32>(A, snext, G, x, y, v, xb);
}

// One in-place step: TXW x 1 tiles (TXW = 64: one wavefront per workgroup, or 256) handed out XCD
// by XCD, as the two-buffer step kernel.
template <typename S, typename Real, bool DEV, bool ODD, bool NT, int TXW>
__global__ __launch_bounds__(TXW) void step_aa_kernel(S* __restrict__ A, const S* __restrict__ snow,
                                                     S* __restrict__ snext, Geo G, Par<Real> P, int tiles_x,
                                                     int ntiles, uint32_t key)
{
    const int q = int(gridDim.x >> 3);
    const int t = int(blockIdx.x & 7) * q + int(blockIdx.x >> 3);
    if (t >= ntiles) return;
    const int y = t / tiles_x;
    const int x = (t - y * tiles_x) * TXW + int(threadIdx.x);
    if (x >= G.nx) return;
    node_update_aa<S, Real, DEV, ODD, NT>(A, snow, snext, G, P, x, y, key);
}

template <typename S, typename Real, bool DEV, int TXW>
void launch_step_aa_w(bool odd, bool nt, S* a, const S* sn, S* sx, const Geo& G, const Par<Real>& P, uint32_t key,
                      hipStream_t st)
{
    const int tx = (G.nx + TXW - 1) / TXW, ntiles = tx * G.ny;
    const int q = (ntiles + 7) / 8;
    const dim3 grid(8 * q), block(TXW);
    if (odd) {
        if (nt) step_aa_kernel<S, Real, DEV, true, true, TXW><<<grid, block, 0, st>>>(a, sn, sx, G, P, tx, ntiles, key);
        else step_aa_kernel<S, Real, DEV, true, false, TXW><<<grid, block, 0, st>>>(a, sn, sx, G, P, tx, ntiles, key);
    } else {
        if (nt) step_aa_kernel<S, Real, DEV, false, true, TXW><<<grid, block, 0, st>>>(a, sn, sx, G, P, tx, ntiles, key);
        else step_aa_kernel<S, Real, DEV, false, false, TXW><<<grid, block, 0, st>>>(a, sn, sx, G, P, tx, ntiles, key);
    }
}

// txw: workgroup width, 64 or 256 nodes (from the lattice's tile shape); nt: non-temporal stores.
template <typename S, typename Real, bool DEV>
hipError_t launch_step_aa(bool odd, bool nt, int txw, void* A, const void* snow, void* snext, const Geo& G,
                          const Par<Real>& P, uint32_t key, hipStream_t st)
{
    if (txw == 64) launch_step_aa_w<S, Real, DEV, 64>(odd, nt, (S*)A, (const S*)snow, (S*)snext, G, P, key, st);
    else launch_step_aa_w<S, Real, DEV, 256>(odd, nt, (S*)A, (const S*)snow, (S*)snext, G, P, key, st);
    return hipGetLastError();
}

}  // namespace clb
