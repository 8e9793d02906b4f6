// clb_inplace.h -- in-place streaming (AA pattern): one population buffer instead of two.
//
// Time t even: the post-streaming population f_i(x, t) is at slot i of node x; the step reads the
// node's own 14 slots and writes f*_i(x) to slot opp(i) of the same node.  Time t odd: f_i(x, t)
// = f*_i(x - e_i, t - 1) is at slot opp(i) of node x - e_i; the step reads it there and writes
// f*_i(x) to slot i of node x + e_i, where the next even step expects f_i(x + e_i, t + 1).  In both
// steps a thread reads and writes the same 14 locations and no other thread touches them, so the
// update is race-free in one buffer.  Populations whose source lies outside a wall are not read
// (the wall step replaces them).  A flow population whose target lies outside a wall stays in slot
// opp(q) of its own node at either parity, where the wall step's mass balance reads it one step
// later; that slot is the one the node's unknown population opp(q) occupies, which no other node
// reads or writes.
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
__host__ __device__ __forceinline__ long long snap_elems(int nx, int ny) { return 8LL * (nx > ny ? nx : ny) * 14; }

// Snapshot offset of population 0 of node (x, y) (population q at + q * len), or -1 if the node lies
// in no band.  x-bands are tried first.
__device__ __forceinline__ long long snap_at(const Geo& G, int x, int y)
{
    const long long len = G.nx > G.ny ? G.nx : G.ny;
    int b = -1, k = 0, j = 0;
    if (!G.perx && (x == 1 || x == 2)) { b = 0; k = x - 1; j = y; }
    else if (!G.perx && (x == G.nx - 2 || x == G.nx - 3)) { b = 1; k = G.nx - 2 - x; j = y; }
    else if (!G.pery && (y == 1 || y == 2)) { b = 2; k = y - 1; j = x; }
    else if (!G.pery && (y == G.ny - 2 || y == G.ny - 3)) { b = 3; k = G.ny - 2 - y; j = x; }
    if (b < 0) return -1;
    return (b * 2 + k) * 14 * len + j;
}

// snap_at for the wall step's neighbours, which always lie in a band (at least 4 nodes across a
// walled direction); a node outside every band would read band 0's first entry, never out of bounds
__device__ __forceinline__ long long snap_at_checked(const Geo& G, int x, int y)
{
    const long long o = snap_at(G, x, y);
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
struct SnapSource {
    const S* snap;
    const S* A;
    template <typename Real>
    __device__ __forceinline__ Real outgoing(const Geo& G, int x, int y, const WallGeom& W, int j) const
    {
        const int k = W.o[j];
        return Real(A[pop_at(G, x, y) + (k == 1 ? 3 : k == 2 ? 4 : k == 3 ? 1 : k == 4 ? 2 : k == 5 ? 7 : k == 6 ? 8 : k == 7 ? 5 : 6) * CW]);
    }
    template <typename Real>
    __device__ __forceinline__ void all(const Geo& G, int x, int y, Real f[9], Real g[5]) const
    {
        const long long len = G.nx > G.ny ? G.nx : G.ny;
        const long long o = snap_at_checked(G, x, y);
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = Real(snap[o + i * len]);
#pragma unroll
        for (int i = 0; i < 5; ++i) g[i] = Real(snap[o + (9 + i) * len]);
    }
    template <typename Real>
    __device__ __forceinline__ void temp(const Geo& G, int x, int y, Real g[5]) const
    {
        const long long len = G.nx > G.ny ? G.nx : G.ny;
        const long long o = snap_at_checked(G, x, y);
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
// onto the edge, as in pull).
struct AANbr {
    long long rm, rc, rp;
    int cm, cc, cp;
};
__device__ __forceinline__ AANbr aa_nbr(const Geo& G, int x, int y)
{
    const int xm = x > 0 ? x - 1 : (G.perx ? G.nx - 1 : 0);
    const int xp = x < G.nx - 1 ? x + 1 : (G.perx ? 0 : G.nx - 1);
    const int ym = y > 0 ? y - 1 : (G.pery ? G.ny - 1 : 0);
    const int yp = y < G.ny - 1 ? y + 1 : (G.pery ? 0 : G.ny - 1);
    return {(long long)ym * G.row, (long long)y * G.row, (long long)yp * G.row, chunk_col(xm), chunk_col(x), chunk_col(xp)};
}
// offset of the node one step along (dx, dy) (each -1, 0 or +1, known at compile time after unrolling)
__device__ __forceinline__ long long aa_at(const AANbr& n, int dx, int dy)
{
    return (dy < 0 ? n.rm : (dy > 0 ? n.rp : n.rc)) + (dx < 0 ? n.cm : (dx > 0 ? n.cp : n.cc));
}

// Post-streaming populations of node (x, y) at a time of parity ODD.  At a wall node the unknown
// ones are read from a clamped neighbour and are meaningless: the wall step replaces them.
template <typename S, typename Real, bool ODD>
__device__ __forceinline__ void load_aa(const S* __restrict__ A, const Geo& G, int x, int y, Real f[9], Real g[5])
{
    if (!ODD) {
        const long long o = pop_at(G, x, y);
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = Real(A[o + i * CW]);
#pragma unroll
        for (int i = 0; i < 5; ++i) g[i] = Real(A[o + (9 + i) * CW]);
        poison_unknown<Real>(G, x, y, f, g);
        return;
    }
    const AANbr n = aa_nbr(G, x, y);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = Real(A[aa_at(n, -ex_of(i), -ey_of(i)) + opp_of(i) * CW]);
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = Real(A[aa_at(n, -ex_of(i), -ey_of(i)) + (9 + opp_of(i)) * CW]);
    poison_unknown<Real>(G, x, y, f, g);
}

// Store the node's rounded post-collision values v (f* then g*) for the next time step, and copy
// those that stream into a snapshot band node into the next snapshot.
template <typename S, bool ODD, bool NT>
__device__ __forceinline__ void store_aa(S* __restrict__ A, S* __restrict__ snext, const Geo& G, int x, int y,
                                         const S v[14])
{
    if (!ODD) {
        const long long o = pop_at(G, x, y);
#pragma unroll
        for (int q = 0; q < 14; ++q) {
            const int slot = q < 9 ? opp_of(q) : 9 + opp_of(q - 9);
            if (NT) __builtin_nontemporal_store(v[q], A + o + slot * CW);
            else A[o + slot * CW] = v[q];
        }
    } else {
        const AANbr n = aa_nbr(G, x, y);
        // targets beyond a wall: a flow population is kept in slot opp(q) of the node itself (the
        // wall step's mass balance reads it there), a temperature one is dropped; only wall nodes
        // have any
        const bool okxm = G.perx || x > 0, okxp = G.perx || x < G.nx - 1;
        const bool okym = G.pery || y > 0, okyp = G.pery || y < G.ny - 1;
#pragma unroll
        for (int q = 0; q < 14; ++q) {
            const int i = q < 9 ? q : q - 9;
            const int dx = ex_of(i), dy = ey_of(i);
            const bool ok = (dx < 0 ? okxm : (dx > 0 ? okxp : true)) && (dy < 0 ? okym : (dy > 0 ? okyp : true));
            if (!ok) {
                if (q < 9) {
                    if (NT) __builtin_nontemporal_store(v[q], A + aa_at(n, 0, 0) + opp_of(q) * CW);
                    else A[aa_at(n, 0, 0) + opp_of(q) * CW] = v[q];
                }
                continue;
            }
            if (NT) __builtin_nontemporal_store(v[q], A + aa_at(n, dx, dy) + q * CW);
            else A[aa_at(n, dx, dy) + q * CW] = v[q];
        }
    }
    // only nodes within one step of a band can stream into it
    const bool near = (!G.perx && (x <= 3 || x >= G.nx - 4)) || (!G.pery && (y <= 3 || y >= G.ny - 4));
    if (!near) return;
    // per neighbour offset d = -1, 0, +1: the snapshot base of the column band holding column x + d
    // (or -1) and the position of row y + d along it (or -1 outside a wall), and likewise for rows
    const long long len = G.nx > G.ny ? G.nx : G.ny;
    long long cbase[3], rbase[3];
    int ypos[3], xpos[3];
#pragma unroll
    for (int d = -1; d <= 1; ++d) {
        const int tx = x + d, ty = y + d;
        cbase[d + 1] = G.perx ? -1 : (tx == 1 || tx == 2) ? (0 * 2 + tx - 1) * 14 * len
                                  : (tx == G.nx - 2 || tx == G.nx - 3) ? (1 * 2 + G.nx - 2 - tx) * 14 * len : -1;
        rbase[d + 1] = G.pery ? -1 : (ty == 1 || ty == 2) ? (2 * 2 + ty - 1) * 14 * len
                                  : (ty == G.ny - 2 || ty == G.ny - 3) ? (3 * 2 + G.ny - 2 - ty) * 14 * len : -1;
        ypos[d + 1] = ty >= 0 && ty < G.ny ? ty : (G.pery ? (ty < 0 ? G.ny - 1 : 0) : -1);
        xpos[d + 1] = tx >= 0 && tx < G.nx ? tx : (G.perx ? (tx < 0 ? G.nx - 1 : 0) : -1);
    }
#pragma unroll
    for (int q = 0; q < 14; ++q) {
        const int i = q < 9 ? q : q - 9;
        const int dx = ex_of(i) + 1, dy = ey_of(i) + 1;
        // a node can lie in a column band and a row band: both copies are written
        if (cbase[dx] >= 0 && ypos[dy] >= 0) snext[cbase[dx] + q * len + ypos[dy]] = v[q];
        if (rbase[dy] >= 0 && xpos[dx] >= 0) snext[rbase[dy] + q * len + xpos[dx]] = v[q];
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
