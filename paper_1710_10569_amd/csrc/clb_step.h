// clb_step.h -- the tiled step kernel and its launch shapes.
//
// A workgroup updates a tile of TXW x (TY * SPT) nodes: TXW consecutive nodes of a row per thread
// row (TXW is a multiple of the 64-lane wavefront, so every wavefront covers one 64-node storage
// chunk and reads and writes 64 consecutive values per population), TY thread rows, and SPT nodes
// per thread stacked TY rows apart.  Tiles are numbered row-major over the lattice and handed to
// workgroups XCD by XCD: the dispatcher places workgroup b on XCD b mod 8, so workgroup b takes
// tile (b mod 8) * q + b / 8 (q = tiles per XCD).  Each XCD then sweeps one contiguous band of
// rows, and the values that two neighbouring tiles share at their edge -- every population with an
// x component is read one node off the chunk -- are fetched once into that XCD's L2 instead of
// once per XCD.
#pragma once

#include "clb_device.h"

namespace clb {

// tx x ty threads, spt nodes per thread (ty rows apart), nt: non-temporal stores, wpe: minimum
// waves per SIMD the register allocation must allow (0: compiler's choice); spt = 2 variants pull
// both nodes' 28 values before computing either, to double the loads in flight per thread.
struct TileShape { int tx, ty, spt, nt, wpe; };

// The compiled shapes (the autotuner chooses among them).  11-13 are one-wavefront workgroups (one
// 64-node chunk of a row each): the finest dispatch granularity, which plain streaming copies
// on MI355X favour over 256-thread workgroups.
constexpr int kNumShapes = 14;
__host__ __device__ constexpr TileShape tile_shape(int i)
{
    return i == 0 ? TileShape{64, 4, 1, 0, 0}
         : i == 1 ? TileShape{128, 2, 1, 0, 0}
         : i == 2 ? TileShape{256, 1, 1, 0, 0}
         : i == 3 ? TileShape{256, 1, 2, 0, 0}
         : i == 4 ? TileShape{128, 4, 1, 0, 0}
         : i == 5 ? TileShape{256, 2, 1, 0, 0}
         : i == 6 ? TileShape{256, 1, 1, 1, 0}
         : i == 7 ? TileShape{64, 4, 2, 0, 0}
         : i == 8 ? TileShape{256, 1, 1, 0, 8}
         : i == 9 ? TileShape{256, 1, 1, 1, 8}
         : i == 10 ? TileShape{128, 2, 1, 1, 8}
         : i == 11 ? TileShape{64, 1, 1, 1, 0}
         : i == 12 ? TileShape{64, 1, 1, 0, 0}
                   : TileShape{64, 1, 1, 1, 8};
}

inline int tiles_x_of(const Geo& G, const TileShape& s) { return (G.nx + s.tx - 1) / s.tx; }
inline int tiles_y_of(const Geo& G, const TileShape& s) { return (G.ny + s.ty * s.spt - 1) / (s.ty * s.spt); }

template <typename S, typename Real, bool DEV, int TXW, int TY, int SPT, bool NT, int WPE>
__global__ __launch_bounds__(TXW * TY, WPE) void step_tile_kernel(const S* __restrict__ src, S* __restrict__ dst,
                                                                 Geo G, Par<Real> P, int tiles_x, int ntiles,
                                                                 uint32_t key)
{
    const int q = int(gridDim.x >> 3);
    const int t = int(blockIdx.x & 7) * q + int(blockIdx.x >> 3);
    if (t >= ntiles) return;
    const int tyi = t / tiles_x, txi = t - tyi * tiles_x;
    const int x = txi * TXW + int(threadIdx.x % TXW);
    const int y0 = tyi * (TY * SPT) + int(threadIdx.x / TXW);
    if (x >= G.nx) return;
    if (SPT == 1) {
        if (y0 < G.ny) node_update<S, Real, DEV, NT>(src, dst, G, P, x, y0, key);
    } else {
        const int y1 = y0 + TY;
        if (y1 < G.ny) node_update2<S, Real, DEV, NT>(src, dst, G, P, x, y0, y1, key);
        else if (y0 < G.ny) node_update<S, Real, DEV, NT>(src, dst, G, P, x, y0, key);
    }
}

// Enqueue one step from src into dst with shape SH; key = step_key(number of steps taken before).
template <typename S, typename Real, bool DEV, int SH>
hipError_t launch_step_shape(const void* src, void* dst, const Geo& G, const Par<Real>& P, uint32_t key, hipStream_t st)
{
    constexpr TileShape sh = tile_shape(SH);
    const int tx = tiles_x_of(G, sh), ntiles = tx * tiles_y_of(G, sh);
    const int q = (ntiles + 7) / 8;
    step_tile_kernel<S, Real, DEV, sh.tx, sh.ty, sh.spt, sh.nt != 0, (sh.wpe > 0 ? sh.wpe : 1)><<<dim3(8 * q), dim3(sh.tx * sh.ty), 0, st>>>(
        (const S*)src, (S*)dst, G, P, tx, ntiles, key);
    return hipGetLastError();
}

template <typename S, typename Real, bool DEV>
hipError_t launch_step_any(int shape, const void* src, void* dst, const Geo& G, const Par<Real>& P, uint32_t key,
                           hipStream_t st)
{
    switch (shape) {
    case 0: return launch_step_shape<S, Real, DEV, 0>(src, dst, G, P, key, st);
    case 1: return launch_step_shape<S, Real, DEV, 1>(src, dst, G, P, key, st);
    case 2: return launch_step_shape<S, Real, DEV, 2>(src, dst, G, P, key, st);
    case 3: return launch_step_shape<S, Real, DEV, 3>(src, dst, G, P, key, st);
    case 4: return launch_step_shape<S, Real, DEV, 4>(src, dst, G, P, key, st);
    case 5: return launch_step_shape<S, Real, DEV, 5>(src, dst, G, P, key, st);
    case 6: return launch_step_shape<S, Real, DEV, 6>(src, dst, G, P, key, st);
    case 7: return launch_step_shape<S, Real, DEV, 7>(src, dst, G, P, key, st);
    case 8: return launch_step_shape<S, Real, DEV, 8>(src, dst, G, P, key, st);
    case 9: return launch_step_shape<S, Real, DEV, 9>(src, dst, G, P, key, st);
    case 10: return launch_step_shape<S, Real, DEV, 10>(src, dst, G, P, key, st);
    case 11: return launch_step_shape<S, Real, DEV, 11>(src, dst, G, P, key, st);
    case 12: return launch_step_shape<S, Real, DEV, 12>(src, dst, G, P, key, st);
    default: return launch_step_shape<S, Real, DEV, 13>(src, dst, G, P, key, st);
    }
}

// Temperature-only step (prescribed velocity): 256 x 1 tiles in the same XCD order, the five g
// populations read and written per node.
template <typename S, typename Real, bool DEV>
__global__ __launch_bounds__(256) void step_T_kernel(const S* __restrict__ src, S* __restrict__ dst, Geo G,
                                                    Par<Real> P, int tiles_x, int ntiles, uint32_t key)
{
    const int q = int(gridDim.x >> 3);
    const int t = int(blockIdx.x & 7) * q + int(blockIdx.x >> 3);
    if (t >= ntiles) return;
    const int y = t / tiles_x;
    const int x = (t - y * tiles_x) * 256 + int(threadIdx.x);
    if (x >= G.nx) return;
    node_update_T<S, Real, DEV, false>(src, dst, G, P, x, y, key);
}

template <typename S, typename Real, bool DEV>
hipError_t launch_step_T(const void* src, void* dst, const Geo& G, const Par<Real>& P, uint32_t key, hipStream_t st)
{
    const int tx = (G.nx + 255) / 256, ntiles = tx * G.ny;
    const int q = (ntiles + 7) / 8;
    step_T_kernel<S, Real, DEV><<<dim3(8 * q), dim3(256), 0, st>>>((const S*)src, (S*)dst, G, P, tx, ntiles, key);
    return hipGetLastError();
}

}  // namespace clb
