// clb_batch.hip -- many lattices of uneven size resident in one HBM pool, advanced together.
//
// Memory: one pool (allocated by the library or handed in, e.g. a torch tensor) is carved by a
// first-fit free list into per-lattice regions: two population buffers (rows of 64-node chunks
// of 14 populations, on 256-byte boundaries) and an FP64 snapshot of (u_x, u_y, T) for the
// residual test.  Admission is
// that allocation succeeding inside the budget.
//
// Device tables: one entry per slot (geometry, buffer offsets, current buffer, tile width, and the
// lattice's parameters in the arithmetic type), and a tile list ordered by slot and, within a
// lattice, row-major.  Every tile is 256 threads: row tiles of 64 x 4, 128 x 2 or 256 x 1 nodes, or
// eight 32-node runs of wrapped rows, chosen per lattice (the autotuner picks the mapping per size
// class).
//
// Step schedules, all running the same per-node update (node_update), so a lattice's result does
// not depend on the schedule or on the other lattices:
//   grouped     one launch per time step over every tile of every lattice, tiles handed to XCDs in
//               contiguous bands (as in the single-lattice kernel);
//   each        one launch per lattice per time step (the schedule a one-lattice-at-a-time caller
//               would use);
//   persistent  when at least kResidentMinCount lattices of at most kResidentMaxNodes nodes are
//               resident (one per CU or more), each of them is owned by one workgroup of
//               1024 threads that runs all the steps of the call inside one launch, with a
//               workgroup barrier between steps (all its waves share one CU and its L1, so no
//               cross-workgroup synchronisation or agent-scope cache maintenance is needed, and a
//               small lattice's two buffers stay in that XCD's L2); larger lattices take the grouped
//               launches, on the batch's stream, while the resident kernel runs on a second stream.
//               (Measured on MI355X, FP32-SR cavities: 512 lattices of 32^2 run 2x faster resident
//               than grouped, 256 of 64^2 13 % faster, 128^2 lattices 13 % slower; fewer small
//               lattices than CUs leave CUs idle, and then grouped launches are faster.)
#include "clb_internal.h"
#include "clb_aux.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <vector>

namespace clb {

struct BatchLat {
    Geo G;
    long long off[2];   // element offsets of the two population buffers in the pool
    long long snap;     // byte offset of the FP64 (u_x, u_y, T) snapshot in the pool
    int cur;            // buffer holding the current post-collision state
    uint32_t step;      // steps taken before the current call (low 32 bits): the rounding key base
    int tw_log2;        // tile width 1 << tw_log2 (6, 7 or 8), tile rows 256 >> tw_log2; 0: wrapped rows
    int tiles_x, ntiles;
    int halves;         // 32-node runs per row, ceil(nx / 32) (wrapped rows)
    double inv_halves;  // 1 / halves
    int aa;             // 1: in-place lattice (off[0] only, snapshot copies at sn[0], sn[1])
    int xbands;         // in place: the snapshot keeps the column bands (aa_column_bands)
    long long sn[2];    // element offsets of the in-place snapshot copies
};

template <typename Real>
struct BatchEntry {
    BatchLat L;
    Par<Real> P;
};

struct TileRef { int lat, tile; };

constexpr int BNT = 256;

// Node of thread `lane` of work item `tile` of a lattice; false if none.  Row tiles: width
// 1 << tw_log2, BNT >> tw_log2 rows.  Wrapped rows (tw_log2 = 0): the rows are cut into runs of 32
// nodes starting at x = 0, 32, 64, ... (the halves of the storage chunks; a row's last run may be
// short), all runs of all rows are numbered in row-major order, and each half-wavefront takes one
// run, the sequence shifted by one run: tile t takes runs 8t - 1 .. 8t + 6.  The last run of a row
// and the first of the next thus share one wavefront, and only that wavefront takes the wall
// branch of the two x-wall nodes (in row tiles each of them costs its own wavefront); every
// half-wavefront reads and writes one aligned 32-node half of a chunk, i.e. whole cache lines, for
// any nx.  Where nx is a multiple of 32 this is node k = 256 t + lane - 32 in row-major order.
__device__ __forceinline__ bool batch_node(const BatchLat& L, int tile, int lane, int& x, int& y)
{
    if (L.tw_log2 == 0) {
        const int q = tile * (BNT / 32) + (lane >> 5) - 1;   // run of this half-wavefront
        if (q < 0 || q >= L.halves * L.G.ny) return false;
        y = int(double(q) * L.inv_halves);
        int h = q - y * L.halves;
        if (h < 0) { --y; h += L.halves; }
        else if (h >= L.halves) { ++y; h -= L.halves; }
        x = (h << 5) + (lane & 31);
        return x < L.G.nx;
    }
    const int tyi = tile / L.tiles_x, txi = tile - tyi * L.tiles_x;
    x = (txi << L.tw_log2) + (lane & ((1 << L.tw_log2) - 1));
    y = tyi * (BNT >> L.tw_log2) + (lane >> L.tw_log2);
    return x < L.G.nx && y < L.G.ny;
}

// AA: the batch holds in-place lattices (a separate instantiation, so that batches without them keep
// the register budget of the two-buffer update alone).  UNIT: every lattice has s_b = s3 = s4 =
// lambda2 = 1 (the collision skips the moments those rates send to equilibrium).  REST (with UNIT):
// every wall of every lattice is at rest, so the wall step takes u_w = 0 at compile time.
template <typename S, typename Real, bool DEV, bool NT, bool AA, bool UNIT = false, bool REST = false>
__device__ __forceinline__ void batch_tile(S* __restrict__ pool, const BatchEntry<Real>& E, int tile, int s)
{
    int x = 0, y = 0;
    const bool valid = batch_node(E.L, tile, int(threadIdx.x), x, y);
    if (!AA || !E.L.aa) {
        // select the buffers without indexing off[] by a runtime value (which would put the entry
        // in private memory); every lane of the wavefront takes part (node_update_wave)
        const bool c = (E.L.cur ^ (s & 1)) != 0;
        const long long o_src = c ? E.L.off[1] : E.L.off[0];
        const long long o_dst = c ? E.L.off[0] : E.L.off[1];
        node_update_wave<S, Real, DEV, NT, UNIT, true, REST>(pool + o_src, pool + o_dst, E.L.G, E.P, x, y, valid,
                                                             step_key(E.L.step + uint32_t(s)));
        return;
    }
    // the lattice's own step count sets the in-place form and the snapshot copies
    const uint32_t t = E.L.step + uint32_t(s);
    const bool odd = (t & 1u) != 0;
    S* A = pool + E.L.off[0];
    const S* snow = pool + (odd ? E.L.sn[1] : E.L.sn[0]);
    S* snext = pool + (odd ? E.L.sn[0] : E.L.sn[1]);
    const bool xb = E.L.xbands != 0;
    if (odd) node_update_aa_wave<S, Real, DEV, true, NT, true, UNIT, REST>(A, snow, snext, E.L.G, E.P, x, y, valid, xb, step_key(t));
    else node_update_aa_wave<S, Real, DEV, false, NT, true, UNIT, REST>(A, snow, snext, E.L.G, E.P, x, y, valid, xb, step_key(t));
}

template <typename S, typename Real, bool DEV, bool NT, bool AA, bool UNIT = false, bool REST = false>
__global__ __launch_bounds__(BNT) void batch_step_kernel(S* __restrict__ pool, const BatchEntry<Real>* __restrict__ lats,
                                                       const TileRef* __restrict__ tiles, int tile_base, int ntiles,
                                                       int s)
{
    const int q = int(gridDim.x >> 3);
    const int t = int(blockIdx.x & 7) * q + int(blockIdx.x >> 3);
    if (t >= ntiles) return;
    const TileRef r = tiles[tile_base + t];
    const BatchEntry<Real> E = lats[r.lat];
    batch_tile<S, Real, DEV, NT, AA, UNIT, REST>(pool, E, r.tile, s);
}

// After a call of nsteps steps: flip the current-buffer index of every listed slot if nsteps is
// odd, and advance its step count.
template <typename Real>
__global__ void batch_advance_kernel(BatchEntry<Real>* lats, const int* slots, int n, int nsteps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        lats[slots[i]].L.cur ^= nsteps & 1;
        lats[slots[i]].L.step += uint32_t(nsteps);
    }
}

__global__ void batch_zero_kernel(unsigned* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Workgroup-resident steps: workgroup i owns lattice slots[i] and advances it nsteps steps.
constexpr int RNT = 1024;
constexpr long long kResidentMaxNodes = 64 * 64;
constexpr int kResidentMinCount = 256;

template <typename S, typename Real, bool DEV, bool AA>
__global__ __launch_bounds__(RNT) void batch_resident_kernel(S* __restrict__ pool, const BatchEntry<Real>* __restrict__ lats,
                                                           const int* __restrict__ slots, int nslots, int nsteps)
{
    if (int(blockIdx.x) >= nslots) return;
    const BatchEntry<Real> E = lats[slots[blockIdx.x]];
    const int nx = E.L.G.nx, n = E.L.G.nx * E.L.G.ny;
    for (int s = 0; s < nsteps; ++s) {
        if (AA && E.L.aa) {
            const uint32_t t = E.L.step + uint32_t(s);
            const bool odd = (t & 1u) != 0;
            S* A = pool + E.L.off[0];
            const S* snow = pool + (odd ? E.L.sn[1] : E.L.sn[0]);
            S* snext = pool + (odd ? E.L.sn[0] : E.L.sn[1]);
            for (int k = int(threadIdx.x); k < n; k += RNT) {
                const int y = k / nx, x = k - y * nx;
                if (odd) node_update_aa<S, Real, DEV, true, false>(A, snow, snext, E.L.G, E.P, x, y, step_key(t));
                else node_update_aa<S, Real, DEV, false, false>(A, snow, snext, E.L.G, E.P, x, y, step_key(t));
            }
            __syncthreads();
            continue;
        }
        const bool c = (E.L.cur ^ (s & 1)) != 0;
        const S* src = pool + (c ? E.L.off[1] : E.L.off[0]);
        S* dst = pool + (c ? E.L.off[0] : E.L.off[1]);
        for (int k = int(threadIdx.x); k < n; k += RNT) {
            const int y = k / nx, x = k - y * nx;
            node_update<S, Real, DEV, false>(src, dst, E.L.G, E.P, x, y, step_key(E.L.step + uint32_t(s)));
        }
        // every store of step s is visible to every load of step s + 1: all waves of the workgroup
        // are on one CU and share its L1
        __syncthreads();
    }
}

// Residual of every resident lattice in one launch: at each node the moments of the current step
// (pull, wall step, macroscopic, as in clb_moments) are compared with the lattice's FP64 snapshot,
// which is then overwritten; per lattice the maxima of |u_x - u_x'|, |u_y - u_y'| (together),
// |T - T'| and a non-finite flag are combined with atomic max on their IEEE bit patterns (all
// values are non-negative, so the integer order is the numeric order and the result does not
// depend on the order of the updates).
template <typename S, typename Real, bool DEV, bool AA>
__global__ __launch_bounds__(BNT) void batch_residual_kernel(S* __restrict__ pool, const BatchEntry<Real>* __restrict__ lats,
                                                           const TileRef* __restrict__ tiles, int ntiles,
                                                           unsigned long long* __restrict__ res)
{
    const int q = int(gridDim.x >> 3);
    const int t = int(blockIdx.x & 7) * q + int(blockIdx.x >> 3);
    if (t >= ntiles) return;   // uniform over the workgroup
    const TileRef r = tiles[t];
    const BatchEntry<Real> E = lats[r.lat];
    int x, y;
    double du = 0.0, dT = 0.0, bad = 0.0;
    if (batch_node(E.L, r.tile, int(threadIdx.x), x, y)) {
        Real f[9], g[5];
        if (AA && E.L.aa) {
            const bool odd = (E.L.step & 1u) != 0;
            const S* A = pool + E.L.off[0];
            if (odd) load_aa<S, Real, true>(A, E.L.G, x, y, f, g);
            else load_aa<S, Real, false>(A, E.L.G, x, y, f, g);
            if (on_wall(E.L.G, x, y)) {
                if (odd) wall_step_nb<Real, DEV>(DirectSource<S, true>{A}, E.L.G, E.P, x, y, f, g);
                else wall_step_nb<Real, DEV>(DirectSource<S, false>{A}, E.L.G, E.P, x, y, f, g);
            }
        } else {
            const S* src = pool + (E.L.cur ? E.L.off[1] : E.L.off[0]);
            pull(src, E.L.G, x, y, f, g);
            if (on_wall(E.L.G, x, y)) wall_step<S, Real, DEV>(src, E.L.G, E.P, x, y, f, g);
        }
        const Macro<Real, DEV> m = macro<Real, DEV>(f, g, E.P);
        const double ux = double(m.ux), uy = double(m.uy), T = double(E.P.TR) + double(m.dT);
        double* snap = reinterpret_cast<double*>(reinterpret_cast<char*>(pool) + E.L.snap);
        const long long n = (long long)E.L.G.nx * E.L.G.ny, k = (long long)y * E.L.G.nx + x;
        du = fmax(fabs(ux - snap[k]), fabs(uy - snap[n + k]));
        dT = fabs(T - snap[2 * n + k]);
        bad = (__builtin_isfinite(double(m.rho)) && __builtin_isfinite(ux) && __builtin_isfinite(uy) &&
               __builtin_isfinite(T)) ? 0.0 : 1.0;
        snap[k] = ux;
        snap[n + k] = uy;
        snap[2 * n + k] = T;
    }
    for (int o = 32; o > 0; o >>= 1) {
        du = fmax(du, __shfl_xor(du, o, 64));
        dT = fmax(dT, __shfl_xor(dT, o, 64));
        bad = fmax(bad, __shfl_xor(bad, o, 64));
    }
    __shared__ double red[BNT / 64][3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { red[wave][0] = du; red[wave][1] = dT; red[wave][2] = bad; }
    __syncthreads();
    if (threadIdx.x < 3) {
        double v = red[0][threadIdx.x];
        for (int w = 1; w < BNT / 64; ++w) v = fmax(v, red[w][threadIdx.x]);
        atomicMax(res + 3 * r.lat + threadIdx.x, (unsigned long long)__double_as_longlong(v));
    }
}

__global__ void batch_zero64_kernel(unsigned long long* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace clb

using namespace clb;

// ---------------------------------------------------------------------------------------------
// Host side.

namespace {

struct BatchSlot {
    bool used = false;
    clb_desc desc{};
    Params par;
    size_t alloc_off = 0, alloc_bytes = 0;   // byte range in the pool
    long long off[2] = {0, 0};               // element offsets of the population buffers
    size_t snap_off = 0;                     // byte offset of the FP64 snapshot (3 n doubles)
    long long sn[2] = {0, 0};                // in-place lattices: element offsets of the snapshot copies
    int cur = 0;
    long long steps = 0;
    bool has_snap = false;
    int tw_log2 = 8;
};

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Pool bytes of one lattice: two population buffers (in place: one, plus two snapshot copies of
// the wall-adjacent bands) and the FP64 residual snapshot.
size_t slot_bytes(const clb_desc& d, size_t* buf_bytes_out, size_t* band_bytes_out = nullptr)
{
    const size_t eb = elem_bytes(d.precision);
    const size_t buf = align_up(size_t(buffer_elems(d.nx, d.ny)) * eb);
    const size_t band = align_up(size_t(snap_elems(d.nx, d.ny)) * eb);
    const size_t snap = align_up(size_t(3) * d.nx * d.ny * sizeof(double));
    if (buf_bytes_out) *buf_bytes_out = buf;
    if (band_bytes_out) *band_bytes_out = band;
    return d.in_place ? buf + 2 * band + snap : 2 * buf + snap;
}

// Default mapping of a lattice until the autotuner or the caller sets one.  With walls in x: wrapped
// rows, which put the two x-wall ends of consecutive rows into one wavefront (half the wavefronts
// that take the wall branch of row tiles) and keep every access line-aligned for any nx.  Measured
// on the 32 cavities of the served mix (sides 34-864, MI355X): two-buffer SR 41.4 GLUPS wrapped
// against 38.9 with 64-wide rows, FP32 46.2 against 46.5; in place SR 38.1 against 35.7, FP32
// 49.4 against 47.2.  Periodic in x: row tiles about as wide as the lattice.  The autotuner
// cannot time in-place lattices (its timing launches would advance them), so they keep this.
int default_tw_log2(const clb_desc& d)
{
    if (d.west.kind != CLB_PERIODIC) return 0;
    if (d.in_place) return 6;
    return d.nx <= 96 ? 6 : (d.nx <= 192 ? 7 : 8);
}

// Whether an in-place lattice keeps the column bands of its snapshot.  Not needed when every x-wall
// edge node finds its inner neighbours x + dx and x + 2 dx in its own wavefront in the grouped step:
// under wrapped rows (runs of 32 from x = 0) and row tiles (64-node rows per wavefront) the west
// wall sits at a run's first node, and the east wall at position (nx - 1) mod 32 (resp. 64) >= 2
// unless nx mod 32 is 1 or 2; lattices small enough for the workgroup-resident step (whose
// node-to-lane mapping gives no such guarantee) keep them.  Fixed at admission, so the choice holds
// whatever mapping or schedule steps the lattice later.
bool aa_column_bands(const clb_desc& d)
{
    if (!d.in_place || d.west.kind == CLB_PERIODIC) return false;
    const int r = d.nx % 32;
    return d.nx < 4 || r == 1 || r == 2 || (long long)d.nx * d.ny <= kResidentMaxNodes;
}

int size_class(const clb_desc& d)
{
    int c = 0;
    while ((1 << c) < d.nx) ++c;
    int e = 0;
    while ((1 << e) < d.ny) ++e;
    return c * 64 + e;
}

}  // namespace

struct clb_batch {
    int capacity = 0;
    int precision = CLB_FP32_DEV;
    size_t budget = 0;       // pool bytes available to lattices
    size_t used_bytes = 0;
    char* pool = nullptr;
    bool own_pool = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<BatchSlot> slots;
    std::map<size_t, size_t> free_list;   // byte offset -> length
    void* d_lats = nullptr;
    TileRef* d_tiles = nullptr;
    size_t tiles_cap = 0;
    std::vector<TileRef> tiles;
    std::vector<int> first_tile, ntiles;
    int* d_active = nullptr;              // slots in use (for the advance kernel)
    int n_active = 0;
    bool dirty = true;
    hipStream_t side = nullptr;           // second stream for the workgroup-resident kernel
    hipEvent_t fork = nullptr, join = nullptr;
    int* d_small = nullptr;               // slots run by the resident kernel
    std::vector<int> small_slots;
    std::vector<TileRef> tiles_big;       // tiles of the other lattices (grouped launches)
    TileRef* d_tiles_big = nullptr;
    size_t tiles_big_cap = 0;
    double* d_fields = nullptr;
    size_t fields_cap = 0;                // doubles
    double* d_partials = nullptr;
    int partials_cap = 0;
    double* d_diag = nullptr;
    unsigned long long* d_res = nullptr;  // 3 per slot: residual of u, of T, non-finite flag
    hipEvent_t ev[2] = {nullptr, nullptr};
    std::map<int, int> tw_by_class;       // autotuned tile width (log2) per size class
    bool nontemporal = false;
    bool nt_chosen = false;               // store form set by the caller or the autotuner
    bool has_aa = false;                  // some resident lattice streams in place
    bool unit_rates = false;              // every resident lattice has s_b = s3 = s4 = lambda2 = 1
    bool rest_walls = false;              // every wall of every resident lattice is at rest
};

namespace {

int alloc_range(clb_batch* b, size_t bytes, size_t* off)
{
    for (auto it = b->free_list.begin(); it != b->free_list.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t roff = it->first + bytes;
            b->free_list.erase(it);
            if (rest) b->free_list[roff] = rest;
            b->used_bytes += bytes;
            return CLB_OK;
        }
    }
    return CLB_ENOMEM;
}

void free_range(clb_batch* b, size_t off, size_t bytes)
{
    b->used_bytes -= bytes;
    auto it = b->free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != b->free_list.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        b->free_list.erase(nx);
    }
    if (it != b->free_list.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            b->free_list.erase(it);
        }
    }
}

size_t entry_bytes(int precision) { return precision == CLB_FP32_DEV ? sizeof(BatchEntry<float>) : sizeof(BatchEntry<double>); }

template <typename Real>
BatchEntry<Real> make_entry(const BatchSlot& s, int tw_log2)
{
    BatchEntry<Real> E;
    E.L.G = make_geo(s.desc);
    E.L.off[0] = s.off[0];
    E.L.off[1] = s.off[1];
    E.L.snap = (long long)s.snap_off;
    E.L.aa = s.desc.in_place ? 1 : 0;
    E.L.xbands = aa_column_bands(s.desc) ? 1 : 0;
    E.L.sn[0] = s.sn[0];
    E.L.sn[1] = s.sn[1];
    E.L.cur = s.cur;
    E.L.step = uint32_t(s.steps);
    E.L.tw_log2 = tw_log2;
    E.L.halves = (s.desc.nx + 31) / 32;
    E.L.inv_halves = 1.0 / double(E.L.halves);
    if (tw_log2 == 0) {
        // runs -1 .. halves ny - 1, eight per tile
        E.L.tiles_x = 0;
        E.L.ntiles = int(((long long)E.L.halves * s.desc.ny + 1 + BNT / 32 - 1) / (BNT / 32));
    } else {
        const int tw = 1 << tw_log2, th = BNT >> tw_log2;
        E.L.tiles_x = (s.desc.nx + tw - 1) / tw;
        E.L.ntiles = E.L.tiles_x * ((s.desc.ny + th - 1) / th);
    }
    E.P = make_par<Real>(s.desc, s.par);
    return E;
}

// Rebuild and upload the slot table and the tile list (stream-ordered).
int upload_tables(clb_batch* b)
{
    const int cap = b->capacity;
    std::vector<char> host(entry_bytes(b->precision) * cap, 0);
    b->tiles.clear();
    b->first_tile.assign(cap, 0);
    b->ntiles.assign(cap, 0);
    std::vector<int> active;
    size_t resident = 0;
    b->has_aa = false;
    bool all_unit = true, all_rest = true;
    for (int i = 0; i < cap; ++i) {
        BatchSlot& s = b->slots[i];
        if (!s.used) continue;
        active.push_back(i);
        resident += s.alloc_bytes;
        b->has_aa = b->has_aa || s.desc.in_place;
        all_unit = all_unit && s.par.s_b == 1.0 && s.par.s3 == 1.0 && s.par.s4 == 1.0 && s.par.lam2 == 1.0;
        for (const clb_edge* e : {&s.desc.west, &s.desc.east, &s.desc.south, &s.desc.north})
            all_rest = all_rest && (e->kind == CLB_PERIODIC || (e->ux == 0.0 && e->uy == 0.0));
        int nt;
        if (b->precision == CLB_FP32_DEV) {
            BatchEntry<float> E = make_entry<float>(s, s.tw_log2);
            std::memcpy(host.data() + i * sizeof E, &E, sizeof E);
            nt = E.L.ntiles;
        } else {
            BatchEntry<double> E = make_entry<double>(s, s.tw_log2);
            std::memcpy(host.data() + i * sizeof E, &E, sizeof E);
            nt = E.L.ntiles;
        }
        b->first_tile[i] = int(b->tiles.size());
        b->ntiles[i] = nt;
        for (int t = 0; t < nt; ++t) b->tiles.push_back(TileRef{i, t});
    }
    // unless chosen: non-temporal stores once the resident lattices outgrow the 256 MiB Infinity
    // Cache (the next step's input cannot stay there anyway), and always for FP64 storage
    if (!b->nt_chosen)
        b->nontemporal = resident > (size_t(256) << 20) || b->precision == CLB_FP64 || b->precision == CLB_FP64_DEV;
    CLB_HIP(hipMemcpyAsync(b->d_lats, host.data(), host.size(), hipMemcpyHostToDevice, b->stream));
    if (b->tiles.size() > b->tiles_cap) {
        CLB_HIP(hipStreamSynchronize(b->stream));
        (void)hipFree(b->d_tiles);
        b->d_tiles = nullptr;
        const size_t cap_t = std::max<size_t>(b->tiles.size() * 5 / 4, 1024);
        CLB_HIP(hipMalloc((void**)&b->d_tiles, cap_t * sizeof(TileRef)));
        b->tiles_cap = cap_t;
    }
    if (!b->tiles.empty())
        CLB_HIP(hipMemcpyAsync(b->d_tiles, b->tiles.data(), b->tiles.size() * sizeof(TileRef), hipMemcpyHostToDevice, b->stream));
    if (!active.empty())
        CLB_HIP(hipMemcpyAsync(b->d_active, active.data(), active.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
    b->n_active = int(active.size());
    b->unit_rates = all_unit;
    b->rest_walls = all_rest;
    // split for the persistent schedule: small lattices are workgroup-resident, the rest grouped
    b->small_slots.clear();
    b->tiles_big.clear();
    int nsmall = 0;
    for (int i : active)
        if ((long long)b->slots[i].desc.nx * b->slots[i].desc.ny <= kResidentMaxNodes) ++nsmall;
    const bool use_resident = nsmall >= kResidentMinCount;
    for (int i : active) {
        const BatchSlot& s = b->slots[i];
        if (use_resident && (long long)s.desc.nx * s.desc.ny <= kResidentMaxNodes) {
            b->small_slots.push_back(i);
        } else {
            for (int t = 0; t < b->ntiles[i]; ++t) b->tiles_big.push_back(TileRef{i, t});
        }
    }
    if (!b->small_slots.empty())
        CLB_HIP(hipMemcpyAsync(b->d_small, b->small_slots.data(), b->small_slots.size() * sizeof(int),
                               hipMemcpyHostToDevice, b->stream));
    if (b->tiles_big.size() > b->tiles_big_cap) {
        CLB_HIP(hipStreamSynchronize(b->stream));
        CLB_HIP(hipStreamSynchronize(b->side));
        (void)hipFree(b->d_tiles_big);
        b->d_tiles_big = nullptr;
        const size_t cap_t = std::max<size_t>(b->tiles_big.size() * 5 / 4, 1024);
        CLB_HIP(hipMalloc((void**)&b->d_tiles_big, cap_t * sizeof(TileRef)));
        b->tiles_big_cap = cap_t;
    }
    if (!b->tiles_big.empty())
        CLB_HIP(hipMemcpyAsync(b->d_tiles_big, b->tiles_big.data(), b->tiles_big.size() * sizeof(TileRef),
                               hipMemcpyHostToDevice, b->stream));
    b->dirty = false;
    return CLB_OK;
}

// Occupancy of the grouped step.  FP32 storage with FP32 arithmetic needs 47-51 VGPRs, so 8 wavefronts
// per SIMD would fit; at most 6 are faster (512-cavity batch, one MI355X: two buffers 1.040 -> 1.005 ms
// per step, in place 1.109 -> 1.090; 5 or 4 are no better), as fewer streams are in flight per CU.  The
// cap is dynamic LDS the kernel does not use: a CU's 160 KiB hold 6 such allocations, i.e. 6
// workgroups of BNT threads (one wavefront per SIMD each).  The FP64-arithmetic forms are held to 5
// wavefronts by their registers already, and an extra cap makes them slower.
template <typename S, typename Real>
constexpr size_t occupancy_lds()
{
    return sizeof(S) == 4 && sizeof(Real) == 4 ? size_t(160 * 1024 / 6) / 512 * 512 : 0;
}

template <typename S, typename Real, bool DEV>
hipError_t grouped_launch(clb_batch* b, const TileRef* tiles, int tile_base, int ntiles, int s)
{
    const int q = (ntiles + 7) / 8;
    const dim3 grid(8 * q), block(BNT);
    S* pool = (S*)b->pool;
    constexpr size_t lds = occupancy_lds<S, Real>();
    const BatchEntry<Real>* lats = (const BatchEntry<Real>*)b->d_lats;
    if (b->has_aa && b->unit_rates && b->rest_walls) {
        if (b->nontemporal) batch_step_kernel<S, Real, DEV, true, true, true, true><<<grid, block, lds, b->stream>>>(pool, lats, tiles, tile_base, ntiles, s);
        else batch_step_kernel<S, Real, DEV, false, true, true, true><<<grid, block, lds, b->stream>>>(pool, lats, tiles, tile_base, ntiles, s);
    } else if (b->has_aa && b->unit_rates) {
        if (b->nontemporal) batch_step_kernel<S, Real, DEV, true, true, true><<<grid, block, lds, b->stream>>>(pool, lats, tiles, tile_base, ntiles, s);
        else batch_step_kernel<S, Real, DEV, false, true, true><<<grid, block, lds, b->stream>>>(pool, lats, tiles, tile_base, ntiles, s);
    } else if (b->has_aa) {
        if (b->nontemporal) batch_step_kernel<S, Real, DEV, true, true><<<grid, block, lds, b->stream>>>(pool, lats, tiles, tile_base, ntiles, s);
        else batch_step_kernel<S, Real, DEV, false, true><<<grid, block, lds, b->stream>>>(pool, lats, tiles, tile_base, ntiles, s);
    } else if (b->unit_rates && b->rest_walls) {
        if (b->nontemporal) batch_step_kernel<S, Real, DEV, true, false, true, true><<<grid, block, lds, b->stream>>>(pool, lats, tiles, tile_base, ntiles, s);
        else batch_step_kernel<S, Real, DEV, false, false, true, true><<<grid, block, lds, b->stream>>>(pool, lats, tiles, tile_base, ntiles, s);
    } else if (b->unit_rates) {
        if (b->nontemporal) batch_step_kernel<S, Real, DEV, true, false, true><<<grid, block, lds, b->stream>>>(pool, lats, tiles, tile_base, ntiles, s);
        else batch_step_kernel<S, Real, DEV, false, false, true><<<grid, block, lds, b->stream>>>(pool, lats, tiles, tile_base, ntiles, s);
    } else {
        if (b->nontemporal) batch_step_kernel<S, Real, DEV, true, false><<<grid, block, lds, b->stream>>>(pool, lats, tiles, tile_base, ntiles, s);
        else batch_step_kernel<S, Real, DEV, false, false><<<grid, block, lds, b->stream>>>(pool, lats, tiles, tile_base, ntiles, s);
    }
    return hipGetLastError();
}

hipError_t grouped_any(clb_batch* b, int tile_base, int ntiles, int s, const TileRef* tiles = nullptr)
{
    if (ntiles <= 0) return hipSuccess;
    if (!tiles) tiles = b->d_tiles;
    switch (b->precision) {
    case CLB_FP64: return grouped_launch<double, double, false>(b, tiles, tile_base, ntiles, s);
    case CLB_FP64_DEV: return grouped_launch<double, double, true>(b, tiles, tile_base, ntiles, s);
    case CLB_FP32_SR: return grouped_launch<float, double, true>(b, tiles, tile_base, ntiles, s);
    default: return grouped_launch<float, float, true>(b, tiles, tile_base, ntiles, s);
    }
}

template <typename S, typename Real, bool DEV>
hipError_t resident_launch(clb_batch* b, int nsteps, hipStream_t st)
{
    const int ns = int(b->small_slots.size());
    if (b->has_aa)
        batch_resident_kernel<S, Real, DEV, true><<<dim3(ns), dim3(RNT), 0, st>>>(
            (S*)b->pool, (const BatchEntry<Real>*)b->d_lats, b->d_small, ns, nsteps);
    else
        batch_resident_kernel<S, Real, DEV, false><<<dim3(ns), dim3(RNT), 0, st>>>(
            (S*)b->pool, (const BatchEntry<Real>*)b->d_lats, b->d_small, ns, nsteps);
    return hipGetLastError();
}

hipError_t resident_any(clb_batch* b, int nsteps, hipStream_t st)
{
    if (b->small_slots.empty() || nsteps <= 0) return hipSuccess;
    switch (b->precision) {
    case CLB_FP64: return resident_launch<double, double, false>(b, nsteps, st);
    case CLB_FP64_DEV: return resident_launch<double, double, true>(b, nsteps, st);
    case CLB_FP32_SR: return resident_launch<float, double, true>(b, nsteps, st);
    default: return resident_launch<float, float, true>(b, nsteps, st);
    }
}

hipError_t advance_all(clb_batch* b, int nsteps)
{
    if (b->n_active == 0) return hipSuccess;
    const int nb = (b->n_active + 255) / 256;
    if (b->precision == CLB_FP32_DEV)
        batch_advance_kernel<float><<<nb, 256, 0, b->stream>>>((BatchEntry<float>*)b->d_lats, b->d_active, b->n_active, nsteps);
    else
        batch_advance_kernel<double><<<nb, 256, 0, b->stream>>>((BatchEntry<double>*)b->d_lats, b->d_active, b->n_active, nsteps);
    return hipGetLastError();
}

void advance_host(clb_batch* b, long long n)
{
    for (auto& s : b->slots)
        if (s.used) {
            s.steps += n;
            if (n & 1) s.cur ^= 1;
        }
}

int check_slot(clb_batch* b, int slot)
{
    if (!b) { set_error("batch is NULL"); return CLB_EINVAL; }
    if (slot < 0 || slot >= b->capacity || !b->slots[slot].used) { set_error("slot %d is not in use", slot); return CLB_EINVAL; }
    return CLB_OK;
}

int ensure_fields(clb_batch* b, size_t doubles)
{
    if (b->fields_cap >= doubles) return CLB_OK;
    CLB_HIP(hipStreamSynchronize(b->stream));
    (void)hipFree(b->d_fields);
    b->d_fields = nullptr;
    CLB_HIP(hipMalloc((void**)&b->d_fields, doubles * sizeof(double)));
    b->fields_cap = doubles;
    return CLB_OK;
}

enum { MODE_GROUPED = 0, MODE_EACH = 1, MODE_PERSISTENT = 2 };

int step_impl(clb_batch* b, int mode, long long n)
{
    if (n < 0) { set_error("negative step count"); return CLB_EINVAL; }
    if (n == 0) return CLB_OK;
    if (b->dirty) {
        const int rc = upload_tables(b);
        if (rc) return rc;
    }
    if (b->tiles.empty()) return CLB_OK;
    if (mode == MODE_PERSISTENT) {
        // small lattices: one resident launch per chunk on the side stream; big ones: grouped
        // launches on the main stream, concurrently
        const long long chunk = 1 << 20;
        long long done = 0;
        while (done < n) {
            const int k = int(std::min(chunk, n - done));
            if (!b->small_slots.empty()) {
                CLB_HIP(hipEventRecord(b->fork, b->stream));
                CLB_HIP(hipStreamWaitEvent(b->side, b->fork, 0));
                CLB_HIP(resident_any(b, k, b->side));
                CLB_HIP(hipEventRecord(b->join, b->side));
            }
            for (int s = 0; s < k; ++s)
                CLB_HIP(grouped_any(b, 0, int(b->tiles_big.size()), s, b->d_tiles_big));
            if (!b->small_slots.empty()) CLB_HIP(hipStreamWaitEvent(b->stream, b->join, 0));
            CLB_HIP(advance_all(b, k));
            advance_host(b, k);
            done += k;
        }
        return CLB_OK;
    }
    // in chunks, so the call-relative step index passed to the kernels stays within int
    const long long chunk = 1 << 20;
    for (long long done = 0; done < n;) {
        const int k = int(std::min(chunk, n - done));
        for (int s = 0; s < k; ++s) {
            if (mode == MODE_GROUPED) {
                CLB_HIP(grouped_any(b, 0, int(b->tiles.size()), s));
            } else {
                for (int i = 0; i < b->capacity; ++i)
                    if (b->slots[i].used) CLB_HIP(grouped_any(b, b->first_tile[i], b->ntiles[i], s));
            }
        }
        CLB_HIP(advance_all(b, k));
        advance_host(b, k);
        done += k;
    }
    return CLB_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// C ABI.

extern "C" int clb_batch_footprint(const clb_desc* desc, size_t* bytes)
{
    clear_error();
    if (!bytes) { set_error("NULL argument"); return CLB_EINVAL; }
    const int rc = validate_desc(desc);
    if (rc) return rc;
    *bytes = slot_bytes(*desc, nullptr);
    return CLB_OK;
}

extern "C" void clb_batch_destroy(clb_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->own_pool) (void)hipFree(b->pool);
    (void)hipFree(b->d_lats);
    (void)hipFree(b->d_tiles);
    (void)hipFree(b->d_active);
    (void)hipFree(b->d_small);
    (void)hipFree(b->d_tiles_big);
    if (b->side) (void)hipStreamSynchronize(b->side);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->side) (void)hipStreamDestroy(b->side);
    (void)hipFree(b->d_fields);
    (void)hipFree(b->d_partials);
    (void)hipFree(b->d_diag);
    (void)hipFree(b->d_res);
    if (b->ev[0]) (void)hipEventDestroy(b->ev[0]);
    if (b->ev[1]) (void)hipEventDestroy(b->ev[1]);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

static int batch_create_impl(int capacity, int precision, size_t budget, void* pool, size_t pool_bytes, void* hip_stream,
                             clb_batch* b)
{
    if (capacity <= 0 || capacity > (1 << 20)) { set_error("capacity must be in [1, 2^20]"); return CLB_EINVAL; }
    if (precision != CLB_FP64 && precision != CLB_FP32_DEV && precision != CLB_FP64_DEV && precision != CLB_FP32_SR) {
        set_error("unknown precision %d", precision);
        return CLB_EINVAL;
    }
    b->capacity = capacity;
    b->precision = precision;
    b->slots.resize(capacity);
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        CLB_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        b->own_stream = true;
    }
    if (pool) {
        if (pool_bytes < kAlign || (reinterpret_cast<uintptr_t>(pool) % kAlign) != 0) {
            set_error("external pool must be 256-byte aligned and at least 256 bytes");
            return CLB_EINVAL;
        }
        b->pool = (char*)pool;
        b->budget = pool_bytes / kAlign * kAlign;
    } else {
        if (budget < kAlign) { set_error("budget must be at least 256 bytes"); return CLB_EINVAL; }
        b->budget = budget / kAlign * kAlign;
        if (hipMalloc((void**)&b->pool, b->budget) != hipSuccess) {
            (void)hipGetLastError();
            set_error("pool allocation of %zu bytes failed", b->budget);
            return CLB_ENOMEM;
        }
        b->own_pool = true;
    }
    b->free_list[0] = b->budget;
    CLB_HIP(hipMalloc(&b->d_lats, entry_bytes(precision) * capacity));
    CLB_HIP(hipMemsetAsync(b->d_lats, 0, entry_bytes(precision) * capacity, b->stream));
    CLB_HIP(hipMalloc((void**)&b->d_active, sizeof(int) * capacity));
    CLB_HIP(hipMalloc((void**)&b->d_small, sizeof(int) * capacity));
    CLB_HIP(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
    CLB_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    CLB_HIP(hipEventCreateWithFlags(&b->join, hipEventDisableTiming));
    CLB_HIP(hipMalloc((void**)&b->d_diag, DIAG_SLOTS * sizeof(double)));
    CLB_HIP(hipMalloc((void**)&b->d_res, sizeof(unsigned long long) * 3 * capacity));
    CLB_HIP(hipEventCreate(&b->ev[0]));
    CLB_HIP(hipEventCreate(&b->ev[1]));
    b->nontemporal = precision == CLB_FP64 || precision == CLB_FP64_DEV;
    return CLB_OK;
}

extern "C" int clb_batch_create(int capacity, int precision, size_t hbm_budget_bytes, void* pool, size_t pool_bytes,
                                void* hip_stream, clb_batch** out)
{
    clear_error();
    if (!out) { set_error("out is NULL"); return CLB_EINVAL; }
    *out = nullptr;
    clb_batch* b = new (std::nothrow) clb_batch;
    if (!b) { set_error("host allocation failed"); return CLB_ENOMEM; }
    const int rc = batch_create_impl(capacity, precision, hbm_budget_bytes, pool, pool_bytes, hip_stream, b);
    if (rc) {
        clb_batch_destroy(b);
        return rc;
    }
    *out = b;
    return CLB_OK;
}

extern "C" int clb_batch_add(clb_batch* b, const clb_desc* desc, double tau_nu, double tau_alpha, double g_beta,
                             double Ma, int* slot)
{
    clear_error();
    if (!b || !slot) { set_error("NULL argument"); return CLB_EINVAL; }
    int rc = validate_desc(desc);
    if (rc) return rc;
    if (desc->precision != b->precision) { set_error("lattice precision differs from the batch's"); return CLB_EINVAL; }
    if (desc->prescribed_u) { set_error("temperature-only lattices (prescribed_u) are single-lattice only"); return CLB_EINVAL; }
    rc = check_params(tau_nu, tau_alpha, g_beta, Ma);
    if (rc) return rc;
    int free_slot = -1;
    for (int i = 0; i < b->capacity; ++i)
        if (!b->slots[i].used) { free_slot = i; break; }
    if (free_slot < 0) { set_error("batch is full (%d slots)", b->capacity); return CLB_ENOMEM; }
    BatchSlot s;
    size_t buf_bytes = 0, band_bytes = 0;
    const size_t bytes = slot_bytes(*desc, &buf_bytes, &band_bytes);
    if (buf_bytes >= (size_t(1) << 32)) {
        // the grouped step addresses a lattice's buffers with 32-bit byte offsets
        set_error("a batch lattice's population buffer must be under 4 GiB (this one needs %zu bytes); "
                  "use a single lattice (clb_create)", buf_bytes);
        return CLB_EINVAL;
    }
    size_t off = 0;
    if (alloc_range(b, bytes, &off) != CLB_OK) {
        set_error("lattice needs %zu bytes; %zu of %zu bytes in use", bytes, b->used_bytes, b->budget);
        return CLB_ENOMEM;
    }
    const size_t n = size_t(desc->nx) * desc->ny;
    rc = ensure_fields(b, 4 * n);
    if (rc) { free_range(b, off, bytes); return rc; }
    const size_t eb = elem_bytes(desc->precision);
    s.used = true;
    s.desc = *desc;
    s.par.tau_nu = tau_nu;
    s.par.tau_alpha = tau_alpha;
    s.par.g_beta = g_beta;
    s.par.Ma = Ma;
    s.alloc_off = off;
    s.alloc_bytes = bytes;
    s.off[0] = (long long)(off / eb);
    if (desc->in_place) {
        s.off[1] = s.off[0];
        s.sn[0] = (long long)((off + buf_bytes) / eb);
        s.sn[1] = (long long)((off + buf_bytes + band_bytes) / eb);
        s.snap_off = off + buf_bytes + 2 * band_bytes;
    } else {
        s.off[1] = (long long)((off + buf_bytes) / eb);
        s.snap_off = off + 2 * buf_bytes;
    }
    auto it = b->tw_by_class.find(size_class(*desc));
    s.tw_log2 = !desc->in_place && it != b->tw_by_class.end() ? it->second : default_tw_log2(*desc);
    b->slots[free_slot] = s;
    b->dirty = true;
    *slot = free_slot;
    rc = clb_batch_init(b, free_slot, nullptr, nullptr, nullptr);
    if (rc) {
        b->slots[free_slot].used = false;
        free_range(b, off, bytes);
        return rc;
    }
    return CLB_OK;
}

extern "C" int clb_batch_set_relaxation(clb_batch* b, int slot, double s_b, double s3, double s4, double lambda2)
{
    clear_error();
    int rc = check_slot(b, slot);
    if (rc) return rc;
    const double v[4] = {s_b, s3, s4, lambda2};
    for (double r : v)
        if (!std::isfinite(r) || r <= 0.0 || r >= 2.0) { set_error("relaxation rates must lie in (0, 2)"); return CLB_EINVAL; }
    Params& p = b->slots[slot].par;
    p.s_b = s_b;
    p.s3 = s3;
    p.s4 = s4;
    p.lam2 = lambda2;
    b->dirty = true;
    return CLB_OK;
}

extern "C" int clb_batch_set_body_force(clb_batch* b, int slot, double Fvx, double Fvy)
{
    clear_error();
    int rc = check_slot(b, slot);
    if (rc) return rc;
    if (!std::isfinite(Fvx) || !std::isfinite(Fvy)) { set_error("body force must be finite"); return CLB_EINVAL; }
    b->slots[slot].par.Fvx = Fvx;
    b->slots[slot].par.Fvy = Fvy;
    b->dirty = true;
    return CLB_OK;
}

// Moments (rho, u_x, u_y, T) of a slot's current step into b->d_fields.
static hipError_t slot_moments(clb_batch* b, const BatchSlot& s)
{
    const clb_desc& d = s.desc;
    const size_t eb = elem_bytes(d.precision);
    const Geo G = make_geo(d);
    if (d.in_place) {
        const bool odd = (s.steps & 1) != 0;
        return enqueue_moments_aa(d, s.par, odd, b->pool + s.off[0] * eb, G, b->d_fields, b->stream);
    }
    return enqueue_moments(d, s.par, b->pool + s.off[s.cur] * eb, G, b->d_fields, b->stream);
}

extern "C" int clb_batch_init(clb_batch* b, int slot, const double* rho, const double* u, const double* T)
{
    clear_error();
    int rc = check_slot(b, slot);
    if (rc) return rc;
    BatchSlot& s = b->slots[slot];
    const clb_desc& d = s.desc;
    const size_t n = size_t(d.nx) * d.ny;
    std::vector<double> host(4 * n);
    for (size_t k = 0; k < n; ++k) {
        host[k] = rho ? rho[k] : 1.0;
        host[n + k] = u ? u[k] : 0.0;
        host[2 * n + k] = u ? u[n + k] : 0.0;
        host[3 * n + k] = T ? T[k] : d.T0;
    }
    for (size_t k = 0; k < 4 * n; ++k)
        if (!std::isfinite(host[k]) || (k < n && host[k] <= 0.0)) {
            set_error("initial fields must be finite with rho > 0");
            return CLB_EINVAL;
        }
    rc = ensure_fields(b, 4 * n);
    if (rc) return rc;
    const size_t eb = elem_bytes(d.precision);
    // both population buffers, or the in-place buffer and its snapshot copies: everything below the
    // residual snapshot
    CLB_HIP(hipMemsetAsync(b->pool + s.off[0] * eb, 0, s.snap_off - size_t(s.off[0]) * eb, b->stream));
    CLB_HIP(hipMemcpyAsync(b->d_fields, host.data(), 4 * n * sizeof(double), hipMemcpyHostToDevice, b->stream));
    const Geo G = make_geo(d);
    s.cur = 0;
    s.steps = 0;
    if (d.in_place)
        CLB_HIP(enqueue_init_aa(d, s.par, b->pool + s.off[0] * eb, b->pool + s.sn[0] * eb, G, b->d_fields, b->stream));
    else
        CLB_HIP(enqueue_init(d, s.par, b->pool + s.off[0] * eb, G, b->d_fields, b->stream));
    // the snapshot starts as the initial (u_x, u_y, T), so the first residual measures the first chunk
    CLB_HIP(slot_moments(b, s));
    CLB_HIP(hipMemcpyAsync(b->pool + s.snap_off, b->d_fields + n, 3 * n * sizeof(double), hipMemcpyDeviceToDevice,
                           b->stream));
    CLB_HIP(hipStreamSynchronize(b->stream));
    s.cur = 0;
    s.steps = 0;
    s.has_snap = true;
    b->dirty = true;
    return CLB_OK;
}

extern "C" int clb_batch_remove(clb_batch* b, int slot)
{
    clear_error();
    int rc = check_slot(b, slot);
    if (rc) return rc;
    BatchSlot& s = b->slots[slot];
    free_range(b, s.alloc_off, s.alloc_bytes);
    s = BatchSlot();
    b->dirty = true;
    return CLB_OK;
}

extern "C" int clb_batch_step(clb_batch* b, long long n)
{
    clear_error();
    if (!b) { set_error("batch is NULL"); return CLB_EINVAL; }
    return step_impl(b, MODE_GROUPED, n);
}

extern "C" int clb_batch_step_each(clb_batch* b, long long n)
{
    clear_error();
    if (!b) { set_error("batch is NULL"); return CLB_EINVAL; }
    return step_impl(b, MODE_EACH, n);
}

extern "C" int clb_batch_step_persistent(clb_batch* b, long long n)
{
    clear_error();
    if (!b) { set_error("batch is NULL"); return CLB_EINVAL; }
    return step_impl(b, MODE_PERSISTENT, n);
}

extern "C" int clb_batch_check(clb_batch* b)
{
    clear_error();
    if (!b) { set_error("batch is NULL"); return CLB_EINVAL; }
    CLB_HIP(hipStreamSynchronize(b->stream));
    CLB_HIP(hipGetLastError());
    return CLB_OK;
}

extern "C" int clb_batch_time_steps(clb_batch* b, int mode, long long n, double* ms)
{
    clear_error();
    if (!b || !ms) { set_error("NULL argument"); return CLB_EINVAL; }
    if (mode < MODE_GROUPED || mode > MODE_PERSISTENT || n <= 0) { set_error("bad mode or step count"); return CLB_EINVAL; }
    if (b->dirty) {
        const int rc = upload_tables(b);
        if (rc) return rc;
    }
    CLB_HIP(hipEventRecord(b->ev[0], b->stream));
    const int rc = step_impl(b, mode, n);
    if (rc) return rc;
    CLB_HIP(hipEventRecord(b->ev[1], b->stream));
    CLB_HIP(hipEventSynchronize(b->ev[1]));
    float t = 0.0f;
    CLB_HIP(hipEventElapsedTime(&t, b->ev[0], b->ev[1]));
    *ms = t;
    return CLB_OK;
}

extern "C" int clb_batch_synchronize(clb_batch* b)
{
    clear_error();
    if (!b) { set_error("batch is NULL"); return CLB_EINVAL; }
    CLB_HIP(hipStreamSynchronize(b->stream));
    return CLB_OK;
}

extern "C" int clb_batch_info(clb_batch* b, int* count, size_t* used_bytes, size_t* budget_bytes, long long* sites)
{
    clear_error();
    if (!b) { set_error("batch is NULL"); return CLB_EINVAL; }
    int c = 0;
    long long ns = 0;
    for (auto& s : b->slots)
        if (s.used) {
            ++c;
            ns += (long long)s.desc.nx * s.desc.ny;
        }
    if (count) *count = c;
    if (used_bytes) *used_bytes = b->used_bytes;
    if (budget_bytes) *budget_bytes = b->budget;
    if (sites) *sites = ns;
    return CLB_OK;
}

extern "C" int clb_batch_moments(clb_batch* b, int slot, double* rho, double* u, double* T)
{
    clear_error();
    int rc = check_slot(b, slot);
    if (rc) return rc;
    BatchSlot& s = b->slots[slot];
    const clb_desc& d = s.desc;
    const size_t n = size_t(d.nx) * d.ny;
    rc = ensure_fields(b, 4 * n);
    if (rc) return rc;
    CLB_HIP(slot_moments(b, s));
    if (rho) CLB_HIP(hipMemcpyAsync(rho, b->d_fields, n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    if (u) CLB_HIP(hipMemcpyAsync(u, b->d_fields + n, 2 * n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    if (T) CLB_HIP(hipMemcpyAsync(T, b->d_fields + 3 * n, n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    CLB_HIP(hipStreamSynchronize(b->stream));
    return CLB_OK;
}

extern "C" int clb_batch_diagnostics(clb_batch* b, int slot, int snapshot, clb_diag* out)
{
    clear_error();
    int rc = check_slot(b, slot);
    if (rc) return rc;
    if (!out) { set_error("NULL argument"); return CLB_EINVAL; }
    BatchSlot& s = b->slots[slot];
    const clb_desc& d = s.desc;
    const size_t n = size_t(d.nx) * d.ny;
    rc = ensure_fields(b, 4 * n);
    if (rc) return rc;
    const Geo G = make_geo(d);
    const int nb = diag_blocks(G);
    if (b->partials_cap < nb) {
        CLB_HIP(hipStreamSynchronize(b->stream));
        (void)hipFree(b->d_partials);
        b->d_partials = nullptr;
        CLB_HIP(hipMalloc((void**)&b->d_partials, size_t(nb) * DIAG_SLOTS * sizeof(double)));
        b->partials_cap = nb;
    }
    double* snap = (double*)(b->pool + s.snap_off);
    CLB_HIP(slot_moments(b, s));
    CLB_HIP(enqueue_diag(b->d_fields, snap, s.has_snap ? 1 : 0, G, b->d_partials, b->d_diag, b->stream));
    double r[DIAG_SLOTS];
    CLB_HIP(hipMemcpyAsync(r, b->d_diag, sizeof r, hipMemcpyDeviceToHost, b->stream));
    if (snapshot) CLB_HIP(hipMemcpyAsync(snap, b->d_fields + n, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, b->stream));
    CLB_HIP(hipStreamSynchronize(b->stream));
    if (snapshot) s.has_snap = true;
    unpack_diag(r, s.steps, out);
    if (out->nonfinite) {
        set_error("slot %d: non-finite density, velocity or temperature at step %lld", slot, s.steps);
        return CLB_EDIVERGED;
    }
    return CLB_OK;
}

extern "C" int clb_batch_set_tile_width(clb_batch* b, int slot, int tile_width)
{
    clear_error();
    int rc = check_slot(b, slot);
    if (rc) return rc;
    const int lg = tile_width == 64 ? 6 : tile_width == 128 ? 7 : tile_width == 256 ? 8 : tile_width == 0 ? 0 : -1;
    if (lg < 0) { set_error("tile width must be 64, 128, 256 or 0 (wrapped rows)"); return CLB_EINVAL; }
    b->slots[slot].tw_log2 = lg;
    b->dirty = true;
    return CLB_OK;
}

extern "C" int clb_batch_get_tile_width(clb_batch* b, int slot, int* tile_width)
{
    clear_error();
    int rc = check_slot(b, slot);
    if (rc) return rc;
    if (!tile_width) { set_error("NULL argument"); return CLB_EINVAL; }
    const int lg = b->slots[slot].tw_log2;
    *tile_width = lg == 0 ? 0 : 1 << lg;
    return CLB_OK;
}

// For every size class present, time the grouped step over that class's lattices with each tile
// width (state unchanged: reads the current buffers, writes the spare ones) and keep the fastest.
// Tile mappings and store form are timed on the two-buffer lattices only: their timing launches
// read the current state and write the spare buffer, so the state is untouched.  An in-place
// lattice would be advanced by them; in-place lattices keep their mappings (and take the store
// form chosen for the rest).
static int autotune_two_buffer(clb_batch* b, int launches)
{
    std::map<int, std::vector<int>> classes;
    for (int i = 0; i < b->capacity; ++i)
        if (b->slots[i].used) classes[size_class(b->slots[i].desc)].push_back(i);
    for (auto& kv : classes) {
        int best = -1;
        double best_t = 0.0;
        for (int lg : {6, 7, 8, 0}) {
            std::vector<bool> keep(b->capacity, false);
            for (int i : kv.second) keep[i] = true;
            // restrict the tables to this class with width lg
            std::vector<int> saved_tw(b->capacity);
            std::vector<char> saved_used(b->capacity);
            for (int i = 0; i < b->capacity; ++i) {
                saved_tw[i] = b->slots[i].tw_log2;
                saved_used[i] = b->slots[i].used;
                if (b->slots[i].used && !keep[i]) b->slots[i].used = false;
                if (keep[i]) b->slots[i].tw_log2 = lg;
            }
            int rc = upload_tables(b);
            for (int i = 0; i < b->capacity; ++i) {
                b->slots[i].used = saved_used[i] != 0;
                b->slots[i].tw_log2 = saved_tw[i];
            }
            if (rc) { b->dirty = true; return rc; }
            const int nt = int(b->tiles.size());
            for (int w = 0; w < 2; ++w) CLB_HIP(grouped_any(b, 0, nt, 0));
            CLB_HIP(hipEventRecord(b->ev[0], b->stream));
            for (int r = 0; r < launches; ++r) CLB_HIP(grouped_any(b, 0, nt, 0));
            CLB_HIP(hipEventRecord(b->ev[1], b->stream));
            CLB_HIP(hipEventSynchronize(b->ev[1]));
            float ms = 0.0f;
            CLB_HIP(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
            if (best < 0 || ms < best_t) { best = lg; best_t = ms; }
        }
        b->tw_by_class[kv.first] = best;
        for (int i : kv.second) b->slots[i].tw_log2 = best;
    }
    b->dirty = true;
    int rc = upload_tables(b);
    if (rc) return rc;
    // store form over the whole batch
    const int nt = int(b->tiles.size());
    if (nt == 0) return CLB_OK;
    double t_store[2] = {0.0, 0.0};
    for (int v = 0; v < 2; ++v) {
        b->nontemporal = v != 0;
        for (int w = 0; w < 2; ++w) CLB_HIP(grouped_any(b, 0, nt, 0));
        CLB_HIP(hipEventRecord(b->ev[0], b->stream));
        for (int r = 0; r < launches; ++r) CLB_HIP(grouped_any(b, 0, nt, 0));
        CLB_HIP(hipEventRecord(b->ev[1], b->stream));
        CLB_HIP(hipEventSynchronize(b->ev[1]));
        float ms = 0.0f;
        CLB_HIP(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
        t_store[v] = ms;
    }
    b->nontemporal = t_store[1] < t_store[0];
    b->nt_chosen = true;
    return CLB_OK;
}

extern "C" int clb_batch_autotune(clb_batch* b, int launches)
{
    clear_error();
    if (!b || launches <= 0) { set_error("bad arguments"); return CLB_EINVAL; }
    // hide the in-place lattices for the duration
    std::vector<int> hidden;
    for (int i = 0; i < b->capacity; ++i)
        if (b->slots[i].used && b->slots[i].desc.in_place) {
            b->slots[i].used = false;
            hidden.push_back(i);
        }
    const int rc = autotune_two_buffer(b, launches);
    for (int i : hidden) b->slots[i].used = true;
    b->dirty = true;
    if (rc) return rc;
    return upload_tables(b);
}

extern "C" int clb_batch_set_nontemporal(clb_batch* b, int nontemporal)
{
    clear_error();
    if (!b) { set_error("batch is NULL"); return CLB_EINVAL; }
    b->nontemporal = nontemporal != 0;
    b->nt_chosen = true;
    return CLB_OK;
}

extern "C" int clb_batch_get_nontemporal(clb_batch* b, int* nontemporal)
{
    clear_error();
    if (!b || !nontemporal) { set_error("NULL argument"); return CLB_EINVAL; }
    if (b->dirty) {
        // the default store form follows the resident footprint, fixed when the tables are built
        const int rc = upload_tables(b);
        if (rc) return rc;
    }
    *nontemporal = b->nontemporal ? 1 : 0;
    return CLB_OK;
}

template <typename S, typename Real, bool DEV>
static hipError_t residual_launch(clb_batch* b)
{
    const int nt = int(b->tiles.size());
    const int q = (nt + 7) / 8;
    if (b->has_aa)
        batch_residual_kernel<S, Real, DEV, true><<<dim3(8 * q), dim3(BNT), 0, b->stream>>>(
            (S*)b->pool, (const BatchEntry<Real>*)b->d_lats, b->d_tiles, nt, b->d_res);
    else
        batch_residual_kernel<S, Real, DEV, false><<<dim3(8 * q), dim3(BNT), 0, b->stream>>>(
            (S*)b->pool, (const BatchEntry<Real>*)b->d_lats, b->d_tiles, nt, b->d_res);
    return hipGetLastError();
}

extern "C" int clb_batch_residuals(clb_batch* b, double* du, double* dT, int* nonfinite)
{
    clear_error();
    if (!b) { set_error("batch is NULL"); return CLB_EINVAL; }
    if (b->dirty) {
        const int rc = upload_tables(b);
        if (rc) return rc;
    }
    const int n3 = 3 * b->capacity;
    batch_zero64_kernel<<<(n3 + 255) / 256, 256, 0, b->stream>>>(b->d_res, n3);
    CLB_HIP(hipGetLastError());
    if (!b->tiles.empty()) {
        switch (b->precision) {
        case CLB_FP64: CLB_HIP((residual_launch<double, double, false>(b))); break;
        case CLB_FP64_DEV: CLB_HIP((residual_launch<double, double, true>(b))); break;
        case CLB_FP32_SR: CLB_HIP((residual_launch<float, double, true>(b))); break;
        default: CLB_HIP((residual_launch<float, float, true>(b))); break;
        }
    }
    std::vector<unsigned long long> host(n3);
    CLB_HIP(hipMemcpyAsync(host.data(), b->d_res, n3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, b->stream));
    CLB_HIP(hipStreamSynchronize(b->stream));
    for (int i = 0; i < b->capacity; ++i) {
        const bool used = b->slots[i].used;
        double v[3];
        std::memcpy(v, &host[3 * i], sizeof v);
        if (du) du[i] = used ? v[0] : -1.0;
        if (dT) dT[i] = used ? v[1] : -1.0;
        if (nonfinite) nonfinite[i] = used && v[2] > 0.0 ? 1 : 0;
    }
    return CLB_OK;
}
