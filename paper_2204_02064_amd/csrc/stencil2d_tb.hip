// 2D radius-1 Jacobi stencils (Eq. 2, the 5-point star and the 9-point box of
// tab:domain), temporally blocked persistent kernel for small grids.
//
// On a small grid a step costs a few microseconds, almost all of it the
// latency of the halo exchange between CUs (a store that other CUs must see,
// then their loads), so the persistent kernel exchanges only every K steps:
// each wavefront owns a tile of OW = 64 - 2K columns x H rows and holds the
// tile plus a ring of K ghost columns and rows in registers (lane l keeps
// column x0 - K + l, rows y0 - K .. y0 + H + K - 1); it then takes K Jacobi
// steps on that block with no exchange at all (neighbours along y in the
// lane's registers, along x by DPP lane shifts).  Each step leaves the cells
// one row and one column further in from the block's edge exact, so after K
// steps the owned tile is exact: the ghost ring is recomputed instead of
// exchanged (overlapped temporal blocking).  The tile is then stored into
// the other of two grid buffers, and one device-wide barrier precedes the
// next block's loads.  The grid lives in the two buffers between blocks (on
// a small grid, in the caches); the paper's register cache holds each block
// for K steps.
//
// Every cell is summed in ascending (dy, dx) order, one multiply then FMAs,
// as the per-step baseline does, so the two agree bit for bit.  Ring cells
// and clamped copies outside the grid are never updated.
#include <algorithm>
#include <type_traits>
#include <new>
#include <vector>

#include "barrier.hpp"
#include "common.hpp"
#include "stencil_api.hpp"

namespace perks {
namespace {

constexpr int TBW = 4;   // waves per workgroup

template <typename T>
struct TB2DParams {
    gmem<T> *buf0;   // the caller's grid
    gmem<T> *buf1;   // second buffer of the same extents (ring copied in)
    unsigned *sync;
    int64_t steps;
    int nx, ny;
    int ntx, nty;    // tiles along x (OW columns) and y (H rows)
    T w[9];          // [dy + 1][dx + 1]
};

// One Jacobi step of a block of RB rows x 64 lanes, in place.  Rows 0 and
// RB - 1 lack a neighbour row and lanes 0 and 63 a neighbour column: their
// new values are not exact and are never used (they lie outside the region
// that is still exact after this step), so the lane shifts give the edge
// lane 0 for its missing neighbour.
template <typename T, bool BOX, int RB>
__device__ __forceinline__ void tb_step(T (&u)[RB], const T (&w)[9], bool lane_in, int y0, int ny) {
    T pv = u[0], pw = from_west0(pv), pe = from_east0(pv);
    T cv = u[1], cw = from_west0(cv), ce = from_east0(cv);
#pragma unroll
    for (int i = 1; i < RB - 1; ++i) {
        const T nv = u[i + 1];
        const T nw = from_west0(nv), ne = from_east0(nv);
        T acc;
        if constexpr (BOX) {
            acc = w[0] * pw;
            acc = fma_t(w[1], pv, acc);
            acc = fma_t(w[2], pe, acc);
            acc = fma_t(w[3], cw, acc);
            acc = fma_t(w[4], cv, acc);
            acc = fma_t(w[5], ce, acc);
            acc = fma_t(w[6], nw, acc);
            acc = fma_t(w[7], nv, acc);
            acc = fma_t(w[8], ne, acc);
        } else {
            acc = w[1] * pv;
            acc = fma_t(w[3], cw, acc);
            acc = fma_t(w[4], cv, acc);
            acc = fma_t(w[5], ce, acc);
            acc = fma_t(w[7], nv, acc);
        }
        const int y = y0 + i;
        u[i] = (lane_in && y >= 1 && y <= ny - 2) ? acc : cv;
        pv = cv;
        pw = cw;
        pe = ce;
        cv = nv;
        cw = nw;
        ce = ne;
    }
}

// The same step with every new row written into its own old row's register:
// each old row is visited once, top to bottom, and adds its terms to the new
// rows it touches (three rolling accumulators); new row i is complete, and
// old row i dead, once old row i+1 has been visited.  tb_step instead holds
// each old row in a copy while its new value takes another register, which
// in a loop over steps makes the compiler rotate every row back (FP64 tall
// blocks then need twice their registers).  Sums, rows updated and rows kept
// are tb_step's, so the two give the same bits.
// done(integral_constant<int, i>) is called once new row i is in u[i] (rows
// 1 .. RB-2, in order), so that a caller can store it while later rows are
// still being computed.
template <typename T, bool BOX, int RB, class Done>
__device__ __forceinline__ void tb_step_roll(T (&u)[RB], const T (&w)[9], bool lane_in, int y0, int ny,
                                             Done &&done) {
    T acc[3] = {T(0), T(0), T(0)};   // each starts with a product before use
    static_for<0, RB>([&](auto jc) {
        constexpr int j = decltype(jc)::value;   // old row visited
        const T v = u[j];
        const T vw = from_west0(v), ve = from_east0(v);
        if constexpr (j + 1 <= RB - 2) {   // new row j+1: its dy = -1 terms, the first a product
            T &a = acc[(j + 1) % 3];
            if constexpr (BOX) {
                a = w[0] * vw;
                a = fma_t(w[1], v, a);
                a = fma_t(w[2], ve, a);
            } else {
                a = w[1] * v;
            }
        }
        if constexpr (j >= 1 && j <= RB - 2) {   // new row j: dy = 0
            T &a = acc[j % 3];
            a = fma_t(w[3], vw, a);
            a = fma_t(w[4], v, a);
            a = fma_t(w[5], ve, a);
        }
        if constexpr (j >= 2) {   // new row j-1: dy = +1, then it replaces old row j-1
            T &a = acc[(j - 1) % 3];
            if constexpr (BOX) {
                a = fma_t(w[6], vw, a);
                a = fma_t(w[7], v, a);
                a = fma_t(w[8], ve, a);
            } else {
                a = fma_t(w[7], v, a);
            }
            const int y = y0 + j - 1;
            u[j - 1] = (lane_in && y >= 1 && y <= ny - 2) ? a : u[j - 1];
            done(std::integral_constant<int, j - 1>{});
        }
        settle(acc);   // this row's terms here (not sunk below later rows' shifts)
    });
}

// One block of K (kk <= K) steps of tile t of a grid: load the tile and its
// ghost ring from src, step, store the owned cells into dst.
// ROLL: steps by tb_step_roll (fewer registers for 16-row FP64 blocks, more
// waves: the batched kernel), else by tb_step (fewer for 8-row ones).
template <typename T, bool BOX, int K, int H, bool ROLL = false>
__device__ __forceinline__ void tb_tile(const gmem<T> *src, gmem<T> *dst, int nx, int ny, int ntx, int t, int kk,
                                        int lane, const T (&w)[9]) {
    constexpr int RB = H + 2 * K, OW = 64 - 2 * K;
    const int tx = t % ntx, ty = t / ntx;
    const int xg = 1 + OW * tx - K + lane;   // this lane's column
    const int y0 = 1 + H * ty - K;           // the block's first row
    const int xc = min(max(xg, 0), nx - 1);
    T u[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        const int yc = min(max(y0 + i, 0), ny - 1);
        u[i] = ld_coh(src + (size_t)yc * nx + xc);
    }
    const bool lane_in = xg >= 1 && xg <= nx - 2;
    for (int j = 0; j < kk; ++j) {
        if constexpr (ROLL) tb_step_roll<T, BOX, RB>(u, w, lane_in, y0, ny, [](auto) {});
        else tb_step<T, BOX, RB>(u, w, lane_in, y0, ny);
    }
    const bool own = lane_in && lane >= K && lane < K + OW;
#pragma unroll
    for (int i = K; i < K + H; ++i) {
        const int y = y0 + i;
        if (own && y >= 1 && y <= ny - 2) st_coh(dst + (size_t)y * nx + xg, u[i]);
    }
}

// The owned cells of tile t from the second buffer back into the grid (the
// same wave stored them there).
template <int K, int H, typename T>
__device__ __forceinline__ void tb_copy_back(gmem<T> *buf0, const gmem<T> *buf1, int nx, int ny, int ntx, int t,
                                             int lane) {
    constexpr int OW = 64 - 2 * K;
    const int tx = t % ntx, ty = t / ntx;
    const int xg = 1 + OW * tx - K + lane;
    const int y0 = 1 + H * ty - K;
    const bool own = xg >= 1 && xg <= nx - 2 && lane >= K && lane < K + OW;
    for (int i = K; i < K + H; ++i) {
        const int y = y0 + i;
        if (own && y >= 1 && y <= ny - 2) {
            const size_t e = (size_t)y * nx + xg;
            buf0[e] = ld_coh(buf1 + e);
        }
    }
}

template <typename T, bool BOX, int K, int H>
__global__ __launch_bounds__(TBW * 64) void stencil2d_tb(TB2DParams<T> p) {
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gw = blockIdx.x * TBW + wave, nw = gridDim.x * TBW;
    const int ntiles = p.ntx * p.nty;
    T w[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = p.w[k];
    GridSync gs;
    gs.init(p.sync);
    int64_t blk = 0;
    for (int64_t s0 = 0; s0 < p.steps; s0 += K, ++blk) {
        const int kk = (int)std::min<int64_t>(K, p.steps - s0);
        const gmem<T> *src = opaque((blk & 1) ? p.buf1 : p.buf0);
        gmem<T> *dst = opaque((blk & 1) ? p.buf0 : p.buf1);
        for (int t = gw; t < ntiles; t += nw) tb_tile<T, BOX, K, H>(src, dst, p.nx, p.ny, p.ntx, t, kk, lane, w);
        gs.sync();
    }
    if (blk & 1)   // the result is in the second buffer
        for (int t = gw; t < ntiles; t += nw) tb_copy_back<K, H>(p.buf0, p.buf1, p.nx, p.ny, p.ntx, t, lane);
    gs.finish();
}

// Register-resident variant, for grids whose tiles all have a wave of their
// own (the plan checks it): each wave keeps its block in registers for the
// whole run.  After a block of K steps it stores only the band of owned
// cells within K of its tile's edge (into the other buffer), and after the
// barrier loads only its ghost ring back from there (the neighbours' bands);
// the last block stores the whole owned tile.  The cells and their
// arithmetic are those of stencil2d_tb, so the two agree bit for bit, but a
// block moves the band and the ring instead of the whole block and tile.
// Element e of a wave-uniform row start: a scalar base plus a 32-bit vector
// offset (a 64-bit vector address per row would cost two registers a row).
template <typename T>
__device__ __forceinline__ gmem<T> *row_at(gmem<T> *row, int e) {
    return (gmem<T> *)((gmem<char> *)row + (unsigned)e * (unsigned)sizeof(T));
}

template <typename T, bool BOX, int K, int H>
__global__ __launch_bounds__(TBW * 64) void stencil2d_tbr(TB2DParams<T> p) {
    constexpr int RB = H + 2 * K, OW = 64 - 2 * K;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // waves past the last tile (ty >= nty) step a block of clamped copies and
    // store nothing: their owned rows lie past the grid
    const int t = blockIdx.x * TBW + wave;
    T w[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = p.w[k];
    GridSync gs;
    gs.init(p.sync);
    const int tx = t % p.ntx, ty = t / p.ntx;
    const int xg = 1 + OW * tx - K + lane;   // this lane's column
    const int y0 = 1 + H * ty - K;           // the block's first row
    const int xc = min(max(xg, 0), p.nx - 1);
    const bool lane_in = xg >= 1 && xg <= p.nx - 2;
    const bool own = lane_in && lane >= K && lane < K + OW;
    const bool side = lane < 2 * K || lane >= OW;       // (owned lanes) within K of the west / east edge
    const bool ring_lane = lane < K || lane >= K + OW;  // ghost columns
    T u[RB];
    {
        gmem<T> *src = opaque(p.buf0);
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int yc = min(max(y0 + i, 0), p.ny - 1);
            u[i] = ld_coh(row_at(src + (size_t)yc * p.nx, xc));
        }
    }
    settle(u);   // the loads land here, in the registers the steps use
    // Every block ends with the ring loads, the last one too (its values go
    // unused): no branch around them, so each load writes its row's register.
    int64_t blk = 0;
    for (int64_t s0 = 0; s0 < p.steps; s0 += K, ++blk) {
        const int kk = (int)std::min<int64_t>(K, p.steps - s0);
        const bool last = s0 + K >= p.steps;
        gmem<T> *dst = opaque((blk & 1) ? p.buf0 : p.buf1);
        // the block's last step stores each owned row as soon as it is final
        // (its band part; every owned cell in the last block), overlapping
        // the writes with the rows still to come.  Owned rows are K .. K+H-1;
        // the band is rows K .. 2K-1 and H .. H+K-1, and the side lanes.
        for (int j = 0; j + 1 < kk; ++j) tb_step_roll<T, BOX, RB>(u, w, lane_in, y0, p.ny, [](auto) {});
        tb_step_roll<T, BOX, RB>(u, w, lane_in, y0, p.ny, [&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if constexpr (i >= K && i < K + H) {
                const int y = y0 + i;
                const bool band = last || side || i < 2 * K || i >= H;
                if (own && band && y >= 1 && y <= p.ny - 2) st_coh(row_at(dst + (size_t)y * p.nx, xg), u[i]);
            }
        });
        gs.sync();
        // the ghost rows in every lane, then the ghost columns' owned rows in
        // their lanes only
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            if (i < K || i >= K + H) {
                const int yc = min(max(y0 + i, 0), p.ny - 1);
                u[i] = ld_coh(row_at(dst + (size_t)yc * p.nx, xc));
            }
        }
        if (ring_lane) {
#pragma unroll
            for (int i = K; i < K + H; ++i) {
                const int yc = min(max(y0 + i, 0), p.ny - 1);
                u[i] = ld_coh(row_at(dst + (size_t)yc * p.nx, xc));
            }
        }
        settle(u);
    }
    if (blk & 1)   // the result is in the second buffer
        tb_copy_back<K, H>(p.buf0, p.buf1, p.nx, p.ny, p.ntx, t, lane);
    gs.finish();
}

// Many grids in one launch: the tiles of every grid form one range (grid i's
// tiles start at tile_base[i]), taken by the waves in turn; one barrier per
// block for all of them.
template <typename T>
struct TBGrid {
    gmem<T> *buf0, *buf1;
    int nx, ny, ntx, tile_base;
};

template <typename T>
struct TBBatchParams {
    const TBGrid<T> *grids;
    int count, ntiles;
    unsigned *sync;
    int64_t steps;
    T w[9];
};

// Grid of global tile t: the last i with grids[i].tile_base <= t.
template <typename T>
__device__ __forceinline__ int tb_locate(const TBGrid<T> *g, int count, int t) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g[mid].tile_base <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The fixed ring of grid g into its second buffer (by one wave; the first
// block writes only interior cells there, and the second, the first to read
// the second buffer, follows a device barrier).
template <typename T>
__device__ __forceinline__ void tb_copy_ring(const TBGrid<T> &g, int lane) {
    const int nx = g.nx, ny = g.ny;
    const size_t last = (size_t)(ny - 1) * nx;
    for (int x = lane; x < nx; x += 64) {
        st_coh(g.buf1 + x, g.buf0[x]);
        st_coh(g.buf1 + last + x, g.buf0[last + x]);
    }
    for (int y = 1 + lane; y < ny - 1; y += 64) {
        const size_t r = (size_t)y * nx;
        st_coh(g.buf1 + r, g.buf0[r]);
        st_coh(g.buf1 + r + nx - 1, g.buf0[r + nx - 1]);
    }
}

template <typename T, bool BOX, int K, int H>
__global__ __launch_bounds__(TBW * 64) void stencil2d_tb_batched(TBBatchParams<T> p) {
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gw = blockIdx.x * TBW + wave, nw = gridDim.x * TBW;
    T w[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = p.w[k];
    GridSync gs;
    gs.init(p.sync);
    // each grid's ring goes to its second buffer with the wave of its first tile
    for (int t = gw; t < p.ntiles; t += nw) {
        const TBGrid<T> g = p.grids[tb_locate(p.grids, p.count, t)];
        if (t == g.tile_base) tb_copy_ring(g, lane);
    }
    int64_t blk = 0;
    for (int64_t s0 = 0; s0 < p.steps; s0 += K, ++blk) {
        const int kk = (int)std::min<int64_t>(K, p.steps - s0);
        for (int t = gw; t < p.ntiles; t += nw) {
            const TBGrid<T> g = p.grids[tb_locate(p.grids, p.count, t)];
            const gmem<T> *src = opaque((blk & 1) ? g.buf1 : g.buf0);
            gmem<T> *dst = opaque((blk & 1) ? g.buf0 : g.buf1);
            tb_tile<T, BOX, K, H, true>(src, dst, g.nx, g.ny, g.ntx, t - g.tile_base, kk, lane, w);
        }
        gs.sync();
    }
    if (blk & 1) {
        for (int t = gw; t < p.ntiles; t += nw) {
            const TBGrid<T> g = p.grids[tb_locate(p.grids, p.count, t)];
            tb_copy_back<K, H>(g.buf0, g.buf1, g.nx, g.ny, g.ntx, t - g.tile_base, lane);
        }
    }
    gs.finish();
}

template <typename T, bool BOX, int K>
const void *pick_tb_h(int h) {
    switch (h) {
        case 8: return reinterpret_cast<const void *>(&stencil2d_tb<T, BOX, K, 8>);
        case 16: return reinterpret_cast<const void *>(&stencil2d_tb<T, BOX, K, 16>);
        default: return nullptr;
    }
}

template <typename T, bool BOX>
const void *pick_tb(int k, int h) {
    switch (k) {
        case 2: return pick_tb_h<T, BOX, 2>(h);
        case 4: return pick_tb_h<T, BOX, 4>(h);
        case 8: return pick_tb_h<T, BOX, 8>(h);
        default: return nullptr;
    }
}

// Register-resident instantiations: the small-grid tiles, and 32- and
// 56-row tiles for large grids (whose tiles must all be co-resident).
template <typename T, bool BOX>
const void *pick_tbr(int k, int h) {
#define PERKS_TBR(K_, H_) \
    if (k == K_ && h == H_) return reinterpret_cast<const void *>(&stencil2d_tbr<T, BOX, K_, H_>);
    PERKS_TBR(2, 8) PERKS_TBR(4, 8) PERKS_TBR(8, 8) PERKS_TBR(2, 16) PERKS_TBR(4, 16) PERKS_TBR(8, 16)
    PERKS_TBR(2, 32) PERKS_TBR(4, 32) PERKS_TBR(2, 56) PERKS_TBR(4, 56)
#undef PERKS_TBR
    return nullptr;
}

template <typename T, bool BOX>
const void *pick_tb_batched(int k, int h) {
    if (k == 4 && h == 16) return reinterpret_cast<const void *>(&stencil2d_tb_batched<T, BOX, 4, 16>);
    if (k == 8 && h == 16) return reinterpret_cast<const void *>(&stencil2d_tb_batched<T, BOX, 8, 16>);
    return nullptr;
}

struct PlanTB {
    int k = 0, h = 0, ntx = 0, nty = 0, wgs = 0;
    bool resident = false;   // stencil2d_tbr: every tile in its own wave's registers
    const void *fn = nullptr;
};

template <typename T>
int plan_tb(const perks_shape &s, bool box, const perks_tuning *tu, PlanTB *pl) {
    if (s.ndim != 2) return set_error(PERKS_E_UNSUPPORTED, "the temporally blocked kernel is 2D");
    // defaults measured on MI355X (2d5pt and 2d9pt, FP64 and FP32, register
    // resident): up to 2^18 interior cells K = 8 on 8-row tiles (256^2: 1.25
    // us per step FP64), up to 2^20 K = 8 on 16-row tiles (1024^2: 2.05 us
    // FP64, 1.65 FP32), above that K = 4 on 56-row tiles, which only the
    // resident kernel has (3072^2: 6.7 us per step FP64, 5.4 FP32); a grid
    // whose 56-row tiles do not all fit takes 8-row streamed tiles when asked
    // for temporal blocking
    const int64_t interior = (s.nx - 2) * (s.ny - 2);
    const bool hdef = !(tu && tu->rows_per_lane > 0);
    pl->k = (tu && tu->steps_per_sync > 0) ? tu->steps_per_sync : (interior < (int64_t(1) << 20) ? 8 : 4);
    pl->h = !hdef ? tu->rows_per_lane
                  : interior <= (int64_t(1) << 18) ? 8 : interior < (int64_t(1) << 20) ? 16 : 56;
    // max_cached_tiles < 0 keeps the grid in its buffers (streamed blocks);
    // a positive cap below the tile count does too
    const int64_t cap_tiles = (tu && tu->max_cached_tiles != 0) ? tu->max_cached_tiles : INT64_MAX;
    if (tu && tu->waves_per_wg != 0 && tu->waves_per_wg != TBW)
        return set_error(PERKS_E_UNSUPPORTED, "the temporally blocked kernel uses %d waves per workgroup", TBW);
    if (tu && tu->sync != 0 && tu->sync != 1)
        return set_error(PERKS_E_UNSUPPORTED, "the temporally blocked kernel synchronises with a grid barrier");
    const int ow = 64 - 2 * pl->k;
    pl->ntx = (int)((s.nx - 2 + ow - 1) / ow);
    pl->nty = (int)((s.ny - 2 + pl->h - 1) / pl->h);
    int64_t tiles = (int64_t)pl->ntx * pl->nty;
    if (tiles > INT32_MAX) return set_error(PERKS_E_UNSUPPORTED, "grid too large for this kernel");
    DeviceFacts f;
    int rc = device_facts(&f);
    if (rc) return rc;
    int occ = 0;
    // the register-resident kernel when every tile gets a wave of its own
    const void *fr = box ? pick_tbr<T, true>(pl->k, pl->h) : pick_tbr<T, false>(pl->k, pl->h);
    if (fr && tiles <= cap_tiles) {
        PERKS_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fr, TBW * 64, 0));
        const int wpc = (tu && tu->wgs_per_cu > 0) ? std::min(tu->wgs_per_cu, occ) : occ;
        if (occ >= 1 && tiles <= (int64_t)f.cus * wpc * TBW) {
            pl->resident = true;
            pl->fn = fr;
            pl->wgs = (int)((tiles + TBW - 1) / TBW);
            return PERKS_OK;
        }
    }
    pl->fn = box ? pick_tb<T, true>(pl->k, pl->h) : pick_tb<T, false>(pl->k, pl->h);
    if (!pl->fn && hdef) {   // the default depth is resident only: stream 8-row tiles instead
        pl->h = 8;
        pl->nty = (int)((s.ny - 2 + pl->h - 1) / pl->h);
        tiles = (int64_t)pl->ntx * pl->nty;
        if (tiles > INT32_MAX) return set_error(PERKS_E_UNSUPPORTED, "grid too large for this kernel");
        pl->fn = box ? pick_tb<T, true>(pl->k, pl->h) : pick_tb<T, false>(pl->k, pl->h);
    }
    if (!pl->fn)
        return set_error(PERKS_E_UNSUPPORTED, fr ? "temporal blocking with %d rows per lane needs every tile "
                                                   "co-resident (steps_per_sync %d)"
                                                 : "temporal blocking takes steps_per_sync 2, 4 or 8 and "
                                                   "rows_per_lane 8, 16, 32 or 56 (got %d, %d)",
                         fr ? pl->h : pl->k, fr ? pl->k : pl->h);
    PERKS_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, pl->fn, TBW * 64, 0));
    if (occ < 1) return set_error(PERKS_E_NOTCORESIDENT, "temporally blocked kernel does not fit a CU");
    const int wpc = (tu && tu->wgs_per_cu > 0) ? std::min(tu->wgs_per_cu, occ) : occ;
    pl->wgs = (int)std::max<int64_t>(1, std::min<int64_t>((tiles + TBW - 1) / TBW, (int64_t)f.cus * wpc));
    return PERKS_OK;
}

}  // namespace

template <typename T>
int run2d_tb(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, bool box, hipStream_t st,
             const perks_tuning *tu) {
    PlanTB pl;
    int rc = plan_tb<T>(s, box, tu, &pl);
    if (rc) return rc;
    const size_t cells = (size_t)s.nx * s.ny;
    T *other = (T *)scratch(SLOT_WIDE, cells * sizeof(T));
    unsigned *sync = (unsigned *)scratch(SLOT_SYNC, SYNC_BYTES);
    if (!other || !sync) return PERKS_E_NOMEM;
    // the second buffer needs the fixed ring: copy the whole grid once
    PERKS_HIP_TRY(hipMemcpyAsync(other, grid, cells * sizeof(T), hipMemcpyDeviceToDevice, st));
    TB2DParams<T> p{};
    p.buf0 = to_global(grid);
    p.buf1 = to_global(other);
    p.sync = sync;
    p.steps = steps;
    p.nx = (int)s.nx;
    p.ny = (int)s.ny;
    p.ntx = pl.ntx;
    p.nty = pl.nty;
    for (int k = 0; k < 9; ++k) p.w[k] = (T)coeffs[k];
    return launch_coop(pl.fn, pl.wgs, TBW * 64, &p, st);
}

namespace {

// Batched grids: K steps per exchange and 16-row tiles (throughput: the
// fewest bytes per step, the blocks' reads and writes spread over every
// grid's tiles).
constexpr int TB_BATCH_K = 8, TB_BATCH_H = 16;

// The grid table of a batch (second buffers carved from `other`, 64-element
// aligned), the kernel, its grid size and the bytes of second buffers.
template <typename T>
struct TBBatchShape {
    std::vector<TBGrid<T>> g;
    int64_t tiles = 0;
    size_t cells = 0;   // elements of the second buffers
    const void *fn = nullptr;
    int wgs = 0;
};

template <typename T>
int tb_batch_shape(T *const *grids, const perks_shape *shapes, int count, bool box, TBBatchShape<T> *b) {
    b->fn = box ? pick_tb_batched<T, true>(TB_BATCH_K, TB_BATCH_H) : pick_tb_batched<T, false>(TB_BATCH_K, TB_BATCH_H);
    DeviceFacts f;
    int rc = device_facts(&f);
    if (rc) return rc;
    int occ = 0;
    PERKS_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, b->fn, TBW * 64, 0));
    if (occ < 1) return set_error(PERKS_E_NOTCORESIDENT, "batched temporally blocked kernel does not fit a CU");
    constexpr int OW = 64 - 2 * TB_BATCH_K;
    b->g.assign(count, TBGrid<T>{});
    for (int i = 0; i < count; ++i) {
        TBGrid<T> &g = b->g[i];
        g.nx = (int)shapes[i].nx;
        g.ny = (int)shapes[i].ny;
        g.ntx = (int)((shapes[i].nx - 2 + OW - 1) / OW);
        const int nty = (int)((shapes[i].ny - 2 + TB_BATCH_H - 1) / TB_BATCH_H);
        g.tile_base = (int)b->tiles;
        g.buf0 = to_global(grids[i]);
        b->tiles += (int64_t)g.ntx * nty;
        b->cells += ((size_t)shapes[i].nx * shapes[i].ny + 63) / 64 * 64;
        if (b->tiles > INT32_MAX) return set_error(PERKS_E_UNSUPPORTED, "batch too large for this kernel");
    }
    b->wgs = (int)std::max<int64_t>(1, std::min<int64_t>((b->tiles + TBW - 1) / TBW, (int64_t)f.cus * occ));
    return PERKS_OK;
}

template <typename T>
void tb_batch_carve(TBBatchShape<T> *b, T *other) {
    for (TBGrid<T> &g : b->g) {
        g.buf1 = to_global(other);
        other += ((size_t)g.nx * g.ny + 63) / 64 * 64;
    }
}

template <typename T>
TBBatchParams<T> tb_batch_params(const TBBatchShape<T> &b, const TBGrid<T> *table, unsigned *sync, int64_t steps,
                                 const double *coeffs) {
    TBBatchParams<T> p{};
    p.grids = table;
    p.count = (int)b.g.size();
    p.ntiles = (int)b.tiles;
    p.sync = sync;
    p.steps = steps;
    for (int k = 0; k < 9; ++k) p.w[k] = (T)coeffs[k];
    return p;
}

__global__ __launch_bounds__(256) void tb_zero_words(unsigned *w, int m) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < m) w[i] = 0u;
}

}  // namespace

template <typename T>
int run2d_tb_batched(T *const *grids, const perks_shape *shapes, int count, const double *coeffs, int64_t steps,
                     bool box, hipStream_t st) {
    TBBatchShape<T> b;
    int rc = tb_batch_shape(grids, shapes, count, box, &b);
    if (rc) return rc;
    const size_t meta = (sizeof(TBGrid<T>) * count + 255) / 256 * 256;
    char *blk = (char *)scratch(SLOT_WIDE, meta + b.cells * sizeof(T));
    unsigned *sync = (unsigned *)scratch(SLOT_SYNC, SYNC_BYTES);
    if (!blk || !sync) return PERKS_E_NOMEM;
    tb_batch_carve(&b, (T *)(blk + meta));
    PERKS_HIP_TRY(hipStreamSynchronize(st));   // the block may still be read by an earlier launch
    PERKS_HIP_TRY(hipMemcpy(blk, b.g.data(), sizeof(TBGrid<T>) * count, hipMemcpyHostToDevice));
    TBBatchParams<T> p = tb_batch_params(b, (const TBGrid<T> *)blk, sync, steps, coeffs);
    return launch_coop(b.fn, b.wgs, TBW * 64, &p, st);
}


// A batch plan: its own device block (barrier words, grid table, second
// buffers) and its launch as a one-node HIP graph with the cooperative
// attribute (or a direct cooperative launch where the runtime refuses one).
struct StencilBatchPlan {
    int device = -1;
    bool f64 = false;
    void *mem = nullptr;
    unsigned *sync = nullptr;
    const void *fn = nullptr;
    int wgs = 0, count = 0;
    int64_t steps = 0;
    uint64_t epochs_used = 0;
    TBBatchParams<float> pf{};
    TBBatchParams<double> pd{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

template <typename T>
int tb_batch_create(T *const *grids, const perks_shape *shapes, int count, const double *coeffs, int64_t steps,
                    bool box, StencilBatchPlan **out) {
    *out = nullptr;
    TBBatchShape<T> b;
    int rc = tb_batch_shape(grids, shapes, count, box, &b);
    if (rc) return rc;
    auto *P = new (std::nothrow) StencilBatchPlan();
    if (!P) return set_error(PERKS_E_NOMEM, "plan allocation failed");
    (void)hipGetDevice(&P->device);
    P->f64 = sizeof(T) == 8;
    P->fn = b.fn;
    P->wgs = b.wgs;
    P->count = count;
    P->steps = steps;
    const size_t meta = (sizeof(TBGrid<T>) * count + 255) / 256 * 256;
    const size_t bytes = SYNC_BYTES + meta + b.cells * sizeof(T);
    do {
        if (hipMalloc(&P->mem, bytes) != hipSuccess) {
            (void)hipGetLastError();
            P->mem = nullptr;
            rc = set_error(PERKS_E_NOMEM, "batch plan: hipMalloc of %zu bytes failed", bytes);
            break;
        }
        char *base = (char *)P->mem;
        P->sync = (unsigned *)base;
        tb_batch_carve(&b, (T *)(base + SYNC_BYTES + meta));
        if (hipMemset(P->mem, 0, SYNC_BYTES) != hipSuccess ||
            hipMemcpy(base + SYNC_BYTES, b.g.data(), sizeof(TBGrid<T>) * count, hipMemcpyHostToDevice) !=
                hipSuccess) {
            (void)hipGetLastError();
            rc = set_error(PERKS_E_HIP, "batch plan: uploading the grid table failed");
            break;
        }
        const TBBatchParams<T> p = tb_batch_params(b, (const TBGrid<T> *)(base + SYNC_BYTES), P->sync, steps, coeffs);
        void *args[1];
        if constexpr (sizeof(T) == 8) {
            P->pd = p;
            args[0] = &P->pd;
        } else {
            P->pf = p;
            args[0] = &P->pf;
        }
        hipKernelNodeParams kp{};
        kp.func = const_cast<void *>(P->fn);
        kp.gridDim = dim3(P->wgs);
        kp.blockDim = dim3(TBW * 64);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        hipGraphNode_t node;
        hipLaunchAttributeValue v{};
        v.cooperative = 1;
        if (hipGraphCreate(&P->graph, 0) != hipSuccess ||
            hipGraphAddKernelNode(&node, P->graph, nullptr, 0, &kp) != hipSuccess ||
            hipGraphKernelNodeSetAttribute(node, hipKernelNodeAttributeCooperative, &v) != hipSuccess ||
            hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGetLastError();
            if (P->exec) (void)hipGraphExecDestroy(P->exec);
            if (P->graph) (void)hipGraphDestroy(P->graph);
            P->exec = nullptr;
            P->graph = nullptr;
        }
    } while (false);
    if (rc) {
        tb_batch_destroy(P);
        return rc;
    }
    *out = P;
    return PERKS_OK;
}

int tb_batch_run(StencilBatchPlan *P, hipStream_t st) {
    if (P->count == 0 || P->steps == 0) return PERKS_OK;
    // barrier epochs are 32-bit: start again from zeroed words well before
    // they could wrap (a fill kernel, so the reset is stream-ordered)
    const uint64_t per_run = (uint64_t)(P->steps / TB_BATCH_K + 2);
    P->epochs_used += per_run;
    if (P->epochs_used > (uint64_t(1) << 31)) {
        hipLaunchKernelGGL(tb_zero_words, dim3((SYNC_BYTES / 4 + 255) / 256), dim3(256), 0, st, P->sync,
                           (int)(SYNC_BYTES / 4));
        P->epochs_used = per_run;
    }
    note_persistent_launch(P->wgs, P->sync);
    if (P->exec) {
        PERKS_HIP_TRY(hipGraphLaunch(P->exec, st));
        return PERKS_OK;
    }
    void *args[1] = {P->f64 ? (void *)&P->pd : (void *)&P->pf};
    const hipError_t e = hipLaunchCooperativeKernel(P->fn, dim3(P->wgs), dim3(TBW * 64), args, 0, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(e == hipErrorCooperativeLaunchTooLarge ? PERKS_E_NOTCORESIDENT : PERKS_E_HIP,
                         "batched stencil launch: %s", hipGetErrorString(e));
    }
    return PERKS_OK;
}

int tb_batch_graph(StencilBatchPlan *P, void **graph) {
    if (!P->graph) return set_error(PERKS_E_UNSUPPORTED, "the runtime refused a cooperative graph node");
    *graph = (void *)P->graph;
    return PERKS_OK;
}

void tb_batch_destroy(StencilBatchPlan *P) {
    if (!P) return;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->mem) {
        forget_persistent_launch(P->sync);
        (void)hipDeviceSynchronize();
        (void)hipFree(P->mem);
    }
    delete P;
}

template <typename T>
int plan2d_tb_query(const perks_shape &s, bool box, const perks_tuning *tu, perks_stencil_plan *plan) {
    PlanTB pl;
    int rc = plan_tb<T>(s, box, tu, &pl);
    if (rc) return rc;
    const int64_t tiles = (int64_t)pl.ntx * pl.nty;
    const int64_t rb = pl.h + 2 * pl.k, ow = 64 - 2 * pl.k;
    plan->wgs = pl.wgs;
    plan->waves_per_wg = TBW;
    plan->rows_per_lane = pl.h;
    plan->planes_per_lane = 1;
    plan->tiles = tiles;
    plan->interior_cells = (s.nx - 2) * (s.ny - 2);
    if (pl.resident) {
        // every tile in registers; per block its band stored and its ghost ring loaded
        plan->cached_tiles = tiles;
        plan->cached_cells = plan->interior_cells;
        const int64_t k2 = 2 * pl.k;
        plan->halo_bytes_per_step =
            tiles * (k2 * ow + k2 * (pl.h - k2) + k2 * 64 + k2 * pl.h) * (int64_t)sizeof(T) / pl.k;
    } else {
        // between blocks the grid lives in its two buffers: each tile's block
        // read and its owned cells written, once per K steps
        plan->cached_tiles = 0;
        plan->cached_cells = 0;
        plan->halo_bytes_per_step = tiles * (64 * rb + ow * pl.h) * (int64_t)sizeof(T) / pl.k;
    }
    plan->sync = 3;
    plan->lds_rows_per_lane = 0;
    return PERKS_OK;
}

template int run2d_tb<float>(float *, const double *, const perks_shape &, int64_t, bool, hipStream_t,
                             const perks_tuning *);
template int run2d_tb<double>(double *, const double *, const perks_shape &, int64_t, bool, hipStream_t,
                              const perks_tuning *);
template int plan2d_tb_query<float>(const perks_shape &, bool, const perks_tuning *, perks_stencil_plan *);
template int run2d_tb_batched<float>(float *const *, const perks_shape *, int, const double *, int64_t, bool,
                                     hipStream_t);
template int tb_batch_create<float>(float *const *, const perks_shape *, int, const double *, int64_t, bool,
                                    StencilBatchPlan **);
template int tb_batch_create<double>(double *const *, const perks_shape *, int, const double *, int64_t, bool,
                                     StencilBatchPlan **);
template int run2d_tb_batched<double>(double *const *, const perks_shape *, int, const double *, int64_t, bool,
                                      hipStream_t);
template int plan2d_tb_query<double>(const perks_shape &, bool, const perks_tuning *, perks_stencil_plan *);

}  // namespace perks
