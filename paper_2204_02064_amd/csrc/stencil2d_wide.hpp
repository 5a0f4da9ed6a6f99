// 2D Jacobi stencils of radius 2 to 4 (the rest of tab:domain's 2D suite:
// the 2ds9pt, 2d13pt and 2d17pt stars, radius 2, 3 and 4, and the 2d25pt
// box, radius 2): the persistent kernel and the per-step baseline, both built
// on one tile routine so that they round identically.
//
// Tiling.  The interior (cells at distance >= r from the border; the ring of
// width r is the fixed Dirichlet boundary) is cut into wave tiles of 64
// columns x RC rows.  Lane l owns column x0+l and keeps the tile's RC cells
// of that column in registers (Sec. 4.2.1's vertical run per thread).
// Neighbours up to r rows away are in the lane's own registers or in the r
// halo rows above and below; neighbours up to r columns away arrive by r
// chained DPP lane shifts, the k-th shift feeding the edge lane the halo
// column at distance k (so after k shifts lane 0 holds x0-k and lane j < k
// the halo column at distance k-j).
//
// Halo exchange.  The grid's own two buffers serve as the face buffers: step
// s reads buffer s%2 and writes buffer (s+1)%2; a cached tile writes only its
// edge band (the r outermost rows and columns of its valid cells) there, and
// neighbours read their halo rows (coalesced) and halo columns (staged in LDS
// through the wave) from it after the step's device barrier.  Cells past a
// ragged tile's last valid row or column hold the grid's own values there
// (ring cells, which never change) and are never updated.
//
// Cache mode.  When every tile has its own wavefront (tiles <= co-resident
// waves) the tile stays in registers for the whole launch and HBM carries
// only the edge bands.  Otherwise every tile streams: read from buffer s%2,
// written whole to buffer (s+1)%2, one barrier per step (the per-step
// baseline fused into one launch).
#pragma once

#include <type_traits>
#include <utility>

#include "barrier.hpp"
#include "common.hpp"

namespace perks {

template <typename T, int R>
struct WideW {
    T w[(2 * R + 1) * (2 * R + 1)];   // [dy + R][dx + R]
};

template <typename T, int R>
struct Wide2DParams {
    gmem<T> *buf0;    // the caller's grid
    gmem<T> *buf1;    // second buffer of the same extents (ring copied in)
    unsigned *sync;   // barrier words
    int64_t steps;
    int nx, ny;       // full extents
    int ntx, nty;     // tiles along x and y
    int cached;       // 1: one tile per wave kept in registers; 0: all tiles stream
    gmem<T> *cols;    // cached: two step-parity copies of every tile's edge-column block
    WideW<T, R> W;
};

// Rows per lane of the tile (RC) and their valid count on this tile.
struct WideTile {
    int x0, y0, wx, hy;
};

template <int RC>
__device__ __forceinline__ WideTile wide_tile_of(int t, int ntx, int nx, int ny, int r) {
    WideTile tl;
    const int tx = t % ntx, ty = t / ntx;
    tl.x0 = r + 64 * tx;
    tl.y0 = r + RC * ty;
    tl.wx = min(64, nx - r - tl.x0);
    tl.hy = min(RC, ny - r - tl.y0);
    return tl;
}

// One Jacobi step of a lane's strip: u[i] is the old value of row y0+i on
// entry and its new value on exit.  hr (LDS, this lane's column, stride 64):
// entry k < R is old row y0-R+k, entry R+k old row y0+RC+k (held in LDS
// rather than registers, which the cache needs).  cw / ce (LDS): the halo
// column at distance k+1 west / east of
// the tile, row j at [k*NJ + j + J0] (J0 = R: rows -R .. RC+R-1 for the box;
// J0 = 0: rows 0 .. RC-1 for a star).  A new value is the sum over dy
// ascending, then dx ascending, of w[dy][dx] * old[y+dy][x+dx], its first
// term a product and the others FMAs.  Rows i >= hy, and every row of a lane
// with !live, keep their old values.
//
// Old rows are visited once each, top to bottom; each is shifted sideways
// (r DPP moves per direction) and its products are added to the 2r+1 new
// rows it touches, whose accumulators roll through 2r+1 registers.  New row
// i is complete once old row i+r has been visited; by then old row i has
// been consumed, so the new value takes its register.
//
// ACC selects the 3D use (one z layer of a 3D stencil): the new values are
// not written into u but added to out (FIRST: out = the layer's sum); wt(dy,
// dx) returns the layer's weight.
template <typename T, int R, bool BOX, int RC, bool ACC = false, bool FIRST = false, class WF>
__device__ __forceinline__ void wide_rows_impl(T (&u)[RC], const T *hr, const T *cw, const T *ce, WF &&wt, int hy,
                                               bool live, T (&out)[RC]) {
    constexpr int S = 2 * R + 1;
    constexpr int NJ = BOX ? RC + 2 * R : RC;
    constexpr int J0 = BOX ? R : 0;
    constexpr int JS = BOX ? -R : 0;   // first row that is shifted sideways
    T acc[S];
    // the halo columns of the next shifted row are read from LDS one row
    // ahead, so their latency overlaps this row's arithmetic
    T hw[R], he[R];
    static_for<0, R>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        hw[k] = cw[k * NJ + JS + J0];
        he[k] = ce[k * NJ + JS + J0];
    });
    T vn = hr[0];   // the next halo row's value, read one row ahead
    static_for<0, RC + 2 * R>([&](auto jc) {
        constexpr int j = decltype(jc)::value - R;   // old row, -R .. RC+R-1
        T v;
        if constexpr (j < 0 || j >= RC) v = vn;
        else v = u[j];
        constexpr int jn = j + 1;
        if constexpr (jn < 0) vn = hr[(jn + R) * 64];
        else if constexpr (jn >= RC && jn < RC + R) vn = hr[(R + jn - RC) * 64];
        constexpr bool SIDE = BOX || (j >= 0 && j < RC);
        constexpr bool NEXT = BOX ? j + 1 < RC + R : (j + 1 >= 0 && j + 1 < RC);
        T sh[S];   // sh[dx + R] = old[j][x + dx]
        sh[R] = v;
        if constexpr (SIDE) {
            T cwk[R], cek[R];
            static_for<0, R>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                cwk[k] = hw[k];
                cek[k] = he[k];
                if constexpr (NEXT) {
                    hw[k] = cw[k * NJ + j + 1 + J0];
                    he[k] = ce[k * NJ + j + 1 + J0];
                }
            });
            T a = v, b = v;
            static_for<1, R + 1>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                a = from_west(a, cwk[k - 1]);
                b = from_east(b, cek[k - 1]);
                sh[R - k] = a;
                sh[R + k] = b;
            });
        }
        // add old row j's terms to new rows i = j - dy, dy = R .. -R
        static_for<0, S>([&](auto dc) {
            constexpr int dy = R - decltype(dc)::value;
            constexpr int i = j - dy;
            if constexpr (i >= 0 && i < RC) {
                constexpr int slot = i % S;
                if constexpr (BOX) {
                    static_for<0, S>([&](auto xc) {
                        constexpr int dx = decltype(xc)::value - R;
                        const T w = wt(dy, dx);
                        if constexpr (dy == -R && dx == -R) acc[slot] = w * sh[dx + R];
                        else acc[slot] = fma_t(w, sh[dx + R], acc[slot]);
                    });
                } else if constexpr (dy == 0) {
                    static_for<0, S>([&](auto xc) {
                        constexpr int dx = decltype(xc)::value - R;
                        acc[slot] = fma_t(wt(0, dx), sh[dx + R], acc[slot]);
                    });
                } else {
                    const T w = wt(dy, 0);
                    if constexpr (dy == -R) acc[slot] = w * v;
                    else acc[slot] = fma_t(w, v, acc[slot]);
                }
            }
        });
        if constexpr (j - R >= 0 && j - R < RC) {
            constexpr int i = j - R;
            if constexpr (!ACC) u[i] = (live && i < hy) ? acc[i % S] : u[i];
            else if constexpr (FIRST) out[i] = acc[i % S];
            else out[i] = out[i] + acc[i % S];
        }
        // this row's products are computed here: without the tie the
        // compiler sinks every row's FMAs below all the shifts, keeping each
        // row's shifted values live at once
        settle(acc);
    });
}

template <typename T, int R, bool BOX, int RC>
__device__ __forceinline__ void wide_rows(T (&u)[RC], const T *hr, const T *cw, const T *ce, const WideW<T, R> &W,
                                          int hy, bool live) {
    constexpr int S = 2 * R + 1;
    wide_rows_impl<T, R, BOX, RC>(u, hr, cw, ce, [&](int dy, int dx) { return W.w[(dy + R) * S + dx + R]; }, hy,
                                  live, u);
}

// Element offset of (row y, column x) with both clamped into the grid (reads
// past a ragged tile's edge land on the ring and are never used).
__device__ __forceinline__ size_t wide_at(int y, int x, int nx, int ny) {
    return (size_t)min(y, ny - 1) * (size_t)nx + (size_t)min(x, nx - 1);
}

// Start of row y (clamped into the grid) of a buffer; y and the tile
// geometry are wave-uniform, so this is a scalar address and each access
// adds only the lane's column.
template <typename P>
__device__ __forceinline__ P wide_row(P buf, int y, int nx, int ny) {
    return buf + (size_t)min(y, ny - 1) * (size_t)nx;
}

// Loads the halo of one tile from `src`: the R rows above and below into
// registers, the R columns on each side into the wave's LDS (k fastest, so
// that R neighbouring lanes read one row's R cells together). Where `cwb`
// (`ceb`) is given, the west (east) columns of the tile's own rows come from
// that neighbour's edge-column block instead ([k][row], written by
// wide_cols_store), read with contiguous lanes; corners and rows past a
// ragged tile's end still come from `src`.
template <typename T, int R, bool BOX, int RC>
__device__ __forceinline__ void wide_halo(const gmem<T> *src, const WideTile &tl, int nx, int ny, int lane, T *hr,
                                          T *cw, T *ce, const gmem<T> *cwb = nullptr,
                                          const gmem<T> *ceb = nullptr) {
    constexpr int NJ = BOX ? RC + 2 * R : RC;
    constexpr int J0 = BOX ? R : 0;
    const int xl = min(tl.x0 + lane, nx - 1);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        hr[k * 64] = ld_coh(wide_row(src, tl.y0 - R + k, nx, ny) + xl);
        hr[(R + k) * 64] = ld_coh(wide_row(src, tl.y0 + RC + k, nx, ny) + xl);
    }
    constexpr int PER_SIDE = R * NJ;
#pragma unroll
    for (int e0 = 0; e0 < 2 * PER_SIDE; e0 += 64) {
        const int e = e0 + lane;
        if (e < 2 * PER_SIDE) {
            const int side = e >= PER_SIDE;
            const int rem = e - side * PER_SIDE;
            const int jj = rem / R, k = rem - jj * R;
            const bool banded = (side ? ceb : cwb) != nullptr && jj >= J0 && jj < J0 + tl.hy;
            if (!banded) {
                const int y = max(tl.y0 + jj - J0, 0);
                const int x = side ? tl.x0 + 64 + k : tl.x0 - 1 - k;
                const T val = ld_coh(src + wide_at(y, x, nx, ny));
                (side ? ce : cw)[k * NJ + jj] = val;
            }
        }
    }
    if (cwb || ceb) {
        constexpr int BAND = R * RC;
#pragma unroll
        for (int e0 = 0; e0 < 2 * BAND; e0 += 64) {
            const int e = e0 + lane;
            if (e < 2 * BAND) {
                const int side = e >= BAND;
                const int rem = e - side * BAND;
                const int k = rem / RC, i = rem - k * RC;
                const gmem<T> *b = side ? ceb : cwb;
                if (b && i < tl.hy) (side ? ce : cw)[k * NJ + J0 + i] = ld_coh(b + rem);
            }
        }
    }
    compiler_fence();
}

// Writes the tile's R westmost and R eastmost columns (lanes k and 63 - k,
// all RC rows) as one contiguous block [side][k][row] for the neighbours'
// next step. The block is transposed through the wave's LDS (`stage`, at
// least 2 R RC elements, free once the step's rows are done) so that the
// store is coalesced instead of one cell per row.
template <typename T, int R, int RC>
__device__ __forceinline__ void wide_cols_store(gmem<T> *blk, int lane, const T (&u)[RC], T *stage) {
    constexpr int BAND = R * RC;
    const bool west = lane < R, east = lane >= 64 - R;
    if (west || east) {
        T *q = stage + (west ? lane * RC : BAND + (63 - lane) * RC);
#pragma unroll
        for (int i = 0; i < RC; ++i) q[i] = u[i];
    }
    compiler_fence();
#pragma unroll
    for (int e0 = 0; e0 < 2 * BAND; e0 += 64) {
        const int e = e0 + lane;
        if (e < 2 * BAND) st_coh(blk + e, stage[e]);
    }
    compiler_fence();
}

template <typename T, int RC>
__device__ __forceinline__ void wide_load(const gmem<T> *src, const WideTile &tl, int nx, int ny, int lane,
                                          T (&u)[RC]) {
    const int xl = min(tl.x0 + lane, nx - 1);
#pragma unroll
    for (int i = 0; i < RC; ++i) u[i] = ld_coh(wide_row(src, tl.y0 + i, nx, ny) + xl);
}

// Stores the tile's valid cells (EDGE: only those within R of the tile's
// valid edges, the cells its neighbours read; ROWS: of those only the R top
// and bottom rows, the side columns going through wide_cols_store).
template <typename T, int R, int RC, bool EDGE, bool COH, bool ROWS = false>
__device__ __forceinline__ void wide_store(gmem<T> *dst, const WideTile &tl, int nx, int lane, const T (&u)[RC]) {
    const bool lane_ok = lane < tl.wx;
    const bool side = !ROWS && (lane < R || lane >= tl.wx - R);
#pragma unroll
    for (int i = 0; i < RC; ++i) {
        bool ok = lane_ok && i < tl.hy;
        if (EDGE) ok = ok && (side || i < R || i >= tl.hy - R);
        if (ok) {
            gmem<T> *q = dst + (size_t)(tl.y0 + i) * (size_t)nx + tl.x0;
            if (COH) st_coh(q + lane, u[i]);
            else q[lane] = u[i];
        }
    }
}

template <typename T, int R, bool BOX, int RC>
struct WideLds {
    static constexpr int NJ = BOX ? RC + 2 * R : RC;
    T c[2][R * NJ];   // west / east halo columns
    T rows[2 * R][64];   // halo rows above (k < R) and below
};

// Waves per SIMD a tile depth is built for (the register budget of a wave is
// 512 / that): deeper tiles hold more of the grid per wave, shallower ones
// leave more waves to hide each row's latency. The shallowest depth runs
// five FP64 or six FP32 waves per SIMD.
template <typename T, int RC>
struct WideOcc {
    static constexpr int value = RC <= 24 ? (sizeof(T) == 4 ? 6 : 5) : RC <= 32 ? 4 : RC <= 48 ? 3 : 2;
};

// Whether cached tiles exchange their side columns as contiguous blocks
// (wide_cols_store). Off for FP64 radius 4, whose kernels it pushes further
// past the register budget (measured slower there).
template <typename T, int R>
constexpr bool wide_cols_on() {
    return !(sizeof(T) == 8 && R >= 4);
}

template <typename T, int R, bool BOX, int RC, int WAVES>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(WideOcc<T, RC>::value))) void
stencil2d_wide(Wide2DParams<T, R> p) {
    __shared__ WideLds<T, R, BOX, RC> lds[WAVES];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gw = blockIdx.x * WAVES + wave, nw = gridDim.x * WAVES;
    const int ntiles = p.ntx * p.nty;
    constexpr int BAND2 = 2 * R * RC;   // one tile's edge-column block
    T *cw = lds[wave].c[0], *ce = lds[wave].c[1];   // contiguous: cw also stages BAND2 elements
    GridSync gs;
    gs.init(p.sync);
    T u[RC];
    T *hr = &lds[wave].rows[0][lane];
    if (p.cached && gw < ntiles) {
        const WideTile tl = wide_tile_of<RC>(gw, p.ntx, p.nx, p.ny, R);
        wide_load<T, RC>(p.buf0, tl, p.nx, p.ny, lane, u);
    }
    for (int64_t s = 0; s < p.steps; ++s) {
        const gmem<T> *src = opaque((s & 1) ? p.buf1 : p.buf0);
        gmem<T> *dst = opaque((s & 1) ? p.buf0 : p.buf1);
        for (int t = gw; t < ntiles; t += nw) {
            const WideTile tl = wide_tile_of<RC>(t, p.ntx, p.nx, p.ny, R);
            if (!p.cached) wide_load<T, RC>(src, tl, p.nx, p.ny, lane, u);
            // cached tiles after the first step: side columns from the
            // neighbours' blocks of the previous step (step 0 reads the
            // caller's grid, which holds every cell)
            const gmem<T> *cwb = nullptr, *ceb = nullptr;
            if (wide_cols_on<T, R>() && p.cols && s > 0) {
                const int tx = t % p.ntx;
                const gmem<T> *blocks = p.cols + (size_t)(s & 1) * ntiles * BAND2;
                if (tx > 0) cwb = blocks + (size_t)(t - 1) * BAND2 + R * RC;
                if (tx < p.ntx - 1) ceb = blocks + (size_t)(t + 1) * BAND2;
            }
            wide_halo<T, R, BOX, RC>(src, tl, p.nx, p.ny, lane, hr, cw, ce, cwb, ceb);
            wide_rows<T, R, BOX, RC>(u, hr, cw, ce, p.W, tl.hy, lane < tl.wx);
            if (wide_cols_on<T, R>() && p.cached && p.cols) {
                wide_store<T, R, RC, true, true, true>(dst, tl, p.nx, lane, u);
                wide_cols_store<T, R, RC>(p.cols + ((size_t)((s + 1) & 1) * ntiles + t) * BAND2, lane, u, cw);
            } else if (p.cached) {
                wide_store<T, R, RC, true, true>(dst, tl, p.nx, lane, u);
            } else {
                wide_store<T, R, RC, false, true>(dst, tl, p.nx, lane, u);
            }
        }
        gs.sync();
    }
    // results into the caller's grid (every read of the last step is done)
    if (p.cached) {
        if (gw < ntiles) {
            const WideTile tl = wide_tile_of<RC>(gw, p.ntx, p.nx, p.ny, R);
            wide_store<T, R, RC, false, false>(p.buf0, tl, p.nx, lane, u);
        }
    } else if (p.steps & 1) {
        for (int t = gw; t < ntiles; t += nw) {
            const WideTile tl = wide_tile_of<RC>(t, p.ntx, p.nx, p.ny, R);
            wide_load<T, RC>(p.buf1, tl, p.nx, p.ny, lane, u);
            wide_store<T, R, RC, false, false>(p.buf0, tl, p.nx, lane, u);
        }
    }
    gs.finish();
}

// Per-step baseline: one launch per step, one tile per wave, src -> dst.
template <typename T, int R>
struct Wide2DStep {
    const gmem<T> *src;
    gmem<T> *dst;
    int nx, ny, ntx, nty;
    WideW<T, R> W;
};

template <typename T, int R, bool BOX, int RC, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void stencil2d_wide_step(Wide2DStep<T, R> p) {
    __shared__ WideLds<T, R, BOX, RC> lds[WAVES];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = blockIdx.x * WAVES + wave;
    if (t >= p.ntx * p.nty) return;
    T *cw = lds[wave].c[0], *ce = lds[wave].c[1];
    const WideTile tl = wide_tile_of<RC>(t, p.ntx, p.nx, p.ny, R);
    T u[RC];
    T *hr = &lds[wave].rows[0][lane];
    wide_load<T, RC>(p.src, tl, p.nx, p.ny, lane, u);
    wide_halo<T, R, BOX, RC>(p.src, tl, p.nx, p.ny, lane, hr, cw, ce);
    wide_rows<T, R, BOX, RC>(u, hr, cw, ce, p.W, tl.hy, lane < tl.wx);
    wide_store<T, R, RC, false, false>(p.dst, tl, p.nx, lane, u);
}

// ---------------------------------------------------------------------------
// Host side.
constexpr int WW = 4;          // waves per workgroup (persistent)
constexpr int WWB = 4;         // waves per workgroup (baseline)
constexpr int WRB = 16;        // tile depth of the baseline
constexpr int WR_DEPTHS[4] = {24, 32, 48, 80};   // tile depths of the persistent kernel

template <typename T, int R, bool BOX>
const void *wide_fn(int rc) {
    switch (rc) {
        case 24: return reinterpret_cast<const void *>(&stencil2d_wide<T, R, BOX, 24, WW>);
        case 32: return reinterpret_cast<const void *>(&stencil2d_wide<T, R, BOX, 32, WW>);
        case 48: return reinterpret_cast<const void *>(&stencil2d_wide<T, R, BOX, 48, WW>);
        case 80: return reinterpret_cast<const void *>(&stencil2d_wide<T, R, BOX, 80, WW>);
        default: return nullptr;
    }
}

struct PlanWide {
    int rc = 0, wgs = 0, ntx = 0, nty = 0, cached = 0;
    const void *fn = nullptr;
};

template <typename T, int R, bool BOX>
int plan_wide(const perks_shape &s, const perks_tuning *tu, PlanWide *pl) {
    DeviceFacts f;
    int rc = device_facts(&f);
    if (rc) return rc;
    if (tu && tu->waves_per_wg != 0 && tu->waves_per_wg != WW)
        return set_error(PERKS_E_UNSUPPORTED, "wide 2D stencils use %d waves per workgroup", WW);
    if (tu && tu->sync > 1) return set_error(PERKS_E_UNSUPPORTED, "wide 2D stencils synchronise with a grid barrier");
    const int want = tu ? tu->rows_per_lane : 0;
    if (want && !wide_fn<T, R, BOX>(want))
        return set_error(PERKS_E_UNSUPPORTED, "wide 2D stencils keep 24, 32, 48 or 80 rows per lane (got %d)", want);
    const long long nxi = s.nx - 2 * R, nyi = s.ny - 2 * R;
    pl->ntx = (int)((nxi + 63) / 64);
    auto tiles = [&](int h) { return (long long)pl->ntx * ((nyi + h - 1) / h); };
    // co-resident waves = cacheable tiles
    auto cap_of = [&](const void *fn) -> long long {
        int occ = 0;
        if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, WW * 64, 0) != hipSuccess || occ < 1)
            return 0;
        return (long long)f.cus * occ * WW;
    };
    const bool stream_all = tu && tu->max_cached_tiles != 0;   // < 0: none cached; > 0: fewer than all -> stream
    int chosen = 0;
    for (int h : WR_DEPTHS) {
        if (want && h != want) continue;
        const long long cap = cap_of(wide_fn<T, R, BOX>(h));
        if (!cap) continue;
        if (!chosen && (tiles(h) <= cap || want)) chosen = h;
    }
    if (!chosen) chosen = want ? 0 : WR_DEPTHS[0];   // streams
    const void *fn = wide_fn<T, R, BOX>(chosen);
    const long long cap = cap_of(fn);
    if (!cap) return set_error(PERKS_E_UNSUPPORTED, "no wide 2D kernel fits the device");
    pl->rc = chosen;
    pl->nty = (int)((nyi + chosen - 1) / chosen);
    const long long nt = tiles(chosen);
    pl->cached = (!stream_all && nt <= cap) ? 1 : 0;
    if (tu && tu->max_cached_tiles > 0 && tu->max_cached_tiles >= nt && nt <= cap) pl->cached = 1;
    pl->wgs = (int)std::min<long long>((nt + WW - 1) / WW, cap / WW);   // all co-resident
    pl->fn = fn;
    return PERKS_OK;
}

template <typename T, int R>
void fill_wide(WideW<T, R> &W, const double *c) {
    for (int i = 0; i < (2 * R + 1) * (2 * R + 1); ++i) W.w[i] = (T)c[i];
}

template <typename T, int R, bool BOX>
int run_wide(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, hipStream_t st,
             const perks_tuning *tu) {
    PlanWide pl;
    int rc = plan_wide<T, R, BOX>(s, tu, &pl);
    if (rc) return rc;
    const size_t cells = (size_t)s.nx * s.ny;
    // the second grid buffer, then (cached tiles) two step-parity copies of
    // every tile's edge-column block of 2 R RC cells
    const size_t cols_off = (cells * sizeof(T) + 255) & ~(size_t)255;
    const bool cols = pl.cached && wide_cols_on<T, R>();
    const size_t cols_bytes = cols ? (size_t)2 * pl.ntx * pl.nty * (2 * R * pl.rc) * sizeof(T) : 0;
    char *ws = (char *)scratch(SLOT_WIDE, cols_off + cols_bytes);
    T *other = (T *)ws;
    unsigned *sync = (unsigned *)scratch(SLOT_SYNC, SYNC_BYTES);
    if (!other || !sync) return PERKS_E_NOMEM;
    // the second buffer needs the fixed ring (and, for streamed tiles, nothing
    // else): copy the whole grid once
    PERKS_HIP_TRY(hipMemcpyAsync(other, grid, cells * sizeof(T), hipMemcpyDeviceToDevice, st));
    Wide2DParams<T, R> p{};
    p.buf0 = to_global(grid);
    p.buf1 = to_global(other);
    p.sync = sync;
    p.steps = steps;
    p.nx = (int)s.nx;
    p.ny = (int)s.ny;
    p.ntx = pl.ntx;
    p.nty = pl.nty;
    p.cached = pl.cached;
    p.cols = cols ? to_global((T *)(ws + cols_off)) : nullptr;
    fill_wide(p.W, coeffs);
    return launch_coop(pl.fn, pl.wgs, WW * 64, &p, st);
}

template <typename T, int R, bool BOX>
int baseline_wide(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, hipStream_t st) {
    const size_t cells = (size_t)s.nx * s.ny;
    T *other = (T *)scratch(SLOT_PINGPONG, cells * sizeof(T));
    if (!other) return PERKS_E_NOMEM;
    Wide2DStep<T, R> p{};
    p.nx = (int)s.nx;
    p.ny = (int)s.ny;
    p.ntx = (int)((s.nx - 2 * R + 63) / 64);
    p.nty = (int)((s.ny - 2 * R + WRB - 1) / WRB);
    fill_wide(p.W, coeffs);
    PERKS_HIP_TRY(hipMemcpyAsync(other, grid, cells * sizeof(T), hipMemcpyDeviceToDevice, st));
    const int wgs = (p.ntx * p.nty + WWB - 1) / WWB;
    T *a = grid, *b = other;
    for (int64_t k = 0; k < steps; ++k) {
        p.src = to_global((const T *)a);
        p.dst = to_global(b);
        hipLaunchKernelGGL((stencil2d_wide_step<T, R, BOX, WRB, WWB>), dim3(wgs), dim3(WWB * 64), 0, st, p);
        std::swap(a, b);
    }
    PERKS_HIP_TRY(hipGetLastError());
    if (a != grid) PERKS_HIP_TRY(hipMemcpyAsync(grid, a, cells * sizeof(T), hipMemcpyDeviceToDevice, st));
    return PERKS_OK;
}

template <typename T, int R, bool BOX>
int plan_wide_query(const perks_shape &s, const perks_tuning *tu, perks_stencil_plan *plan) {
    PlanWide pl;
    int rc = plan_wide<T, R, BOX>(s, tu, &pl);
    if (rc) return rc;
    const int64_t nxi = s.nx - 2 * R, nyi = s.ny - 2 * R;
    const int ntiles = pl.ntx * pl.nty;
    plan->wgs = pl.wgs;
    plan->waves_per_wg = WW;
    plan->rows_per_lane = pl.rc;
    plan->planes_per_lane = 1;
    plan->tiles = ntiles;
    plan->cached_tiles = pl.cached ? ntiles : 0;
    plan->cached_cells = pl.cached ? nxi * nyi : 0;
    plan->interior_cells = nxi * nyi;
    // per step: each tile writes its edge band and reads its halo (R rows
    // above and below, R columns on each side, plus the corners for the box)
    int64_t face = 0;
    for (int t = 0; t < ntiles; ++t) {
        const int tx = t % pl.ntx, ty = t / pl.ntx;
        const int64_t wx = std::min<int64_t>(64, nxi - 64 * tx), hy = std::min<int64_t>(pl.rc, nyi - pl.rc * ty);
        const int64_t band = wx * hy - std::max<int64_t>(0, wx - 2 * R) * std::max<int64_t>(0, hy - 2 * R);
        const int64_t halo = 2 * R * wx + 2 * R * hy + (BOX ? 4 * R * R : 0);
        face += pl.cached ? band + halo : 2 * wx * hy + halo;
    }
    plan->halo_bytes_per_step = face * (int64_t)sizeof(T);
    plan->sync = 1;
    plan->lds_rows_per_lane = 0;
    return PERKS_OK;
}

}  // namespace perks
