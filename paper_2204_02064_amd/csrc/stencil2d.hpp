// 2D radius-1 Jacobi stencils (Eq. 2 and the 2d9pt box of tab:domain) on
// gfx950: the tile arithmetic and the persistent kernel.
// (Their per-step baseline is the radius-2..4 family's per-step kernel run at
// radius 1, which sums the same terms in the same order.)
//
// Tiling.  The interior (x in [1,nx-2], y in [1,ny-2]) is cut into wave tiles
// of 64 columns x R rows.  Lane l of the wavefront owns column x0+l and keeps
// the tile's R cells of that column in registers ("each thread computes a
// vertical run of cells", Sec. 4.2.1): north/south neighbours are in the
// lane's own registers, west/east neighbours arrive through DPP lane shifts,
// and the tile's outer neighbours (halo) come from face buffers.
//
// Face buffers hold tile edges in global coordinates, double-buffered by step
// parity:  rowbuf[par][slot][x]  (slot 2ty+1 = top edge row of tile row ty,
// 2ty+2 = its bottom edge row, 0 and 2*nty+1 = the fixed ring rows) and
// colbuf[par][slot][y] (the same for tile columns; edge columns are stored
// transposed so that they are written and read contiguously, Sec. 4.2.2).
// Tile (tx,ty) reads its north halo row from slot 2ty, south from 2ty+3, west
// column from slot 2tx, east from 2tx+3.  Corner cells needed by the 9-point
// box are the end entries of those rows/columns.
#pragma once

#include <vector>

#include "barrier.hpp"
#include "common.hpp"

#ifndef PERKS_SCHED_ROWS
#define PERKS_SCHED_ROWS 4
#endif

namespace perks {

// Rows of a cached tile that may live in LDS (the PERKS_MIX tier), per wave:
// 8 waves x (28 x 64) doubles or (56 x 64) floats = 112 KiB, next to the halo
// columns.
template <typename T>
struct LdsRows {
    static constexpr int value = sizeof(T) == 8 ? 28 : 56;
};

template <typename T>
struct Weights2D {
    T w[9];  // [dy+1][dx+1]
};

// Rolling state of one old row at this lane: value and its west/east values.
template <typename T>
struct RowVal {
    T c, w, e;
};

// Updates rows 0..nrows-1 of u in place (one Jacobi step for one lane strip).
//   u[0..nrows-1] old values on entry, new values on exit.
//   above         old row above row 0 with its west/east values; on exit the
//                 old value of row nrows-1 (so chunks can be chained).
//   below         old row below row nrows-1 (south halo or next chunk's row).
//   lw, le        LDS: west / east halo column, entry j <-> row j-1 (j=0..nrows+1).
// FULL means nrows == RC; otherwise the last row's south neighbour is picked
// with a wave-uniform select (never a register-array index that depends on a
// run-time value, which would move the array to scratch memory).
// Terms are summed in ascending (dy, dx) order, one multiply then FMAs, the
// order of the radius-2..4 tile routine too, so the per-step baseline (that
// routine at radius 1) rounds identically.
// Returns the new value of row nrows-1 (the tile's bottom edge when the strip
// ends the tile), taken from the computed values rather than from u.
template <typename T, int RC, bool BOX, bool FULL>
__device__ __forceinline__ T compute_rows(T (&u)[RC], int nrows, RowVal<T> &above, T below, const T *lw,
                                          const T *le, const Weights2D<T> &W) {
    // acc carries the south-row terms of the row being computed; they are
    // accumulated while the old south row is still live, so that each new
    // value can take its old value's register (no second register set).
    T acc;
    if (BOX) {
        acc = W.w[0] * above.w;
        acc = fma_t(W.w[1], above.c, acc);
        acc = fma_t(W.w[2], above.e, acc);
    } else {
        acc = W.w[1] * above.c;
    }
    T last = T(0);
    T c = u[0];
    T cw = from_west(c, lw[1]);
    T ce = from_east(c, le[1]);
#pragma unroll
    for (int i = 0; i < RC; ++i) {
        if (FULL || i < nrows) {
            T n;
            if (i + 1 < RC)
                n = (FULL || i + 1 < nrows) ? u[i + 1] : below;
            else
                n = below;
            acc = fma_t(W.w[3], cw, acc);
            acc = fma_t(W.w[4], c, acc);
            acc = fma_t(W.w[5], ce, acc);
            // south-row terms of row i+1 come from old row i: take them now, so
            // old row i is dead before the new value of row i is complete
            T nxt;
            if (BOX) {
                nxt = W.w[0] * cw;
                nxt = fma_t(W.w[1], c, nxt);
                nxt = fma_t(W.w[2], ce, nxt);
            } else {
                nxt = W.w[1] * c;
            }
            above.c = c;
            above.w = cw;
            above.e = ce;
            T nw = n, ne = n;
            if (BOX || (i + 1 < RC && (FULL || i + 1 < nrows))) {
                nw = from_west(n, lw[i + 2]);
                ne = from_east(n, le[i + 2]);
            }
            if (BOX) {
                acc = fma_t(W.w[6], nw, acc);
                acc = fma_t(W.w[7], n, acc);
                acc = fma_untied(W.w[8], ne, acc);
            } else {
                acc = fma_untied(W.w[7], n, acc);
            }
            u[i] = acc;
            if (FULL ? (i == RC - 1) : true) last = (FULL || i == nrows - 1) ? acc : last;
            acc = nxt;
            c = n;
            cw = nw;
            ce = ne;
        }
        // bound how far the scheduler may hoist loads and products across
        // rows: every hoisted row costs registers the cache needs
        if ((i % PERKS_SCHED_ROWS) == PERKS_SCHED_ROWS - 1) __builtin_amdgcn_sched_barrier(0);
    }
    return last;
}

// ---------------------------------------------------------------------------
struct Tile2D {
    int tx, ty, x0, y0, wx, hy;
};

template <typename T>
struct Stencil2DParams {
    gmem<T> *grid;
    gmem<T> *rowbuf;   // [2][2*nty+2][nx]
    gmem<T> *colbuf;   // [2][2*ntx+2][ny]
    unsigned *sync;
    long long steps;
    int nx, ny;
    int ntx, nty;
    int R;             // tile height H (rows per lane): register rows + LDS rows
    int RL;            // rows of a cached tile kept in LDS (rows RREG .. H-1)
    int last_w, last_h;
    int ntiles;
    int cached;        // number of tiles held in registers (tile id < cached)
    unsigned epoch0;   // LL mode: epoch of the initial faces (state 0)
    unsigned ering;    // LL mode: epoch of the fixed ring words of this launch
    Weights2D<T> W;
};

template <typename T>
__device__ __forceinline__ Tile2D tile_of(const Stencil2DParams<T> &p, int t) {
    Tile2D tl;
    tl.tx = t % p.ntx;
    tl.ty = t / p.ntx;
    tl.x0 = 1 + 64 * tl.tx;
    tl.y0 = 1 + p.R * tl.ty;
    tl.wx = (tl.tx == p.ntx - 1) ? p.last_w : 64;
    tl.hy = (tl.ty == p.nty - 1) ? p.last_h : p.R;
    return tl;
}

template <typename T>
__device__ __forceinline__ size_t rb_off(const Stencil2DParams<T> &p, int par, int slot) {
    return ((size_t)par * (2 * p.nty + 2) + slot) * p.nx;
}
template <typename T>
__device__ __forceinline__ size_t cb_off(const Stencil2DParams<T> &p, int par, int slot) {
    return ((size_t)par * (2 * p.ntx + 2) + slot) * p.ny;
}

// Loads the halo of tile tl from parity `par` face buffers: north/south rows
// into registers, west/east columns (rows y0-1..y0+hy) into this wave's LDS.
template <typename T>
__device__ __forceinline__ void load_halo(const Stencil2DParams<T> &p, const Tile2D &tl, int par,
                                          int lane, T &hn, T &hs, T *lw, T *le) {
    const int xl = min(tl.x0 + lane, p.nx - 1);
    hn = ld_coh(p.rowbuf + rb_off(p, par, 2 * tl.ty) + xl);
    hs = ld_coh(p.rowbuf + rb_off(p, par, 2 * tl.ty + 3) + xl);
    const gmem<T> *cw = p.colbuf + cb_off(p, par, 2 * tl.tx) + (tl.y0 - 1);
    const gmem<T> *ce = p.colbuf + cb_off(p, par, 2 * tl.tx + 3) + (tl.y0 - 1);
    for (int j = lane; j < tl.hy + 2; j += 64) {
        lw[j] = ld_coh(cw + j);
        le[j] = ld_coh(ce + j);
    }
    compiler_fence();
}

// Publishes the edges of a tile strip into parity `par` face buffers.
// Rows r0..r0+n-1 of the tile are in u[0..n-1].
template <typename T, int RC, bool FULL>
__device__ __forceinline__ void publish_rows(const Stencil2DParams<T> &p, const Tile2D &tl, int par, int lane,
                                             const T (&u)[RC], int r0, int n, T lastval) {
    gmem<T> *left = p.colbuf + cb_off(p, par, 2 * tl.tx + 1) + tl.y0 + r0;
    gmem<T> *right = p.colbuf + cb_off(p, par, 2 * tl.tx + 2) + tl.y0 + r0;
    const bool in = lane < tl.wx;
#pragma unroll
    for (int i = 0; i < RC; ++i) {
        if (FULL || i < n) {
            if (lane == 0) st_coh(left + i, u[i]);
            if (lane == tl.wx - 1) st_coh(right + i, u[i]);
        }
    }
    if (in && r0 == 0) st_coh(p.rowbuf + rb_off(p, par, 2 * tl.ty + 1) + tl.x0 + lane, u[0]);
    if (in && r0 + n == tl.hy)
        st_coh(p.rowbuf + rb_off(p, par, 2 * tl.ty + 2) + tl.x0 + lane, lastval);
}

// Fixed ring entries of the face buffers, both parities (grid-stride loop
// over all threads of the launch).
template <typename T>
__device__ __forceinline__ void init_ring_faces(const Stencil2DParams<T> &p, const gmem<T> *g) {
    const int nthreads = gridDim.x * blockDim.x;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nrs = 2 * p.nty + 2, ncs = 2 * p.ntx + 2;
    for (int par = 0; par < 2; ++par) {
        for (int x = tid; x < p.nx; x += nthreads) {
            st_coh(p.rowbuf + rb_off(p, par, 0) + x, g[x]);
            st_coh(p.rowbuf + rb_off(p, par, nrs - 1) + x, g[(size_t)(p.ny - 1) * p.nx + x]);
        }
        for (int y = tid; y < p.ny; y += nthreads) {
            st_coh(p.colbuf + cb_off(p, par, 0) + y, g[(size_t)y * p.nx]);
            st_coh(p.colbuf + cb_off(p, par, ncs - 1) + y, g[(size_t)y * p.nx + p.nx - 1]);
        }
        // ring columns inside every row slot, ring rows inside every column slot
        for (int s = tid; s < nrs - 2; s += nthreads) {
            const int ty = s / 2;
            const int y = (s % 2 == 0) ? 1 + p.R * ty : 1 + p.R * ty + ((ty == p.nty - 1) ? p.last_h : p.R) - 1;
            st_coh(p.rowbuf + rb_off(p, par, s + 1) + 0, g[(size_t)y * p.nx]);
            st_coh(p.rowbuf + rb_off(p, par, s + 1) + p.nx - 1, g[(size_t)y * p.nx + p.nx - 1]);
        }
        for (int s = tid; s < ncs - 2; s += nthreads) {
            const int tx = s / 2;
            const int x = (s % 2 == 0) ? 1 + 64 * tx : 1 + 64 * tx + ((tx == p.ntx - 1) ? p.last_w : 64) - 1;
            st_coh(p.colbuf + cb_off(p, par, s + 1) + 0, g[x]);
            st_coh(p.colbuf + cb_off(p, par, s + 1) + p.ny - 1, g[(size_t)(p.ny - 1) * p.nx + x]);
        }
    }
}

// Edges of a tile straight from the grid into parity-0 face buffers.
template <typename T>
__device__ __forceinline__ void publish_initial(const Stencil2DParams<T> &p, const Tile2D &tl, int lane) {
    const gmem<T> *g = p.grid;
    if (lane < tl.wx) {
        st_coh(p.rowbuf + rb_off(p, 0, 2 * tl.ty + 1) + tl.x0 + lane, g[(size_t)tl.y0 * p.nx + tl.x0 + lane]);
        st_coh(p.rowbuf + rb_off(p, 0, 2 * tl.ty + 2) + tl.x0 + lane,
               g[(size_t)(tl.y0 + tl.hy - 1) * p.nx + tl.x0 + lane]);
    }
    for (int j = lane; j < tl.hy; j += 64) {
        const size_t row = (size_t)(tl.y0 + j) * p.nx;
        st_coh(p.colbuf + cb_off(p, 0, 2 * tl.tx + 1) + tl.y0 + j, g[row + tl.x0]);
        st_coh(p.colbuf + cb_off(p, 0, 2 * tl.tx + 2) + tl.y0 + j, g[row + tl.x0 + tl.wx - 1]);
    }
}

// ---------------------------------------------------------------------------
// Low-latency (LL) face exchange: point-to-point synchronisation instead of a
// device-wide barrier.  Every face element is stored as 64-bit words that
// carry 32 data bits and the epoch of the state they belong to (FP32: one
// word, FP64: two).  Aligned 64-bit stores and loads are single-copy atomic,
// so a reader that sees the expected epoch in a word also sees its data: the
// reader polls the halo words themselves, and a step needs no barrier and no
// separate flag round trip.  Ring entries carry an epoch reserved for this
// launch (every launch takes a fresh range of epochs, so a word left by an
// earlier launch, whose layout may differ, is never taken as current).  Neighbour
// dependencies are symmetric (a tile only polls the tiles that also poll it),
// so no tile can run two steps ahead of a reader and overwrite words of a
// parity buffer that reader still needs.
typedef unsigned long long llword;

template <typename T>
struct LLTraits {
    static constexpr int WPE = sizeof(T) / 4;   // 64-bit words per element
};

template <typename T>
__device__ __forceinline__ void ll_store(gmem<llword> *w, T v, unsigned e) {
    const llword tag = (llword)e << 32;
    if constexpr (sizeof(T) == 4) {
        st_coh(w, tag | __float_as_uint(v));
    } else {
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        st_coh(w, tag | (unsigned)b);
        st_coh(w + 1, tag | (unsigned)(b >> 32));
    }
}

// Loads one element; clears ok when `need` and a word is neither of epoch e
// nor a ring word of this launch (epoch er).
template <typename T>
__device__ __forceinline__ T ll_load(const gmem<llword> *w, unsigned e, unsigned er, bool need, bool &ok) {
    if constexpr (sizeof(T) == 4) {
        const llword a = ld_coh(w);
        const unsigned f = (unsigned)(a >> 32);
        if (need && f != e && f != er) ok = false;
        return __uint_as_float((unsigned)a);
    } else {
        const llword a = ld_coh(w), b = ld_coh(w + 1);
        const unsigned fa = (unsigned)(a >> 32), fb = (unsigned)(b >> 32);
        if (need && ((fa != e && fa != er) || (fb != e && fb != er))) ok = false;
        return __longlong_as_double((long long)(((unsigned long long)(unsigned)b << 32) | (unsigned)a));
    }
}

template <typename T>
__device__ __forceinline__ gmem<llword> *ll_row(const Stencil2DParams<T> &p, int par, int slot) {
    return reinterpret_cast<gmem<llword> *>(p.rowbuf) + rb_off(p, par, slot) * LLTraits<T>::WPE;
}
template <typename T>
__device__ __forceinline__ gmem<llword> *ll_col(const Stencil2DParams<T> &p, int par, int slot) {
    return reinterpret_cast<gmem<llword> *>(p.colbuf) + cb_off(p, par, slot) * LLTraits<T>::WPE;
}

// Polls the halo of tile tl (parity par, epoch e) until every word it needs
// is current.  The 5-point star needs no corner: ghost lanes and the end
// entries of the columns are then not waited for (a diagonal tile does not
// depend on this one either).
template <typename T, bool BOX>
__device__ __forceinline__ void load_halo_ll(const Stencil2DParams<T> &p, const Tile2D &tl, int par, unsigned e,
                                             int lane, T &hn, T &hs, T *lw, T *le) {
    constexpr int WPE = LLTraits<T>::WPE;
    const int xl = min(tl.x0 + lane, p.nx - 1);
    const bool need_row = lane < tl.wx || (BOX && lane == tl.wx);
    const gmem<llword> *rn = ll_row(p, par, 2 * tl.ty) + (size_t)xl * WPE;
    const gmem<llword> *rs = ll_row(p, par, 2 * tl.ty + 3) + (size_t)xl * WPE;
    const gmem<llword> *cw = ll_col(p, par, 2 * tl.tx) + (size_t)(tl.y0 - 1) * WPE;
    const gmem<llword> *ce = ll_col(p, par, 2 * tl.tx + 3) + (size_t)(tl.y0 - 1) * WPE;
    const int jlo = BOX ? 0 : 1, jhi = BOX ? tl.hy + 2 : tl.hy + 1;
    while (true) {
        bool ok = true;
        hn = ll_load<T>(rn, e, p.ering, need_row, ok);
        hs = ll_load<T>(rs, e, p.ering, need_row, ok);
        for (int j = lane; j < tl.hy + 2; j += 64) {
            const bool need = j >= jlo && j < jhi;
            lw[j] = ll_load<T>(cw + (size_t)j * WPE, e, p.ering, need, ok);
            le[j] = ll_load<T>(ce + (size_t)j * WPE, e, p.ering, need, ok);
        }
        if (__all(ok)) break;
        __builtin_amdgcn_s_sleep(1);
    }
    compiler_fence();
}

// Edge rows of a strip go straight out; edge column values are gathered in
// LDS (ow / oe, indexed by tile row) and stored coalesced by publish_cols_ll.
template <typename T, int RC, bool FULL>
__device__ __forceinline__ void publish_rows_ll(const Stencil2DParams<T> &p, const Tile2D &tl, int par, unsigned e,
                                                int lane, const T (&u)[RC], int r0, int n, T lastval, T *ow, T *oe) {
    constexpr int WPE = LLTraits<T>::WPE;
#pragma unroll
    for (int i = 0; i < RC; ++i) {
        if (FULL || i < n) {
            if (lane == 0) ow[r0 + i] = u[i];
            if (lane == tl.wx - 1) oe[r0 + i] = u[i];
        }
    }
    if (lane < tl.wx) {
        const size_t xo = (size_t)(tl.x0 + lane) * WPE;
        if (r0 == 0) ll_store(ll_row(p, par, 2 * tl.ty + 1) + xo, u[0], e);
        if (r0 + n == tl.hy) ll_store(ll_row(p, par, 2 * tl.ty + 2) + xo, lastval, e);
    }
}

template <typename T>
__device__ __forceinline__ void publish_cols_ll(const Stencil2DParams<T> &p, const Tile2D &tl, int par, unsigned e,
                                                int lane, const T *ow, const T *oe) {
    constexpr int WPE = LLTraits<T>::WPE;
    compiler_fence();
    gmem<llword> *cl = ll_col(p, par, 2 * tl.tx + 1) + (size_t)tl.y0 * WPE;
    gmem<llword> *cr = ll_col(p, par, 2 * tl.tx + 2) + (size_t)tl.y0 * WPE;
    for (int j = lane; j < tl.hy; j += 64) {
        ll_store(cl + (size_t)j * WPE, ow[j], e);
        ll_store(cr + (size_t)j * WPE, oe[j], e);
    }
    compiler_fence();
}

template <typename T>
__device__ __forceinline__ void init_ring_faces_ll(const Stencil2DParams<T> &p) {
    constexpr int WPE = LLTraits<T>::WPE;
    const gmem<T> *g = p.grid;
    const int nthreads = gridDim.x * blockDim.x;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nrs = 2 * p.nty + 2, ncs = 2 * p.ntx + 2;
    for (int par = 0; par < 2; ++par) {
        for (int x = tid; x < p.nx; x += nthreads) {
            ll_store(ll_row(p, par, 0) + (size_t)x * WPE, g[x], p.ering);
            ll_store(ll_row(p, par, nrs - 1) + (size_t)x * WPE, g[(size_t)(p.ny - 1) * p.nx + x], p.ering);
        }
        for (int y = tid; y < p.ny; y += nthreads) {
            ll_store(ll_col(p, par, 0) + (size_t)y * WPE, g[(size_t)y * p.nx], p.ering);
            ll_store(ll_col(p, par, ncs - 1) + (size_t)y * WPE, g[(size_t)y * p.nx + p.nx - 1], p.ering);
        }
        for (int s = tid; s < nrs - 2; s += nthreads) {
            const int ty = s / 2;
            const int y = (s % 2 == 0) ? 1 + p.R * ty : 1 + p.R * ty + ((ty == p.nty - 1) ? p.last_h : p.R) - 1;
            ll_store(ll_row(p, par, s + 1), g[(size_t)y * p.nx], p.ering);
            ll_store(ll_row(p, par, s + 1) + (size_t)(p.nx - 1) * WPE, g[(size_t)y * p.nx + p.nx - 1], p.ering);
        }
        for (int s = tid; s < ncs - 2; s += nthreads) {
            const int tx = s / 2;
            const int x = (s % 2 == 0) ? 1 + 64 * tx : 1 + 64 * tx + ((tx == p.ntx - 1) ? p.last_w : 64) - 1;
            ll_store(ll_col(p, par, s + 1), g[x], p.ering);
            ll_store(ll_col(p, par, s + 1) + (size_t)(p.ny - 1) * WPE, g[(size_t)(p.ny - 1) * p.nx + x], p.ering);
        }
    }
}

template <typename T>
__device__ __forceinline__ void publish_initial_ll(const Stencil2DParams<T> &p, const Tile2D &tl, int lane) {
    constexpr int WPE = LLTraits<T>::WPE;
    const gmem<T> *g = p.grid;
    const unsigned e = p.epoch0;
    if (lane < tl.wx) {
        const size_t xo = (size_t)(tl.x0 + lane) * WPE;
        ll_store(ll_row(p, 0, 2 * tl.ty + 1) + xo, g[(size_t)tl.y0 * p.nx + tl.x0 + lane], e);
        ll_store(ll_row(p, 0, 2 * tl.ty + 2) + xo, g[(size_t)(tl.y0 + tl.hy - 1) * p.nx + tl.x0 + lane], e);
    }
    for (int j = lane; j < tl.hy; j += 64) {
        const size_t row = (size_t)(tl.y0 + j) * p.nx;
        ll_store(ll_col(p, 0, 2 * tl.tx + 1) + (size_t)(tl.y0 + j) * WPE, g[row + tl.x0], e);
        ll_store(ll_col(p, 0, 2 * tl.tx + 2) + (size_t)(tl.y0 + j) * WPE, g[row + tl.x0 + tl.wx - 1], e);
    }
}

// One step of a cached tile: rows 0..RREG-1 live in registers v, rows
// RREG..hy-1 (at most p.RL) in this wave's LDS rows lt[r][lane] (the
// register + shared-memory cache of PERKS_MIX).  In LL mode the halo is
// polled (epoch e_in) and the faces are tagged e_in + 1; otherwise the step is
// bracketed by device-wide barriers.
template <typename T, int RREG, bool BOX, bool LL>
__device__ __forceinline__ void step_cached(const Stencil2DParams<T> &p, const Tile2D &tl, int par, unsigned e_in,
                                            int lane, T (&v)[RREG], T *lt, T *lw, T *le, T *ow, T *oe) {
    T hn, hs;
    if constexpr (LL) load_halo_ll<T, BOX>(p, tl, par, e_in, lane, hn, hs, lw, le);
    else load_halo(p, tl, par, lane, hn, hs, lw, le);
    const bool ghost = lane >= tl.wx;
    if (tl.wx < 64 && ghost) {
        // ghost lanes carry the east halo column so the DPP east shift of the
        // last real lane picks it up
#pragma unroll
        for (int i = 0; i < RREG; ++i) v[i] = le[i + 1];
        hn = le[0];
        hs = le[tl.hy + 1];
    }
    RowVal<T> above;
    above.c = hn;
    above.w = from_west(hn, lw[0]);
    above.e = from_east(hn, le[0]);
    const int nreg = min(RREG, tl.hy);
    // old value of the row below the register rows
    T below = hs;
    if (tl.hy > RREG) below = ghost ? le[RREG + 1] : lt[lane];
    const unsigned e_out = e_in + 1;
    if (nreg == RREG) {
        const T last = compute_rows<T, RREG, BOX, true>(v, RREG, above, below, lw, le, p.W);
        if constexpr (LL) publish_rows_ll<T, RREG, true>(p, tl, par ^ 1, e_out, lane, v, 0, RREG, last, ow, oe);
        else publish_rows<T, RREG, true>(p, tl, par ^ 1, lane, v, 0, RREG, last);
    } else {
        const T last = compute_rows<T, RREG, BOX, false>(v, nreg, above, below, lw, le, p.W);
        if constexpr (LL) publish_rows_ll<T, RREG, false>(p, tl, par ^ 1, e_out, lane, v, 0, nreg, last, ow, oe);
        else publish_rows<T, RREG, false>(p, tl, par ^ 1, lane, v, 0, nreg, last);
    }
    // LDS rows, 8 at a time, updated in place (the rolling `above` keeps the
    // old last row of the previous chunk)
    constexpr int CH = 8;
    for (int c = RREG; c < tl.hy; c += CH) {
        const int n = min(CH, tl.hy - c);
        T *lr = lt + (c - RREG) * 64 + lane;
        T u[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) u[i] = (i < n) ? (ghost ? le[c + i + 1] : lr[i * 64]) : T(0);
        T bl = hs;
        if (c + n < tl.hy) bl = ghost ? le[c + n + 1] : lr[n * 64];
        const T last = (n == CH) ? compute_rows<T, CH, BOX, true>(u, CH, above, bl, lw + c, le + c, p.W)
                                 : compute_rows<T, CH, BOX, false>(u, n, above, bl, lw + c, le + c, p.W);
#pragma unroll
        for (int i = 0; i < CH; ++i)
            if (i < n) lr[i * 64] = u[i];
        if constexpr (LL) {
            if (n == CH) publish_rows_ll<T, CH, true>(p, tl, par ^ 1, e_out, lane, u, c, CH, last, ow, oe);
            else publish_rows_ll<T, CH, false>(p, tl, par ^ 1, e_out, lane, u, c, n, last, ow, oe);
        } else {
            if (n == CH) publish_rows<T, CH, true>(p, tl, par ^ 1, lane, u, c, CH, last);
            else publish_rows<T, CH, false>(p, tl, par ^ 1, lane, u, c, n, last);
        }
    }
    if constexpr (LL) publish_cols_ll(p, tl, par ^ 1, e_out, lane, ow, oe);
}

// One step of a tile that lives in the grid (the uncached part, Eq. 5's
// D_uncache): streamed through registers CH rows at a time, updated in place.
// In-place is safe because neighbours read this tile only through the face
// buffers, and the rolling `above` state keeps the old value of the last row
// of the previous chunk.
template <typename T, int CH, bool BOX, bool LL>
__device__ __forceinline__ void step_streamed(const Stencil2DParams<T> &p, const Tile2D &tl, int par, unsigned e_in,
                                              int lane, T *lw, T *le, T *ow, T *oe) {
    T hn, hs;
    if constexpr (LL) load_halo_ll<T, BOX>(p, tl, par, e_in, lane, hn, hs, lw, le);
    else load_halo(p, tl, par, lane, hn, hs, lw, le);
    const bool ghost = lane >= tl.wx;
    const int xl = min(tl.x0 + lane, p.nx - 1);
    if (ghost) {
        hn = le[0];
        hs = le[tl.hy + 1];
    }
    RowVal<T> above;
    above.c = hn;
    above.w = from_west(hn, lw[0]);
    above.e = from_east(hn, le[0]);
    T u[CH];
    for (int c = 0; c < tl.hy; c += CH) {
        const int n = min(CH, tl.hy - c);
        gmem<T> *row0 = p.grid + (size_t)(tl.y0 + c) * p.nx + xl;
#pragma unroll
        for (int i = 0; i < CH; ++i)
            u[i] = (i < n) ? (ghost ? le[c + i + 1] : row0[(size_t)i * p.nx]) : T(0);
        T below = hs;
        if (c + n < tl.hy) below = ghost ? le[c + n + 1] : row0[(size_t)n * p.nx];
        const T last = (n == CH) ? compute_rows<T, CH, BOX, true>(u, CH, above, below, lw + c, le + c, p.W)
                                 : compute_rows<T, CH, BOX, false>(u, n, above, below, lw + c, le + c, p.W);
        if (!ghost) {
#pragma unroll
            for (int i = 0; i < CH; ++i)
                if (i < n) row0[(size_t)i * p.nx] = u[i];
        }
        if constexpr (LL) {
            if (n == CH) publish_rows_ll<T, CH, true>(p, tl, par ^ 1, e_in + 1, lane, u, c, CH, last, ow, oe);
            else publish_rows_ll<T, CH, false>(p, tl, par ^ 1, e_in + 1, lane, u, c, n, last, ow, oe);
        } else {
            if (n == CH) publish_rows<T, CH, true>(p, tl, par ^ 1, lane, u, c, CH, last);
            else publish_rows<T, CH, false>(p, tl, par ^ 1, lane, u, c, n, last);
        }
    }
    if constexpr (LL) publish_cols_ll(p, tl, par ^ 1, e_in + 1, lane, ow, oe);
}

// The persistent kernel: one launch runs all steps.  Tiles t < p.cached are
// kept in registers by wave t for the whole run; the remaining tiles are
// assigned round-robin to all waves and streamed through the grid.  LL selects
// point-to-point halo synchronisation; otherwise every step ends with a
// device-wide barrier.
template <typename T, int R, bool BOX, int WAVES, bool LL>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(1, 2))) void stencil2d_persistent(
    Stencil2DParams<T> p) {
    constexpr int HMAX = R + LdsRows<T>::value;
    __shared__ T lds[WAVES][4][HMAX + 2];
    __shared__ T ltile[WAVES][LdsRows<T>::value * 64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gw = blockIdx.x * WAVES + wave;
    const int nwaves = gridDim.x * WAVES;
    T *lw = lds[wave][0];
    T *le = lds[wave][1];
    T *ow = lds[wave][2];
    T *oe = lds[wave][3];
    T *lt = ltile[wave];
    GridSync gs;
    gs.init(p.sync);
    if constexpr (LL) {
        // this launch's epochs: ering (ring words), epoch0 .. epoch0+steps
        // (states); all above the last epoch of the previous launch and above
        // 0, the epoch of freshly zeroed words
        const unsigned base = ld_coh(p.sync + SYNC_LL_EPOCH);
        p.ering = base + 1u;
        p.epoch0 = base + 2u;
        init_ring_faces_ll(p);
        for (int t = gw; t < p.ntiles; t += nwaves) publish_initial_ll(p, tile_of(p, t), lane);
    } else {
        init_ring_faces(p, p.grid);
        for (int t = gw; t < p.ntiles; t += nwaves) publish_initial(p, tile_of(p, t), lane);
    }
    gs.sync();

    const bool has_cached = gw < p.cached;
    T v[R];
    Tile2D ct{};
    if (has_cached) {
        ct = tile_of(p, gw);
        const int xl = min(ct.x0 + lane, p.nx - 1);
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = (i < ct.hy) ? p.grid[(size_t)(ct.y0 + i) * p.nx + xl] : T(0);
        for (int i = R; i < ct.hy; ++i) lt[(i - R) * 64 + lane] = p.grid[(size_t)(ct.y0 + i) * p.nx + xl];
    }
    settle(v);   // the initial loads complete before the time loop
    const int first_streamed = p.cached + gw;
    for (long long s = 0; s < p.steps; ++s) {
        const int par = (int)(s & 1);
        const unsigned e_in = p.epoch0 + (unsigned)s;
        Stencil2DParams<T> q = p;
        q.grid = opaque(q.grid);
        q.rowbuf = opaque(q.rowbuf);
        q.colbuf = opaque(q.colbuf);
        if (has_cached) step_cached<T, R, BOX, LL>(q, ct, par, e_in, lane, v, lt, lw, le, ow, oe);
        for (int t = first_streamed; t < p.ntiles; t += nwaves)
            step_streamed<T, 8, BOX, LL>(q, tile_of(p, t), par, e_in, lane, lw, le, ow, oe);
        if constexpr (!LL) gs.sync();
    }
    if (has_cached && lane < ct.wx) {
#pragma unroll
        for (int i = 0; i < R; ++i)
            if (i < ct.hy) p.grid[(size_t)(ct.y0 + i) * p.nx + ct.x0 + lane] = v[i];
        for (int i = R; i < ct.hy; ++i) p.grid[(size_t)(ct.y0 + i) * p.nx + ct.x0 + lane] = lt[(i - R) * 64 + lane];
    }
    if constexpr (LL) {
        // the next launch starts its epochs above every word written here
        if (blockIdx.x == 0 && threadIdx.x == 0) st_coh(p.sync + SYNC_LL_EPOCH, p.epoch0 + (unsigned)p.steps);
    }
    gs.finish();
}

// ---------------------------------------------------------------------------
// Host planning / launch (2D).
constexpr int W2 = 8;       // wavefronts per workgroup of the persistent kernel

template <typename T> struct RList;
template <> struct RList<double> { static constexpr int v[4] = {8, 16, 32, 48}; };
template <> struct RList<float> { static constexpr int v[5] = {8, 16, 32, 48, 64}; };

template <typename T, int R, bool BOX>
const void *persist2d_fn(bool ll) {
    return ll ? reinterpret_cast<const void *>(&stencil2d_persistent<T, R, BOX, W2, true>)
              : reinterpret_cast<const void *>(&stencil2d_persistent<T, R, BOX, W2, false>);
}

template <typename T, bool BOX>
const void *pick2d(int R, bool ll) {
    switch (R) {
        case 8: return persist2d_fn<T, 8, BOX>(ll);
        case 16: return persist2d_fn<T, 16, BOX>(ll);
        case 32: return persist2d_fn<T, 32, BOX>(ll);
        case 48: return persist2d_fn<T, 48, BOX>(ll);
        default: break;
    }
    if constexpr (std::is_same<T, float>::value) {
        switch (R) {
            case 64: return persist2d_fn<T, 64, BOX>(ll);
            default: break;
        }
    }
    return nullptr;
}

struct Plan2D {
    int R = 0, RL = 0, wgs = 0, ntx = 0, nty = 0, last_w = 0, last_h = 0, ntiles = 0, cached = 0;
    bool ll = true;       // point-to-point halo synchronisation (else a grid barrier per step)
    const void *fn = nullptr;
};

template <typename T>
int plan2d(const perks_shape &s, bool box, const perks_tuning *tu, Plan2D *pl) {
    DeviceFacts f;
    int rc = device_facts(&f);
    if (rc) return rc;
    const int nxi = (int)s.nx - 2, nyi = (int)s.ny - 2;
    pl->ntx = (nxi + 63) / 64;
    pl->last_w = nxi - 64 * (pl->ntx - 1);
    const int want_r = tu ? tu->rows_per_lane : 0;
    const int wgs_per_cu = (tu && tu->wgs_per_cu > 0) ? tu->wgs_per_cu : 1;
    if (tu && tu->waves_per_wg != 0 && tu->waves_per_wg != W2)
        return set_error(PERKS_E_UNSUPPORTED, "2D persistent kernels use %d waves per workgroup", W2);
    if (tu && (tu->sync < 0 || tu->sync > 2)) return set_error(PERKS_E_INVAL, "sync must be 0, 1 or 2");
    pl->ll = !(tu && tu->sync == 1);
    const long long cap = (long long)f.cus * wgs_per_cu * W2;   // co-resident waves = cacheable tiles
    // smallest tile height H with every tile cached: the fewest rows of serial
    // work per wave.  Register rows come from the instantiated depths; above the
    // deepest one the tile continues in LDS (at most LdsRows rows); whatever is
    // still left over streams through HBM.
    const long long per_col = std::max<long long>(1, cap / pl->ntx);
    const int h_min = (int)std::max<long long>(1, (nyi + per_col - 1) / per_col);
    int chosen = 0, rl = 0, deepest = 0;
    for (int r : RList<T>::v) {
        const void *fn = box ? pick2d<T, true>(r, pl->ll) : pick2d<T, false>(r, pl->ll);
        if (!fn) continue;
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, W2 * 64, 0) != hipSuccess || occ < wgs_per_cu)
            continue;
        deepest = r;
        if (want_r) {
            if (r == want_r) chosen = r;
        } else if (!chosen && r >= h_min) {
            chosen = r;
        }
    }
    if (!chosen && !want_r && deepest) {
        chosen = deepest;
        const int lds_rows = (tu && tu->max_cached_tiles < 0) ? 0 : LdsRows<T>::value;
        rl = std::min(h_min - deepest, lds_rows);
    }
    if (!chosen)
        return set_error(PERKS_E_UNSUPPORTED, "no 2D tile depth matches the request (rows_per_lane=%d)", want_r);
    const int H = chosen + rl;
    pl->R = chosen;
    pl->RL = rl;
    pl->nty = (nyi + H - 1) / H;
    pl->last_h = nyi - H * (pl->nty - 1);
    pl->ntiles = pl->ntx * pl->nty;
    long long cached = std::min<long long>(pl->ntiles, cap);
    if (tu && tu->max_cached_tiles < 0) cached = 0;
    if (tu && tu->max_cached_tiles > 0) cached = std::min<long long>(cached, tu->max_cached_tiles);
    pl->cached = (int)cached;
    long long waves = std::min<long long>(pl->ntiles, cap);
    pl->wgs = (int)((waves + W2 - 1) / W2);
    pl->fn = box ? pick2d<T, true>(chosen, pl->ll) : pick2d<T, false>(chosen, pl->ll);
    return pl->fn ? PERKS_OK : set_error(PERKS_E_UNSUPPORTED, "no kernel for this tile depth");
}

template <typename T>
void fill_weights(Weights2D<T> &W, const double *c) {
    for (int i = 0; i < 9; ++i) W.w[i] = (T)c[i];
}

// Bytes of face buffers (and whether they hold epoch-tagged words) that plan
// `pl` needs for extents s.
template <typename T>
size_t faces2d_bytes(const perks_shape &s, const Plan2D &pl) {
    // LL words double the footprint of a face element (data + epoch)
    const size_t mult = pl.ll ? 2 : 1;
    const size_t rb = (size_t)2 * (2 * pl.nty + 2) * s.nx * mult, cb = (size_t)2 * (2 * pl.ntx + 2) * s.ny * mult;
    return (rb + cb) * sizeof(T);
}

// Launches plan `pl` with the given face buffers (faces2d_bytes of them) and
// barrier words (SYNC_BYTES); allocates nothing.
template <typename T>
int run2d_planned(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, const Plan2D &pl, T *faces,
                  unsigned *sync, hipStream_t st) {
    Stencil2DParams<T> p{};
    p.grid = to_global(grid);
    p.nx = (int)s.nx;
    p.ny = (int)s.ny;
    p.ntx = pl.ntx;
    p.nty = pl.nty;
    p.R = pl.R + pl.RL;
    p.RL = pl.RL;
    p.last_w = pl.last_w;
    p.last_h = pl.last_h;
    p.ntiles = pl.ntiles;
    p.cached = pl.cached;
    p.steps = steps;
    fill_weights(p.W, coeffs);
    const size_t mult = pl.ll ? 2 : 1;
    const size_t rb = (size_t)2 * (2 * pl.nty + 2) * s.nx * mult;
    p.rowbuf = to_global(faces);
    p.colbuf = to_global(faces + rb);
    p.sync = sync;
    return launch_coop(pl.fn, pl.wgs, W2 * 64, &p, st);
}

template <typename T>
int run2d(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, bool box, hipStream_t st,
          const perks_tuning *tu) {
    Plan2D pl;
    int rc = plan2d<T>(s, box, tu, &pl);
    if (rc) return rc;
    // LL words and raw values never share a buffer (a raw value read as an
    // LL word could carry any epoch)
    T *faces = (T *)scratch(pl.ll ? SLOT_FACES_LL : SLOT_FACES, faces2d_bytes<T>(s, pl));
    unsigned *sync = (unsigned *)scratch(SLOT_SYNC, SYNC_BYTES);
    if (!faces || !sync) return PERKS_E_NOMEM;
    return run2d_planned<T>(grid, coeffs, s, steps, pl, faces, sync, st);
}

// run2d with the default plan (point-to-point halo words) in caller-provided
// memory: `mem` (device) holds the barrier words (SYNC_BYTES, first) and the
// face buffers; nothing is allocated.  PERKS_E_UNSUPPORTED when the plan
// needs more than `cap` bytes.
template <typename T>
int run2d_in(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, bool box, hipStream_t st,
             void *mem, size_t cap) {
    Plan2D pl;
    int rc = plan2d<T>(s, box, nullptr, &pl);
    if (rc) return rc;
    const size_t need = SYNC_BYTES + faces2d_bytes<T>(s, pl);
    if (need > cap)
        return set_error(PERKS_E_UNSUPPORTED, "the grid needs %zu bytes of scratch, more than the %zu available", need,
                         cap);
    unsigned *sync = (unsigned *)mem;
    rc = run2d_planned<T>(grid, coeffs, s, steps, pl, (T *)((char *)mem + SYNC_BYTES), sync, st);
    if (rc == PERKS_OK) note_persistent_launch(pl.wgs, sync);   // its barrier clock records are in mem
    return rc;
}

template <typename T>
int plan2d_query(const perks_shape &shape, bool box, const perks_tuning *tune, perks_stencil_plan *plan) {
    Plan2D pl;
    int rc = plan2d<T>(shape, box, tune, &pl);
    if (rc) return rc;
    plan->wgs = pl.wgs;
    plan->waves_per_wg = W2;
    plan->rows_per_lane = pl.R + pl.RL;
    plan->planes_per_lane = 1;
    plan->lds_rows_per_lane = pl.RL;
    plan->tiles = pl.ntiles;
    plan->cached_tiles = pl.cached;
    plan->interior_cells = (shape.nx - 2) * (shape.ny - 2);
    int64_t cc = 0, face = 0;
    for (int t = 0; t < pl.ntiles; ++t) {
        const int tx = t % pl.ntx, ty = t / pl.ntx;
        const int64_t wx = tx == pl.ntx - 1 ? pl.last_w : 64, hy = ty == pl.nty - 1 ? pl.last_h : pl.R + pl.RL;
        if (t < pl.cached) cc += wx * hy;
        // per step: 2 edge rows + 2 edge columns written, the same plus corners read
        face += 2 * (2 * wx + 2 * hy) + 4;
    }
    plan->cached_cells = cc;
    plan->halo_bytes_per_step = face * (int64_t)sizeof(T) * (pl.ll ? 2 : 1);
    plan->sync = pl.ll ? 2 : 1;
    return PERKS_OK;
}

}  // namespace perks
