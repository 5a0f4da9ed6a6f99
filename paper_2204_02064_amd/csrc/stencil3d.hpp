// 3D 7-point Jacobi stencil (tab:domain "3d7pt") on gfx950: plane
// arithmetic, the persistent column kernel, the per-step-launch baseline
// kernel, and host planning.
//
// Persistent kernel: column tiling.  The interior is cut into columns of
// 64 (x) x WAVES*RY (y) x dz (z) cells, one workgroup per column (more than
// one per workgroup, in turn, when the grid has more columns than the device
// holds workgroups).  Wave w of the workgroup owns rows [w RY, (w+1) RY) of
// the column, lane l the x position x0 + l, and a lane holds RY cells of each
// plane: y neighbours inside the wave are the lane's own registers, x
// neighbours arrive through DPP lane shifts, z neighbours are the next and
// previous planes of the same lane.
//
// On chip (Eq. 5): the top min(NC, dz) planes of each workgroup's first
// column stay in registers for the whole run; every other plane is streamed:
// read from the grid, updated in place, in chunks of SC planes with the next
// chunk's loads in flight while the current one is computed.
//
// Halo.  Between the waves of a workgroup the y halo goes through LDS plane
// by plane (each wave posts the old values of its edge rows, a workgroup
// barrier, each reads its neighbours'), so only the column's outer faces go
// through global memory, in face buffers in global coordinates,
// double-buffered by step parity:
//   xface[par][slot][z][y]  (slot 2tx+1 / 2tx+2 = west / east edge plane of
//                            the columns at x index tx; 0 and 2*ntx+1 = the
//                            fixed ring)
//   yface[par][slot][z][x], zface[par][slot][y][x]  likewise for y and z.
// A column's faces are staged in LDS (x, y) and registers (z) at the start of
// each step with all loads in flight at once.
#pragma once

#include <algorithm>
#include <utility>

#include "barrier.hpp"
#include "common.hpp"

namespace perks {

template <typename T>
struct Weights3D {
    T zm, ym, xm, c, xp, yp, zp;  // offsets (-1,0,0) (0,-1,0) (0,0,-1) (0,0,0) (0,0,1) (0,1,0) (1,0,0)
};

// One Jacobi step of one z-plane of a lane's block, in place.
//   cur[0..hy-1]  old plane values on entry, new values on exit.
//   part[iy]      on entry: the (dz=-1) term of cell iy, W.zm * old(z-1, y),
//                 already rounded; on exit the same term for the plane above,
//                 W.zm * old(z, y).  Accumulating the terms that an old value
//                 contributes to later cells while it is still live lets each
//                 new value take its old value's register.
//   ym, yp        old values at y0-1 and y0+hy of this plane (halo).
//   znext[iy]     old plane above.
// Terms are summed in ascending (dz, dy, dx) order: one multiply then FMAs,
// exactly as a straight evaluation of the seven-term sum would.
// Returns the new value of cell hy-1 (the tile's north edge row).
template <typename T, int RY, bool FULLY>
__device__ __forceinline__ T compute_plane(T (&cur)[RY], T (&part)[RY], const T (&znext)[RY], int hy, T ym, T yp,
                                           const T *lw, const T *le, const Weights3D<T> &W) {
    T last = T(0);
    T acc_next = fma_t(W.ym, ym, part[0]);   // (dz=-1) then (dy=-1) for cell 0
#pragma unroll
    for (int iy = 0; iy < RY; ++iy) {
        if (FULLY || iy < hy) {
            const T c = cur[iy];
            T acc = acc_next;
            const T w = from_west(c, lw[iy]);
            const T e = from_east(c, le[iy]);
            acc = fma_t(W.xm, w, acc);
            acc = fma_t(W.c, c, acc);
            acc = fma_t(W.xp, e, acc);
            // what old c contributes to later cells: (dy=-1) of cell iy+1 and
            // (dz=-1) of this cell in the plane above
            if (iy + 1 < RY) acc_next = fma_t(W.ym, c, part[iy + 1]);
            part[iy] = W.zm * c;
            T yn;
            if (iy + 1 < RY)
                yn = (FULLY || iy + 1 < hy) ? cur[iy + 1] : yp;
            else
                yn = yp;
            acc = fma_t(W.yp, yn, acc);
            const T nv = fma_untied(W.zp, znext[iy], acc);
            cur[iy] = nv;
            if (FULLY ? (iy == RY - 1) : true) last = (FULLY || iy == hy - 1) ? nv : last;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    return last;
}

// Wave tiles of the per-step baseline: 64 (x) x RY (y) x RZ (z).
struct Tile3D {
    int tx, ty, tz, x0, y0, z0, wx, hy, dz;
};

template <typename T>
struct Step3DParams {
    gmem<T> *src, *dst;
    int nx, ny, nz;
    int ntx, nty, ntz;
    int RY, RZ;
    int last_w, last_h, last_d;
    int ntiles;
    Weights3D<T> W;
};

template <typename T>
__device__ __forceinline__ Tile3D tile3_of(const Step3DParams<T> &p, int t) {
    Tile3D tl;
    tl.tx = t % p.ntx;
    tl.ty = (t / p.ntx) % p.nty;
    tl.tz = t / (p.ntx * p.nty);
    tl.x0 = 1 + 64 * tl.tx;
    tl.y0 = 1 + p.RY * tl.ty;
    tl.z0 = 1 + p.RZ * tl.tz;
    tl.wx = tl.tx == p.ntx - 1 ? p.last_w : 64;
    tl.hy = tl.ty == p.nty - 1 ? p.last_h : p.RY;
    tl.dz = tl.tz == p.ntz - 1 ? p.last_d : p.RZ;
    return tl;
}

// ---------------------------------------------------------------------------
// Persistent column kernel.
constexpr int C3_RY = 4;      // rows per lane
constexpr int C3_WAVES = 8;   // waves per workgroup (two per SIMD)
constexpr int C3_DZMAX = 32;  // deepest column (LDS staging of its faces)
constexpr int C3_SC = 2;      // planes per streamed chunk
// planes of each workgroup's first column kept in LDS (streaming kernel
// only): FP64 5 planes of 8 waves x 4 rows x 64 lanes = 80 KiB, which with
// the 80 KiB of face staging and row exchange fills the 160 KiB of LDS; FP32
// none (its register planes already cover the deepest column)
template <typename T> struct C3Lds { static constexpr int L = sizeof(T) == 8 ? 5 : 0; };
template <typename T> using LdsPlane = T[C3_WAVES][C3_RY][64];
// register-cached planes per lane: NC * RY values of 128 VGPRs
template <typename T> struct C3Cache { static constexpr int NC = sizeof(T) == 8 ? 12 : 32; };

template <typename T>
struct Col3DParams {
    gmem<T> *grid;
    gmem<T> *xface, *yface, *zface;
    unsigned *sync;
    long long steps;
    int nx, ny, nz;
    int ntx, nty, ntz, dz;
    int last_w, last_rows, last_d;
    int ncols, cached;   // cached: workgroups whose first column keeps planes on chip
    int nlds;            // planes of a cached column kept in LDS (below the register planes)
    Weights3D<T> W;
};

struct Col3D {
    int tx, ty, tz, x0, wx, yb, rows, z0, dz;
};

template <typename T>
__device__ __forceinline__ Col3D col_of(const Col3DParams<T> &p, int t) {
    Col3D c;
    c.tx = t % p.ntx;
    c.ty = (t / p.ntx) % p.nty;
    c.tz = t / (p.ntx * p.nty);
    c.x0 = 1 + 64 * c.tx;
    c.wx = c.tx == p.ntx - 1 ? p.last_w : 64;
    c.yb = 1 + C3_WAVES * C3_RY * c.ty;
    c.rows = c.ty == p.nty - 1 ? p.last_rows : C3_WAVES * C3_RY;
    c.z0 = 1 + p.dz * c.tz;
    c.dz = c.tz == p.ntz - 1 ? p.last_d : p.dz;
    return c;
}

// Rows of wave w in column c.  first: its south neighbour is outside the
// workgroup; last: its north neighbour is.
struct WaveRows {
    int y0, hy;
    bool first, last;
};
__device__ __forceinline__ WaveRows rows_of(const Col3D &c, int w) {
    WaveRows r;
    r.y0 = c.yb + w * C3_RY;
    r.hy = min(max(c.rows - w * C3_RY, 0), C3_RY);
    r.first = w == 0;
    r.last = r.hy > 0 && (w + 1) * C3_RY >= c.rows;
    return r;
}

template <typename T>
__device__ __forceinline__ gmem<T> *cxf(const Col3DParams<T> &p, int par, int slot) {
    return p.xface + ((size_t)par * (2 * p.ntx + 2) + slot) * p.nz * p.ny;
}
template <typename T>
__device__ __forceinline__ gmem<T> *cyf(const Col3DParams<T> &p, int par, int slot) {
    return p.yface + ((size_t)par * (2 * p.nty + 2) + slot) * p.nz * p.nx;
}
template <typename T>
__device__ __forceinline__ gmem<T> *czf(const Col3DParams<T> &p, int par, int slot) {
    return p.zface + ((size_t)par * (2 * p.ntz + 2) + slot) * p.ny * p.nx;
}

// Element e (a 32-bit lane offset) of a uniform base: the address stays a
// scalar base plus a 32-bit vector offset instead of a 64-bit vector address.
template <typename T>
__device__ __forceinline__ gmem<T> *at(gmem<T> *base, unsigned e) {
    return (gmem<T> *)((gmem<char> *)base + e * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const gmem<T> *at(const gmem<T> *base, unsigned e) {
    return (const gmem<T> *)((const gmem<char> *)base + e * (unsigned)sizeof(T));
}

template <typename T>
struct ColShared {
    T xs[C3_WAVES][2][C3_DZMAX][C3_RY];   // west / east face of each wave's rows, per plane
    T ysf[2][C3_DZMAX][64];               // south / north face of the column, per plane
    T ex[2][2][C3_WAVES][2][64];          // exchange [slot][plane of the pair][wave]: bottom / top row
};

// The fixed ring (both parities) from the grid.
template <typename T>
__device__ __forceinline__ void init_ring_faces_col(const Col3DParams<T> &p) {
    const size_t nthreads = (size_t)gridDim.x * blockDim.x;
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const gmem<T> *g = p.grid;
    const size_t nx = p.nx, ny = p.ny, nz = p.nz;
    for (int par = 0; par < 2; ++par) {
        for (size_t i = tid; i < nz * ny; i += nthreads) {  // planes x = 0, nx-1; i = z*ny + y
            st_coh(cxf(p, par, 0) + i, g[i * nx]);
            st_coh(cxf(p, par, 2 * p.ntx + 1) + i, g[i * nx + nx - 1]);
        }
        for (size_t i = tid; i < nz * nx; i += nthreads) {  // planes y = 0, ny-1; i = z*nx + x
            const size_t z = i / nx, x = i % nx;
            st_coh(cyf(p, par, 0) + i, g[(z * ny) * nx + x]);
            st_coh(cyf(p, par, 2 * p.nty + 1) + i, g[(z * ny + ny - 1) * nx + x]);
        }
        for (size_t i = tid; i < ny * nx; i += nthreads) {  // planes z = 0, nz-1; i = y*nx + x
            st_coh(czf(p, par, 0) + i, g[i]);
            st_coh(czf(p, par, 2 * p.ntz + 1) + i, g[(nz - 1) * ny * nx + i]);
        }
    }
}

// Parity-0 faces of column c from the grid (wave w's share).
template <typename T>
__device__ __forceinline__ void publish_initial_col(const Col3DParams<T> &p, const Col3D &c, int w, int lane) {
    const WaveRows wr = rows_of(c, w);
    if (wr.hy == 0) return;
    const gmem<T> *g = p.grid;
    const size_t nx = p.nx, ny = p.ny;
    for (int j = lane; j < wr.hy * c.dz; j += 64) {
        const int iz = j / wr.hy, iy = j % wr.hy;
        const size_t zy = (size_t)(c.z0 + iz) * ny + wr.y0 + iy;
        st_coh(cxf(p, 0, 2 * c.tx + 1) + zy, g[zy * nx + c.x0]);
        st_coh(cxf(p, 0, 2 * c.tx + 2) + zy, g[zy * nx + c.x0 + c.wx - 1]);
    }
    if (lane < c.wx) {
        const size_t x = c.x0 + lane;
        for (int iz = 0; iz < c.dz; ++iz) {
            const size_t z = c.z0 + iz;
            if (wr.first) st_coh(cyf(p, 0, 2 * c.ty + 1) + z * nx + x, g[(z * ny + wr.y0) * nx + x]);
            if (wr.last) st_coh(cyf(p, 0, 2 * c.ty + 2) + z * nx + x, g[(z * ny + wr.y0 + wr.hy - 1) * nx + x]);
        }
        for (int iy = 0; iy < wr.hy; ++iy) {
            const size_t y = wr.y0 + iy;
            st_coh(czf(p, 0, 2 * c.tz + 1) + y * nx + x, g[((size_t)c.z0 * ny + y) * nx + x]);
            st_coh(czf(p, 0, 2 * c.tz + 2) + y * nx + x, g[((size_t)(c.z0 + c.dz - 1) * ny + y) * nx + x]);
        }
    }
}

// Stage the x and y faces of column c (parity par) in LDS: every load of the
// workgroup in flight at once, then the LDS writes.
template <typename T>
__device__ __forceinline__ void stage_faces_col(const Col3DParams<T> &p, const Col3D &c, int par, ColShared<T> &sh) {
    constexpr int NT = C3_WAVES * 64;
    constexpr int NXV = C3_WAVES * 2 * C3_DZMAX * C3_RY, NYV = 2 * C3_DZMAX * 64;
    constexpr int KX = (NXV + NT - 1) / NT, KY = (NYV + NT - 1) / NT;
    const int tid = threadIdx.x;
    T xv[KX], yv[KY];
    const gmem<T> *fw = cxf(p, par, 2 * c.tx), *fe = cxf(p, par, 2 * c.tx + 3);
#pragma unroll
    for (int k = 0; k < KX; ++k) {
        const int e = tid + k * NT;
        const int iy = e % C3_RY, iz = (e / C3_RY) % C3_DZMAX, side = (e / (C3_RY * C3_DZMAX)) % 2,
                  w = e / (2 * C3_RY * C3_DZMAX);
        const int hy = min(max(c.rows - w * C3_RY, 0), C3_RY);
        const bool ok = e < NXV && iz < c.dz && iy < hy;
        const unsigned o = (unsigned)(iz * p.ny + w * C3_RY + iy);
        xv[k] = ok ? ld_coh(at((side ? fe : fw) + ((size_t)c.z0 * p.ny + c.yb), o)) : T(0);
    }
    const gmem<T> *fs = cyf(p, par, 2 * c.ty), *fn = cyf(p, par, 2 * c.ty + 3);
#pragma unroll
    for (int k = 0; k < KY; ++k) {
        const int e = tid + k * NT;
        const int x = e % 64, iz = (e / 64) % C3_DZMAX, side = e / (64 * C3_DZMAX);
        const bool ok = e < NYV && iz < c.dz && x < c.wx;
        const unsigned o = (unsigned)(iz * p.nx + x);
        yv[k] = ok ? ld_coh(at((side ? fn : fs) + ((size_t)c.z0 * p.nx + c.x0), o)) : T(0);
    }
    __builtin_amdgcn_sched_barrier(0);
    T *xs = &sh.xs[0][0][0][0];
    T *ys = &sh.ysf[0][0][0];
#pragma unroll
    for (int k = 0; k < KX; ++k)
        if (tid + k * NT < NXV) xs[tid + k * NT] = xv[k];
#pragma unroll
    for (int k = 0; k < KY; ++k)
        if (tid + k * NT < NYV) ys[tid + k * NT] = yv[k];
}

// Old values of the bottom and top rows of one plane of wave w's rows, posted
// for the neighbouring waves (exchange slot `slot`, plane k of the pair).
template <typename T, bool FULL>
__device__ __forceinline__ void post_rows(const WaveRows &wr, int w, int lane, int slot, int k,
                                          const T (&cur)[C3_RY], ColShared<T> &sh) {
    T top = cur[0];
#pragma unroll
    for (int iy = 1; iy < C3_RY; ++iy)
        if (FULL || iy < wr.hy) top = cur[iy];
    sh.ex[slot][k][w][0][lane] = cur[0];
    sh.ex[slot][k][w][1][lane] = top;
}

// Plane iz of wave w's rows, after the exchange: the neighbours' rows, the
// update of cur in place, and the new values of the column's outer faces.
template <typename T, bool FULL>
__device__ __forceinline__ void plane_work(const Col3DParams<T> &p, const Col3D &c, const WaveRows &wr, int w,
                                           int lane, int par, int iz, int slot, int k, T (&cur)[C3_RY],
                                           const T (&znext)[C3_RY], T (&part)[C3_RY], ColShared<T> &sh) {
    constexpr int RY = C3_RY;
    const T ym = wr.first ? sh.ysf[0][iz][lane] : sh.ex[slot][k][w - 1][1][lane];
    const T yp = wr.last ? sh.ysf[1][iz][lane] : sh.ex[slot][k][w + 1][0][lane];
    const T *lw = &sh.xs[w][0][iz][0];
    const T *le = &sh.xs[w][1][iz][0];
    // ghost lanes carry the east face so the last real lane's DPP east shift
    // picks it up (a select: no branch, no exec-mask change per plane)
    const bool ghost = lane >= c.wx;
    T e[RY];
#pragma unroll
    for (int iy = 0; iy < RY; ++iy) e[iy] = le[iy];
    settle(e);   // read by every lane: keeps the select below from becoming a branch
#pragma unroll
    for (int iy = 0; iy < RY; ++iy) cur[iy] = ghost ? e[iy] : cur[iy];
    const T last = compute_plane<T, RY, FULL>(cur, part, znext, wr.hy, ym, yp, lw, le, p.W);
    // The column's new west / east edges and south / north boundary rows go
    // to the LDS slots just consumed (xs[w], ysf), published to global memory
    // in one batch after the last plane; only the bottom and top planes are
    // stored here.  Lane 0 writes its rows into the west slot, lane wx-1
    // into the east one (with wx == 1 lane 0 holds both edges); rows beyond
    // hy are never published.
    if (lane == 0 || lane == c.wx - 1) {
        T *dst = &sh.xs[w][lane == 0 ? 0 : 1][iz][0];
#pragma unroll
        for (int iy = 0; iy < RY; ++iy) dst[iy] = cur[iy];
    }
    if (c.wx == 1 && lane == 0) {
#pragma unroll
        for (int iy = 0; iy < RY; ++iy) sh.xs[w][1][iz][iy] = cur[iy];
    }
    if (wr.first) sh.ysf[0][iz][lane] = cur[0];
    if (wr.last) sh.ysf[1][iz][lane] = last;
    if ((iz == 0 || iz == c.dz - 1) && !ghost) {
        // plane index laundered: the addresses are formed here, not
        // hoisted for every plane of the unrolled cached-plane loop
        int z = __builtin_amdgcn_readfirstlane(iz == 0 ? 1 : 2);
        asm volatile("" : "+s"(z));
        gmem<T> *f = opaque(czf(p, par ^ 1, 2 * c.tz + z) + (size_t)wr.y0 * p.nx);
        const unsigned xo = (unsigned)(c.x0 + lane);
#pragma unroll
        for (int iy = 0; iy < RY; ++iy)
            if (FULL || iy < wr.hy) st_coh(at(f, (unsigned)(iy * p.nx) + xo), cur[iy]);
        if (iz == 0 && c.dz == 1) {
            gmem<T> *f2 = opaque(czf(p, par ^ 1, 2 * c.tz + 2) + (size_t)wr.y0 * p.nx);
#pragma unroll
            for (int iy = 0; iy < RY; ++iy)
                if (FULL || iy < wr.hy) st_coh(at(f2, (unsigned)(iy * p.nx) + xo), cur[iy]);
        }
    }
}


// One or two consecutive planes (iz, and iz + 1 when `two`) of wave w's rows
// behind one workgroup barrier: each wave posts the old values of its edge
// rows of both planes, then updates them (a in place with the plane above
// being b, then b with zn; a alone with zn when !two).  Every wave of the
// workgroup calls this for the same planes; `phase` alternates the exchange
// slot from one call to the next.
template <typename T, bool FULL>
__device__ __forceinline__ void col_pair(const Col3DParams<T> &p, const Col3D &c, const WaveRows &wr, int w,
                                         int lane, int par, int iz, bool two, int &phase, T (&a)[C3_RY],
                                         T (&b)[C3_RY], const T (&zn)[C3_RY], T (&part)[C3_RY], ColShared<T> &sh) {
    const int slot = phase;
    phase ^= 1;
    if (wr.hy > 0) {
        post_rows<T, FULL>(wr, w, lane, slot, 0, a, sh);
        if (two) post_rows<T, FULL>(wr, w, lane, slot, 1, b, sh);
    }
    __syncthreads();
    if (wr.hy == 0) return;
    if (two) {
        plane_work<T, FULL>(p, c, wr, w, lane, par, iz, slot, 0, a, b, part, sh);
        plane_work<T, FULL>(p, c, wr, w, lane, par, iz + 1, slot, 1, b, zn, part, sh);
    } else {
        plane_work<T, FULL>(p, c, wr, w, lane, par, iz, slot, 0, a, zn, part, sh);
    }
}

template <typename T>
__device__ __forceinline__ void col_pair_any(const Col3DParams<T> &p, const Col3D &c, const WaveRows &wr, int w,
                                             int lane, int par, int iz, bool two, int &phase, T (&a)[C3_RY],
                                             T (&b)[C3_RY], const T (&zn)[C3_RY], T (&part)[C3_RY],
                                             ColShared<T> &sh) {
    if (wr.hy == C3_RY)
        col_pair<T, true>(p, c, wr, w, lane, par, iz, two, phase, a, b, zn, part, sh);
    else
        col_pair<T, false>(p, c, wr, w, lane, par, iz, two, phase, a, b, zn, part, sh);
}

// Publish the column's west / east edges and south / north boundary rows,
// gathered in LDS during the step, to parity par ^ 1 (the whole workgroup,
// after a barrier).
template <typename T>
__device__ __forceinline__ void publish_faces_col(const Col3DParams<T> &p, const Col3D &c, int par,
                                                  const ColShared<T> &sh) {
    constexpr int NT = C3_WAVES * 64;
    constexpr int NXV = C3_WAVES * 2 * C3_DZMAX * C3_RY, NYV = 2 * C3_DZMAX * 64;
    const int tid = threadIdx.x;
    gmem<T> *fw = cxf(p, par ^ 1, 2 * c.tx + 1) + ((size_t)c.z0 * p.ny + c.yb);
    gmem<T> *fe = cxf(p, par ^ 1, 2 * c.tx + 2) + ((size_t)c.z0 * p.ny + c.yb);
    const T *xs = &sh.xs[0][0][0][0];
    for (int e = tid; e < NXV; e += NT) {
        const int iy = e % C3_RY, iz = (e / C3_RY) % C3_DZMAX, side = (e / (C3_RY * C3_DZMAX)) % 2,
                  w = e / (2 * C3_RY * C3_DZMAX);
        const int hy = min(max(c.rows - w * C3_RY, 0), C3_RY);
        if (iz < c.dz && iy < hy) st_coh(at(side ? fe : fw, (unsigned)(iz * p.ny + w * C3_RY + iy)), xs[e]);
    }
    gmem<T> *fs = cyf(p, par ^ 1, 2 * c.ty + 1) + ((size_t)c.z0 * p.nx + c.x0);
    gmem<T> *fn = cyf(p, par ^ 1, 2 * c.ty + 2) + ((size_t)c.z0 * p.nx + c.x0);
    const T *ys = &sh.ysf[0][0][0];
    for (int e = tid; e < NYV; e += NT) {
        const int x = e % 64, iz = (e / 64) % C3_DZMAX, side = e / (64 * C3_DZMAX);
        if (iz < c.dz && x < c.wx) st_coh(at(side ? fn : fs, (unsigned)(iz * p.nx + x)), ys[e]);
    }
}

// Loads of streamed planes [j, j + SC) (those below `n`) of wave w's rows.
template <typename T>
__device__ __forceinline__ void load_chunk(const Col3DParams<T> &p, const Col3D &c, const WaveRows &wr, int xl,
                                           int j, int n, T (&buf)[C3_SC][C3_RY]) {
#pragma unroll
    for (int k = 0; k < C3_SC; ++k) {
        const gmem<T> *g = opaque(p.grid + ((size_t)(c.z0 + j + k) * p.ny + wr.y0) * p.nx);
#pragma unroll
        for (int iy = 0; iy < C3_RY; ++iy)
            buf[k][iy] = (j + k < n && iy < wr.hy) ? *at(g, (unsigned)(iy * p.nx + xl)) : T(0);
    }
}

template <typename T>
__device__ __forceinline__ void store_plane(const Col3DParams<T> &p, const Col3D &c, const WaveRows &wr, int lane,
                                            int iz, const T (&v)[C3_RY]) {
    if (lane >= c.wx) return;
    gmem<T> *g = opaque(p.grid + ((size_t)(c.z0 + iz) * p.ny + wr.y0) * p.nx);
#pragma unroll
    for (int iy = 0; iy < C3_RY; ++iy)
        if (iy < wr.hy) *at(g, (unsigned)(iy * p.nx + c.x0 + lane)) = v[iy];
}

// rows[k] = src for the k (runtime, uniform) given; no-op when k >= N.
// Every entry is rewritten with a select, so that no store has a run-time
// index (which would move the whole array to scratch memory).
template <int N, typename T>
__device__ __forceinline__ void put_plane(T (&rows)[N][C3_RY], int k, const T (&src)[C3_RY]) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int iy = 0; iy < C3_RY; ++iy) rows[i][iy] = i == k ? src[iy] : rows[i][iy];
}

// Streamed planes j, j + 1 (those below nstream) of the column from buf, as
// one pair; the plane after buf's last is nxt[0].  The caller has put the
// plane above the last streamed one where the chunk that ends the stream
// looks for it (buf[1] when only plane j remains).
template <typename T>
__device__ __forceinline__ void run_chunk(const Col3DParams<T> &p, const Col3D &c, const WaveRows &wr, int w,
                                          int lane, int par, int j, int nstream, int &phase,
                                          T (&buf)[C3_SC][C3_RY], const T (&nxt)[C3_SC][C3_RY], T (&part)[C3_RY],
                                          ColShared<T> &sh) {
    static_assert(C3_SC == 2, "a streamed chunk is one pair of planes");
    // the chunk's loads complete here, once, not at every later use
#pragma unroll
    for (int k = 0; k < C3_SC; ++k) settle(buf[k]);
    const bool two = j + 1 < nstream;
    T zn[C3_RY];
#pragma unroll
    for (int iy = 0; iy < C3_RY; ++iy) zn[iy] = two ? nxt[0][iy] : buf[1][iy];
    col_pair_any(p, c, wr, w, lane, par, j, two, phase, buf[0], buf[1], zn, part, sh);
    if (wr.hy > 0) {
        store_plane(p, c, wr, lane, j, buf[0]);
        if (two) store_plane(p, c, wr, lane, j + 1, buf[1]);
    }
}

// Cached planes I and I + 1 (I even, compile-time, so that v is indexed
// statically: the planes are expanded by a fold, not by the loop unroller,
// whose size limit would otherwise leave v in scratch memory).  v[ncache]
// holds the plane above the last cached one when ncache < NC.
template <typename T, int NC, int I>
__device__ __forceinline__ void cached_pair(const Col3DParams<T> &p, const Col3D &c, const WaveRows &wr, int w,
                                            int lane, int par, int iz0, int ncache, int &phase, T (&v)[NC][C3_RY],
                                            const T (&zt)[C3_RY], T (&part)[C3_RY], ColShared<T> &sh) {
    static_assert(NC % 2 == 0, "register planes come in pairs");
    if constexpr (I % 2 == 0) {
        if (I < ncache) {
            const bool two = I + 1 < ncache;
            T zn[C3_RY];
#pragma unroll
            for (int iy = 0; iy < C3_RY; ++iy) {
                if constexpr (I + 2 < NC)
                    zn[iy] = two ? v[I + 2][iy] : v[I + 1][iy];
                else
                    zn[iy] = two ? zt[iy] : v[I + 1][iy];
            }
            col_pair_any(p, c, wr, w, lane, par, iz0 + I, two, phase, v[I], v[I + 1], zn, part, sh);
        }
    }
}
template <typename T, int NC, int... I>
__device__ __forceinline__ void cached_planes(const Col3DParams<T> &p, const Col3D &c, const WaveRows &wr, int w,
                                              int lane, int par, int iz0, int ncache, int &phase, T (&v)[NC][C3_RY],
                                              const T (&zt)[C3_RY], T (&part)[C3_RY], ColShared<T> &sh,
                                              std::integer_sequence<int, I...>) {
    (cached_pair<T, NC, I>(p, c, wr, w, lane, par, iz0, ncache, phase, v, zt, part, sh), ...);
}

// One step of column c: the streamed planes (bottom dz - nlds - ncache),
// the LDS-cached ones (next nlds, in lp) and the register-cached ones (top
// ncache, in v[0 .. ncache)).  STREAM = false: the plan has every plane of
// every column in registers (nstream == nlds == 0).
template <typename T, int NC, bool STREAM>
__device__ __forceinline__ void column_step(const Col3DParams<T> &p, const Col3D &c, int w, int lane, int par,
                                            int ncache, int nlds, T (&v)[NC][C3_RY], LdsPlane<T> *lp,
                                            ColShared<T> &sh) {
    constexpr int RY = C3_RY, SC = C3_SC;
    const WaveRows wr = rows_of(c, w);
    const int xl = min(c.x0 + lane, p.nx - 1);
    const int nstream = STREAM ? c.dz - ncache - nlds : 0;
    __syncthreads();   // the previous column's readers are done with sh
    T zb[RY], zt[RY];
    T sa[SC][RY], sb[SC][RY];
    {
        const gmem<T> *fb = czf(p, par, 2 * c.tz) + (size_t)wr.y0 * p.nx;
        const gmem<T> *ft = czf(p, par, 2 * c.tz + 3) + (size_t)wr.y0 * p.nx;
#pragma unroll
        for (int iy = 0; iy < RY; ++iy) {
            zb[iy] = iy < wr.hy ? ld_coh(at(fb, (unsigned)(iy * p.nx + xl))) : T(0);
            zt[iy] = iy < wr.hy ? ld_coh(at(ft, (unsigned)(iy * p.nx + xl))) : T(0);
        }
    }
    if (STREAM && nstream > 0) load_chunk(p, c, wr, xl, 0, nstream, sa);
    stage_faces_col(p, c, par, sh);
    // every load so far (faces, first chunk) completes here, before any
    // store of the step: a wait placed later would also wait for the stores
    settle(zb);
    settle(zt);
    if constexpr (STREAM) {
#pragma unroll
        for (int k = 0; k < SC; ++k) settle(sa[k]);
    }
    __syncthreads();
    T part[RY];
#pragma unroll
    for (int iy = 0; iy < RY; ++iy) part[iy] = p.W.zm * zb[iy];
    int phase = 0;
    if constexpr (STREAM) {
    // old values of the plane above the last streamed plane
    T above[RY];
#pragma unroll
    for (int iy = 0; iy < RY; ++iy) above[iy] = nlds > 0 ? lp[0][w][iy][lane] : ncache > 0 ? v[0][iy] : zt[iy];
    for (int j = 0; j < nstream; j += 2 * SC) {
        if (j + SC < nstream) load_chunk(p, c, wr, xl, j + SC, nstream, sb);
        if (nstream - j <= SC) {
            put_plane<SC>(sa, nstream - j, above);
            put_plane<SC>(sb, nstream - j - SC, above);
        }
        run_chunk(p, c, wr, w, lane, par, j, nstream, phase, sa, sb, part, sh);
        if (j + SC >= nstream) break;
        if (j + 2 * SC < nstream) load_chunk(p, c, wr, xl, j + 2 * SC, nstream, sa);
        if (nstream - j - SC <= SC) {
            put_plane<SC>(sb, nstream - j - SC, above);
            put_plane<SC>(sa, nstream - j - 2 * SC, above);
        }
        run_chunk(p, c, wr, w, lane, par, j + SC, nstream, phase, sb, sa, part, sh);
    }
    // no chunk load is left in flight; telling the compiler so keeps it from
    // waiting for one (and for every store after it) in the cached planes
#pragma unroll
    for (int k = 0; k < SC; ++k) {
        settle(sa[k]);
        settle(sb[k]);
    }
    // LDS planes: read, updated, written back; the plane above the last one
    // is the first register plane or the face above the column
    for (int l = 0; l < nlds; l += 2) {
        const bool two = l + 1 < nlds;
        const int la = l + (two ? 2 : 1);   // the plane above the pair (or the single plane)
        T a[RY], b[RY], zn[RY];
#pragma unroll
        for (int iy = 0; iy < RY; ++iy) {
            a[iy] = lp[l][w][iy][lane];
            b[iy] = two ? lp[l + 1][w][iy][lane] : T(0);
            zn[iy] = la < nlds ? lp[la][w][iy][lane] : ncache > 0 ? v[0][iy] : zt[iy];
        }
        col_pair_any(p, c, wr, w, lane, par, nstream + l, two, phase, a, b, zn, part, sh);
#pragma unroll
        for (int iy = 0; iy < RY; ++iy) {
            lp[l][w][iy][lane] = a[iy];
            if (two) lp[l + 1][w][iy][lane] = b[iy];
        }
    }
    }
    // cached planes: the plane above the last one is v[ncache] (a free slot
    // when ncache < NC; with ncache == 0 there are none and v, which may
    // hold the workgroup's first column, is left alone) or the face above
    if (ncache > 0 && ncache < NC) put_plane<NC>(v, ncache, zt);
    cached_planes<T, NC>(p, c, wr, w, lane, par, nstream + nlds, ncache, phase, v, zt, part, sh,
                         std::make_integer_sequence<int, NC>());
    __syncthreads();
    publish_faces_col(p, c, par, sh);
}

template <typename T, int NC, bool STREAM>
__global__ __launch_bounds__(C3_WAVES * 64) __attribute__((amdgpu_waves_per_eu(1, C3_WAVES / 4))) void
stencil3d_column(Col3DParams<T> p) {
    constexpr int RY = C3_RY;
    __shared__ ColShared<T> sh;
    __shared__ LdsPlane<T> lp[STREAM && C3Lds<T>::L > 0 ? C3Lds<T>::L : 1];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    GridSync gs;
    gs.init(p.sync);
    init_ring_faces_col(p);
    for (int t = blockIdx.x; t < p.ncols; t += gridDim.x) publish_initial_col(p, col_of(p, t), w, lane);
    gs.sync();

    // the first column's top planes, in registers, and the planes below
    // them in LDS
    T v[NC][RY];
    int ncache0 = 0, nlds0 = 0;
    if ((int)blockIdx.x < p.ncols) {
        const Col3D c = col_of(p, blockIdx.x);
        const WaveRows wr = rows_of(c, w);
        ncache0 = (int)blockIdx.x < p.cached ? min(NC, c.dz) : 0;
        nlds0 = STREAM && (int)blockIdx.x < p.cached ? min(p.nlds, c.dz - ncache0) : 0;
        const int xl = min(c.x0 + lane, p.nx - 1);
        const int zc = c.z0 + c.dz - ncache0;
        for (int l = 0; l < nlds0; ++l)
#pragma unroll
            for (int iy = 0; iy < RY; ++iy)
                lp[l][w][iy][lane] =
                    iy < wr.hy ? p.grid[((size_t)(zc - nlds0 + l) * p.ny + wr.y0 + iy) * p.nx + xl] : T(0);
#pragma unroll
        for (int i = 0; i < NC; ++i)
#pragma unroll
            for (int iy = 0; iy < RY; ++iy)
                v[i][iy] = (i < ncache0 && iy < wr.hy)
                               ? p.grid[((size_t)(zc + i) * p.ny + wr.y0 + iy) * p.nx + xl]
                               : T(0);
    }
    // The register cache's initial loads complete here: otherwise their waits
    // land inside the step loop, where each would also wait, every step, for
    // all the stores issued before it (vmcnt counts loads and stores alike).
#pragma unroll
    for (int i = 0; i < NC; ++i) settle(v[i]);
    for (long long s = 0; s < p.steps; ++s) {
        const int par = (int)(s & 1);
        Col3DParams<T> q = p;
        q.grid = opaque(q.grid);
        q.xface = opaque(q.xface);
        q.yface = opaque(q.yface);
        q.zface = opaque(q.zface);
        int k = 0;
        for (int t = blockIdx.x; t < p.ncols; t += gridDim.x, ++k)
            column_step<T, NC, STREAM>(q, col_of(q, t), w, lane, par, k == 0 ? ncache0 : 0, k == 0 ? nlds0 : 0, v,
                                       lp, sh);
        gs.sync();
    }
    if ((int)blockIdx.x < p.ncols && ncache0 + nlds0 > 0) {
        const Col3D c = col_of(p, blockIdx.x);
        const WaveRows wr = rows_of(c, w);
        const int zc = c.z0 + c.dz - ncache0;
        if (lane < c.wx) {
            for (int l = 0; l < nlds0; ++l)
#pragma unroll
                for (int iy = 0; iy < RY; ++iy)
                    if (iy < wr.hy)
                        p.grid[((size_t)(zc - nlds0 + l) * p.ny + wr.y0 + iy) * p.nx + c.x0 + lane] = lp[l][w][iy][lane];
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int iy = 0; iy < RY; ++iy)
                    if (i < ncache0 && iy < wr.hy)
                        p.grid[((size_t)(zc + i) * p.ny + wr.y0 + iy) * p.nx + c.x0 + lane] = v[i][iy];
        }
    }
    gs.finish();
}

// Per-step baseline: one wave per tile, src -> dst.  The west/east faces are
// staged in LDS in the persistent kernel's layout and the same compute_plane
// is applied, so the two paths round identically; every other neighbour is
// read straight from src (ghost lanes read the real east column).
template <typename T, int RY, int RZ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void stencil3d_step(Step3DParams<T> p) {
    __shared__ T hx[WAVES][2][RY * RZ];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = blockIdx.x * WAVES + wave;
    if (t >= p.ntiles) return;
    T *lw = hx[wave][0];
    T *le = hx[wave][1];
    const Tile3D tl = tile3_of(p, t);
    const gmem<T> *src = p.src;
    const size_t nx = p.nx, ny = p.ny;
    const int xl = min(tl.x0 + lane, p.nx - 1);
    for (int j = lane; j < RY * RZ; j += 64) {
        const int iz = j / RY, iy = j % RY;
        if (iz < tl.dz && iy < tl.hy) {
            const size_t row = ((size_t)(tl.z0 + iz) * ny + tl.y0 + iy) * nx;
            lw[j] = src[row + tl.x0 - 1];
            le[j] = src[row + tl.x0 + tl.wx];
        }
    }
    compiler_fence();
    T cur[RY], nxt[RY], part[RY];
    const size_t col = (size_t)tl.y0 * nx + xl;
    const size_t plane = ny * nx;
#pragma unroll
    for (int iy = 0; iy < RY; ++iy) {
        part[iy] = p.W.zm * ((iy < tl.hy) ? src[((size_t)tl.z0 - 1) * plane + col + (size_t)iy * nx] : T(0));
        cur[iy] = (iy < tl.hy) ? src[(size_t)tl.z0 * plane + col + (size_t)iy * nx] : T(0);
    }
    for (int iz = 0; iz < tl.dz; ++iz) {
        const size_t pz = (size_t)(tl.z0 + iz) * plane;
        const T ym = src[pz + col - nx];
        const T yp = src[pz + col + (size_t)tl.hy * nx];
#pragma unroll
        for (int iy = 0; iy < RY; ++iy) nxt[iy] = (iy < tl.hy) ? src[pz + plane + col + (size_t)iy * nx] : T(0);
        if (tl.hy == RY)
            compute_plane<T, RY, true>(cur, part, nxt, RY, ym, yp, lw + iz * RY, le + iz * RY, p.W);
        else
            compute_plane<T, RY, false>(cur, part, nxt, tl.hy, ym, yp, lw + iz * RY, le + iz * RY, p.W);
        if (lane < tl.wx) {
#pragma unroll
            for (int iy = 0; iy < RY; ++iy)
                if (iy < tl.hy) p.dst[pz + col + (size_t)iy * nx] = cur[iy];
        }
#pragma unroll
        for (int iy = 0; iy < RY; ++iy) cur[iy] = nxt[iy];
    }
}

// ---------------------------------------------------------------------------
// Host planning / launch (3D).
constexpr int W3B = 4;    // waves per workgroup, baseline
constexpr int RYB = 4, RZB = 8;

struct PlanCol {
    int dz = 0, ntx = 0, nty = 0, ntz = 0, last_w = 0, last_rows = 0, last_d = 0, ncols = 0, cached = 0, wgs = 0,
        nc = 0, nlds = 0;
    const void *fn = nullptr;
};

// Column depth: the request (planes_per_lane, 1..C3_DZMAX), else the
// shallowest column for which the grid has no more columns than the device
// holds workgroups (so every workgroup's planes can be on chip), else the
// deepest.
template <typename T>
int plan3d(const perks_shape &s, const perks_tuning *tu, PlanCol *pl) {
    DeviceFacts f;
    int rc = device_facts(&f);
    if (rc) return rc;
    if (tu && tu->rows_per_lane && tu->rows_per_lane != C3_RY)
        return set_error(PERKS_E_UNSUPPORTED, "3D: rows_per_lane must be %d (or 0)", C3_RY);
    if (tu && tu->waves_per_wg && tu->waves_per_wg != C3_WAVES)
        return set_error(PERKS_E_UNSUPPORTED, "3D: waves_per_wg must be %d (or 0)", C3_WAVES);
    if (tu && (tu->planes_per_lane < 0 || tu->planes_per_lane > C3_DZMAX))
        return set_error(PERKS_E_UNSUPPORTED, "3D: planes_per_lane (column depth) must be 0..%d", C3_DZMAX);
    constexpr int NC = C3Cache<T>::NC;
    pl->fn = reinterpret_cast<const void *>(&stencil3d_column<T, NC, true>);
    pl->nc = NC;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, pl->fn, C3_WAVES * 64, 0) != hipSuccess || occ < 1) {
        (void)hipGetLastError();
        return set_error(PERKS_E_NOTCORESIDENT, "3D column kernel does not fit a CU");
    }
    const long long cap = (long long)f.cus * std::min(occ, (tu && tu->wgs_per_cu > 0) ? tu->wgs_per_cu : 1);
    const long long nxi = s.nx - 2, nyi = s.ny - 2, nzi = s.nz - 2;
    const int rows = C3_WAVES * C3_RY;
    pl->ntx = (int)((nxi + 63) / 64);
    pl->last_w = (int)(nxi - 64 * (pl->ntx - 1));
    pl->nty = (int)((nyi + rows - 1) / rows);
    pl->last_rows = (int)(nyi - (long long)rows * (pl->nty - 1));
    const long long nxy = (long long)pl->ntx * pl->nty;
    int dz = tu ? tu->planes_per_lane : 0;
    if (!dz) {
        dz = C3_DZMAX;
        for (int d = 1; d <= C3_DZMAX; ++d)
            if (nxy * ((nzi + d - 1) / d) <= cap) {
                dz = d;
                break;
            }
    }
    dz = (int)std::min<long long>(dz, nzi);
    pl->dz = dz;
    pl->ntz = (int)((nzi + dz - 1) / dz);
    pl->last_d = (int)(nzi - (long long)dz * (pl->ntz - 1));
    const long long nc = nxy * pl->ntz;
    if (nc > (1LL << 30)) return set_error(PERKS_E_UNSUPPORTED, "too many columns");
    pl->ncols = (int)nc;
    pl->wgs = (int)std::min(nc, cap);
    long long cached = pl->wgs;
    if (tu && tu->max_cached_tiles < 0) cached = 0;
    if (tu && tu->max_cached_tiles > 0) cached = std::min<long long>(cached, tu->max_cached_tiles);
    pl->cached = (int)cached;
    // every plane of every column in registers: the kernel without the
    // streaming path (less code, fewer registers)
    pl->nlds = pl->cached > 0 ? C3Lds<T>::L : 0;
    if (pl->cached == pl->ncols && dz <= NC) {
        pl->fn = reinterpret_cast<const void *>(&stencil3d_column<T, NC, false>);
        pl->nlds = 0;
    }
    return PERKS_OK;
}

template <typename T>
void fill_weights3(Weights3D<T> &W, const double *c) {
    W.zm = (T)c[(0 * 3 + 1) * 3 + 1];
    W.ym = (T)c[(1 * 3 + 0) * 3 + 1];
    W.xm = (T)c[(1 * 3 + 1) * 3 + 0];
    W.c = (T)c[(1 * 3 + 1) * 3 + 1];
    W.xp = (T)c[(1 * 3 + 1) * 3 + 2];
    W.yp = (T)c[(1 * 3 + 2) * 3 + 1];
    W.zp = (T)c[(2 * 3 + 1) * 3 + 1];
}


template <typename T>
int run3d(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, hipStream_t st,
          const perks_tuning *tu) {
    PlanCol pl;
    int rc = plan3d<T>(s, tu, &pl);
    if (rc) return rc;
    Col3DParams<T> p{};
    p.grid = to_global(grid);
    p.nx = (int)s.nx;
    p.ny = (int)s.ny;
    p.nz = (int)s.nz;
    p.ntx = pl.ntx;
    p.nty = pl.nty;
    p.ntz = pl.ntz;
    p.dz = pl.dz;
    p.last_w = pl.last_w;
    p.last_rows = pl.last_rows;
    p.last_d = pl.last_d;
    p.ncols = pl.ncols;
    p.cached = pl.cached;
    p.nlds = pl.nlds;
    p.steps = steps;
    fill_weights3(p.W, coeffs);
    const size_t fx = (size_t)2 * (2 * pl.ntx + 2) * s.nz * s.ny;
    const size_t fy = (size_t)2 * (2 * pl.nty + 2) * s.nz * s.nx;
    const size_t fz = (size_t)2 * (2 * pl.ntz + 2) * s.ny * s.nx;
    T *faces = (T *)scratch(SLOT_FACES, (fx + fy + fz) * sizeof(T));
    unsigned *sync = (unsigned *)scratch(SLOT_SYNC, SYNC_BYTES);
    if (!faces || !sync) return PERKS_E_NOMEM;
    p.xface = to_global(faces);
    p.yface = to_global(faces + fx);
    p.zface = to_global(faces + fx + fy);
    p.sync = sync;
    return launch_coop(pl.fn, pl.wgs, C3_WAVES * 64, &p, st);
}

template <typename T>
int baseline3d(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, hipStream_t st) {
    const size_t cells = (size_t)s.nx * s.ny * s.nz;
    T *other = (T *)scratch(SLOT_PINGPONG, cells * sizeof(T));
    if (!other) return PERKS_E_NOMEM;
    Step3DParams<T> p{};
    p.nx = (int)s.nx;
    p.ny = (int)s.ny;
    p.nz = (int)s.nz;
    const long long nxi = s.nx - 2, nyi = s.ny - 2, nzi = s.nz - 2;
    p.ntx = (int)((nxi + 63) / 64);
    p.nty = (int)((nyi + RYB - 1) / RYB);
    p.ntz = (int)((nzi + RZB - 1) / RZB);
    p.RY = RYB;
    p.RZ = RZB;
    p.last_w = (int)(nxi - 64LL * (p.ntx - 1));
    p.last_h = (int)(nyi - (long long)RYB * (p.nty - 1));
    p.last_d = (int)(nzi - (long long)RZB * (p.ntz - 1));
    const long long nt = (long long)p.ntx * p.nty * p.ntz;
    if (nt > (1LL << 30)) return set_error(PERKS_E_UNSUPPORTED, "too many tiles");
    p.ntiles = (int)nt;
    fill_weights3(p.W, coeffs);
    PERKS_HIP_TRY(hipMemcpyAsync(other, grid, cells * sizeof(T), hipMemcpyDeviceToDevice, st));
    const int wgs = (int)((nt + W3B - 1) / W3B);
    T *a = grid, *b = other;
    for (int64_t k = 0; k < steps; ++k) {
        p.src = to_global(a);
        p.dst = to_global(b);
        hipLaunchKernelGGL((stencil3d_step<T, RYB, RZB, W3B>), dim3(wgs), dim3(W3B * 64), 0, st, p);
        std::swap(a, b);
    }
    PERKS_HIP_TRY(hipGetLastError());
    if (a != grid) PERKS_HIP_TRY(hipMemcpyAsync(grid, a, cells * sizeof(T), hipMemcpyDeviceToDevice, st));
    return PERKS_OK;
}

template <typename T>
int plan3d_query(const perks_shape &s, const perks_tuning *tu, perks_stencil_plan *plan) {
    PlanCol pl;
    int rc = plan3d<T>(s, tu, &pl);
    if (rc) return rc;
    plan->wgs = pl.wgs;
    plan->waves_per_wg = C3_WAVES;
    plan->rows_per_lane = C3_RY;
    plan->planes_per_lane = pl.dz;
    plan->tiles = pl.ncols;
    plan->cached_tiles = pl.cached;
    plan->interior_cells = (s.nx - 2) * (s.ny - 2) * (s.nz - 2);
    int64_t cc = 0, face = 0;
    for (int t = 0; t < pl.ncols; ++t) {
        const int tx = t % pl.ntx, ty = (t / pl.ntx) % pl.nty, tz = t / (pl.ntx * pl.nty);
        const int64_t wx = tx == pl.ntx - 1 ? pl.last_w : 64,
                      rows = ty == pl.nty - 1 ? pl.last_rows : C3_WAVES * C3_RY,
                      dz = tz == pl.ntz - 1 ? pl.last_d : pl.dz;
        if (t < pl.cached) cc += wx * rows * std::min<int64_t>(dz, pl.nc + pl.nlds);
        // the column's outer faces, written and read once per step
        face += 2 * (2 * rows * dz + 2 * wx * dz + 2 * wx * rows);
    }
    plan->cached_cells = cc;
    plan->halo_bytes_per_step = face * (int64_t)sizeof(T);
    plan->sync = 1;
    plan->lds_rows_per_lane = pl.nlds;   // 3D: planes of each cached column in LDS
    return PERKS_OK;
}

}  // namespace perks
