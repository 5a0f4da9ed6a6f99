// 3D 7-point Jacobi stencil (tab:domain "3d7pt") on gfx950: tile arithmetic,
// persistent kernel, per-step-launch baseline kernel, and host planning.
//
// Tiling.  The interior is cut into wave tiles of 64 (x) x RY (y) x RZ (z)
// cells.  Lane l owns column x0+l and keeps its RY x RZ block in registers:
// y and z neighbours are in the lane's registers, x neighbours arrive through
// DPP lane shifts, and the tile's six outer faces (halo) come from face
// buffers in global coordinates, double-buffered by step parity:
//   xface[par][slot][z][y]  (slot 2tx+1 / 2tx+2 = left / right edge plane of
//                            tile column tx; 0 and 2*ntx+1 = the fixed ring)
//   yface[par][slot][z][x], zface[par][slot][y][x]  likewise for y and z.
// Halo faces are staged in LDS for the step.
#pragma once

#include <algorithm>

#include "barrier.hpp"
#include "common.hpp"

namespace perks {

template <typename T>
struct Weights3D {
    T zm, ym, xm, c, xp, yp, zp;  // offsets (-1,0,0) (0,-1,0) (0,0,-1) (0,0,0) (0,0,1) (0,1,0) (1,0,0)
};

// LDS halo of one wave tile.
template <typename T, int RY, int RZ>
struct Halo3D {
    T xw[RZ * RY], xe[RZ * RY];   // west / east face, [iz][iy]
    T ym[RZ * 64], yp[RZ * 64];   // south / north face (y-1 / y+hy), [iz][lane]
    T zp[RY * 64];                // above face (z+dz), [iy][lane]; the face below is read directly
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
    T acc_next = __builtin_fma(W.ym, ym, part[0]);   // (dz=-1) then (dy=-1) for cell 0
#pragma unroll
    for (int iy = 0; iy < RY; ++iy) {
        if (FULLY || iy < hy) {
            const T c = cur[iy];
            T acc = acc_next;
            const T w = from_west(c, lw[iy]);
            const T e = from_east(c, le[iy]);
            acc = __builtin_fma(W.xm, w, acc);
            acc = __builtin_fma(W.c, c, acc);
            acc = __builtin_fma(W.xp, e, acc);
            // what old c contributes to later cells: (dy=-1) of cell iy+1 and
            // (dz=-1) of this cell in the plane above
            if (iy + 1 < RY) acc_next = __builtin_fma(W.ym, c, part[iy + 1]);
            part[iy] = W.zm * c;
            T yn;
            if (iy + 1 < RY)
                yn = (FULLY || iy + 1 < hy) ? cur[iy + 1] : yp;
            else
                yn = yp;
            acc = __builtin_fma(W.yp, yn, acc);
            const T nv = fma_untied(W.zp, znext[iy], acc);
            cur[iy] = nv;
            if (FULLY ? (iy == RY - 1) : true) last = (FULLY || iy == hy - 1) ? nv : last;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    return last;
}

struct Tile3D {
    int tx, ty, tz, x0, y0, z0, wx, hy, dz;
};

template <typename T>
struct Stencil3DParams {
    T *grid;
    T *src, *dst;      // baseline buffers
    T *xface, *yface, *zface;
    unsigned *sync;
    long long steps;
    int nx, ny, nz;
    int ntx, nty, ntz;
    int RY, RZ;
    int last_w, last_h, last_d;
    int ntiles, cached;
    Weights3D<T> W;
};

template <typename T>
__device__ __forceinline__ Tile3D tile3_of(const Stencil3DParams<T> &p, int t) {
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

template <typename T>
__device__ __forceinline__ T *xf(const Stencil3DParams<T> &p, int par, int slot) {
    return p.xface + ((size_t)par * (2 * p.ntx + 2) + slot) * p.nz * p.ny;
}
template <typename T>
__device__ __forceinline__ T *yf(const Stencil3DParams<T> &p, int par, int slot) {
    return p.yface + ((size_t)par * (2 * p.nty + 2) + slot) * p.nz * p.nx;
}
template <typename T>
__device__ __forceinline__ T *zf(const Stencil3DParams<T> &p, int par, int slot) {
    return p.zface + ((size_t)par * (2 * p.ntz + 2) + slot) * p.ny * p.nx;
}

// Stage the six halo faces of tile tl (parity par) into LDS.
template <typename T, int RY, int RZ>
__device__ __forceinline__ void load_halo3(const Stencil3DParams<T> &p, const Tile3D &tl, int par, int lane,
                                           Halo3D<T, RY, RZ> &h) {
    const int xl = min(tl.x0 + lane, p.nx - 1);
    const T *w = xf(p, par, 2 * tl.tx), *e = xf(p, par, 2 * tl.tx + 3);
    for (int j = lane; j < RY * RZ; j += 64) {
        const int iz = j / RY, iy = j % RY;
        if (iz < tl.dz && iy < tl.hy) {
            const size_t o = (size_t)(tl.z0 + iz) * p.ny + tl.y0 + iy;
            h.xw[j] = ld_coh(w + o);
            h.xe[j] = ld_coh(e + o);
        }
    }
    // y and z faces: four rows of loads in flight at a time (all of them at
    // once would hold 2 (RZ + RY) values per lane in registers next to the
    // cached block)
    const T *ys = yf(p, par, 2 * tl.ty), *yn = yf(p, par, 2 * tl.ty + 3);
#pragma unroll 1
    for (int iz = 0; iz < RZ; iz += 4) {
        T a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (iz + u < tl.dz) {
                const size_t o = (size_t)(tl.z0 + iz + u) * p.nx + xl;
                a[u] = ld_coh(ys + o);
                b[u] = ld_coh(yn + o);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (iz + u < tl.dz) {
                h.ym[(iz + u) * 64 + lane] = a[u];
                h.yp[(iz + u) * 64 + lane] = b[u];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    const T *zb = zf(p, par, 2 * tl.tz), *zt = zf(p, par, 2 * tl.tz + 3);
#pragma unroll 1
    for (int iy = 0; iy < RY; iy += 4) {
        T a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (iy + u < tl.hy) {
                const size_t o = (size_t)(tl.y0 + iy + u) * p.nx + xl;
                b[u] = ld_coh(zt + o);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (iy + u < tl.hy) {
                h.zp[(iy + u) * 64 + lane] = b[u];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    compiler_fence();
}

// Publish the edges of plane iz (values in u[0..hy-1]) of tile tl.
template <typename T, int RY>
__device__ __forceinline__ void publish_plane(const Stencil3DParams<T> &p, const Tile3D &tl, int par, int lane,
                                              const T (&u)[RY], int iz, T last) {

    const bool in = lane < tl.wx;
    const int z = tl.z0 + iz;
    T *left = xf(p, par, 2 * tl.tx + 1) + (size_t)z * p.ny + tl.y0;
    T *right = xf(p, par, 2 * tl.tx + 2) + (size_t)z * p.ny + tl.y0;
#pragma unroll
    for (int iy = 0; iy < RY; ++iy) {
        if (iy < tl.hy) {
            if (lane == 0) st_coh(left + iy, u[iy]);
            if (lane == tl.wx - 1) st_coh(right + iy, u[iy]);
        }
    }
    if (in) {
        const size_t ox = (size_t)z * p.nx + tl.x0 + lane;
        st_coh(yf(p, par, 2 * tl.ty + 1) + ox, u[0]);
        st_coh(yf(p, par, 2 * tl.ty + 2) + ox, last);
        if (iz == 0) {
#pragma unroll
            for (int iy = 0; iy < RY; ++iy)
                if (iy < tl.hy) st_coh(zf(p, par, 2 * tl.tz + 1) + (size_t)(tl.y0 + iy) * p.nx + tl.x0 + lane, u[iy]);
        }
        if (iz == tl.dz - 1) {
#pragma unroll
            for (int iy = 0; iy < RY; ++iy)
                if (iy < tl.hy) st_coh(zf(p, par, 2 * tl.tz + 2) + (size_t)(tl.y0 + iy) * p.nx + tl.x0 + lane, u[iy]);
        }
    }
}

template <typename T>
__device__ void init_ring_faces3(const Stencil3DParams<T> &p) {
    const size_t nthreads = (size_t)gridDim.x * blockDim.x;
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const T *g = p.grid;
    const size_t nx = p.nx, ny = p.ny, nz = p.nz;
    for (int par = 0; par < 2; ++par) {
        for (size_t i = tid; i < nz * ny; i += nthreads) {  // planes x = 0, nx-1; i = z*ny + y
            st_coh(xf(p, par, 0) + i, g[i * nx]);
            st_coh(xf(p, par, 2 * p.ntx + 1) + i, g[i * nx + nx - 1]);
        }
        for (size_t i = tid; i < nz * nx; i += nthreads) {  // planes y = 0, ny-1; i = z*nx + x
            const size_t z = i / nx, x = i % nx;
            st_coh(yf(p, par, 0) + i, g[(z * ny) * nx + x]);
            st_coh(yf(p, par, 2 * p.nty + 1) + i, g[(z * ny + ny - 1) * nx + x]);
        }
        for (size_t i = tid; i < ny * nx; i += nthreads) {  // planes z = 0, nz-1; i = y*nx + x
            st_coh(zf(p, par, 0) + i, g[i]);
            st_coh(zf(p, par, 2 * p.ntz + 1) + i, g[(nz - 1) * ny * nx + i]);
        }
    }
}

template <typename T>
__device__ void publish_initial3(const Stencil3DParams<T> &p, const Tile3D &tl, int lane) {
    const T *g = p.grid;
    const size_t nx = p.nx, ny = p.ny;
    for (int j = lane; j < tl.hy * tl.dz; j += 64) {
        const int iz = j / tl.hy, iy = j % tl.hy;
        const size_t row = ((size_t)(tl.z0 + iz) * ny + tl.y0 + iy) * nx;
        const size_t o = (size_t)(tl.z0 + iz) * ny + tl.y0 + iy;
        st_coh(xf(p, 0, 2 * tl.tx + 1) + o, g[row + tl.x0]);
        st_coh(xf(p, 0, 2 * tl.tx + 2) + o, g[row + tl.x0 + tl.wx - 1]);
    }
    if (lane < tl.wx) {
        const int x = tl.x0 + lane;
        for (int iz = 0; iz < tl.dz; ++iz) {
            const size_t z = tl.z0 + iz;
            st_coh(yf(p, 0, 2 * tl.ty + 1) + z * nx + x, g[(z * ny + tl.y0) * nx + x]);
            st_coh(yf(p, 0, 2 * tl.ty + 2) + z * nx + x, g[(z * ny + tl.y0 + tl.hy - 1) * nx + x]);
        }
        for (int iy = 0; iy < tl.hy; ++iy) {
            const size_t y = tl.y0 + iy;
            st_coh(zf(p, 0, 2 * tl.tz + 1) + y * nx + x, g[((size_t)tl.z0 * ny + y) * nx + x]);
            st_coh(zf(p, 0, 2 * tl.tz + 2) + y * nx + x, g[((size_t)(tl.z0 + tl.dz - 1) * ny + y) * nx + x]);
        }
    }
}

// Step of a register-cached tile: v[iz][iy] holds the block.  FULL tiles
// (hy == RY, dz == RZ) take halo values at compile-time positions; ragged
// tiles select them with wave-uniform conditions.
template <typename T, int RY, int RZ, bool FULL>
__device__ __forceinline__ void planes_cached3(const Stencil3DParams<T> &p, const Tile3D &tl, int par, int lane,
                                               T (&v)[RZ][RY], Halo3D<T, RY, RZ> &h) {
    T part[RY];
    const int xl = min(tl.x0 + lane, p.nx - 1);
    const T *zb = zf(p, par, 2 * tl.tz) + (size_t)tl.y0 * p.nx + xl;
#pragma unroll
    for (int iy = 0; iy < RY; ++iy) part[iy] = p.W.zm * ((FULL || iy < tl.hy) ? ld_coh(zb + (size_t)iy * p.nx) : T(0));
#pragma unroll
    for (int iz = 0; iz < RZ; ++iz) {
        if (FULL || iz < tl.dz) {
            const T ym = h.ym[iz * 64 + lane], yp = h.yp[iz * 64 + lane];
            T last;
            if (iz + 1 < RZ && (FULL || iz + 1 < tl.dz)) {
                last = compute_plane<T, RY, FULL>(v[iz], part, v[iz + 1], tl.hy, ym, yp, h.xw + iz * RY,
                                                  h.xe + iz * RY, p.W);
            } else {
                T zh[RY];
#pragma unroll
                for (int iy = 0; iy < RY; ++iy) zh[iy] = h.zp[iy * 64 + lane];
                last = compute_plane<T, RY, FULL>(v[iz], part, zh, tl.hy, ym, yp, h.xw + iz * RY, h.xe + iz * RY,
                                                  p.W);
            }
            publish_plane<T, RY>(p, tl, par ^ 1, lane, v[iz], iz, last);
        }
    }
}

template <typename T, int RY, int RZ>
__device__ __forceinline__ void step_cached3(const Stencil3DParams<T> &p, const Tile3D &tl, int par, int lane,
                                             T (&v)[RZ][RY], Halo3D<T, RY, RZ> &h) {
    load_halo3<T, RY, RZ>(p, tl, par, lane, h);
    if (lane >= tl.wx) {
        // ghost lanes carry the east face so the last real lane's DPP east
        // shift picks it up
#pragma unroll
        for (int iz = 0; iz < RZ; ++iz)
#pragma unroll
            for (int iy = 0; iy < RY; ++iy) v[iz][iy] = h.xe[iz * RY + iy];
    }
    if (tl.hy == RY && tl.dz == RZ)
        planes_cached3<T, RY, RZ, true>(p, tl, par, lane, v, h);
    else
        planes_cached3<T, RY, RZ, false>(p, tl, par, lane, v, h);
}

// Step of a tile that lives in the grid (uncached): planes streamed through
// registers, updated in place.
template <typename T, int RY, int RZ>
__device__ __forceinline__ void step_streamed3(const Stencil3DParams<T> &p, const Tile3D &tl, int par, int lane,
                                               Halo3D<T, RY, RZ> &h) {
    load_halo3<T, RY, RZ>(p, tl, par, lane, h);
    const bool ghost = lane >= tl.wx;
    const int xl = min(tl.x0 + lane, p.nx - 1);
    const size_t nx = p.nx, ny = p.ny;
    T cur[RY], nxt[RY], part[RY];
#pragma unroll
    for (int iy = 0; iy < RY; ++iy) {
        part[iy] = p.W.zm * ((iy < tl.hy) ? ld_coh(zf(p, par, 2 * tl.tz) + (size_t)(tl.y0 + iy) * p.nx + xl) : T(0));
        cur[iy] = (iy < tl.hy) ? (ghost ? h.xe[iy] : p.grid[((size_t)tl.z0 * ny + tl.y0 + iy) * nx + xl]) : T(0);
    }
    for (int iz = 0; iz < tl.dz; ++iz) {
        if (iz + 1 < tl.dz) {
            const size_t zo = ((size_t)(tl.z0 + iz + 1) * ny + tl.y0) * nx + xl;
#pragma unroll
            for (int iy = 0; iy < RY; ++iy)
                nxt[iy] = (iy < tl.hy) ? (ghost ? h.xe[(iz + 1) * RY + iy] : p.grid[zo + (size_t)iy * nx]) : T(0);
        } else {
#pragma unroll
            for (int iy = 0; iy < RY; ++iy) nxt[iy] = h.zp[iy * 64 + lane];
        }
        const T ym = h.ym[iz * 64 + lane], yp = h.yp[iz * 64 + lane];
        const T last =
            (tl.hy == RY)
                ? compute_plane<T, RY, true>(cur, part, nxt, RY, ym, yp, h.xw + iz * RY, h.xe + iz * RY, p.W)
                : compute_plane<T, RY, false>(cur, part, nxt, tl.hy, ym, yp, h.xw + iz * RY, h.xe + iz * RY, p.W);
        if (!ghost) {
            const size_t zo = ((size_t)(tl.z0 + iz) * ny + tl.y0) * nx + xl;
#pragma unroll
            for (int iy = 0; iy < RY; ++iy)
                if (iy < tl.hy) p.grid[zo + (size_t)iy * nx] = cur[iy];
        }
        publish_plane<T, RY>(p, tl, par ^ 1, lane, cur, iz, last);
#pragma unroll
        for (int iy = 0; iy < RY; ++iy) cur[iy] = nxt[iy];
    }
}

template <typename T, int RY, int RZ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(1, 2))) void stencil3d_persistent(Stencil3DParams<T> p) {
    __shared__ Halo3D<T, RY, RZ> halo[WAVES];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gw = blockIdx.x * WAVES + wave;
    const int nwaves = gridDim.x * WAVES;
    Halo3D<T, RY, RZ> &h = halo[wave];
    GridSync gs;
    gs.init(p.sync);
    init_ring_faces3(p);
    for (int t = gw; t < p.ntiles; t += nwaves) publish_initial3(p, tile3_of(p, t), lane);
    gs.sync();

    const bool has_cached = gw < p.cached;
    T v[RZ][RY];
    Tile3D ct{};
    if (has_cached) {
        ct = tile3_of(p, gw);
        const int xl = min(ct.x0 + lane, p.nx - 1);
#pragma unroll
        for (int iz = 0; iz < RZ; ++iz)
#pragma unroll
            for (int iy = 0; iy < RY; ++iy)
                v[iz][iy] = (iz < ct.dz && iy < ct.hy)
                                ? p.grid[(((size_t)(ct.z0 + iz)) * p.ny + ct.y0 + iy) * p.nx + xl]
                                : T(0);
    }
    for (long long s = 0; s < p.steps; ++s) {
        const int par = (int)(s & 1);
        Stencil3DParams<T> q = p;
        q.grid = opaque(q.grid);
        q.xface = opaque(q.xface);
        q.yface = opaque(q.yface);
        q.zface = opaque(q.zface);
        if (has_cached) step_cached3<T, RY, RZ>(q, ct, par, lane, v, h);
        for (int t = p.cached + gw; t < p.ntiles; t += nwaves) step_streamed3<T, RY, RZ>(q, tile3_of(p, t), par, lane, h);
        gs.sync();
    }
    if (has_cached && lane < ct.wx) {
#pragma unroll
        for (int iz = 0; iz < RZ; ++iz)
#pragma unroll
            for (int iy = 0; iy < RY; ++iy)
                if (iz < ct.dz && iy < ct.hy)
                    p.grid[(((size_t)(ct.z0 + iz)) * p.ny + ct.y0 + iy) * p.nx + ct.x0 + lane] = v[iz][iy];
    }
    gs.finish();
}

// Per-step baseline: one wave per tile, src -> dst.  The west/east faces are
// staged in LDS in the persistent kernel's layout and the same compute_plane
// is applied, so the two paths round identically; every other neighbour is
// read straight from src (ghost lanes read the real east column).
template <typename T, int RY, int RZ, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void stencil3d_step(Stencil3DParams<T> p) {
    __shared__ T hx[WAVES][2][RY * RZ];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = blockIdx.x * WAVES + wave;
    if (t >= p.ntiles) return;
    T *lw = hx[wave][0];
    T *le = hx[wave][1];
    const Tile3D tl = tile3_of(p, t);
    const T *src = p.src;
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

// Tile shapes (rows x planes per lane) and the waves per workgroup each runs
// with.  The deepest tile (4 x 16) fits the register file without spilling
// only in FP32.
struct Tile3Shape {
    int ry, rz, waves;
};
template <typename T> struct R3List;
template <> struct R3List<double> { static constexpr Tile3Shape v[2] = {{4, 4, 8}, {4, 8, 8}}; };
template <> struct R3List<float> { static constexpr Tile3Shape v[3] = {{4, 4, 8}, {4, 8, 8}, {4, 16, 8}}; };

template <typename T>
const void *pick3d(int ry, int rz, int waves) {
    if (waves != 8 || ry != 4) return nullptr;
    if (rz == 4) return reinterpret_cast<const void *>(&stencil3d_persistent<T, 4, 4, 8>);
    if (rz == 8) return reinterpret_cast<const void *>(&stencil3d_persistent<T, 4, 8, 8>);
    if constexpr (sizeof(T) == 4) {
        if (rz == 16) return reinterpret_cast<const void *>(&stencil3d_persistent<T, 4, 16, 8>);
    }
    return nullptr;
}

struct Plan3D {
    int ry = 0, rz = 0, waves = 0, wgs = 0, ntx = 0, nty = 0, ntz = 0, last_w = 0, last_h = 0, last_d = 0, ntiles = 0,
        cached = 0;
    const void *fn = nullptr;
};

template <typename T>
int plan3d(const perks_shape &s, const perks_tuning *tu, Plan3D *pl) {
    DeviceFacts f;
    int rc = device_facts(&f);
    if (rc) return rc;
    const long long nxi = s.nx - 2, nyi = s.ny - 2, nzi = s.nz - 2;
    pl->ntx = (int)((nxi + 63) / 64);
    pl->last_w = (int)(nxi - 64 * (pl->ntx - 1));
    const int want_ry = tu ? tu->rows_per_lane : 0, want_rz = tu ? tu->planes_per_lane : 0;
    const int wgs_per_cu = (tu && tu->wgs_per_cu > 0) ? tu->wgs_per_cu : 1;
    const int want_waves = tu ? tu->waves_per_wg : 0;
    Tile3Shape chosen{0, 0, 0};
    long long cap = 0;
    for (Tile3Shape sh : R3List<T>::v) {
        if (want_waves && want_waves != sh.waves) continue;
        const void *fn = pick3d<T>(sh.ry, sh.rz, sh.waves);
        int occ = 0;
        if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, sh.waves * 64, 0) != hipSuccess ||
            occ < wgs_per_cu)
            continue;
        const long long c = (long long)f.cus * wgs_per_cu * sh.waves;
        const long long nt = pl->ntx * ((nyi + sh.ry - 1) / sh.ry) * ((nzi + sh.rz - 1) / sh.rz);
        if (want_ry || want_rz) {
            if ((!want_ry || want_ry == sh.ry) && (!want_rz || want_rz == sh.rz)) {
                chosen = sh;
                cap = c;
            }
        } else if (nt <= c) {
            chosen = sh;
            cap = c;
            break;
        } else {
            chosen = sh;
            cap = c;
        }
    }
    if (!chosen.ry) return set_error(PERKS_E_UNSUPPORTED, "no 3D tile shape matches the request");
    pl->ry = chosen.ry;
    pl->rz = chosen.rz;
    pl->waves = chosen.waves;
    pl->nty = (int)((nyi + chosen.ry - 1) / chosen.ry);
    pl->ntz = (int)((nzi + chosen.rz - 1) / chosen.rz);
    pl->last_h = (int)(nyi - (long long)chosen.ry * (pl->nty - 1));
    pl->last_d = (int)(nzi - (long long)chosen.rz * (pl->ntz - 1));
    const long long nt = (long long)pl->ntx * pl->nty * pl->ntz;
    if (nt > (1LL << 30)) return set_error(PERKS_E_UNSUPPORTED, "too many tiles");
    pl->ntiles = (int)nt;
    long long cached = std::min<long long>(nt, cap);
    if (tu && tu->max_cached_tiles < 0) cached = 0;
    if (tu && tu->max_cached_tiles > 0) cached = std::min<long long>(cached, tu->max_cached_tiles);
    pl->cached = (int)cached;
    const long long waves = std::min<long long>(nt, cap);
    pl->wgs = (int)((waves + chosen.waves - 1) / chosen.waves);
    pl->fn = pick3d<T>(chosen.ry, chosen.rz, chosen.waves);
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
size_t faces3_elems(const perks_shape &s, int ntx, int nty, int ntz) {
    return (size_t)2 * ((size_t)(2 * ntx + 2) * s.nz * s.ny + (size_t)(2 * nty + 2) * s.nz * s.nx +
                        (size_t)(2 * ntz + 2) * s.ny * s.nx);
}


template <typename T>
int run3d(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, hipStream_t st,
          const perks_tuning *tu) {
    Plan3D pl;
    int rc = plan3d<T>(s, tu, &pl);
    if (rc) return rc;
    Stencil3DParams<T> p{};
    p.grid = grid;
    p.nx = (int)s.nx;
    p.ny = (int)s.ny;
    p.nz = (int)s.nz;
    p.ntx = pl.ntx;
    p.nty = pl.nty;
    p.ntz = pl.ntz;
    p.RY = pl.ry;
    p.RZ = pl.rz;
    p.last_w = pl.last_w;
    p.last_h = pl.last_h;
    p.last_d = pl.last_d;
    p.ntiles = pl.ntiles;
    p.cached = pl.cached;
    p.steps = steps;
    fill_weights3(p.W, coeffs);
    const size_t fx = (size_t)2 * (2 * pl.ntx + 2) * s.nz * s.ny;
    const size_t fy = (size_t)2 * (2 * pl.nty + 2) * s.nz * s.nx;
    const size_t fz = (size_t)2 * (2 * pl.ntz + 2) * s.ny * s.nx;
    T *faces = (T *)scratch(SLOT_FACES, (fx + fy + fz) * sizeof(T));
    unsigned *sync = (unsigned *)scratch(SLOT_SYNC, SYNC_BYTES);
    if (!faces || !sync) return PERKS_E_NOMEM;
    p.xface = faces;
    p.yface = faces + fx;
    p.zface = faces + fx + fy;
    p.sync = sync;
    return launch_coop(pl.fn, pl.wgs, pl.waves * 64, &p, st);
}

template <typename T>
int baseline3d(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, hipStream_t st) {
    const size_t cells = (size_t)s.nx * s.ny * s.nz;
    T *other = (T *)scratch(SLOT_PINGPONG, cells * sizeof(T));
    if (!other) return PERKS_E_NOMEM;
    Stencil3DParams<T> p{};
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
        p.src = a;
        p.dst = b;
        hipLaunchKernelGGL((stencil3d_step<T, RYB, RZB, W3B>), dim3(wgs), dim3(W3B * 64), 0, st, p);
        std::swap(a, b);
    }
    PERKS_HIP_TRY(hipGetLastError());
    if (a != grid) PERKS_HIP_TRY(hipMemcpyAsync(grid, a, cells * sizeof(T), hipMemcpyDeviceToDevice, st));
    return PERKS_OK;
}

template <typename T>
int plan3d_query(const perks_shape &s, const perks_tuning *tu, perks_stencil_plan *plan) {
    Plan3D pl;
    int rc = plan3d<T>(s, tu, &pl);
    if (rc) return rc;
    plan->wgs = pl.wgs;
    plan->waves_per_wg = pl.waves;
    plan->rows_per_lane = pl.ry;
    plan->planes_per_lane = pl.rz;
    plan->tiles = pl.ntiles;
    plan->cached_tiles = pl.cached;
    plan->interior_cells = (s.nx - 2) * (s.ny - 2) * (s.nz - 2);
    int64_t cc = 0, face = 0;
    for (int t = 0; t < pl.ntiles; ++t) {
        int tx = t % pl.ntx, ty = (t / pl.ntx) % pl.nty, tz = t / (pl.ntx * pl.nty);
        int64_t wx = tx == pl.ntx - 1 ? pl.last_w : 64, hy = ty == pl.nty - 1 ? pl.last_h : pl.ry,
                dz = tz == pl.ntz - 1 ? pl.last_d : pl.rz;
        if (t < pl.cached) cc += wx * hy * dz;
        face += 2 * (2 * hy * dz + 2 * wx * dz + 2 * wx * hy);
    }
    plan->cached_cells = cc;
    plan->halo_bytes_per_step = face * (int64_t)sizeof(T);
    plan->sync = 1;
    return PERKS_OK;
}

}  // namespace perks
