// 3D Jacobi stencils beyond the 7-point star (the rest of tab:domain's 3D
// suite): any pattern inside the radius-1 box (3d27pt, the 19-point poisson
// stencil, 3d17pt) and the radius-2 star (3d13pt).  Persistent kernel and
// per-step baseline on one tile routine, so the two round identically.
//
// These kernels stream: every step reads the whole grid from buffer s%2 and
// writes the interior to buffer (s+1)%2; nothing is kept on chip across
// steps.  The persistent kernel removes the per-step launches (one device
// barrier per step instead), which is the part of PERKS that does not need
// a cache.
//
// Tile: 64 columns x RC rows of one z plane, one wavefront.  The new value is
// the sum over the weight box's z layers of that layer's 2D stencil applied
// to plane z+dz: each full layer runs the 2D tile routine of the radius-2..4
// kernels on that plane (rows in registers, chained DPP shifts, halo rows and
// columns staged in LDS) and adds its sums to the output rows; a layer whose
// only weight is its centre (the outer layers of a star) is one FMA per cell.
#pragma once

#include "stencil2d_wide.hpp"

namespace perks {

template <typename T, int R>
struct Wide3W {
    T w[(2 * R + 1) * (2 * R + 1) * (2 * R + 1)];   // [dz + R][dy + R][dx + R]
};

template <typename T, int R>
struct Wide3DParams {
    gmem<T> *buf0;    // the caller's grid
    gmem<T> *buf1;    // second buffer (ring copied in)
    unsigned *sync;
    int64_t steps;
    int nx, ny, nz;
    int ntx, nty;     // tiles per plane along x and y
    Wide3W<T, R> W;
};

template <typename T, int R>
struct Wide3DStep {
    const gmem<T> *src;
    gmem<T> *dst;
    int nx, ny, nz, ntx, nty;
    Wide3W<T, R> W;
};

constexpr int W3RC = 16;   // rows per lane of a 3D tile
constexpr int W3W = 4;     // waves per workgroup (both kernels)

// Launch shape of the persistent kernel, chosen by measurement at 256^3:
// FP64 completes each z layer before the next layer's loads (PIN) to run
// four waves per SIMD; FP32 lets the compiler issue every layer's loads at
// once and runs five.  The per-step baseline keeps the compiler's own
// choices (measured faster there).
template <typename T>
struct Wide3Occ {
    static constexpr int value = sizeof(T) == 4 ? 5 : 4;
    static constexpr bool pin = sizeof(T) == 8;
};

// Tile t: (tx, ty) in its plane, interior plane z = R + t / (ntx * nty).
template <int R>
__device__ __forceinline__ WideTile wide3_tile_of(int t, int ntx, int nty, int nx, int ny, int *z) {
    const int per = ntx * nty;
    *z = R + t / per;
    return wide_tile_of<W3RC>(t % per, ntx, nx, ny, R);
}

// New values of one tile (plane z) from `src` into out[].  BOX: every layer
// is a full (2R+1)^2 box (any radius-1 3D pattern); otherwise a star: the
// centre layer is the 2D star, the other layers hold their centre only.
//
// PIN: each layer's sum is completed before the next layer's loads are
// issued (one layer's rows live at a time: fewer registers, more waves);
// otherwise the compiler may issue every layer's loads at once.  The
// arithmetic, and so the result, is the same either way.
template <typename T, int R, bool BOX, bool PIN>
__device__ __forceinline__ void wide3_tile(const gmem<T> *src, const WideTile &tl, int z, int nx, int ny, int lane,
                                           const Wide3W<T, R> &W, WideLds<T, R, BOX, W3RC> &lds, T (&out)[W3RC]) {
    constexpr int S = 2 * R + 1;
    const size_t plane = (size_t)nx * ny;
    T *cw = lds.c[0], *ce = lds.c[1];
    T *hr = &lds.rows[0][lane];
    const bool live = lane < tl.wx;
    static_for<0, S>([&](auto zc) {
        constexpr int dz = decltype(zc)::value - R;
        const gmem<T> *sp = src + (size_t)(z + dz) * plane;
        T u[W3RC];
        wide_load<T, W3RC>(sp, tl, nx, ny, lane, u);
        if constexpr (BOX || dz == 0) {
            wide_halo<T, R, BOX, W3RC>(sp, tl, nx, ny, lane, hr, cw, ce);
            wide_rows_impl<T, R, BOX, W3RC, true, dz == -R>(
                u, hr, cw, ce, [&](int dy, int dx) { return W.w[((dz + R) * S + dy + R) * S + dx + R]; }, tl.hy,
                live, out);
            compiler_fence();   // the next layer's staging overwrites this layer's LDS
        } else {
            const T w = W.w[((dz + R) * S + R) * S + R];
#pragma unroll
            for (int i = 0; i < W3RC; ++i) {
                if constexpr (dz == -R) out[i] = w * u[i];
                else out[i] = fma_t(w, u[i], out[i]);
            }
        }
        if constexpr (PIN) settle(out);
    });
}

template <typename T, int R, bool BOX>
__global__ __launch_bounds__(W3W * 64) __attribute__((amdgpu_waves_per_eu(Wide3Occ<T>::value))) void stencil3d_wide(
    Wide3DParams<T, R> p) {
    __shared__ WideLds<T, R, BOX, W3RC> lds[W3W];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gw = blockIdx.x * W3W + wave, nw = gridDim.x * W3W;
    const int ntiles = p.ntx * p.nty * (p.nz - 2 * R);
    GridSync gs;
    gs.init(p.sync);
    for (int64_t s = 0; s < p.steps; ++s) {
        const gmem<T> *src = opaque((s & 1) ? p.buf1 : p.buf0);
        gmem<T> *dst = opaque((s & 1) ? p.buf0 : p.buf1);
        for (int t = gw; t < ntiles; t += nw) {
            int z;
            const WideTile tl = wide3_tile_of<R>(t, p.ntx, p.nty, p.nx, p.ny, &z);
            T out[W3RC];
            wide3_tile<T, R, BOX, Wide3Occ<T>::pin>(src, tl, z, p.nx, p.ny, lane, p.W, lds[wave], out);
            wide_store<T, R, W3RC, false, true>(dst + (size_t)z * p.nx * p.ny, tl, p.nx, lane, out);
        }
        gs.sync();
    }
    if (p.steps & 1) {   // the result is in the second buffer: copy the interior back
        for (int t = gw; t < ntiles; t += nw) {
            int z;
            const WideTile tl = wide3_tile_of<R>(t, p.ntx, p.nty, p.nx, p.ny, &z);
            const size_t off = (size_t)z * p.nx * p.ny;
            T u[W3RC];
            wide_load<T, W3RC>(p.buf1 + off, tl, p.nx, p.ny, lane, u);
            wide_store<T, R, W3RC, false, false>(p.buf0 + off, tl, p.nx, lane, u);
        }
    }
    gs.finish();
}

template <typename T, int R, bool BOX>
__global__ __launch_bounds__(W3W * 64) void stencil3d_wide_step(Wide3DStep<T, R> p) {
    __shared__ WideLds<T, R, BOX, W3RC> lds[W3W];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = blockIdx.x * W3W + wave;
    if (t >= p.ntx * p.nty * (p.nz - 2 * R)) return;
    int z;
    const WideTile tl = wide3_tile_of<R>(t, p.ntx, p.nty, p.nx, p.ny, &z);
    T out[W3RC];
    wide3_tile<T, R, BOX, false>(p.src, tl, z, p.nx, p.ny, lane, p.W, lds[wave], out);
    wide_store<T, R, W3RC, false, false>(p.dst + (size_t)z * p.nx * p.ny, tl, p.nx, lane, out);
}

// ---------------------------------------------------------------------------
// Host side.
template <typename T, int R>
void fill_wide3(Wide3W<T, R> &W, const double *c) {
    for (int i = 0; i < (2 * R + 1) * (2 * R + 1) * (2 * R + 1); ++i) W.w[i] = (T)c[i];
}

template <typename T, int R, bool BOX>
int wide3_grid(const perks_shape &s, int *wgs, int *ntx, int *nty, int64_t *ntiles) {
    DeviceFacts f;
    int rc = device_facts(&f);
    if (rc) return rc;
    int occ = 0;
    PERKS_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &occ, reinterpret_cast<const void *>(&stencil3d_wide<T, R, BOX>), W3W * 64, 0));
    if (occ < 1) return set_error(PERKS_E_NOTCORESIDENT, "3D stencil kernel does not fit a CU");
    *ntx = (int)((s.nx - 2 * R + 63) / 64);
    *nty = (int)((s.ny - 2 * R + W3RC - 1) / W3RC);
    *ntiles = (int64_t)*ntx * *nty * (s.nz - 2 * R);
    if (*ntiles > INT32_MAX) return set_error(PERKS_E_UNSUPPORTED, "3D grid too large for this kernel");
    *wgs = (int)std::min<int64_t>((*ntiles + W3W - 1) / W3W, (int64_t)f.cus * occ);
    return PERKS_OK;
}

template <typename T, int R, bool BOX>
int run_wide3(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, hipStream_t st,
              const perks_tuning *tu) {
    if (tu && (tu->rows_per_lane > 0 && tu->rows_per_lane != W3RC))
        return set_error(PERKS_E_UNSUPPORTED, "3D stencils of this pattern use %d rows per lane", W3RC);
    int wgs, ntx, nty;
    int64_t ntiles;
    int rc = wide3_grid<T, R, BOX>(s, &wgs, &ntx, &nty, &ntiles);
    if (rc) return rc;
    const size_t cells = (size_t)s.nx * s.ny * s.nz;
    T *other = (T *)scratch(SLOT_WIDE, cells * sizeof(T));
    unsigned *sync = (unsigned *)scratch(SLOT_SYNC, SYNC_BYTES);
    if (!other || !sync) return PERKS_E_NOMEM;
    PERKS_HIP_TRY(hipMemcpyAsync(other, grid, cells * sizeof(T), hipMemcpyDeviceToDevice, st));
    Wide3DParams<T, R> p{};
    p.buf0 = to_global(grid);
    p.buf1 = to_global(other);
    p.sync = sync;
    p.steps = steps;
    p.nx = (int)s.nx;
    p.ny = (int)s.ny;
    p.nz = (int)s.nz;
    p.ntx = ntx;
    p.nty = nty;
    fill_wide3(p.W, coeffs);
    return launch_coop(reinterpret_cast<const void *>(&stencil3d_wide<T, R, BOX>), wgs, W3W * 64, &p, st);
}

template <typename T, int R, bool BOX>
int baseline_wide3(T *grid, const double *coeffs, const perks_shape &s, int64_t steps, hipStream_t st) {
    const size_t cells = (size_t)s.nx * s.ny * s.nz;
    T *other = (T *)scratch(SLOT_PINGPONG, cells * sizeof(T));
    if (!other) return PERKS_E_NOMEM;
    Wide3DStep<T, R> p{};
    p.nx = (int)s.nx;
    p.ny = (int)s.ny;
    p.nz = (int)s.nz;
    p.ntx = (int)((s.nx - 2 * R + 63) / 64);
    p.nty = (int)((s.ny - 2 * R + W3RC - 1) / W3RC);
    const int64_t ntiles = (int64_t)p.ntx * p.nty * (s.nz - 2 * R);
    if (ntiles > INT32_MAX) return set_error(PERKS_E_UNSUPPORTED, "3D grid too large for this kernel");
    fill_wide3(p.W, coeffs);
    PERKS_HIP_TRY(hipMemcpyAsync(other, grid, cells * sizeof(T), hipMemcpyDeviceToDevice, st));
    const int wgs = (int)((ntiles + W3W - 1) / W3W);
    T *a = grid, *b = other;
    for (int64_t k = 0; k < steps; ++k) {
        p.src = to_global((const T *)a);
        p.dst = to_global(b);
        hipLaunchKernelGGL((stencil3d_wide_step<T, R, BOX>), dim3(wgs), dim3(W3W * 64), 0, st, p);
        std::swap(a, b);
    }
    PERKS_HIP_TRY(hipGetLastError());
    if (a != grid) PERKS_HIP_TRY(hipMemcpyAsync(grid, a, cells * sizeof(T), hipMemcpyDeviceToDevice, st));
    return PERKS_OK;
}

template <typename T, int R, bool BOX>
int plan_wide3_query(const perks_shape &s, const perks_tuning *tu, perks_stencil_plan *plan) {
    if (tu && (tu->rows_per_lane > 0 && tu->rows_per_lane != W3RC))
        return set_error(PERKS_E_UNSUPPORTED, "3D stencils of this pattern use %d rows per lane", W3RC);
    int wgs, ntx, nty;
    int64_t ntiles;
    int rc = wide3_grid<T, R, BOX>(s, &wgs, &ntx, &nty, &ntiles);
    if (rc) return rc;
    const int64_t interior = (s.nx - 2 * R) * (s.ny - 2 * R) * (s.nz - 2 * R);
    plan->wgs = wgs;
    plan->waves_per_wg = W3W;
    plan->rows_per_lane = W3RC;
    plan->planes_per_lane = 1;
    plan->tiles = (int32_t)ntiles;
    plan->cached_tiles = 0;
    plan->cached_cells = 0;
    plan->interior_cells = interior;
    // streamed: the interior read and written once per step (the halo reads
    // of neighbouring planes and tiles come from the caches)
    plan->halo_bytes_per_step = 0;
    plan->sync = 1;
    plan->lds_rows_per_lane = 0;
    return PERKS_OK;
}

}  // namespace perks
