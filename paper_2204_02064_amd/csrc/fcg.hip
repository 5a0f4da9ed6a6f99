// Flexible CG with the learned preconditioner, as one persistent kernel.
//
// FCG(1) (Notay's flexible CG keeping one previous direction): the
// preconditioned residual z = M(r) is made A-orthogonal to the previous
// direction explicitly, p = z - (<z, q_old> / <p_old, q_old>) p_old with
// q = A p, and alpha = <p, r> / <p, q>; this tolerates a preconditioner that
// is not a fixed linear operator.  M is the Jacobi step corrected by the
// convolutional network, z = D^{-1} r + rms(r) * net([r / rms(r), log k]) on
// the H x W grid of unknowns, so a zero network is Jacobi-PCG.  When
// the network fails (<z, r> <= 0 or a non-finite value) the Jacobi step
// z = D^{-1} r replaces it for that iteration; when the residual norm has not
// reached a new minimum for `stall` iterations the kernel ends and the host
// continues from the current iterate with the persistent Jacobi-PCG solver
// (a restart of the direction recurrence, as FCG with a fixed Jacobi step
// would take, at that solver's cost per iteration).
//
// Per iteration, three device-wide barriers: after z and its dot products,
// after q = A p (the new direction formed on the fly where it is gathered)
// and its dot products, after the x / r update and ||r||.  The network runs inside the kernel: each workgroup
// owns 16 x 16 tiles of the grid and computes all six layers of a tile in
// LDS from a 28 x 28 region of r and log k (a halo of one pixel per layer,
// recomputed instead of exchanged), on the matrix cores, so the network adds
// no barrier.  The paper's CG has no preconditioner; this is the learned-
// preconditioner extension.
#include <algorithm>
#include <cmath>

#include "barrier.hpp"
#include "cg_common.hpp"
#include "common.hpp"
#include "nn_common.hpp"

namespace perks {
namespace {

constexpr int FT = 16;             // output tile side
constexpr int FR = FT + 2 * NL;    // 28: side of the layer-0 input region
__shared__ unsigned short fcg_buf_a[FR * FR * NC];
__shared__ unsigned short fcg_buf_b[(FR - 2) * (FR - 2) * NC];
__shared__ double cg_red_fcg[4 * CG_WAVES];
__shared__ double cg_bcast_fcg;

enum { FP_ZR = 0, FP_ZQ, FP_PQ, FP_PR, FP_RR, FP_BB, FP_TRUE, FNPART };

struct FcgParams {
    const int *rowptr;
    const int *colind;
    const double *val;
    const double *b;
    double *x;
    double *r, *z, *p, *p1, *q, *dinv;   // p, p1: the direction, alternating by iteration
    const double *logk;
    const unsigned short *wf;   // packed forward fragments, NL x 5 x 64 x 8 bf16
    const float *bias;          // NL x 16
    double *part;               // FNPART x G
    double *result;
    unsigned *ws;
    int n, H, W, ntx, nty;
    int maxit, stall, use_net;
    double tol;
};

// z on the tile whose first pixel is (tx0, ty0): D^{-1} r + rms * net([r / rms, log k]).
// Layer l reads an (FR - 2l)^2 region and writes the (FR - 2l - 2)^2 region
// inside it; pixels outside the grid are zero in every layer's input (the
// network's zero padding).  Waves take (row, 16-pixel segment) items.
__device__ __forceinline__ void net_tile(const FcgParams &p, int tx0, int ty0, double rms, double inv_rms) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ox = tx0 - NL, oy = ty0 - NL;
    for (int e = tid; e < FR * FR; e += CG_THREADS) {
        const int gy = oy + e / FR, gx = ox + e % FR;
        unsigned c01 = 0u;
        if (gy >= 0 && gy < p.H && gx >= 0 && gx < p.W) {
            const size_t i = (size_t)gy * p.W + gx;
            c01 = (unsigned)to_bf16((float)(ld_coh(p.r + i) * inv_rms)) | ((unsigned)to_bf16((float)p.logk[i]) << 16);
        }
        uint4 *d = reinterpret_cast<uint4 *>(fcg_buf_a + e * NC);
        d[0] = make_uint4(c01, 0u, 0u, 0u);
        d[1] = make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    const int n = lane & 15, g = lane >> 4, cofs = 8 * (g & 1);
    const uint4 *fr = reinterpret_cast<const uint4 *>(p.wf);
    for (int l = 0; l < NL; ++l) {
        const int sin = FR - 2 * l, sout = sin - 2;
        const unsigned short *bin = (l & 1) ? fcg_buf_b : fcg_buf_a;
        unsigned short *bout = (l & 1) ? fcg_buf_a : fcg_buf_b;
        bf16x8 a[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const uint4 v = fr[(l * 5 + q) * 64 + lane];
            a[q] = *reinterpret_cast<const bf16x8 *>(&v);
        }
        float bz[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) bz[j] = p.bias[l * NC + 4 * g + j];
        const int segs = (sout + 15) / 16;
        const int items = sout * segs;
        const int goy = oy + l + 1, gox = ox + l + 1;
        for (int it = wave; it < items; it += CG_WAVES) {
            const int row = it / segs, col = (it % segs) * 16 + n;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const int tap = 2 * q + (g >> 1);
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (tap < 9 && col < sout) {
                    const int iy = row + tap / 3, ix = col + tap % 3;   // (row + 1 + dy, col + 1 + dx)
                    v = *reinterpret_cast<const uint4 *>(bin + (iy * sin + ix) * NC + cofs);
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[q], *reinterpret_cast<const bf16x8 *>(&v), acc, 0, 0,
                                                              0);
            }
            if (col >= sout) continue;
            const int gy = goy + row, gx = gox + col;
            const bool inside = gy >= 0 && gy < p.H && gx >= 0 && gx < p.W;
            if (l < NL - 1) {
                float o[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) o[j] = inside ? fmaxf(acc[j] + bz[j], 0.f) : 0.f;
                uint2 st;
                st.x = (unsigned)to_bf16(o[0]) | ((unsigned)to_bf16(o[1]) << 16);
                st.y = (unsigned)to_bf16(o[2]) | ((unsigned)to_bf16(o[3]) << 16);
                *reinterpret_cast<uint2 *>(bout + (row * sout + col) * NC + 4 * g) = st;
            } else if (g == 0 && inside) {
                const size_t i = (size_t)gy * p.W + gx;   // an own pixel: dinv written by this workgroup
                st_coh(p.z + i, __builtin_fma(rms, (double)(acc[0] + bz[0]), p.dinv[i] * ld_coh(p.r + i)));
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(CG_THREADS) void fcg_persistent(FcgParams p) {
    BarrierClock clk;
    clk.start();
    GroupSync gs;
    gs.init_grid(p.ws, &clk);
    const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
    const int ntiles = p.ntx * p.nty;
    const int own_tiles = g < ntiles ? (ntiles - 1 - g) / G + 1 : 0;
    // Own pixels: the pixels of tiles g, g + G, ...; a fixed thread per pixel.
    auto for_own = [&](auto f) {
        for (int e = tid; e < own_tiles * FT * FT; e += CG_THREADS) {
            const int t = g + (e >> 8) * G;
            const int gy = (t / p.ntx) * FT + ((e & 255) >> 4), gx = (t % p.ntx) * FT + (e & 15);
            if (gy < p.H && gx < p.W) f(gy * p.W + gx);
        }
    };
    auto row_dot = [&](int i, const double *v) {
        double s = 0.0;
        for (int k = p.rowptr[i]; k < p.rowptr[i + 1]; ++k) s = __builtin_fma(p.val[k], v[p.colind[k]], s);
        return s;
    };
    auto post = [&](double (&acc)[2], int s0, int s1) {
        block_sum<2>(acc, cg_red_fcg);
        if (tid == 0) {
            st_coh(p.part + (size_t)s0 * G + g, acc[0]);
            if (s1 >= 0) st_coh(p.part + (size_t)s1 * G + g, acc[1]);
        }
    };

    // setup: D^{-1}, r = b - A x, ||b||^2, ||r||^2
    double a0[2] = {0.0, 0.0};
    for_own([&](int i) {
        double dg = 0.0;
        for (int k = p.rowptr[i]; k < p.rowptr[i + 1]; ++k)
            if (p.colind[k] == i) dg += p.val[k];
        p.dinv[i] = 1.0 / dg;
        p.q[i] = 0.0;   // finite before its first use in <z, q_old> (then weighted by beta = 0)
        const double bi = p.b[i], ri = bi - row_dot(i, p.x);
        st_coh(p.r + i, ri);
        a0[0] = __builtin_fma(bi, bi, a0[0]);
        a0[1] = __builtin_fma(ri, ri, a0[1]);
    });
    post(a0, FP_BB, FP_RR);
    gs.sync<true>();
    const double bnorm = sqrt(grid_total(p.part, FP_BB, G, &cg_bcast_fcg));
    double rr = grid_total(p.part, FP_RR, G, &cg_bcast_fcg);
    int k = 0, status = 1, fallbacks = 0, switched = -1, since = 0;
    bool use_net = p.use_net != 0, have_dir = false;
    double best = INFINITY, pq_old = 0.0;
    if (bnorm == 0.0) {
        for_own([&](int i) { st_coh(p.x + i, 0.0); });
        status = 0;
        rr = 0.0;
    }
    while (status == 1) {
        if (sqrt(rr) <= p.tol * bnorm) { status = 0; break; }
        if (k >= p.maxit) break;
        // z = M(r) and <z, r>, <z, q_old>
        if (use_net) {
            const double rms = sqrt(rr / p.n);
            for (int j = 0; j < own_tiles; ++j) {
                const int t = g + j * G;
                net_tile(p, (t % p.ntx) * FT, (t / p.ntx) * FT, rms, 1.0 / rms);
            }
        } else {
            for_own([&](int i) { st_coh(p.z + i, p.dinv[i] * p.r[i]); });
        }
        __syncthreads();
        double a1[2] = {0.0, 0.0};
        for_own([&](int i) {
            a1[0] = __builtin_fma(p.z[i], p.r[i], a1[0]);
            a1[1] = __builtin_fma(p.z[i], p.q[i], a1[1]);
        });
        post(a1, FP_ZR, FP_ZQ);
        gs.sync<true>();
        double zr = grid_total(p.part, FP_ZR, G, &cg_bcast_fcg);
        double zq = grid_total(p.part, FP_ZQ, G, &cg_bcast_fcg);
        if (use_net && !(zr > 0.0 && isfinite(zr) && isfinite(zq))) {
            ++fallbacks;
            double a2[2] = {0.0, 0.0};
            for_own([&](int i) {
                const double zi = p.dinv[i] * p.r[i];
                st_coh(p.z + i, zi);
                a2[0] = __builtin_fma(zi, p.r[i], a2[0]);
                a2[1] = __builtin_fma(zi, p.q[i], a2[1]);
            });
            post(a2, FP_ZR, FP_ZQ);
            gs.sync<true>();
            zr = grid_total(p.part, FP_ZR, G, &cg_bcast_fcg);
            zq = grid_total(p.part, FP_ZQ, G, &cg_bcast_fcg);
        }
        // new direction p = z - beta p_old, A-orthogonal to the previous one,
        // formed on the fly where q = A p gathers it (no barrier of its own):
        // p alternates between two buffers so p_old stays intact until every
        // workgroup has gathered it; own rows of p are stored.
        const double beta = have_dir ? zq / pq_old : 0.0;
        double *pn = (k & 1) ? p.p1 : p.p;
        const double *po = (k & 1) ? p.p : p.p1;
        auto pval = [&](int c) { return have_dir ? __builtin_fma(-beta, po[c], p.z[c]) : p.z[c]; };
        double a3[2] = {0.0, 0.0};
        for_own([&](int i) {
            double s = 0.0;
            for (int kk = p.rowptr[i]; kk < p.rowptr[i + 1]; ++kk) s = __builtin_fma(p.val[kk], pval(p.colind[kk]), s);
            const double pi = pval(i);
            st_coh(pn + i, pi);
            p.q[i] = s;
            a3[0] = __builtin_fma(pi, s, a3[0]);
            a3[1] = __builtin_fma(pi, p.r[i], a3[1]);
        });
        post(a3, FP_PQ, FP_PR);
        gs.sync<true>();
        const double pq = grid_total(p.part, FP_PQ, G, &cg_bcast_fcg);
        const double pr = grid_total(p.part, FP_PR, G, &cg_bcast_fcg);
        if (!(pq > 0.0) || !isfinite(pq)) { status = 2; break; }
        const double alpha = pr / pq;
        double a4[2] = {0.0, 0.0};
        for_own([&](int i) {
            st_coh(p.x + i, __builtin_fma(alpha, pn[i], p.x[i]));
            const double ri = __builtin_fma(-alpha, p.q[i], p.r[i]);
            st_coh(p.r + i, ri);
            a4[0] = __builtin_fma(ri, ri, a4[0]);
        });
        post(a4, FP_RR, -1);
        gs.sync<true>();
        rr = grid_total(p.part, FP_RR, G, &cg_bcast_fcg);
        pq_old = pq;
        have_dir = true;
        ++k;
        const double rn = sqrt(rr);
        if (rn < best) {
            best = rn;
            since = 0;
        } else {
            ++since;
        }
        if (use_net && since >= p.stall) {   // the host continues with Jacobi-PCG
            switched = k;
            status = 3;
            break;
        }
    }
    // true residual
    gs.sync<true>();
    double a5[2] = {0.0, 0.0};
    for_own([&](int i) {
        const double d = p.b[i] - row_dot(i, p.x);
        a5[0] = __builtin_fma(d, d, a5[0]);
    });
    post(a5, FP_TRUE, -1);
    gs.sync<true>();
    const double tt = grid_total(p.part, FP_TRUE, G, &cg_bcast_fcg);
    if (g == 0 && tid == 0) {
        p.result[0] = k;
        p.result[1] = status;
        p.result[2] = bnorm > 0.0 ? sqrt(rr) / bnorm : 0.0;
        p.result[3] = bnorm > 0.0 ? sqrt(tt) / bnorm : 0.0;
        p.result[4] = bnorm;
        p.result[5] = fallbacks;
        p.result[6] = switched;
    }
    if (g == 0 && tid == 0) st_coh(p.ws + SYNC_EPOCH, gs.epoch);
    clk.publish(p.ws);
}

// z = D^{-1} r + rms(r) * net(...) once, with the tile routine the FCG kernel
// applies in every iteration: `rr` = ||r||^2 comes from fcg_rr, one
// workgroup per 16 x 16 tile.
__global__ __launch_bounds__(CG_THREADS) void fcg_rr(FcgParams p) {
    double a[1] = {0.0};
    for (int i = threadIdx.x; i < p.n; i += CG_THREADS) a[0] = __builtin_fma(p.r[i], p.r[i], a[0]);
    block_sum<1>(a, cg_red_fcg);
    if (threadIdx.x == 0) p.part[0] = a[0];
}

__global__ __launch_bounds__(CG_THREADS) void fcg_precond(FcgParams p) {
    const double rr = p.part[0];
    const int t = blockIdx.x;
    if (rr > 0.0) {
        const double rms = sqrt(rr / p.n);
        net_tile(p, (t % p.ntx) * FT, (t / p.ntx) * FT, rms, 1.0 / rms);
    } else {
        // r = 0: the network input is undefined; z = D^{-1} r = 0
        for (int e = threadIdx.x; e < FT * FT; e += CG_THREADS) {
            const int gy = (t / p.ntx) * FT + e / FT, gx = (t % p.ntx) * FT + e % FT;
            if (gy < p.H && gx < p.W) p.z[(size_t)gy * p.W + gx] = 0.0;
        }
    }
}

}  // namespace
}  // namespace perks

using namespace perks;

extern "C" {

int perks_fcg_precondition(const float *nn_params, const double *r, const double *logk, const double *dinv,
                           int32_t H, int32_t W, double *z, void *stream) {
    if (!nn_params || !r || !logk || !dinv || !z) return set_error(PERKS_E_INVAL, "NULL argument");
    if (H < 1 || W < 1 || (int64_t)H * W > INT32_MAX) return set_error(PERKS_E_INVAL, "bad grid extents");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    FcgParams p{};
    p.ntx = (W + FT - 1) / FT;
    p.nty = (H + FT - 1) / FT;
    const size_t frag = (size_t)NL * 5 * 64 * 8 * sizeof(unsigned short);
    const size_t bytes = 64 * sizeof(double) + 2 * frag + NL * NC * sizeof(float) + 1024;
    char *base = (char *)scratch(SLOT_FCG, bytes);
    if (!base) return PERKS_E_NOMEM;
    p.part = (double *)base;
    unsigned short *wf = (unsigned short *)(p.part + 64);
    unsigned short *wb = wf + frag / sizeof(unsigned short);   // backward fragments (unused here)
    float *bias = (float *)(wb + frag / sizeof(unsigned short));
    p.wf = wf;
    p.bias = bias;
    p.r = const_cast<double *>(r);
    p.z = z;
    p.dinv = const_cast<double *>(dinv);
    p.logk = logk;
    p.n = H * W;
    p.H = H;
    p.W = W;
    hipLaunchKernelGGL(nn_pack, dim3((NL * 5 * 64 * 8 + 255) / 256), dim3(256), 0, st, nn_params, wf, wb, bias);
    hipLaunchKernelGGL(fcg_rr, dim3(1), dim3(CG_THREADS), 0, st, p);
    hipLaunchKernelGGL(fcg_precond, dim3(p.ntx * p.nty), dim3(CG_THREADS), 0, st, p);
    PERKS_HIP_TRY(hipGetLastError());
    return PERKS_OK;
}

int perks_fcg_solve(const perks_csr *A, const void *b, void *x, double tol, int32_t maxit, const float *nn_params,
                    const double *logk, int32_t H, int32_t W, int32_t stall, void *stream, perks_cg_result *out) {
    if (!A || !b || !x) return set_error(PERKS_E_INVAL, "A, b and x must not be NULL");
    if (A->dt != PERKS_F64) return set_error(PERKS_E_UNSUPPORTED, "FP64 matrices only");
    if (H < 1 || W < 1 || (int64_t)H * W != A->n)
        return set_error(PERKS_E_INVAL, "the grid (H x W) must hold exactly the n unknowns");
    if (A->nnz > 0 && (!A->rowptr || !A->colind || !A->val)) return set_error(PERKS_E_INVAL, "NULL CSR array");
    if (nn_params && !logk) return set_error(PERKS_E_INVAL, "logk is required with a network");
    if (!(tol >= 0.0) || !std::isfinite(tol) || maxit < 0 || stall < 1)
        return set_error(PERKS_E_INVAL, "tol >= 0, maxit >= 0 and stall >= 1 required");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    DeviceFacts f;
    int rc = device_facts(&f);
    if (rc) return rc;
    int occ = 0;
    PERKS_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(&fcg_persistent),
                                                               CG_THREADS, 0));
    if (occ < 1) return set_error(PERKS_E_NOTCORESIDENT, "FCG kernel does not fit one workgroup per CU");
    FcgParams p{};
    p.ntx = (W + FT - 1) / FT;
    p.nty = (H + FT - 1) / FT;
    const int G = std::min(std::min(f.cus, SYNC_MAX_WGS), p.ntx * p.nty);
    const size_t nv = ((size_t)A->n + 63) / 64 * 64;
    const size_t frag = (size_t)NL * 5 * 64 * 8 * sizeof(unsigned short);
    const size_t bytes = 6 * nv * sizeof(double) + ((size_t)FNPART * G + 64) * sizeof(double) + 2 * frag +
                         NL * NC * sizeof(float) + 1024;
    char *base = (char *)scratch(SLOT_FCG, bytes);
    if (!base) return PERKS_E_NOMEM;
    unsigned *ws = (unsigned *)scratch(SLOT_SYNC, SYNC_BYTES);
    if (!ws) return PERKS_E_NOMEM;
    double *d = (double *)base;
    p.r = d;
    p.z = d + nv;
    p.p = d + 2 * nv;
    p.q = d + 3 * nv;
    p.dinv = d + 4 * nv;
    p.p1 = d + 5 * nv;
    p.part = d + 6 * nv;
    p.result = p.part + (size_t)FNPART * G;
    unsigned short *wf = (unsigned short *)(p.result + 64);
    unsigned short *wb = wf + frag / sizeof(unsigned short);   // backward fragments (unused here)
    float *bias = (float *)(wb + frag / sizeof(unsigned short));
    p.wf = wf;
    p.bias = bias;
    if (nn_params)
        hipLaunchKernelGGL(nn_pack, dim3((NL * 5 * 64 * 8 + 255) / 256), dim3(256), 0, st, nn_params, wf, wb, bias);
    p.rowptr = A->rowptr;
    p.colind = A->colind;
    p.val = (const double *)A->val;
    p.b = (const double *)b;
    p.x = (double *)x;
    p.logk = logk;
    p.ws = ws;
    p.n = (int)A->n;
    p.H = H;
    p.W = W;
    p.maxit = maxit;
    p.stall = stall;
    p.use_net = nn_params ? 1 : 0;
    p.tol = tol;
    void *args[] = {&p};
    note_persistent_launch(G, nullptr);
    hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&fcg_persistent), dim3(G),
                                              dim3(CG_THREADS), args, 0, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(e == hipErrorCooperativeLaunchTooLarge ? PERKS_E_NOTCORESIDENT : PERKS_E_HIP,
                         "FCG launch: %s", hipGetErrorString(e));
    }
    double h[8] = {0};
    PERKS_HIP_TRY(hipMemcpyAsync(h, p.result, 7 * sizeof(double), hipMemcpyDeviceToHost, st));
    PERKS_HIP_TRY(hipStreamSynchronize(st));
    perks_barrier_stats_t bs;
    int rcb = read_barrier_stats(G, nullptr, st, &bs);
    if (rcb) return rcb;
    const int s = (int)h[1];
    int iters = (int)h[0];
    double relres = h[2], relres_true = h[3];
    int status = s == 2 ? PERKS_BREAKDOWN : (s == 0 && h[3] <= tol) ? PERKS_OK : PERKS_NOT_CONVERGED;
    if (s == 3 && iters < maxit) {
        // the network stalled: Jacobi-PCG from the current iterate for the
        // remaining iterations
        perks_cg_result cg{};
        status = perks_cg_solve(A, b, x, tol, maxit - iters, PERKS_PRECOND_JACOBI, PERKS_PREC_F64, stream, &cg);
        if (status < 0) return status;
        iters += cg.iters;
        relres = cg.relres;
        relres_true = cg.relres_true;
    }
    if (out) {
        out->iters = iters;
        out->status = status;
        out->restarts = 0;
        out->wgs = G;
        out->relres = relres;
        out->relres_true = relres_true;
        out->cached_nnz_frac = 0.0;
        out->fallbacks = (int)h[5];
        out->switched_at = (int)h[6];
        out->barrier_cycles = (int64_t)bs.wait_cycles;   // the FCG launch (not the Jacobi-PCG tail)
    }
    return status;
}

}  // extern "C"
