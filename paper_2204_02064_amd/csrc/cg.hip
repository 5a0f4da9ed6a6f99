// Conjugate gradient (Sec. 2.2.2, Sec. 4.3): the fused persistent solver and
// the host-looped multi-kernel baseline, FP64, CSR matrices.
//
// Persistent solver, per iteration (two device-wide barriers):
//   phase 1  q = A p on the workgroup's rows, gathering p_j = z_j + beta*pold_j
//            on the fly (z = r unpreconditioned, z = D^{-1} r for Jacobi), so
//            the update of p needs no barrier of its own; the new p of the
//            workgroup's own rows is stored to the other p buffer; partial p.q.
//   barrier  every workgroup sums the partials in the same fixed order -> alpha
//   phase 2  x += alpha p, r -= alpha q, z = D^{-1} r on own rows; partials r.z, r.r
//   barrier  -> beta and the (uniform) convergence decision.
// The row partition is a merge-path split of (rows + nonzeros) into equal
// shares, searched once at kernel start (the paper keeps its thread-block
// search result for the whole solve because A is static, Sec. 4.3.2).  The
// first part of the workgroup's slice of A (values and column indices) is
// copied into LDS once and read from there every iteration (the on-chip
// cache of A); the rest streams from L2 / Infinity Cache / HBM.
#include <algorithm>
#include <cmath>
#include <vector>

#include "barrier.hpp"
#include "common.hpp"

namespace perks {
namespace {

constexpr int CG_WAVES = 8;
constexpr int CG_THREADS = CG_WAVES * 64;
enum { PART_PQ = 0, PART_RZ = 1, PART_RR = 2, PART_BB = 3, PART_TRUE = 4, NPART = 5 };

struct CgParams {
    const int *rowptr;
    const int *colind;
    const double *val;
    const double *b;
    double *x;
    double *r;      // residual
    double *z;      // preconditioned residual (== r when unpreconditioned)
    double *q;      // A p (own rows)
    double *p0, *p1;
    double *dinv;   // inverse diagonal (Jacobi)
    double *part;   // [NPART][G]
    double *result; // [8] iters, status, relres, relres_true, rho, ...
    unsigned *sync;
    int n;
    int nnz;
    int maxit;
    int precond;
    int lds_nnz;    // capacity of the LDS cache of A (nonzeros per workgroup)
    double tol;
};

// Sum over the 64 lanes of a wave (butterfly; every lane gets the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over groups of L lanes (L a power of two, runtime-uniform).
__device__ __forceinline__ double group_sum(double v, int L) {
    for (int off = L >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic workgroup sum of up to 3 values: waves reduce, then wave 0
// adds the wave totals in wave order.  Returns the sums to thread 0 only.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *lds_red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) lds_red[k * CG_WAVES + wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int w = 0; w < CG_WAVES; ++w) s += lds_red[k * CG_WAVES + w];
            v[k] = s;
        }
    }
    __syncthreads();
}

// Every workgroup sums the G partials of slot `slot` in the same order
// (lanes take strided shares, then a butterfly): identical bits everywhere.
__device__ __forceinline__ double grid_total(const double *part, int slot, double *lds_bcast) {
    const int G = gridDim.x;
    if (threadIdx.x < 64) {
        double s = 0.0;
        for (int i = threadIdx.x; i < G; i += 64) s += ld_coh(part + (size_t)slot * G + i);
        s = wave_sum(s);
        if (threadIdx.x == 0) *lds_bcast = s;
    }
    __syncthreads();
    const double t = *lds_bcast;
    __syncthreads();
    return t;
}

// First row of share g when rows + nonzeros are split into G equal shares:
// the smallest i with i + rowptr[i] >= g * (n + nnz) / G (merge-path diagonal).
__device__ int merge_split(const int *rowptr, int n, int nnz, int g, int G) {
    const long long target = (long long)g * ((long long)n + nnz) / G;
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((long long)mid + rowptr[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int pick_group(int rows, int nnz) {
    const int avg = rows > 0 ? (nnz + rows - 1) / rows : 1;
    int L = 1;
    while (L < avg && L < 64) L <<= 1;
    return L;
}

// The workgroup's LDS copy of (the first CG_LDS_NNZ entries of) its slice of A.
constexpr int CG_LDS_NNZ = 13312;   // 156 KiB of the 160 KiB LDS
__shared__ double cg_lval[CG_LDS_NNZ];
__shared__ int cg_lcol[CG_LDS_NNZ];

// y_i for rows [r0, r1) with L lanes per row: sum_k a_k * v(col_k), where
// v(j) is produced by `fetch`.  Matrix entries k < kc come from the LDS copy.
template <typename F, typename S>
__device__ __forceinline__ void spmv_rows(const CgParams &p, int r0, int r1, int L, int kbase, int kc, F fetch,
                                          S sink) {
    const int tid = threadIdx.x;
    const int gl = tid & (L - 1);
    const int rows_per_pass = CG_THREADS / L;
    for (int row0 = r0; row0 < r1; row0 += rows_per_pass) {
        const int i = row0 + tid / L;
        double s = 0.0;
        if (i < r1) {
            const int kb = p.rowptr[i], ke = p.rowptr[i + 1];
            for (int k = kb + gl; k < ke; k += L) {
                const int kk = k - kbase;
                double a;
                int c;
                if (kk < kc) {
                    a = cg_lval[kk];
                    c = cg_lcol[kk];
                } else {
                    a = p.val[k];
                    c = p.colind[k];
                }
                s = __builtin_fma(a, fetch(c), s);
            }
        }
        s = group_sum(s, L);
        if (i < r1 && gl == 0) sink(i, s);
    }
}

template <bool JACOBI>
__global__ __launch_bounds__(CG_THREADS) void cg_persistent(CgParams p) {
    __shared__ double red[4 * CG_WAVES];
    __shared__ double bcast;
    GridSync gs;
    gs.init(p.sync);
    const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
    const int r0 = merge_split(p.rowptr, p.n, p.nnz, g, G);
    const int r1 = merge_split(p.rowptr, p.n, p.nnz, g + 1, G);
    const int kbase = p.rowptr[r0];
    const int my_nnz = p.rowptr[r1] - kbase;
    const int L = pick_group(r1 - r0, my_nnz);
    // on-chip cache of this workgroup's slice of A
    const int kc = min(my_nnz, p.lds_nnz);
    for (int k = tid; k < kc; k += CG_THREADS) {
        cg_lval[k] = p.val[kbase + k];
        cg_lcol[k] = p.colind[kbase + k];
    }
    __syncthreads();

    // phase 0: r = b - A x, z, p_{-1} = 0, partials b.b, r.z, r.r
    double acc0[3] = {0.0, 0.0, 0.0};
    spmv_rows(p, r0, r1, L, kbase, kc, [&](int c) { return p.x[c]; },
              [&](int i, double s) { p.q[i] = s; });
    __syncthreads();
    for (int i = r0 + tid; i < r1; i += CG_THREADS) {
        const double bi = p.b[i];
        const double ri = bi - p.q[i];
        const double zi = JACOBI ? p.dinv[i] * ri : ri;
        if (JACOBI) {
            p.r[i] = ri;            // read back only by this thread
            st_coh(p.z + i, zi);    // gathered by other workgroups
        } else {
            st_coh(p.r + i, ri);
        }
        st_coh(p.p1 + i, 0.0);
        acc0[0] = __builtin_fma(bi, bi, acc0[0]);
        acc0[1] = __builtin_fma(ri, zi, acc0[1]);
        acc0[2] = __builtin_fma(ri, ri, acc0[2]);
    }
    block_sum<3>(acc0, red);
    if (tid == 0) {
        st_coh(p.part + (size_t)PART_BB * G + g, acc0[0]);
        st_coh(p.part + (size_t)PART_RZ * G + g, acc0[1]);
        st_coh(p.part + (size_t)PART_RR * G + g, acc0[2]);
    }
    gs.sync();
    const double bb = grid_total(p.part, PART_BB, &bcast);
    double rho = grid_total(p.part, PART_RZ, &bcast);
    double rr = grid_total(p.part, PART_RR, &bcast);
    const double bnorm = sqrt(bb);
    double beta = 0.0;
    int k = 0, status = 1;
    const double *zsrc = JACOBI ? p.z : p.r;
    if (bnorm == 0.0) status = 0;
    while (status == 1) {
        if (sqrt(rr) <= p.tol * bnorm) { status = 0; break; }
        if (k >= p.maxit) break;
        double *pn = (k & 1) ? p.p1 : p.p0;        // p_k
        const double *po = (k & 1) ? p.p0 : p.p1;  // p_{k-1}
        // phase 1: q = A p_k with p_k formed on the fly; own p_k stored
        double acc1[1] = {0.0};
        spmv_rows(p, r0, r1, L, kbase, kc,
                  [&](int c) { return __builtin_fma(beta, ld_coh(po + c), ld_coh(zsrc + c)); },
                  [&](int i, double s) {
                      const double pi = __builtin_fma(beta, ld_coh(po + i), ld_coh(zsrc + i));
                      p.q[i] = s;
                      st_coh(pn + i, pi);
                      acc1[0] = __builtin_fma(pi, s, acc1[0]);
                  });
        block_sum<1>(acc1, red);
        if (tid == 0) st_coh(p.part + (size_t)PART_PQ * G + g, acc1[0]);
        gs.sync();
        const double pq = grid_total(p.part, PART_PQ, &bcast);
        if (!(pq > 0.0) || !isfinite(pq)) { status = 2; break; }
        const double alpha = rho / pq;
        // phase 2: x, r, z updates on own rows
        double acc2[2] = {0.0, 0.0};
        for (int i = r0 + tid; i < r1; i += CG_THREADS) {
            const double pi = ld_coh(pn + i);
            const double qi = p.q[i];
            // x is read by other workgroups for the final true residual
            st_coh(p.x + i, __builtin_fma(alpha, pi, ld_coh(p.x + i)));
            const double ri = __builtin_fma(-alpha, qi, JACOBI ? p.r[i] : ld_coh(p.r + i));
            double zi = ri;
            if (JACOBI) {
                p.r[i] = ri;
                zi = p.dinv[i] * ri;
                st_coh(p.z + i, zi);
            } else {
                st_coh(p.r + i, ri);
            }
            acc2[0] = __builtin_fma(ri, zi, acc2[0]);
            acc2[1] = __builtin_fma(ri, ri, acc2[1]);
        }
        block_sum<2>(acc2, red);
        if (tid == 0) {
            st_coh(p.part + (size_t)PART_RZ * G + g, acc2[0]);
            st_coh(p.part + (size_t)PART_RR * G + g, acc2[1]);
        }
        gs.sync();
        const double rho_new = grid_total(p.part, PART_RZ, &bcast);
        rr = grid_total(p.part, PART_RR, &bcast);
        ++k;
        if (JACOBI && !(rho_new > 0.0) && rr > 0.0) { status = 2; break; }
        beta = rho_new / rho;
        rho = rho_new;
    }
    // true residual ||b - A x|| (x of other workgroups read coherently)
    double acc3[1] = {0.0};
    gs.sync();
    spmv_rows(p, r0, r1, L, kbase, kc, [&](int c) { return ld_coh(p.x + c); },
              [&](int i, double s) {
                  const double d = p.b[i] - s;
                  acc3[0] = __builtin_fma(d, d, acc3[0]);
              });
    block_sum<1>(acc3, red);
    if (tid == 0) st_coh(p.part + (size_t)PART_TRUE * G + g, acc3[0]);
    gs.sync();
    const double tt = grid_total(p.part, PART_TRUE, &bcast);
    if (g == 0 && tid == 0) {
        p.result[0] = k;
        p.result[1] = status;
        p.result[2] = bnorm > 0.0 ? sqrt(rr) / bnorm : 0.0;
        p.result[3] = bnorm > 0.0 ? sqrt(tt) / bnorm : 0.0;
        p.result[4] = bnorm;
    }
    gs.finish();
}

// ---------------------------------------------------------------------------
// Baseline kernels (one launch each per iteration).
struct BaseScalars {
    double rho, pq, alpha, beta, rr, bb, rho_new, status;
};

__global__ __launch_bounds__(256) void base_spmv(const int *rowptr, const int *colind, const double *val, int n,
                                                 int L, const double *v, double *y, const double *pvec,
                                                 double *part) {
    // y = A v; part[block] = sum_i pvec_i * y_i (when pvec != nullptr)
    const int tid = threadIdx.x, gl = tid & (L - 1);
    const int i = blockIdx.x * (256 / L) + tid / L;
    double s = 0.0;
    if (i < n) {
        for (int k = rowptr[i] + gl; k < rowptr[i + 1]; k += L) s = __builtin_fma(val[k], v[colind[k]], s);
    }
    s = group_sum(s, L);
    double d = 0.0;
    if (i < n && gl == 0) {
        y[i] = s;
        if (pvec) d = pvec[i] * s;
    }
    if (part) {
        __shared__ double red[4];
        d = wave_sum(d);
        if ((tid & 63) == 0) red[tid >> 6] = d;
        __syncthreads();
        if (tid == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

__global__ __launch_bounds__(256) void base_reduce(const double *part, int m, double *out) {
    // out = sum of m partials (one block, fixed order)
    __shared__ double red[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) s += part[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

__global__ void base_alpha(BaseScalars *s) {
    if (!(s->pq > 0.0) || !isfinite(s->pq)) s->status = 2;
    s->alpha = s->rho / s->pq;
}

__global__ __launch_bounds__(256) void base_update(int n, const BaseScalars *s, const double *pv, const double *q,
                                                   double *x, double *r, double *z, const double *dinv,
                                                   double *part_rz, double *part_rr) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    double a = 0.0, c = 0.0;
    if (i < n && s->status == 1.0) {
        const double alpha = s->alpha;
        x[i] = __builtin_fma(alpha, pv[i], x[i]);
        const double ri = __builtin_fma(-alpha, q[i], r[i]);
        r[i] = ri;
        const double zi = dinv ? dinv[i] * ri : ri;
        if (dinv) z[i] = zi;
        a = ri * zi;
        c = ri * ri;
    }
    __shared__ double red[8];
    a = wave_sum(a);
    c = wave_sum(c);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = a;
        red[4 + (threadIdx.x >> 6)] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part_rz[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
        part_rr[blockIdx.x] = red[4] + red[5] + red[6] + red[7];
    }
}

__global__ void base_beta(BaseScalars *s) {
    s->beta = s->rho_new / s->rho;
    s->rho = s->rho_new;
}

__global__ __launch_bounds__(256) void base_pupdate(int n, const BaseScalars *s, const double *z, double *pv) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n && s->status == 1.0) pv[i] = __builtin_fma(s->beta, pv[i], z[i]);
}

__global__ __launch_bounds__(256) void base_init(int n, const double *b, const double *ax, double *r, double *z,
                                                 double *pv, const double *dinv, double *part_bb,
                                                 double *part_rz, double *part_rr) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    double a = 0.0, c = 0.0, d = 0.0;
    if (i < n) {
        const double ri = b[i] - ax[i];
        r[i] = ri;
        const double zi = dinv ? dinv[i] * ri : ri;
        if (dinv) z[i] = zi;
        pv[i] = zi;
        a = b[i] * b[i];
        c = ri * zi;
        d = ri * ri;
    }
    __shared__ double red[12];
    a = wave_sum(a);
    c = wave_sum(c);
    d = wave_sum(d);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = a;
        red[4 + (threadIdx.x >> 6)] = c;
        red[8 + (threadIdx.x >> 6)] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part_bb[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
        part_rz[blockIdx.x] = red[4] + red[5] + red[6] + red[7];
        part_rr[blockIdx.x] = red[8] + red[9] + red[10] + red[11];
    }
}

__global__ __launch_bounds__(256) void invert_diagonal(const int *rowptr, const int *colind, const double *val,
                                                       int n, double *dinv) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
        if (colind[k] == i) d += val[k];
    dinv[i] = 1.0 / d;
}

__global__ __launch_bounds__(256) void true_residual_part(const int *rowptr, const int *colind, const double *val,
                                                          int n, const double *x, const double *b, double *part) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    double d = 0.0;
    if (i < n) {
        double s = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) s = __builtin_fma(val[k], x[colind[k]], s);
        const double e = b[i] - s;
        d = e * e;
    }
    __shared__ double red[4];
    d = wave_sum(d);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------------------
int check_csr(const perks_csr *A, const void *b, const void *x, double tol, int maxit, int precond) {
    if (!A || !b || !x) return set_error(PERKS_E_INVAL, "A, b and x must not be NULL");
    if (A->n < 0 || A->nnz < 0) return set_error(PERKS_E_INVAL, "negative matrix size");
    if (A->n > 0 && (!A->rowptr || !A->colind || (A->nnz > 0 && !A->val)))
        return set_error(PERKS_E_INVAL, "CSR arrays must not be NULL");
    if (A->n >= (int64_t(1) << 31) - 1 || A->nnz >= (int64_t(1) << 31) - 1)
        return set_error(PERKS_E_INVAL, "32-bit CSR indices limit n and nnz to < 2^31");
    if (A->dt != PERKS_F64) return set_error(PERKS_E_UNSUPPORTED, "this entry point solves FP64 matrices");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return set_error(PERKS_E_INVAL, "tol must be finite and >= 0");
    if (maxit < 0) return set_error(PERKS_E_INVAL, "maxit must be >= 0");
    if (precond != PERKS_PRECOND_NONE && precond != PERKS_PRECOND_JACOBI)
        return set_error(PERKS_E_INVAL, "unknown preconditioner %d", precond);
    return PERKS_OK;
}

struct CgWork {
    double *r, *z, *q, *p0, *p1, *dinv, *part, *result;
};

int cg_work(int64_t n, int G, CgWork *w) {
    const size_t nv = (size_t)n + 64;
    const size_t bytes = (6 * nv + (size_t)NPART * std::max(G, 1) + 64) * sizeof(double);
    double *base = (double *)scratch(SLOT_CG_VEC, bytes);
    if (!base) return PERKS_E_NOMEM;
    w->r = base;
    w->z = base + nv;
    w->q = base + 2 * nv;
    w->p0 = base + 3 * nv;
    w->p1 = base + 4 * nv;
    w->dinv = base + 5 * nv;
    w->part = base + 6 * nv;
    w->result = w->part + (size_t)NPART * std::max(G, 1);
    return PERKS_OK;
}

void fill_result(perks_cg_result *out, int iters, int status, int restarts, int wgs, double relres,
                 double reltrue, double frac) {
    if (!out) return;
    out->iters = iters;
    out->status = status;
    out->restarts = restarts;
    out->wgs = wgs;
    out->relres = relres;
    out->relres_true = reltrue;
    out->cached_nnz_frac = frac;
    out->reserved = 0;
}

}  // namespace
}  // namespace perks

using namespace perks;

extern "C" {

int perks_cg_solve(const perks_csr *A, const void *b, void *x, double tol, int32_t maxit, int32_t precond,
                   void *stream, perks_cg_result *out) {
    int rc = check_csr(A, b, x, tol, maxit, precond);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (A->n == 0) {
        fill_result(out, 0, PERKS_OK, 0, 0, 0.0, 0.0, 0.0);
        return PERKS_OK;
    }
    DeviceFacts f;
    rc = device_facts(&f);
    if (rc) return rc;
    const bool jac = precond == PERKS_PRECOND_JACOBI;
    const void *fn = jac ? reinterpret_cast<const void *>(&cg_persistent<true>)
                         : reinterpret_cast<const void *>(&cg_persistent<false>);
    // LDS: static cache of A (12 B per nonzero)
    const int lds_nnz = CG_LDS_NNZ;
    int occ = 0;
    PERKS_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, CG_THREADS, 0));
    if (occ < 1) return set_error(PERKS_E_NOTCORESIDENT, "CG kernel does not fit one workgroup per CU");
    // one workgroup per CU, fewer for small systems (at least ~4 rows per thread)
    int G = f.cus;
    const int64_t min_rows = (int64_t)CG_THREADS;
    if (A->n / min_rows < G) G = (int)std::max<int64_t>(1, A->n / min_rows);
    if (G > SYNC_MAX_WGS) G = SYNC_MAX_WGS;
    CgWork w;
    rc = cg_work(A->n, G, &w);
    if (rc) return rc;
    unsigned *sync = (unsigned *)scratch(SLOT_SYNC, SYNC_BYTES);
    if (!sync) return PERKS_E_NOMEM;
    const int nb = (int)((A->n + 255) / 256);
    if (jac) hipLaunchKernelGGL(invert_diagonal, dim3(nb), dim3(256), 0, st, A->rowptr, A->colind,
                                (const double *)A->val, (int)A->n, w.dinv);
    CgParams p{};
    p.rowptr = A->rowptr;
    p.colind = A->colind;
    p.val = (const double *)A->val;
    p.b = (const double *)b;
    p.x = (double *)x;
    p.r = w.r;
    p.z = jac ? w.z : w.r;
    p.q = w.q;
    p.p0 = w.p0;
    p.p1 = w.p1;
    p.dinv = w.dinv;
    p.part = w.part;
    p.result = w.result;
    p.sync = sync;
    p.n = (int)A->n;
    p.nnz = (int)A->nnz;
    p.precond = precond;
    p.lds_nnz = lds_nnz;
    p.tol = tol;
    int total = 0, restarts = 0, status = PERKS_NOT_CONVERGED;
    double h[8] = {0};
    for (;;) {
        p.maxit = maxit - total;
        void *args[] = {&p};
        hipError_t e = hipLaunchCooperativeKernel(fn, dim3(G), dim3(CG_THREADS), args, 0, st);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(e == hipErrorCooperativeLaunchTooLarge ? PERKS_E_NOTCORESIDENT : PERKS_E_HIP,
                             "CG launch: %s", hipGetErrorString(e));
        }
        PERKS_HIP_TRY(hipMemcpyAsync(h, w.result, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
        PERKS_HIP_TRY(hipStreamSynchronize(st));
        total += (int)h[0];
        status = (int)h[1];
        if (status == 2) {
            status = PERKS_BREAKDOWN;
            break;
        }
        if (h[3] <= tol) {
            status = PERKS_OK;
            break;
        }
        if (total >= maxit) {
            status = PERKS_NOT_CONVERGED;
            break;
        }
        ++restarts;   // recursive residual converged but the true one did not
    }
    // share of A's nonzeros held in LDS
    const double cached = std::min<double>((double)A->nnz, (double)lds_nnz * G);
    fill_result(out, total, status, restarts, G, h[2], h[3], A->nnz ? cached / (double)A->nnz : 0.0);
    return status;
}

int perks_cg_solve_baseline(const perks_csr *A, const void *b, void *x, double tol, int32_t maxit, int32_t precond,
                            int32_t check_every, void *stream, perks_cg_result *out) {
    int rc = check_csr(A, b, x, tol, maxit, precond);
    if (rc) return rc;
    if (check_every < 1) return set_error(PERKS_E_INVAL, "check_every must be >= 1");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int n = (int)A->n;
    if (n == 0) {
        fill_result(out, 0, PERKS_OK, 0, 0, 0.0, 0.0, 0.0);
        return PERKS_OK;
    }
    const bool jac = precond == PERKS_PRECOND_JACOBI;
    const int nb = (n + 255) / 256;
    const int avg = (int)((A->nnz + n - 1) / n);
    int L = 1;
    while (L < avg && L < 64) L <<= 1;
    const int nbs = (n + (256 / L) - 1) / (256 / L);
    CgWork w;
    rc = cg_work(A->n, std::max(nb, nbs) * 3 + 64, &w);
    if (rc) return rc;
    double *part_a = w.part, *part_b = w.part + std::max(nb, nbs) + 16, *part_c = part_b + std::max(nb, nbs) + 16;
    BaseScalars *S = reinterpret_cast<BaseScalars *>(w.result);
    const double *val = (const double *)A->val;
    double *xd = (double *)x;
    double *z = jac ? w.z : w.r;
    const double *dinv = jac ? w.dinv : nullptr;
    if (jac) hipLaunchKernelGGL(invert_diagonal, dim3(nb), dim3(256), 0, st, A->rowptr, A->colind, val, n, w.dinv);
    int total = 0, restarts = 0, status = PERKS_NOT_CONVERGED;
    double relres = 0.0, reltrue = 0.0;
    for (;;) {
        // (re)start: r = b - A x, z, p = z, rho = r.z
        hipLaunchKernelGGL(base_spmv, dim3(nbs), dim3(256), 0, st, A->rowptr, A->colind, val, n, L, xd, w.q,
                           (const double *)nullptr, (double *)nullptr);
        hipLaunchKernelGGL(base_init, dim3(nb), dim3(256), 0, st, n, (const double *)b, w.q, w.r, w.z, w.p0, dinv,
                           part_a, part_b, part_c);
        hipLaunchKernelGGL(base_reduce, dim3(1), dim3(256), 0, st, part_a, nb, &S->bb);
        hipLaunchKernelGGL(base_reduce, dim3(1), dim3(256), 0, st, part_b, nb, &S->rho);
        hipLaunchKernelGGL(base_reduce, dim3(1), dim3(256), 0, st, part_c, nb, &S->rr);
        double hs[8];
        PERKS_HIP_TRY(hipMemcpyAsync(hs, S, sizeof(BaseScalars), hipMemcpyDeviceToHost, st));
        PERKS_HIP_TRY(hipStreamSynchronize(st));
        const double bnorm = std::sqrt(hs[5]);
        double rr = hs[4];
        hs[7] = 1.0;
        PERKS_HIP_TRY(hipMemcpyAsync(&S->status, &hs[7], sizeof(double), hipMemcpyHostToDevice, st));
        if (bnorm == 0.0) {
            PERKS_HIP_TRY(hipMemsetAsync(xd, 0, (size_t)n * sizeof(double), st));
            status = PERKS_OK;
            relres = reltrue = 0.0;
            break;
        }
        int k = 0;
        bool conv = std::sqrt(rr) <= tol * bnorm, broke = false;
        while (!conv && total + k < maxit) {
            hipLaunchKernelGGL(base_spmv, dim3(nbs), dim3(256), 0, st, A->rowptr, A->colind, val, n, L, w.p0, w.q,
                               (const double *)w.p0, part_a);
            hipLaunchKernelGGL(base_reduce, dim3(1), dim3(256), 0, st, part_a, nbs, &S->pq);
            hipLaunchKernelGGL(base_alpha, dim3(1), dim3(1), 0, st, S);
            hipLaunchKernelGGL(base_update, dim3(nb), dim3(256), 0, st, n, S, w.p0, w.q, xd, w.r, w.z, dinv, part_b,
                               part_c);
            hipLaunchKernelGGL(base_reduce, dim3(1), dim3(256), 0, st, part_b, nb, &S->rho_new);
            hipLaunchKernelGGL(base_reduce, dim3(1), dim3(256), 0, st, part_c, nb, &S->rr);
            hipLaunchKernelGGL(base_beta, dim3(1), dim3(1), 0, st, S);
            hipLaunchKernelGGL(base_pupdate, dim3(nb), dim3(256), 0, st, n, S, z, w.p0);
            ++k;
            if (k % check_every == 0 || total + k >= maxit) {
                PERKS_HIP_TRY(hipMemcpyAsync(hs, S, sizeof(BaseScalars), hipMemcpyDeviceToHost, st));
                PERKS_HIP_TRY(hipStreamSynchronize(st));
                if (hs[7] != 1.0) {
                    broke = true;
                    break;
                }
                conv = std::sqrt(hs[4]) <= tol * bnorm;
            }
        }
        PERKS_HIP_TRY(hipGetLastError());
        PERKS_HIP_TRY(hipMemcpyAsync(hs, S, sizeof(BaseScalars), hipMemcpyDeviceToHost, st));
        hipLaunchKernelGGL(true_residual_part, dim3(nb), dim3(256), 0, st, A->rowptr, A->colind, val, n, xd,
                           (const double *)b, part_a);
        hipLaunchKernelGGL(base_reduce, dim3(1), dim3(256), 0, st, part_a, nb, &S->pq);
        double tr = 0.0;
        PERKS_HIP_TRY(hipMemcpyAsync(&tr, &S->pq, sizeof(double), hipMemcpyDeviceToHost, st));
        PERKS_HIP_TRY(hipStreamSynchronize(st));
        total += k;
        relres = std::sqrt(hs[4]) / bnorm;
        reltrue = std::sqrt(tr) / bnorm;
        if (broke) {
            status = PERKS_BREAKDOWN;
            break;
        }
        if (reltrue <= tol) {
            status = PERKS_OK;
            break;
        }
        if (total >= maxit) {
            status = PERKS_NOT_CONVERGED;
            break;
        }
        ++restarts;
    }
    fill_result(out, total, status, restarts, 0, relres, reltrue, 0.0);
    return status;
}

}  // extern "C"
