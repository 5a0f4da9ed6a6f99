// Conjugate gradient (Sec. 2.2.2, Sec. 4.3): the fused persistent solver and
// the host-looped multi-kernel baseline, FP64, CSR matrices.
//
// Persistent solver, per iteration (three device-wide barriers):
//   phase P  p = z + beta p on own rows (z = r unpreconditioned, z = D^{-1} r
//            for Jacobi)
//   barrier  every workgroup's p complete
//   phase 1  q = A p on the workgroup's rows (one gather of p per nonzero);
//            partial p.q
//   barrier  every workgroup sums the partials in the same fixed order -> alpha
//   phase 2  x += alpha p, r -= alpha q, z = D^{-1} r on own rows; partials r.z, r.r
//   barrier  -> beta and the (uniform) convergence decision.
// Forming p where it is gathered instead (p_j = z_j + beta pold_j inside the
// SpMV, no barrier of its own) costs a second gather per nonzero; measured on
// gfx950 it was slower on both a 7-point Poisson matrix (4%) and a random
// sparse matrix (2.1x), so the solver takes the extra barrier.
// The row partition is a merge-path split of (rows + nonzeros) into equal
// shares, searched once at kernel start (the paper keeps its thread-block
// search result for the whole solve because A is static, Sec. 4.3.2).  The
// first part of the workgroup's slice of A (values and column indices) is
// copied into LDS once and read from there every iteration (the on-chip
// cache of A); the rest streams from L2 / Infinity Cache / HBM.
#include <algorithm>
#include <cmath>
#include <new>
#include <mutex>
#include <vector>

#include "cg_device.hpp"

namespace perks {

// The register-resident FP64 solver kernel (cg_reg.hip) and its launch
// shape: threads per workgroup, rows per thread.
const void *cg_reg_kernel(bool jacobi, bool mixed, int *threads, int *rows_per_thread);

namespace {

// ---------------------------------------------------------------------------
// Baseline kernels (one launch each per iteration).
struct BaseScalars {
    double rho, pq, alpha, beta, rr, bb, rho_new, status;
};

// y = A v for the rows of this block (U rows per group of L lanes, loads of
// all U rows issued before use); part[block] = sum_i pvec_i * y_i when pvec
// is given.
constexpr int BASE_U = 4;
template <typename T>
__global__ __launch_bounds__(256) void base_spmv(const int *rowptr, const int *colind, const T *val, int n, int L,
                                                 const T *v, T *y, const T *pvec, double *part) {
    const int tid = threadIdx.x, gl = tid & (L - 1);
    const int rpp = 256 / L;
    const int row0 = blockIdx.x * rpp * BASE_U;
    int kb[BASE_U], ke[BASE_U];
    T s[BASE_U];
    int len = 0;
#pragma unroll
    for (int u = 0; u < BASE_U; ++u) {
        const int i = row0 + u * rpp + tid / L;
        kb[u] = 0;
        ke[u] = 0;
        s[u] = T(0);
        if (i < n) {
            kb[u] = rowptr[i] + gl;
            ke[u] = rowptr[i + 1];
        }
        len = max(len, ke[u] - kb[u]);
    }
    for (int j = 0; j < len; j += L) {
#pragma unroll
        for (int u = 0; u < BASE_U; ++u) {
            const int k = kb[u] + j;
            if (k < ke[u]) s[u] = fma_t(val[k], v[colind[k]], s[u]);
        }
    }
    double d = 0.0;
#pragma unroll
    for (int u = 0; u < BASE_U; ++u) {
        const T t = group_sum(s[u], L);
        const int i = row0 + u * rpp + tid / L;
        if (i < n && gl == 0) {
            y[i] = t;
            if (pvec) d = __builtin_fma((double)pvec[i], (double)t, d);
        }
    }
    if (part) {
        __shared__ double red[4];
        d = wave_sum(d);
        if ((tid & 63) == 0) red[tid >> 6] = d;
        __syncthreads();
        if (tid == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

// out = sum of m partials (one block, fixed order; eight independent loads
// in flight per thread).
__global__ __launch_bounds__(1024) void base_reduce(const double *part, int m, double *out) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i0 = 0; i0 < m; i0 += 1024 * 8) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * 1024 + (int)threadIdx.x;
            t[u] = i < m ? part[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s += t[u];
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int w = 0; w < 16; ++w) r += red[w];
        *out = r;
    }
}

__global__ void base_alpha(BaseScalars *s) {
    if (!(s->pq > 0.0) || !isfinite(s->pq)) s->status = 2;
    s->alpha = s->rho / s->pq;
}

template <typename T>
__global__ __launch_bounds__(256) void base_update(int n, const BaseScalars *s, const T *pv, const T *q, T *x, T *r,
                                                   T *z, const T *dinv, double *part_rz, double *part_rr) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    double a = 0.0, c = 0.0;
    if (i < n && s->status == 1.0) {
        const T alpha = (T)s->alpha;
        x[i] = fma_t(alpha, pv[i], x[i]);
        const T ri = fma_t(-alpha, q[i], r[i]);
        r[i] = ri;
        const T zi = dinv ? dinv[i] * ri : ri;
        if (dinv) z[i] = zi;
        a = (double)ri * (double)zi;
        c = (double)ri * (double)ri;
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

template <typename T>
__global__ __launch_bounds__(256) void base_pupdate(int n, const BaseScalars *s, const T *z, T *pv) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n && s->status == 1.0) pv[i] = fma_t((T)s->beta, pv[i], z[i]);
}

// Mixed-precision baseline steps.  r64 = b - ax (ax NULL: 0; r64 NULL: not
// stored); part = sum of r64^2.
__global__ __launch_bounds__(256) void base_resid(int n, const double *b, const double *ax, double *r64,
                                                  double *part) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    double d = 0.0;
    if (i < n) {
        const double ri = ax ? b[i] - ax[i] : b[i];
        if (r64) r64[i] = ri;
        d = ri * ri;
    }
    __shared__ double red[4];
    d = wave_sum(d);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Residual replacement: r32 = float(sc r64), z32, d32 = 0, the direction
// p32 multiplied by ratio (a power of two: exact); partial r.z and r.r in FP64.
__global__ __launch_bounds__(256) void base_mixed_replace(int n, const double *r64, double sc, float ratio, float *r,
                                                          float *z, float *pv, float *d, const float *dinv,
                                                          double *part_rz, double *part_rr) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    double a = 0.0, c = 0.0;
    if (i < n) {
        const float ri = (float)(r64[i] * sc);
        r[i] = ri;
        const float zi = dinv ? dinv[i] * ri : ri;
        if (dinv) z[i] = zi;
        pv[i] = pv[i] * ratio;
        d[i] = 0.0f;
        a = (double)ri * (double)zi;
        c = (double)ri * (double)ri;
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

// beta after a replacement: rho_new is the new residual's r.z, rho the last
// r.z of the recurrence (in the old units: ratio2 = (s'/s)^2); the first
// replacement starts the recurrence (beta 0).
__global__ void base_replace_beta(BaseScalars *s, double ratio2, int first) {
    s->beta = first ? 0.0 : s->rho_new / (s->rho * ratio2);
    s->rho = s->rho_new;
    s->status = 1.0;
}

__global__ __launch_bounds__(256) void base_xupdate(int n, double *x, const float *d, double sc) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = x[i] + (double)d[i] / sc;
}

__global__ __launch_bounds__(256) void zero_words(unsigned *w, int m) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < m) w[i] = 0u;
}

__global__ __launch_bounds__(256) void to_f32(int64_t m, const double *a, float *o) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) o[i] = (float)a[i];
}

__global__ __launch_bounds__(256) void invert_diagonal32(const int *rowptr, const int *colind, const double *val,
                                                         int n, float *dinv) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double dg = 0.0;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
        if (colind[k] == i) dg += val[k];
    dinv[i] = (float)(1.0 / dg);
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
int check_csr(const perks_csr *A, const void *b, const void *x, double tol, int maxit, int precond,
              int precision) {
    if (!A) return set_error(PERKS_E_INVAL, "A must not be NULL");
    if (A->n < 0 || A->nnz < 0) return set_error(PERKS_E_INVAL, "negative matrix size");
    if (A->n > 0 && (!b || !x)) return set_error(PERKS_E_INVAL, "b and x must not be NULL");
    if (A->n > 0 && (!A->rowptr || !A->colind || (A->nnz > 0 && !A->val)))
        return set_error(PERKS_E_INVAL, "CSR arrays must not be NULL");
    if (A->n >= (int64_t(1) << 31) - 1 || A->nnz >= (int64_t(1) << 31) - 1)
        return set_error(PERKS_E_INVAL, "32-bit CSR indices limit n and nnz to < 2^31");
    if (A->dt != PERKS_F64) return set_error(PERKS_E_UNSUPPORTED, "this entry point solves FP64 matrices");
    if (A->spmv < 0 || A->spmv > 2) return set_error(PERKS_E_INVAL, "spmv must be 0, 1 or 2 (got %d)", A->spmv);
    if (!(tol >= 0.0) || !std::isfinite(tol)) return set_error(PERKS_E_INVAL, "tol must be finite and >= 0");
    if (maxit < 0) return set_error(PERKS_E_INVAL, "maxit must be >= 0");
    if (precond != PERKS_PRECOND_NONE && precond != PERKS_PRECOND_JACOBI)
        return set_error(PERKS_E_INVAL, "unknown preconditioner %d", precond);
    if (precision != PERKS_PREC_F64 && precision != PERKS_PREC_MIXED)
        return set_error(PERKS_E_INVAL, "unknown precision %d", precision);
    return PERKS_OK;
}

// Work area of one problem: the partial-sum table (NPART per workgroup) and
// 64 result words, then the vectors.  FP64 solver: r, z, q, p, dinv (n
// doubles each), the sliced-ELL values and indices.  Mixed solver: r64 (n
// doubles); r, z, q, p, d, dinv (n floats each); the FP32 copy of A's values
// (nnz floats); the sliced-ELL FP32 values and indices, and the FP64 values of
// the same layout.  Every vector starts on a 256-byte boundary.
size_t vec_len(int64_t n) { return ((size_t)n + 63) / 64 * 64 + 64; }

size_t inst_bytes(int64_t n, int64_t nnz, int parts, bool mixed) {
    const size_t nv = vec_len(n);
    const size_t np = ((size_t)NPART * std::max(parts, 1) + 64 + 31) / 32 * 32;
    const size_t ns = (sell_capacity(nnz, std::max(parts, 1)) + 63) / 64 * 64;
    size_t bytes = (np + 64) * sizeof(double);
    if (mixed)
        bytes += nv * sizeof(double) + 6 * nv * sizeof(float) + (((size_t)nnz + 63) / 64 * 64) * sizeof(float) +
                 ns * (sizeof(float) + sizeof(int) + sizeof(double));
    else
        bytes += 5 * nv * sizeof(double) + ns * (sizeof(double) + sizeof(int));
    bytes += nv * sizeof(int);   // sperm
    return (bytes + 255) / 256 * 256;
}

void carve(char *base, int64_t n, int64_t nnz, int parts, bool mixed, CgInst *w) {
    const size_t nv = vec_len(n);
    const size_t np = ((size_t)NPART * std::max(parts, 1) + 64 + 31) / 32 * 32;
    const size_t ns = (sell_capacity(nnz, std::max(parts, 1)) + 63) / 64 * 64;
    w->part = (double *)base;
    w->result = w->part + np;
    char *v = (char *)(w->result + 64);
    if (mixed) {
        w->r64 = (double *)v;
        float *f = (float *)(v + nv * sizeof(double));
        w->r32 = f;
        w->z32 = f + nv;
        w->q32 = f + 2 * nv;
        w->p32 = f + 3 * nv;
        w->d32 = f + 4 * nv;
        w->dinv32 = f + 5 * nv;
        w->val32 = f + 6 * nv;
        w->sval32 = w->val32 + ((size_t)nnz + 63) / 64 * 64;
        w->scol = (int *)(w->sval32 + ns);
        w->sperm = w->scol + ns;
        w->sval64 = (double *)(w->sperm + nv);   // FP64 values of the sliced-ELL layout
    } else {
        double *d = (double *)v;
        w->r = d;
        w->z = d + nv;
        w->q = d + 2 * nv;
        w->p = d + 3 * nv;
        w->dinv = d + 4 * nv;
        w->sval64 = d + 5 * nv;
        w->scol = (int *)(w->sval64 + ns);
        w->sperm = w->scol + ns;
    }
}

using CgWork = CgInst;

// Work area of a single solve, in the library's scratch slot.
int cg_work(int64_t n, int64_t nnz, int parts, bool mixed, CgWork *w) {
    *w = CgWork{};
    char *base = (char *)scratch(SLOT_CG_VEC, inst_bytes(n, nnz, parts, mixed));
    if (!base) return PERKS_E_NOMEM;
    carve(base, n, nnz, parts, mixed, w);
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
    out->fallbacks = 0;
    out->switched_at = -1;
    out->barrier_cycles = 0;
}

// Result words (iters, status, relres, relres_true, ||b||, restarts/outer)
// -> perks_cg_result; returns the status code.
int result_from_words(const double *h, int wgs, double cached_frac, perks_cg_result *out) {
    const int st = (int)h[1];
    const int status = st == 2 ? PERKS_BREAKDOWN : st == 0 ? PERKS_OK : PERKS_NOT_CONVERGED;
    fill_result(out, (int)h[0], status, (int)h[5], wgs, h[2], h[3], cached_frac);
    return status;
}

int launch_error(hipError_t e) {
    (void)hipGetLastError();
    return set_error(e == hipErrorCooperativeLaunchTooLarge ? PERKS_E_NOTCORESIDENT : PERKS_E_HIP, "CG launch: %s",
                     hipGetErrorString(e));
}

template <bool MERGE>
const void *persistent_fn_t(bool jac, bool mixed) {
    if (mixed) return jac ? reinterpret_cast<const void *>(&cg_persistent<true, true, MERGE>)
                          : reinterpret_cast<const void *>(&cg_persistent<false, true, MERGE>);
    return jac ? reinterpret_cast<const void *>(&cg_persistent<true, false, MERGE>)
               : reinterpret_cast<const void *>(&cg_persistent<false, false, MERGE>);
}

// The persistent solver kernel; the merge-path SpMV is built into separate
// instances, so the other layouts do not carry its registers.
const void *persistent_fn(bool jac, bool mixed, bool merge = false) {
    return merge ? persistent_fn_t<true>(jac, mixed) : persistent_fn_t<false>(jac, mixed);
}

const void *batched_fn(bool jac, bool mixed) {
    if (mixed) return jac ? reinterpret_cast<const void *>(&cg_batched<true, true>)
                          : reinterpret_cast<const void *>(&cg_batched<false, true>);
    return jac ? reinterpret_cast<const void *>(&cg_batched<true, false>)
               : reinterpret_cast<const void *>(&cg_batched<false, false>);
}

// Workgroups the device holds at once for a CG kernel (one per CU).
int cg_capacity(const void *fn, int *cap) {
    DeviceFacts f;
    int rc = device_facts(&f);
    if (rc) return rc;
    int occ = 0;
    PERKS_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, CG_THREADS, 0));
    if (occ < 1) return set_error(PERKS_E_NOTCORESIDENT, "CG kernel does not fit one workgroup per CU");
    *cap = std::min(f.cus, SYNC_MAX_WGS);
    return PERKS_OK;
}

// Group size for one problem: the whole device, fewer for small systems (at
// least one row per thread).
int cg_group_size(int cap, int64_t n) {
    int g = cap;
    if (n / CG_THREADS < g) g = (int)std::max<int64_t>(1, n / CG_THREADS);
    return g;
}

// Matrices (by their device arrays, order, nonzeros and grid size) whose
// slices the register-resident solver could not take: later solves of the
// same matrix go straight to the memory-resident solver.  Only a hint: the
// solver checks eligibility itself.
struct NoregKey {
    const void *rowptr, *colind;
    int64_t n, nnz;
    int G, device;
};
std::mutex g_noreg_mu;
std::vector<NoregKey> g_noreg;

bool noreg_known(const perks_csr *A, int G) {
    int dev = -1;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(g_noreg_mu);
    for (const NoregKey &k : g_noreg)
        if (k.rowptr == A->rowptr && k.colind == A->colind && k.n == A->n && k.nnz == A->nnz && k.G == G &&
            k.device == dev)
            return true;
    return false;
}

void noreg_remember(const perks_csr *A, int G) {
    int dev = -1;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(g_noreg_mu);
    if (g_noreg.size() >= 256) g_noreg.erase(g_noreg.begin());
    g_noreg.push_back({A->rowptr, A->colind, A->n, A->nnz, G, dev});
}

struct Capture {
    const int *iters = nullptr;
    int n = 0;
    double *x = nullptr, *r = nullptr;
};

int cg_persistent_solve(const perks_csr *A, const void *b, void *x, double tol, int maxit, bool jac, bool mixed,
                        hipStream_t st, perks_cg_result *out, const Capture &capture = Capture()) {
    const void *fn = persistent_fn(jac, mixed, A->spmv == 2);
    int cap = 0;
    int rc = cg_capacity(fn, &cap);
    if (rc) return rc;
    const int G = cg_group_size(cap, A->n);
    CgInst p;
    rc = cg_work(A->n, A->nnz, G, mixed, &p);
    if (rc) return rc;
    unsigned *ws = (unsigned *)scratch(SLOT_SYNC, SYNC_BYTES);
    if (!ws) return PERKS_E_NOMEM;
    p.rowptr = A->rowptr;
    p.colind = A->colind;
    p.spmv = A->spmv;
    p.val = (const double *)A->val;
    p.b = (const double *)b;
    p.x = (double *)x;
    p.n = (int)A->n;
    p.nnz = (int)A->nnz;
    p.maxit = maxit;
    p.max_outer = PERKS_MIXED_MAX_OUTER;
    p.tol = tol;
    p.update_tol = PERKS_MIXED_UPDATE_TOL;
    p.cap_iters = capture.iters;
    p.ncap = capture.n;
    p.cap_x = capture.x;
    p.cap_r = capture.r;
    // the kernel reads the problem description from device memory (in the
    // spare result words)
    static_assert(sizeof(CgInst) <= 48 * sizeof(double), "problem description outgrew the result block");
    CgInst *pdev = reinterpret_cast<CgInst *>(p.result + 16);
    PERKS_HIP_TRY(hipMemcpyAsync(pdev, &p, sizeof(CgInst), hipMemcpyHostToDevice, st));
    void *args[] = {&pdev, &ws};
    note_persistent_launch(G, nullptr);
    double h[8] = {0};
    // first the solver with register-resident own rows when the rows per
    // workgroup suggest they fit (it reports CG_STATUS_NOREG and leaves after
    // its set-up when a slice does not)
    bool done = false;
    int reg_threads = 0, reg_rows = 0;
    const void *fr = A->spmv != 0 ? nullptr : cg_reg_kernel(jac, mixed, &reg_threads, &reg_rows);
    if (fr && (double)A->n / G <= 0.95 * reg_threads * reg_rows && !noreg_known(A, G)) {
        hipError_t e = hipLaunchCooperativeKernel(fr, dim3(G), dim3(reg_threads), args, 0, st);
        if (e != hipSuccess) return launch_error(e);
        PERKS_HIP_TRY(hipMemcpyAsync(h, p.result, 6 * sizeof(double), hipMemcpyDeviceToHost, st));
        PERKS_HIP_TRY(hipStreamSynchronize(st));
        done = (int)h[1] != CG_STATUS_NOREG;
        if (!done) noreg_remember(A, G);
    }
    if (!done) {
        hipError_t e = hipLaunchCooperativeKernel(fn, dim3(G), dim3(CG_THREADS), args, 0, st);
        if (e != hipSuccess) return launch_error(e);
        PERKS_HIP_TRY(hipMemcpyAsync(h, p.result, 6 * sizeof(double), hipMemcpyDeviceToHost, st));
        PERKS_HIP_TRY(hipStreamSynchronize(st));
    }
    const double lds = mixed ? CG_LDS_NNZ32 : CG_LDS_NNZ;
    const double cached = std::min<double>((double)A->nnz, lds * G);
    const int status = result_from_words(h, G, A->nnz ? cached / (double)A->nnz : 0.0, out);
    if (out) {
        perks_barrier_stats_t bs;
        rc = read_barrier_stats(G, nullptr, st, &bs);
        if (rc) return rc;
        out->barrier_cycles = (int64_t)bs.wait_cycles;
    }
    return status;
}

struct BaseShape {
    int n, nb, L, nbs;
    double *part_a, *part_b, *part_c;
    BaseScalars *S;
};

// Launch shape of the baseline kernels: L lanes per row (the power of two at
// or above the mean row length, at most 64), nb blocks of 256 rows for the
// vector kernels, nbs SpMV blocks of (256 / L) * BASE_U rows (more than nb
// when L > 4: the partial-sum arrays are sized for the larger).
void base_dims(const perks_csr *A, int *n, int *nb, int *L, int *nbs) {
    *n = (int)A->n;
    *nb = (*n + 255) / 256;
    const int avg = (int)((A->nnz + *n - 1) / *n);
    *L = 1;
    while (*L < avg && *L < 64) *L <<= 1;
    *nbs = (*n + (256 / *L) * BASE_U - 1) / ((256 / *L) * BASE_U);
}

BaseShape base_shape(const perks_csr *A, const CgWork &w) {
    BaseShape b{};
    base_dims(A, &b.n, &b.nb, &b.L, &b.nbs);
    const int m = std::max(b.nb, b.nbs);
    b.part_a = w.part;
    b.part_b = w.part + m + 16;
    b.part_c = b.part_b + m + 16;
    b.S = reinterpret_cast<BaseScalars *>(w.result);
    return b;
}

// Partial-sum entries the baseline needs: three arrays of max(nb, nbs) + 16.
int base_parts(const perks_csr *A) {
    int n, nb, L, nbs;
    base_dims(A, &n, &nb, &L, &nbs);
    return 3 * (std::max(nb, nbs) + 16) + 16;
}

int cg_baseline_f64(const perks_csr *A, const void *b, void *x, double tol, int maxit, bool jac, int check_every,
                    hipStream_t st, perks_cg_result *out) {
    CgWork w;
    int rc = cg_work(A->n, A->nnz, base_parts(A), false, &w);
    if (rc) return rc;
    const BaseShape B = base_shape(A, w);
    const int n = B.n, nb = B.nb, nbs = B.nbs, L = B.L;
    BaseScalars *S = B.S;
    const double *val = (const double *)A->val;
    double *xd = (double *)x;
    double *z = jac ? w.z : w.r;
    const double *dinv = jac ? w.dinv : nullptr;
    if (jac) hipLaunchKernelGGL(invert_diagonal, dim3(nb), dim3(256), 0, st, A->rowptr, A->colind, val, n, w.dinv);
    int total = 0, restarts = 0, status = PERKS_NOT_CONVERGED;
    double relres = 0.0, reltrue = 0.0;
    for (;;) {
        // (re)start: r = b - A x, z, p = z, rho = r.z
        hipLaunchKernelGGL(base_spmv<double>, dim3(nbs), dim3(256), 0, st, A->rowptr, A->colind, val, n, L, xd, w.q,
                           (const double *)nullptr, (double *)nullptr);
        hipLaunchKernelGGL(base_init, dim3(nb), dim3(256), 0, st, n, (const double *)b, w.q, w.r, w.z, w.p, dinv,
                           B.part_a, B.part_b, B.part_c);
        hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_a, nb, &S->bb);
        hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_b, nb, &S->rho);
        hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_c, nb, &S->rr);
        double hs[8];
        PERKS_HIP_TRY(hipMemcpyAsync(hs, S, sizeof(BaseScalars), hipMemcpyDeviceToHost, st));
        PERKS_HIP_TRY(hipStreamSynchronize(st));
        const double bnorm = std::sqrt(hs[5]);
        double rr = hs[4];
        hs[7] = 1.0;
        PERKS_HIP_TRY(hipMemcpyAsync(&S->status, &hs[7], sizeof(double), hipMemcpyHostToDevice, st));
        if (bnorm == 0.0) {
            PERKS_HIP_TRY(hipMemsetAsync(xd, 0, (size_t)n * sizeof(double), st));
            PERKS_HIP_TRY(hipStreamSynchronize(st));
            status = PERKS_OK;
            relres = reltrue = 0.0;
            break;
        }
        int k = 0;
        bool conv = std::sqrt(rr) <= tol * bnorm, broke = false;
        while (!conv && total + k < maxit) {
            hipLaunchKernelGGL(base_spmv<double>, dim3(nbs), dim3(256), 0, st, A->rowptr, A->colind, val, n, L, w.p,
                               w.q, (const double *)w.p, B.part_a);
            hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_a, nbs, &S->pq);
            hipLaunchKernelGGL(base_alpha, dim3(1), dim3(1), 0, st, S);
            hipLaunchKernelGGL(base_update<double>, dim3(nb), dim3(256), 0, st, n, S, w.p, w.q, xd, w.r, w.z, dinv,
                               B.part_b, B.part_c);
            hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_b, nb, &S->rho_new);
            hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_c, nb, &S->rr);
            hipLaunchKernelGGL(base_beta, dim3(1), dim3(1), 0, st, S);
            hipLaunchKernelGGL(base_pupdate<double>, dim3(nb), dim3(256), 0, st, n, S, (const double *)z, w.p);
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
                           (const double *)b, B.part_a);
        hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_a, nb, &S->pq);
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
        if (total >= maxit || k == 0) {   // no budget, or a cycle without progress
            status = PERKS_NOT_CONVERGED;
            break;
        }
        ++restarts;
    }
    fill_result(out, total, status, restarts, 0, relres, reltrue, 0.0);
    return status;
}

// Host-looped mixed-precision solve: the same algorithm as the persistent one
// (residual replacement around one FP32 recurrence) with one kernel per step,
// the host deciding every replacement and, every check_every iterations,
// whether the recursive residual has fallen enough for the next one.
int cg_baseline_mixed(const perks_csr *A, const void *b, void *x, double tol, int maxit, bool jac, int check_every,
                      hipStream_t st, perks_cg_result *out) {
    CgWork w;
    int rc = cg_work(A->n, A->nnz, base_parts(A), true, &w);
    if (rc) return rc;
    const BaseShape B = base_shape(A, w);
    const int n = B.n, nb = B.nb, nbs = B.nbs, L = B.L;
    BaseScalars *S = B.S;
    const double *val = (const double *)A->val;
    double *xd = (double *)x;
    float *z = jac ? w.z32 : w.r32;
    const float *dinv = jac ? w.dinv32 : nullptr;
    const int nbv = (int)((A->nnz + 255) / 256);
    if (A->nnz > 0) hipLaunchKernelGGL(to_f32, dim3(nbv), dim3(256), 0, st, (int64_t)A->nnz, val, w.val32);
    if (jac)
        hipLaunchKernelGGL(invert_diagonal32, dim3(nb), dim3(256), 0, st, A->rowptr, A->colind, val, n, w.dinv32);
    PERKS_HIP_TRY(hipMemsetAsync(w.p32, 0, (size_t)n * sizeof(float), st));
    PERKS_HIP_TRY(hipMemsetAsync(w.d32, 0, (size_t)n * sizeof(float), st));
    double hs[8];
    // ||b||
    hipLaunchKernelGGL(base_resid, dim3(nb), dim3(256), 0, st, n, (const double *)b, (const double *)nullptr,
                       (double *)nullptr, B.part_a);
    hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_a, nb, &S->bb);
    PERKS_HIP_TRY(hipMemcpyAsync(hs, S, sizeof(BaseScalars), hipMemcpyDeviceToHost, st));
    PERKS_HIP_TRY(hipStreamSynchronize(st));
    const double bnorm = std::sqrt(hs[5]);
    if (bnorm == 0.0) {
        PERKS_HIP_TRY(hipMemsetAsync(xd, 0, (size_t)n * sizeof(double), st));
        PERKS_HIP_TRY(hipStreamSynchronize(st));
        fill_result(out, 0, PERKS_OK, 0, 0, 0.0, 0.0, 0.0);
        return PERKS_OK;
    }
    int k = 0, outer = 0, stall = 0, status = PERKS_NOT_CONVERGED;
    double rn = 0.0, best = INFINITY, sc = 1.0;
    bool broke = false;
    for (;;) {
        // replacement: x += d / s, then r64 = b - A x in FP64 (A x lands in r64 first)
        if (outer > 0) hipLaunchKernelGGL(base_xupdate, dim3(nb), dim3(256), 0, st, n, xd, (const float *)w.d32, sc);
        hipLaunchKernelGGL(base_spmv<double>, dim3(nbs), dim3(256), 0, st, A->rowptr, A->colind, val, n, L,
                           (const double *)xd, w.r64, (const double *)nullptr, (double *)nullptr);
        hipLaunchKernelGGL(base_resid, dim3(nb), dim3(256), 0, st, n, (const double *)b, (const double *)w.r64,
                           w.r64, B.part_a);
        hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_a, nb, &S->rr);
        PERKS_HIP_TRY(hipMemcpyAsync(hs, S, sizeof(BaseScalars), hipMemcpyDeviceToHost, st));
        PERKS_HIP_TRY(hipStreamSynchronize(st));
        rn = std::sqrt(hs[4]);
        if (rn <= tol * bnorm) {
            status = PERKS_OK;
            break;
        }
        if (broke) {
            status = PERKS_BREAKDOWN;
            break;
        }
        if (rn < best) {
            best = rn;
            stall = 0;
        } else if (++stall >= PERKS_MIXED_STALL) {
            break;
        }
        if (k >= maxit || outer >= PERKS_MIXED_MAX_OUTER) break;
        int ex;
        (void)std::frexp(rn, &ex);
        const double sc_new = std::ldexp(1.0, 1 - ex);
        const double ratio = outer == 0 ? 1.0 : sc_new / sc;   // first: p is 0
        hipLaunchKernelGGL(base_mixed_replace, dim3(nb), dim3(256), 0, st, n, (const double *)w.r64, sc_new,
                           (float)ratio, w.r32, w.z32, w.p32, w.d32, dinv, B.part_b, B.part_c);
        hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_b, nb, &S->rho_new);
        hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_c, nb, &S->rr);
        hipLaunchKernelGGL(base_replace_beta, dim3(1), dim3(1), 0, st, S, ratio * ratio, outer == 0 ? 1 : 0);
        PERKS_HIP_TRY(hipMemcpyAsync(hs, S, sizeof(BaseScalars), hipMemcpyDeviceToHost, st));
        PERKS_HIP_TRY(hipStreamSynchronize(st));
        sc = sc_new;
        double rmax = std::sqrt(hs[4]);
        int j = 0;
        for (;;) {
            hipLaunchKernelGGL(base_pupdate<float>, dim3(nb), dim3(256), 0, st, n, S, (const float *)z, w.p32);
            hipLaunchKernelGGL(base_spmv<float>, dim3(nbs), dim3(256), 0, st, A->rowptr, A->colind,
                               (const float *)w.val32, n, L, (const float *)w.p32, w.q32, (const float *)w.p32,
                               B.part_a);
            hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_a, nbs, &S->pq);
            hipLaunchKernelGGL(base_alpha, dim3(1), dim3(1), 0, st, S);
            hipLaunchKernelGGL(base_update<float>, dim3(nb), dim3(256), 0, st, n, S, (const float *)w.p32,
                               (const float *)w.q32, w.d32, w.r32, w.z32, dinv, B.part_b, B.part_c);
            hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_b, nb, &S->rho_new);
            hipLaunchKernelGGL(base_reduce, dim3(1), dim3(1024), 0, st, B.part_c, nb, &S->rr);
            ++k;
            ++j;
            if (j % check_every == 0 || k >= maxit) {
                PERKS_HIP_TRY(hipMemcpyAsync(hs, S, sizeof(BaseScalars), hipMemcpyDeviceToHost, st));
                PERKS_HIP_TRY(hipStreamSynchronize(st));
                const double rnorm = std::sqrt(hs[4]);
                if (hs[7] != 1.0 || (jac && !(hs[6] > 0.0) && rnorm > 0.0)) {
                    broke = true;
                    break;
                }
                rmax = std::max(rmax, rnorm);
                if (rnorm <= PERKS_MIXED_UPDATE_TOL * rmax || rnorm <= tol * bnorm * sc || k >= maxit) break;
            }
            hipLaunchKernelGGL(base_beta, dim3(1), dim3(1), 0, st, S);
        }
        PERKS_HIP_TRY(hipGetLastError());
        ++outer;
    }
    PERKS_HIP_TRY(hipGetLastError());
    fill_result(out, k, status, outer, 0, rn / bnorm, rn / bnorm, 0.0);
    return status;
}

// ---------------------------------------------------------------------------
// Batched solve: many problems in one persistent launch.
//
// Schedule (host, deterministic).  One workgroup streams a slice of A from
// memory far slower than it reads it from its LDS copy, and a problem spread
// over many workgroups pays for every barrier; so each problem gets the
// fewest workgroups whose LDS holds all of its matrix, k_i =
// ceil(nnz_i / (LDS nonzeros per workgroup, less padding)) (at most G, at
// least one row per lane), and the problems, largest predicted work
// (nnz * sqrt(n)) first, are packed first-fit into "phases" of at most G
// workgroups.  Workgroup g runs its phase-0 task, then its phase-1 task, and
// so on: a group's members are all in the same phase, every workgroup takes
// the phases in the same order, so no wait can be circular.  A problem whose
// matrix alone exceeds the whole device's LDS gets all G workgroups, a phase
// of its own.
struct BatchSchedule {
    std::vector<int> task_ptr;   // G + 1
    std::vector<CgTask> tasks;
    std::vector<int> wgs;        // workgroups per problem (0: empty problem)
    int phases = 0;
    int groups = 0;
};

BatchSchedule make_schedule(const std::vector<int64_t> &n, const std::vector<int64_t> &nnz, int G, bool mixed) {
    const int m = (int)n.size();
    BatchSchedule S;
    S.wgs.assign(m, 0);
    const int64_t lds_nnz = (mixed ? CG_LDS_NNZ32 : CG_LDS_NNZ) * 7 / 8;   // room for sliced-ELL padding
    std::vector<double> w(m, 0.0);
    std::vector<int> order;
    for (int i = 0; i < m; ++i) {
        if (n[i] == 0) continue;
        w[i] = (double)std::max<int64_t>(nnz[i], 1) * std::sqrt((double)n[i]);
        int64_t k = (nnz[i] + lds_nnz - 1) / lds_nnz;
        k = std::min<int64_t>(k, std::max<int64_t>(1, n[i] / 64));
        S.wgs[i] = (int)std::max<int64_t>(1, std::min<int64_t>(k, G));
        order.push_back(i);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
    std::vector<std::vector<CgTask>> per(G);
    int used = G, group = 0;   // start a new phase at the first problem
    for (int i : order) {
        const int k = S.wgs[i];
        if (used + k > G) {
            used = 0;
            ++S.phases;
        }
        for (int r = 0; r < k; ++r) per[used + r].push_back(CgTask{i, r, k, k > 1 ? group : 0});
        if (k > 1) ++group;
        used += k;
    }
    S.groups = group;
    S.task_ptr.assign(G + 1, 0);
    for (int g = 0; g < G; ++g) {
        S.task_ptr[g + 1] = S.task_ptr[g] + (int)per[g].size();
        S.tasks.insert(S.tasks.end(), per[g].begin(), per[g].end());
    }
    return S;
}

}  // namespace
}  // namespace perks

using namespace perks;

// Opaque plan of a batched solve: device memory (barrier words, problem table,
// schedule, results, work vectors) and the launch, kept as a one-node HIP
// graph with the cooperative attribute.
struct perks_cg_batch {
    int device = -1;
    int count = 0;
    int G = 0;
    bool mixed = false;
    void *mem = nullptr;
    double *results = nullptr;            // 8 words per problem
    unsigned *ws = nullptr;
    const void *fn = nullptr;
    CgBatch params{};
    std::vector<int> wgs;
    std::vector<double> cached_frac;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t epochs_used = 0;
};

extern "C" {

int perks_cg_batch_create(const perks_csr *As, const void *const *bs, void *const *xs, int32_t count, double tol,
                          int32_t maxit, int32_t precond, int32_t precision, perks_cg_batch **plan) {
    if (!plan) return set_error(PERKS_E_INVAL, "plan must not be NULL");
    *plan = nullptr;
    if (count < 0) return set_error(PERKS_E_INVAL, "count must be >= 0");
    if (count > 0 && (!As || !bs || !xs)) return set_error(PERKS_E_INVAL, "As, bs and xs must not be NULL");
    for (int i = 0; i < count; ++i) {
        int rc = check_csr(&As[i], bs[i], xs[i], tol, maxit, precond, precision);
        if (rc) return set_error(rc, "problem %d: %s", i, last_error());
    }
    if ((int64_t)maxit * 6 + 64LL * PERKS_MIXED_MAX_OUTER > (int64_t(1) << 30))
        return set_error(PERKS_E_INVAL, "maxit too large for a batched solve (barrier epoch range)");
    const bool jac = precond == PERKS_PRECOND_JACOBI, mixed = precision == PERKS_PREC_MIXED;
    auto *P = new (std::nothrow) perks_cg_batch();
    if (!P) return set_error(PERKS_E_NOMEM, "plan allocation failed");
    P->count = count;
    P->mixed = mixed;
    P->fn = batched_fn(jac, mixed);
    int rc = PERKS_OK;
    do {
        if (hipGetDevice(&P->device) != hipSuccess) { rc = set_error(PERKS_E_HIP, "no current HIP device"); break; }
        rc = cg_capacity(P->fn, &P->G);
        if (rc) break;
        std::vector<int64_t> n(count), nnz(count);
        for (int i = 0; i < count; ++i) {
            n[i] = As[i].n;
            nnz[i] = As[i].nnz;
        }
        BatchSchedule S = make_schedule(n, nnz, P->G, mixed);
        P->wgs = S.wgs;
        // device memory: sync words | problems | tasks | task_ptr | results | work areas
        auto up = [](size_t b) { return (b + 255) / 256 * 256; };
        const size_t o_inst = up(SYNC_BYTES);
        const size_t o_tasks = o_inst + up(sizeof(CgInst) * std::max(count, 1));
        const size_t o_ptr = o_tasks + up(sizeof(CgTask) * std::max<size_t>(S.tasks.size(), 1));
        const size_t o_res = o_ptr + up(sizeof(int) * (P->G + 1));
        size_t o_work = o_res + up(sizeof(double) * 8 * std::max(count, 1));
        std::vector<size_t> work_off(count);
        size_t total = o_work;
        for (int i = 0; i < count; ++i) {
            work_off[i] = total;
            if (n[i] > 0) total += inst_bytes(n[i], nnz[i], std::max(S.wgs[i], 1), mixed);
        }
        if (hipMalloc(&P->mem, total) != hipSuccess) {
            (void)hipGetLastError();
            rc = set_error(PERKS_E_NOMEM, "batched solve: hipMalloc of %zu bytes failed", total);
            break;
        }
        char *base = (char *)P->mem;
        std::vector<CgInst> inst(count);
        P->cached_frac.assign(count, 0.0);
        for (int i = 0; i < count; ++i) {
            CgInst &p = inst[i];
            p = CgInst{};
            if (n[i] > 0) carve(base + work_off[i], n[i], nnz[i], std::max(S.wgs[i], 1), mixed, &p);
            p.result = (double *)(base + o_res) + 8 * (size_t)i;
            p.rowptr = As[i].rowptr;
            p.colind = As[i].colind;
            p.spmv = As[i].spmv;
            p.val = (const double *)As[i].val;
            p.b = (const double *)bs[i];
            p.x = (double *)xs[i];
            p.n = (int)n[i];
            p.nnz = (int)nnz[i];
            p.maxit = maxit;
            p.max_outer = PERKS_MIXED_MAX_OUTER;
            p.tol = tol;
            p.update_tol = PERKS_MIXED_UPDATE_TOL;
            const double lds = mixed ? CG_LDS_NNZ32 : CG_LDS_NNZ;
            if (nnz[i] > 0) P->cached_frac[i] = std::min<double>((double)nnz[i], lds * S.wgs[i]) / (double)nnz[i];
        }
        // problems with n = 0 report a converged empty solve
        std::vector<double> res(8 * (size_t)std::max(count, 1), 0.0);
        P->results = (double *)(base + o_res);
        P->ws = (unsigned *)base;
        if (hipMemset(P->mem, 0, SYNC_BYTES) != hipSuccess ||
            hipMemcpy(base + o_inst, inst.data(), sizeof(CgInst) * count, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(base + o_tasks, S.tasks.data(), sizeof(CgTask) * S.tasks.size(), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(base + o_ptr, S.task_ptr.data(), sizeof(int) * (P->G + 1), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(base + o_res, res.data(), sizeof(double) * 8 * count, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            rc = set_error(PERKS_E_HIP, "batched solve: uploading the schedule failed");
            break;
        }
        P->params.inst = (const CgInst *)(base + o_inst);
        P->params.tasks = (const CgTask *)(base + o_tasks);
        P->params.task_ptr = (const int *)(base + o_ptr);
        P->params.ws = P->ws;
        const int64_t span = 6 * (int64_t)maxit + 4 * PERKS_MIXED_MAX_OUTER + 64;
        if (S.groups >= SYNC_MAX_WGS || (S.groups + 2) * span >= (int64_t(1) << 31)) {
            rc = set_error(PERKS_E_UNSUPPORTED, "batch too large for the barrier epoch range (%d groups)", S.groups);
            break;
        }
        P->params.epoch_span = (unsigned)span;
        P->params.ngroups = S.groups;
        // the launch as a graph node with the cooperative attribute (falls back
        // to a direct cooperative launch per run if the runtime refuses it)
        hipKernelNodeParams kp{};
        void *args[] = {&P->params};
        kp.func = const_cast<void *>(P->fn);
        kp.gridDim = dim3(P->G);
        kp.blockDim = dim3(CG_THREADS);
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
        perks_cg_batch_destroy(P);
        return rc;
    }
    *plan = P;
    return PERKS_OK;
}

int perks_cg_batch_run(perks_cg_batch *P, void *stream) {
    if (!P) return set_error(PERKS_E_INVAL, "plan must not be NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != P->device)
        return set_error(PERKS_E_INVAL, "the plan belongs to device %d", P->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (P->count == 0) return PERKS_OK;
    // barrier epochs are 32-bit: start again from zeroed words well before
    // they could wrap (a fill kernel, so the reset is stream-ordered)
    const uint64_t per_run = (uint64_t)(P->params.ngroups + 1) * P->params.epoch_span + 2;
    P->epochs_used += per_run;
    if (P->epochs_used > (uint64_t(1) << 31)) {
        hipLaunchKernelGGL(zero_words, dim3((SYNC_BYTES / 4 + 255) / 256), dim3(256), 0, st, P->ws,
                           (int)(SYNC_BYTES / 4));
        P->epochs_used = per_run;
    }
    note_persistent_launch(P->G, P->ws);
    if (P->exec) {
        PERKS_HIP_TRY(hipGraphLaunch(P->exec, st));
    } else {
        void *args[] = {&P->params};
        hipError_t e = hipLaunchCooperativeKernel(P->fn, dim3(P->G), dim3(CG_THREADS), args, 0, st);
        if (e != hipSuccess) return launch_error(e);
    }
    return PERKS_OK;
}

int perks_cg_batch_results(perks_cg_batch *P, perks_cg_result *outs, void *stream) {
    if (!P) return set_error(PERKS_E_INVAL, "plan must not be NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (P->count == 0) return PERKS_OK;
    std::vector<double> h(8 * (size_t)P->count);
    PERKS_HIP_TRY(hipMemcpyAsync(h.data(), P->results, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    PERKS_HIP_TRY(hipStreamSynchronize(st));
    int worst = PERKS_OK;
    perks_barrier_stats_t bs;
    const int rc = read_barrier_stats(P->G, P->ws, st, &bs);
    if (rc) return rc;
    for (int i = 0; i < P->count; ++i) {
        perks_cg_result r;
        const int s = result_from_words(&h[8 * (size_t)i], P->wgs[i], P->cached_frac[i], &r);
        r.barrier_cycles = (int64_t)bs.wait_cycles;   // the launch's mean over workgroups
        if (outs) outs[i] = r;
        if (s == PERKS_BREAKDOWN || (s == PERKS_NOT_CONVERGED && worst == PERKS_OK)) worst = s;
    }
    return worst;
}

int perks_cg_batch_graph(perks_cg_batch *P, void **graph) {
    if (!P || !graph) return set_error(PERKS_E_INVAL, "plan and graph must not be NULL");
    if (!P->graph) return set_error(PERKS_E_UNSUPPORTED, "the runtime refused a cooperative graph node");
    *graph = (void *)P->graph;
    return PERKS_OK;
}

int perks_cg_batch_destroy(perks_cg_batch *P) {
    if (!P) return PERKS_OK;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->mem) {
        forget_persistent_launch(P->ws);
        (void)hipDeviceSynchronize();
        (void)hipFree(P->mem);
    }
    delete P;
    return PERKS_OK;
}

int perks_cg_solve_batched(const perks_csr *As, const void *const *bs, void *const *xs, int32_t count, double tol,
                           int32_t maxit, int32_t precond, int32_t precision, void *stream, perks_cg_result *outs) {
    perks_cg_batch *P = nullptr;
    int rc = perks_cg_batch_create(As, bs, xs, count, tol, maxit, precond, precision, &P);
    if (rc) return rc;
    rc = perks_cg_batch_run(P, stream);
    if (rc == PERKS_OK) rc = perks_cg_batch_results(P, outs, stream);
    perks_cg_batch_destroy(P);
    return rc;
}

}  // extern "C"

namespace perks {
namespace {
}  // namespace
}  // namespace perks


extern "C" {

int perks_cg_solve(const perks_csr *A, const void *b, void *x, double tol, int32_t maxit, int32_t precond,
                   int32_t precision, void *stream, perks_cg_result *out) {
    int rc = check_csr(A, b, x, tol, maxit, precond, precision);
    if (rc) return rc;
    if (A->n == 0) {
        fill_result(out, 0, PERKS_OK, 0, 0, 0.0, 0.0, 0.0);
        return PERKS_OK;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const bool jac = precond == PERKS_PRECOND_JACOBI;
    return cg_persistent_solve(A, b, x, tol, maxit, jac, precision == PERKS_PREC_MIXED, st, out);
}

int perks_cg_solve_capture(const perks_csr *A, const void *b, void *x, double tol, int32_t maxit, int32_t precond,
                           const int32_t *cap_iters, int32_t ncap, double *cap_x, double *cap_r, void *stream,
                           perks_cg_result *out) {
    int rc = check_csr(A, b, x, tol, maxit, precond, PERKS_PREC_F64);
    if (rc) return rc;
    if (ncap < 0 || (ncap > 0 && (!cap_iters || !cap_x || !cap_r)))
        return set_error(PERKS_E_INVAL, "capture arrays must not be NULL when ncap > 0");
    if (A->n == 0) {
        fill_result(out, 0, PERKS_OK, 0, 0, 0.0, 0.0, 0.0);
        return PERKS_OK;
    }
    Capture c;
    c.iters = cap_iters;
    c.n = ncap;
    c.x = cap_x;
    c.r = cap_r;
    return cg_persistent_solve(A, b, x, tol, maxit, precond == PERKS_PRECOND_JACOBI, false,
                               reinterpret_cast<hipStream_t>(stream), out, c);
}

int perks_cg_solve_baseline(const perks_csr *A, const void *b, void *x, double tol, int32_t maxit, int32_t precond,
                            int32_t precision, int32_t check_every, void *stream, perks_cg_result *out) {
    int rc = check_csr(A, b, x, tol, maxit, precond, precision);
    if (rc) return rc;
    if (check_every < 1) return set_error(PERKS_E_INVAL, "check_every must be >= 1");
    if (A->n == 0) {
        fill_result(out, 0, PERKS_OK, 0, 0, 0.0, 0.0, 0.0);
        return PERKS_OK;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const bool jac = precond == PERKS_PRECOND_JACOBI;
    if (precision == PERKS_PREC_MIXED) return cg_baseline_mixed(A, b, x, tol, maxit, jac, check_every, st, out);
    return cg_baseline_f64(A, b, x, tol, maxit, jac, check_every, st, out);
}

}  // extern "C"
