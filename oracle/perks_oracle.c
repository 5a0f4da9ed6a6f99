/*
 * CPU oracle for the PERKS hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, double-precision reference implementations of what the GPU
 * library computes.  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this file's library.  It shares no code, header or
 * constant with the GPU path and must never be used as a fallback for it.
 *
 * Built with  gcc -O2 -ffp-contract=off  so that every multiply and add is a
 * separately rounded double operation (no fused multiply-add).
 *
 * Paper: "PERKS: a Locality-Optimized Execution Model for Iterative
 * Memory-bound GPU Applications" (ICS '23).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Iterative stencil (Sec. 2.2, Eq. 1 and Eq. 2; Listing 1 keeps an input and
 * an output buffer, i.e. a Jacobi sweep: step k+1 reads only step k).
 *
 * grid   : full extents nz x ny x nx (nz = 1 for 2D), x fastest, updated in
 *          place with the result after `steps` sweeps.
 * w      : dense (2r+1)^ndim weight box, [dz][dy][dx], offsets -r..r; zero
 *          entries are unused points.
 * Cells within distance r of the border form a fixed Dirichlet ring (the
 * paper does not state a boundary condition; this is the reading used).
 * Every interior cell becomes  sum over (dz,dy,dx) ascending of w*in[c+o].
 * threads: host threads sharing each sweep's rows (1 = the plain loop).
 * Returns 0, or -1 on bad arguments / allocation failure.                   */
int oracle_stencil_threads(double *grid, int ndim, int64_t nx, int64_t ny, int64_t nz,
                           const double *w, int r, int64_t steps, int threads)
{
    if (!grid || !w || r < 1 || steps < 0 || (ndim != 2 && ndim != 3) || threads < 1) return -1;
    if (ndim == 2) nz = 1;
    if (nx < 2 * r + 1 || ny < 2 * r + 1 || (ndim == 3 && nz < 2 * r + 1)) return -1;
    const int64_t plane = nx * ny, total = plane * nz;
    const int bw = 2 * r + 1;
    const int nzw = (ndim == 3) ? bw : 1;
    double *a = grid;
    double *b = (double *)malloc((size_t)total * sizeof(double));
    if (!b) return -1;
    memcpy(b, a, (size_t)total * sizeof(double));          /* ring carried over */
    const int64_t z0 = (ndim == 3) ? r : 0, z1 = (ndim == 3) ? nz - r : 1;
    const int64_t rows_per_plane = ny - 2 * r, rows = (z1 - z0) * rows_per_plane;
    for (int64_t t = 0; t < steps; ++t) {
        /* interior rows (z, y) are independent within a sweep: with threads > 1
         * they are shared among threads; every cell's sum is the same. */
#pragma omp parallel for num_threads(threads) schedule(static)
        for (int64_t zy = 0; zy < rows; ++zy) {
            const int64_t z = z0 + zy / rows_per_plane, y = r + zy % rows_per_plane;
            for (int64_t x = r; x < nx - r; ++x) {
                double acc = 0.0;
                for (int dz = 0; dz < nzw; ++dz)
                    for (int dy = 0; dy < bw; ++dy)
                        for (int dx = 0; dx < bw; ++dx) {
                            double wt = w[(dz * bw + dy) * bw + dx];
                            if (wt == 0.0) continue;
                            int64_t zz = (ndim == 3) ? z + dz - r : 0;
                            int64_t idx = zz * plane + (y + dy - r) * nx + (x + dx - r);
                            acc = acc + wt * a[idx];
                        }
                b[z * plane + y * nx + x] = acc;
            }
        }
        double *tmp = a; a = b; b = tmp;
    }
    if (a != grid) {                       /* odd number of sweeps */
        memcpy(grid, a, (size_t)total * sizeof(double));
        free(a);
    } else {
        free(b);
    }
    return 0;
}

int oracle_stencil(double *grid, int ndim, int64_t nx, int64_t ny, int64_t nz,
                   const double *w, int r, int64_t steps)
{
    return oracle_stencil_threads(grid, ndim, nx, ny, nz, w, r, steps, 1);
}

/* ------------------------------------------------------------------------ */
/* Building blocks of conjugate gradient.                                    */

/* Pairwise (recursive halving) summation of x[i]*y[i]: a fixed order. */
static double dot_rec(const double *x, const double *y, int64_t n)
{
    if (n <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s = s + x[i] * y[i];
        return s;
    }
    int64_t h = n / 2;
    return dot_rec(x, y, h) + dot_rec(x + h, y + h, n - h);
}

double oracle_dot(const double *x, const double *y, int64_t n)
{
    return n > 0 ? dot_rec(x, y, n) : 0.0;
}

/* y = A x for CSR A (row pointers and column indices 32-bit). */
void oracle_spmv(int64_t n, const int32_t *rowptr, const int32_t *colind,
                 const double *val, const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) s = s + val[k] * x[colind[k]];
        y[i] = s;
    }
}

/* Conjugate gradient for SPD A (Sec. 2.2.2; the commented algorithm of the
 * paper, Hestenes-Stiefel form), optionally with the Jacobi preconditioner
 * z = D^{-1} r.  The paper prints the stopping test inverted and absolute;
 * the reading used here is: iterate while ||r||_2 > tol * ||b||_2 and
 * k < maxit, on the recursively updated residual.  On leaving the loop the
 * true residual b - A x is formed; if it still exceeds the tolerance and
 * iterations remain, CG restarts from the current x (the restart counts
 * toward maxit).
 *
 * x      : in: initial guess, out: final iterate.
 * out[0] : iterations, out[1] : final recursive relative residual,
 * out[2] : true relative residual ||b-Ax||/||b||, out[3] : restarts.
 * Returns 0 converged, 1 not converged within maxit, 2 breakdown
 * (p'Ap <= 0, or z'r <= 0 with the preconditioner, or non-finite), -1 bad
 * arguments.                                                                  */
int oracle_cg(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
              const double *b, double *x, double tol, int maxit, int precond, double *out)
{
    if (n < 0 || !rowptr || !b || !x || !out || maxit < 0 || !(tol >= 0.0)) return -1;
    out[0] = 0; out[1] = 0; out[2] = 0; out[3] = 0;
    if (n == 0) return 0;
    double *r = malloc((size_t)n * sizeof(double));
    double *z = malloc((size_t)n * sizeof(double));
    double *p = malloc((size_t)n * sizeof(double));
    double *q = malloc((size_t)n * sizeof(double));
    double *dinv = malloc((size_t)n * sizeof(double));
    if (!r || !z || !p || !q || !dinv) { free(r); free(z); free(p); free(q); free(dinv); return -1; }
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) if (colind[k] == i) d = d + val[k];
        dinv[i] = 1.0 / d;
    }
    const double bnorm = sqrt(oracle_dot(b, b, n));
    int status = 1, k = 0, restarts = 0;
    double relrec = 0.0, reltrue = 0.0;
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        status = 0;
        goto done;
    }
    for (;;) {
        /* (re)start: r = b - A x, z = M^{-1} r, p = z */
        oracle_spmv(n, rowptr, colind, val, x, q);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        for (int64_t i = 0; i < n; ++i) z[i] = precond ? dinv[i] * r[i] : r[i];
        for (int64_t i = 0; i < n; ++i) p[i] = z[i];
        double rho = oracle_dot(r, z, n);
        double rnorm = sqrt(oracle_dot(r, r, n));
        relrec = rnorm / bnorm;
        while (k < maxit && rnorm > tol * bnorm) {
            oracle_spmv(n, rowptr, colind, val, p, q);            /* q = A p   */
            double pq = oracle_dot(p, q, n);
            if (!(pq > 0.0) || !isfinite(pq)) { status = 2; goto truth; }
            double alpha = rho / pq;
            for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
            for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
            for (int64_t i = 0; i < n; ++i) z[i] = precond ? dinv[i] * r[i] : r[i];
            double rho_new = oracle_dot(r, z, n);
            rnorm = sqrt(oracle_dot(r, r, n));
            if (precond && !(rho_new > 0.0) && rnorm > 0.0) { status = 2; ++k; goto truth; }
            double beta = rho_new / rho;
            for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
            rho = rho_new;
            ++k;
        }
        relrec = rnorm / bnorm;
    truth:
        oracle_spmv(n, rowptr, colind, val, x, q);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        reltrue = sqrt(oracle_dot(r, r, n)) / bnorm;
        if (status == 2) break;
        if (reltrue <= tol) { status = 0; break; }
        if (k >= maxit) { status = 1; break; }
        ++restarts;
    }
done:
    out[0] = k; out[1] = relrec; out[2] = reltrue; out[3] = restarts;
    free(r); free(z); free(p); free(q); free(dinv);
    return status;
}

/* Dense Cholesky solve A x = b (textbook A = L L^T, forward and back
 * substitution), A row-major n x n.  Used to check CG on tiny SPD systems.
 * Returns 0, or 1 if A is not positive definite.                           */
int oracle_chol_solve(int64_t n, const double *A, const double *b, double *x)
{
    double *L = calloc((size_t)(n * n), sizeof(double));
    double *yv = malloc((size_t)n * sizeof(double));
    if (!L || !yv) { free(L); free(yv); return -1; }
    for (int64_t j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int64_t k = 0; k < j; ++k) s = s - L[j * n + k] * L[j * n + k];
        if (!(s > 0.0)) { free(L); free(yv); return 1; }
        double d = sqrt(s);
        L[j * n + j] = d;
        for (int64_t i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int64_t k = 0; k < j; ++k) t = t - L[i * n + k] * L[j * n + k];
            L[i * n + j] = t / d;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        double t = b[i];
        for (int64_t k = 0; k < i; ++k) t = t - L[i * n + k] * yv[k];
        yv[i] = t / L[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double t = yv[i];
        for (int64_t k = i + 1; k < n; ++k) t = t - L[k * n + i] * x[k];
        x[i] = t / L[i * n + i];
    }
    free(L); free(yv);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Mixed-precision conjugate gradient with FP64 residual replacement.  The
 * paper computes CG in one precision; this is the mixed-precision extension
 * of its CG solver, so every choice below is a reading, not the paper's.
 * One CG recurrence runs in FP32; at chosen points its recursive residual is
 * replaced by the true residual computed in FP64 from an FP64 iterate
 * ("reliable updates": Sleijpen and van der Vorst 1996; van der Vorst and
 * Ye 2000), and the search direction is kept across the replacement, so the
 * Krylov space built so far is not thrown away:
 *
 *   replacement (FP64):  x = x + d / s;  r = b - A x;  stop when
 *                        ||r|| <= tol ||b||;  new scale s' = 2^-floor(log2
 *                        ||r||) (exact, keeps FP32 far from under/overflow);
 *                        r32 = float(s' r), z32 = M r32, d = 0, the
 *                        direction p32 multiplied by s'/s (exact), and
 *                        beta = (r32, z32) / (rho s'^2 / s^2), rho being the
 *                        last (r32, z32) of the recurrence before the
 *                        replacement (rescaled to the new units); the first
 *                        replacement starts the recurrence (p = z, beta 0).
 *   iteration (FP32):    p = z + beta p;  q = A32 p;  alpha = rho / (p, q);
 *                        d += alpha p;  r32 -= alpha q;  z32 = M r32, with
 *                        A32 = float(A), FP32 vectors and arithmetic, and
 *                        dot products, alpha and beta in FP64 (a product of
 *                        two floats is exact in double).
 *   trigger:             a replacement follows the iteration after which
 *                        ||r32|| <= update_tol * (largest ||r32|| since the
 *                        last replacement), or ||r32|| / s <= tol ||b|| (the
 *                        recursion claims convergence), or the iteration
 *                        budget is spent, or the recurrence broke down.
 *   stagnation:          MIXED_STALL replacements in a row whose true
 *                        residual is not below every earlier one end the
 *                        solve as not converged (FP32 cannot resolve the
 *                        system), as does reaching max_outer replacements.
 *
 * The Jacobi preconditioner, when asked for, is z = dinv32 * r in FP32 with
 * dinv32 = float(1 / diag).
 *
 * out[0] : total FP32 iterations, out[1] : last ||r||/||b|| (the true FP64
 * residual), out[2] : same as out[1], out[3] : replacements after the first
 * residual (the FP32 segments run).
 * hist   : if not NULL, hist[j] = ||r_j||/||b|| at the j-th residual
 *          computation, the first one included (max_outer + 1 entries).
 * Returns 0 converged, 1 not converged, 2 breakdown, -1 bad arguments.     */
#define MIXED_STALL 3

/* pairwise FP64 sum of double(x_i) * double(y_i) for float vectors */
static double dot32_rec(const float *x, const float *y, int64_t n)
{
    if (n <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s = s + (double)x[i] * (double)y[i];
        return s;
    }
    int64_t h = n / 2;
    return dot32_rec(x, y, h) + dot32_rec(x + h, y + h, n - h);
}

static double dot32(const float *x, const float *y, int64_t n)
{
    return n > 0 ? dot32_rec(x, y, n) : 0.0;
}

int oracle_cg_mixed(int64_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                    const double *b, double *x, double tol, int maxit, int precond,
                    double update_tol, int max_outer, double *out, double *hist)
{
    if (n < 0 || !rowptr || !b || !x || !out || maxit < 0 || !(tol >= 0.0) ||
        !(update_tol > 0.0) || max_outer < 1) return -1;
    out[0] = 0; out[1] = 0; out[2] = 0; out[3] = 0;
    if (n == 0) return 0;
    const int64_t nnz = rowptr[n];
    float *a32 = malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(float));
    double *r = malloc((size_t)n * sizeof(double));
    double *ax = malloc((size_t)n * sizeof(double));
    float *rr = malloc((size_t)n * sizeof(float));
    float *z = malloc((size_t)n * sizeof(float));
    float *p = malloc((size_t)n * sizeof(float));
    float *q = malloc((size_t)n * sizeof(float));
    float *d = malloc((size_t)n * sizeof(float));
    float *dinv = malloc((size_t)n * sizeof(float));
    int status = 1, k = 0, outer = 0, stall = 0, broke = 0;
    double rel = 0.0;
    if (!a32 || !r || !ax || !rr || !z || !p || !q || !d || !dinv) { status = -1; goto done; }
    for (int64_t e = 0; e < nnz; ++e) a32[e] = (float)val[e];
    for (int64_t i = 0; i < n; ++i) {
        double dd = 0.0;
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) if (colind[e] == i) dd = dd + val[e];
        dinv[i] = (float)(1.0 / dd);
        d[i] = 0.0f;
        p[i] = 0.0f;
    }
    const double bnorm = sqrt(oracle_dot(b, b, n));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        status = 0;
        goto done;
    }
    double s = 1.0, rho = 0.0, best = INFINITY;
    for (;;) {
        /* replacement: fold the FP32 correction into x, true residual in FP64 */
        for (int64_t i = 0; i < n; ++i) x[i] = x[i] + (double)d[i] / s;
        oracle_spmv(n, rowptr, colind, val, x, ax);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - ax[i];
        const double rn = sqrt(oracle_dot(r, r, n));
        rel = rn / bnorm;
        if (hist) hist[outer] = rel;
        if (rn <= tol * bnorm) { status = 0; break; }
        if (broke) { status = 2; break; }
        if (rn < best) { best = rn; stall = 0; }
        else if (++stall >= MIXED_STALL) { status = 1; break; }
        if (k >= maxit || outer >= max_outer) { status = 1; break; }
        /* restart the recurrence's residual from r, keep its direction */
        const double s_new = ldexp(1.0, -ilogb(rn));
        const double ratio = outer == 0 ? 1.0 : s_new / s;   /* first: p is 0 */
        for (int64_t i = 0; i < n; ++i) {
            rr[i] = (float)(r[i] * s_new);
            z[i] = precond ? dinv[i] * rr[i] : rr[i];
            d[i] = 0.0f;
            p[i] = p[i] * (float)ratio;
        }
        const double rho_r = dot32(rr, z, n);
        double beta = outer == 0 ? 0.0 : rho_r / (rho * ratio * ratio);
        rho = rho_r;
        s = s_new;
        double rmax = sqrt(dot32(rr, rr, n));
        /* FP32 iterations until the next replacement */
        for (;;) {
            const float bf = (float)beta;
            for (int64_t i = 0; i < n; ++i) p[i] = z[i] + bf * p[i];
            for (int64_t i = 0; i < n; ++i) {
                float t = 0.0f;
                for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) t = t + a32[e] * p[colind[e]];
                q[i] = t;
            }
            const double pq = dot32(p, q, n);
            if (!(pq > 0.0) || !isfinite(pq)) { broke = 1; break; }
            const float af = (float)(rho / pq);
            for (int64_t i = 0; i < n; ++i) {
                d[i] = d[i] + af * p[i];
                rr[i] = rr[i] - af * q[i];
                z[i] = precond ? dinv[i] * rr[i] : rr[i];
            }
            const double rho_new = dot32(rr, z, n);
            const double rnorm = sqrt(dot32(rr, rr, n));
            ++k;
            if (precond && !(rho_new > 0.0) && rnorm > 0.0) { broke = 1; break; }
            if (rnorm > rmax) rmax = rnorm;
            if (rnorm <= update_tol * rmax || rnorm <= tol * bnorm * s || k >= maxit) break;
            beta = rho_new / rho;
            rho = rho_new;
        }
        ++outer;
    }
done:
    out[0] = k; out[1] = rel; out[2] = rel; out[3] = outer;
    free(a32); free(r); free(ax); free(rr); free(z); free(p); free(q); free(d); free(dinv);
    return status;
}
