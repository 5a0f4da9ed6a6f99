/*
 * perks.h -- C ABI of the MI355X (gfx950) PERKS library (libperks.so).
 *
 * PERKS ("PERsistent KernelS", ICS '23) runs an iterative memory-bound solver
 * as one persistent kernel: the time loop moves from the host into the kernel
 * (Sec. 3, fig:exemodel), a device-wide synchronisation replaces each per-step
 * kernel relaunch, and the data that step k produces and step k+1 consumes is
 * kept on chip (registers / LDS) between steps (Sec. 3, "what/where to
 * cache"), so only halo, boundary and spill traffic reaches HBM (Eq. 5).
 *
 * Conventions for every entry point
 *   - Pointers named "device" point to device memory owned by the caller; the
 *     library never frees them.  Pointers named "host" point to host memory.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Stencil calls are
 *     asynchronous on it; CG calls synchronise it before returning (they fill
 *     a host result struct).
 *   - Scratch state (halo buffers, barrier words, the baseline's second
 *     buffer, CG work vectors) is owned by the library, allocated on first use
 *     per device and grown as needed.  Calls that overlap in time on one device
 *     share it and therefore race: issue them on one stream or serialise them.
 *   - Return value: 0 (PERKS_OK) on success, a positive "completed with a
 *     condition" code, or a negative error code.  No C++ exception or abort
 *     crosses this boundary; perks_last_error() gives a detail string for the
 *     last failing call on the calling thread.
 */
#ifndef PERKS_H
#define PERKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PERKS_OK = 0,
    PERKS_NOT_CONVERGED = 1,      /* CG: maxit reached; x holds the last iterate      */
    PERKS_BREAKDOWN = 2,          /* CG: p'Ap <= 0 (A not SPD) or a non-finite value  */
    PERKS_E_INVAL = -1,           /* bad argument (null pointer, shape, dtype, ...)   */
    PERKS_E_NOMEM = -2,           /* scratch allocation failed                        */
    PERKS_E_HIP = -3,             /* a HIP runtime call failed (detail string)        */
    PERKS_E_NOTCORESIDENT = -4,   /* the persistent grid cannot be co-resident        */
    PERKS_E_UNSUPPORTED = -5      /* valid request outside what this build supports   */
};

typedef enum { PERKS_F32 = 0, PERKS_F64 = 1 } perks_dtype;

/* Full extents of a grid INCLUDING its fixed boundary ring.  ndim = 2: the
 * array is [ny][nx]; ndim = 3: [nz][ny][nx]; x is the fastest index.  nz is
 * ignored for ndim = 2. */
typedef struct {
    int32_t ndim;
    int32_t reserved;
    int64_t nx, ny, nz;
} perks_shape;

/* Launch plan knobs; pass NULL (or zero fields) for the library's choice.
 * These are the paper's tuning parameters: thread blocks per SM / occupancy
 * (Sec. 4.1.1, Sec. 5.4), how much of the domain each thread caches, and the
 * cache level (PERKS_SM / PERKS_REG / PERKS_MIX, Sec. 6.2.1). */
typedef struct perks_tuning {
    int32_t waves_per_wg;     /* wavefronts per workgroup (1..16)                      */
    int32_t wgs_per_cu;       /* co-resident workgroups per CU used by the plan        */
    int32_t rows_per_lane;    /* cells each lane keeps in registers along y            */
    int32_t planes_per_lane;  /* 3D: cells each lane keeps along z                     */
    int32_t sync;             /* 0 auto, 1 grid barrier, 2 neighbour flags             */
    int32_t max_cached_tiles; /* <0: none cached (all tiles stream through HBM);
                                 0: as many as fit; >0: at most this many              */
    int32_t reserved[2];
} perks_tuning;

/* Plan a call would use (for reporting and for the performance model). */
typedef struct {
    int32_t wgs;              /* persistent grid size (workgroups)                    */
    int32_t waves_per_wg;
    int32_t rows_per_lane;
    int32_t planes_per_lane;
    int64_t tiles;            /* wave tiles covering the interior                     */
    int64_t cached_tiles;     /* tiles held in registers across steps                 */
    int64_t cached_cells;     /* interior cells held on chip                          */
    int64_t interior_cells;
    int64_t halo_bytes_per_step;  /* face traffic written + read per step             */
    int32_t sync;             /* 1 grid barrier per step, 2 point-to-point halo words */
    int32_t lds_rows_per_lane;/* rows of each cached tile held in LDS (PERKS_MIX)     */
} perks_stencil_plan;

/*
 * perks_stencil_run -- `steps` Jacobi sweeps of an explicit stencil, in place.
 *
 * Computes x^{k+1} = F(x^k) (Sec. 2.2, Eq. 1) with F the weighted box sum of
 * Eq. 2 (2D 5-point) generalised to a radius-1 weight box: every interior cell
 * becomes sum_{o in box} coeffs[o] * x^k[c + o]; the ring of width 1 is a fixed
 * Dirichlet boundary.  Step k+1 reads only step k (Listing 1 keeps separate
 * input and output buffers).
 *   grid    device, [nz][ny][nx] (or [ny][nx]) of float or double per `dt`;
 *           read as the initial state, overwritten with the state after `steps`.
 *   coeffs  host, 3^ndim doubles, [dz][dy][dx] with offsets -1..1 (dx fastest);
 *           Eq. 2's E is offset dx=+1, N is dy=+1.  Zeros mark unused points.
 *           Supported patterns: 2D 5-point star, 2D 9-point box, 3D 7-point
 *           star (others -> PERKS_E_UNSUPPORTED).  FP32 grids use the weights
 *           rounded to float.
 *   steps   >= 0; 0 leaves grid untouched.
 * Every extent must be >= 3.  The whole run is ONE kernel launch.
 */
int perks_stencil_run(void *grid, const double *coeffs, perks_shape shape, int64_t steps,
                      perks_dtype dt, void *stream, const perks_tuning *tune);

/* Same computation, host-looped: one kernel launch per step over ping-pong
 * buffers (the per-step-launch baseline the paper compares against, Sec. 3,
 * fig:exemodel left).  Bitwise identical result to perks_stencil_run. */
int perks_stencil_run_baseline(void *grid, const double *coeffs, perks_shape shape,
                               int64_t steps, perks_dtype dt, void *stream);

/* Fill *plan (host) with the plan perks_stencil_run would use. */
int perks_stencil_plan_query(const double *coeffs, perks_shape shape, perks_dtype dt,
                             const perks_tuning *tune, perks_stencil_plan *plan);

/* Sparse matrix in CSR form (0-based, 32-bit indices, column indices of a row
 * in any order).  rowptr, colind, val are device pointers; val holds float or
 * double per `dt`. */
typedef struct {
    int64_t n, nnz;
    const int32_t *rowptr;
    const int32_t *colind;
    const void *val;
    perks_dtype dt;
    int32_t reserved;
} perks_csr;

typedef struct {
    int32_t iters;            /* CG iterations performed (restarts included)          */
    int32_t status;           /* PERKS_OK / PERKS_NOT_CONVERGED / PERKS_BREAKDOWN     */
    int32_t restarts;         /* restarts after a true-residual check failed          */
    int32_t wgs;              /* persistent grid size used                            */
    double relres;            /* final recursive ||r|| / ||b||                        */
    double relres_true;       /* ||b - A x|| / ||b|| recomputed at exit               */
    double cached_nnz_frac;   /* share of A's nonzeros held on chip                   */
    double reserved;
} perks_cg_result;

enum { PERKS_PRECOND_NONE = 0, PERKS_PRECOND_JACOBI = 1 };

/*
 * perks_cg_solve -- conjugate gradient for SPD A (Sec. 2.2.2, Sec. 4.3).
 *
 * Hestenes-Stiefel CG as in the paper's CG algorithm, with its stopping test
 * read as: iterate while ||r||_2 > tol * ||b||_2 and iterations < maxit.  At
 * exit the true residual is recomputed; if it exceeds tol and iterations
 * remain, CG restarts from the current x.  The whole solve is one persistent
 * kernel launch per (re)start: SpMV, dot products (a fixed-order all-reduce
 * inside the kernel) and AXPYs are fused, the matrix slice of each workgroup is
 * cached on chip, and workgroups synchronise with a device-wide barrier.
 *   A       host struct describing device CSR arrays (FP64 only in this build).
 *   b       device, n doubles.      x  device, n doubles: initial guess in,
 *           solution out.
 *   precond PERKS_PRECOND_NONE or PERKS_PRECOND_JACOBI (z = D^{-1} r).
 *   out     host, filled on return (may be NULL).
 * Returns PERKS_OK, PERKS_NOT_CONVERGED, PERKS_BREAKDOWN or an error.
 */
int perks_cg_solve(const perks_csr *A, const void *b, void *x, double tol, int32_t maxit,
                   int32_t precond, void *stream, perks_cg_result *out);

/* Same solve, host-looped: separate kernels per step (SpMV, dot products,
 * AXPYs) launched every iteration, scalars kept on the device, and the host
 * reading the residual norm back every `check_every` iterations (>= 1) to
 * decide convergence -- the multi-kernel structure the paper fuses (Sec. 3.1,
 * "Practicality of PERKS"). */
int perks_cg_solve_baseline(const perks_csr *A, const void *b, void *x, double tol,
                            int32_t maxit, int32_t precond, int32_t check_every, void *stream,
                            perks_cg_result *out);

/* Device facts the planner uses (host struct, filled from the current device). */
typedef struct {
    int32_t cus;
    int32_t lds_per_cu;
    int32_t regs_per_cu;      /* 32-bit registers per CU                              */
    int32_t l2_bytes;
    int64_t hbm_bytes;
    char arch[64];
} perks_device_info;

int perks_device_query(perks_device_info *info);

/* Message for a return code, and the detail string of the last failing call
 * on this thread (never NULL). */
const char *perks_strerror(int code);
const char *perks_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PERKS_H */
