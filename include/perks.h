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
    PERKS_E_UNSUPPORTED = -5      /* valid request outside what the library supports  */
};

typedef enum { PERKS_F32 = 0, PERKS_F64 = 1 } perks_dtype;

/* Full extents of a grid INCLUDING its fixed boundary ring.  ndim = 2: the
 * array is [ny][nx]; ndim = 3: [nz][ny][nx]; x is the fastest index.  nz is
 * ignored for ndim = 2.  radius: the stencil's radius r (0 is read as 1);
 * the weight box has (2r+1)^ndim entries and the ring is r cells wide. */
typedef struct {
    int32_t ndim;
    int32_t radius;
    int64_t nx, ny, nz;
} perks_shape;

/* Launch plan knobs; pass NULL (or zero fields) for the library's choice.
 * These are the paper's tuning parameters: thread blocks per SM / occupancy
 * (Sec. 4.1.1, Sec. 5.4), how much of the domain each thread caches, and the
 * cache level (PERKS_SM / PERKS_REG / PERKS_MIX, Sec. 6.2.1). */
typedef struct perks_tuning {
    int32_t waves_per_wg;     /* wavefronts per workgroup (1..16)                      */
    int32_t wgs_per_cu;       /* co-resident workgroups per CU used by the plan        */
    int32_t rows_per_lane;    /* cells each lane keeps in registers along y (3D: 4;
                                 radius-2..4 kernels: 24, 32, 48 or 80)                */
    int32_t planes_per_lane;  /* 3D: column depth, planes per column (1..32; 0 auto)   */
    int32_t sync;             /* 0 auto, 1 grid barrier, 2 neighbour flags             */
    int32_t max_cached_tiles; /* <0: none cached (all tiles stream through HBM);
                                 0: as many as fit; >0: at most this many (3D: columns
                                 whose top planes stay in registers)                   */
    int32_t kernel;           /* 2D radius 1: 0 the library's choice, 1 the radius-1
                                 kernel (LDS rows, point-to-point halos), 2 the
                                 radius-2..4 kernel run at radius 1 (grid barrier,
                                 24/32/48/80 register rows), 3 the temporally blocked
                                 kernel (tiles of 64 - 2K columns x rows_per_lane (8,
                                 16, 32 or 56) rows, each wave taking K steps on its
                                 tile and a K-wide ghost ring in registers between
                                 grid barriers; K = steps_per_sync).  When every tile
                                 has a wave of its own the blocks stay in registers
                                 for the whole run and each exchange moves only the
                                 K-wide bands (32 and 56 rows exist only so);
                                 otherwise (or with max_cached_tiles < 0) each block
                                 is loaded from and stored to the grid's two buffers.
                                 With every field of the struct zero (or tune NULL)
                                 the library takes kernel 3 when the interior holds
                                 < 2^20 cells, or when its default plan (K = 4, 56
                                 rows) keeps every tile in registers, else kernel 2
                                 when it caches every tile, else kernel 1; any other
                                 nonzero field selects kernel 1 unless kernel = 2
                                 or 3.                                                */
    int32_t steps_per_sync;   /* kernel 3: K, steps between exchanges (2, 4 or 8; 0
                                 means 8 below 2^20 interior cells, else 4); its
                                 rows_per_lane 0 means 8 (up to 2^18 cells), 16
                                 (below 2^20) or 56                                   */
} perks_tuning;

/* Plan a call would use (for reporting and for the performance model). */
typedef struct {
    int32_t wgs;              /* persistent grid size (workgroups)                    */
    int32_t waves_per_wg;
    int32_t rows_per_lane;
    int32_t planes_per_lane;
    int64_t tiles;            /* wave tiles covering the interior (3D: columns)       */
    int64_t cached_tiles;     /* tiles (3D: columns) with cells held in registers     */
    int64_t cached_cells;     /* interior cells held on chip                          */
    int64_t interior_cells;
    int64_t halo_bytes_per_step;  /* face traffic written + read per step             */
    int32_t sync;             /* 1 grid barrier per step, 2 point-to-point halo words,
                                 3 a grid barrier every steps_per_sync steps (kernel
                                 3; halo_bytes_per_step then counts the tiles' block
                                 reads and writes per step)                           */
    int32_t lds_rows_per_lane;/* rows of each cached tile held in LDS (PERKS_MIX)     */
} perks_stencil_plan;

/*
 * perks_stencil_run -- `steps` Jacobi sweeps of an explicit stencil, in place.
 *
 * Computes x^{k+1} = F(x^k) (Sec. 2.2, Eq. 1) with F the weighted box sum of
 * Eq. 2 (2D 5-point) generalised to a radius-r weight box: every interior cell
 * becomes sum_{o in box} coeffs[o] * x^k[c + o]; the ring of width r is a fixed
 * Dirichlet boundary.  Step k+1 reads only step k (Listing 1 keeps separate
 * input and output buffers).
 *   grid    device, [nz][ny][nx] (or [ny][nx]) of float or double per `dt`;
 *           read as the initial state, overwritten with the state after `steps`.
 *   shape   extents and radius r = max(1, shape.radius).
 *   coeffs  host, (2r+1)^ndim doubles, [dz][dy][dx] with offsets -r..r (dx
 *           fastest); Eq. 2's E is offset dx=+1, N is dy=+1.  Zeros mark
 *           unused points.  Supported patterns (tab:domain): r = 1: the 2D
 *           5-point star, the 2D 9-point box, the 3D 7-point star; 2D r = 2,
 *           3, 4: the stars (2ds9pt, 2d13pt, 2d17pt: no weight off both
 *           axes) and r = 2: the 5x5 box (2d25pt); 3D r = 2: the star
 *           (3d13pt), which runs persistent but streams the grid through HBM
 *           every step (no on-chip cache; plan.cached_tiles = 0).  Others,
 *           including the 3D radius-1 patterns beyond the 7-point star
 *           (3d27pt, poisson, 3d17pt: their kernel is disabled), ->
 *           PERKS_E_UNSUPPORTED.  FP32 grids use the weights rounded to float.
 *   steps   >= 0; 0 leaves grid untouched.
 * Every extent must be >= 2r+1.  The whole run is ONE kernel launch.
 */
int perks_stencil_run(void *grid, const double *coeffs, perks_shape shape, int64_t steps,
                      perks_dtype dt, void *stream, const perks_tuning *tune);

/*
 * perks_stencil_run_noalloc -- perks_stencil_run for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The persistent radius-1 2D kernel
 * (2d5pt or 2d9pt weights, any radius-1 2D pattern; the plan perks_stencil_run
 * takes with tuning.kernel = 1: register and LDS rows, point-to-point halo
 * words) runs with its barrier words and halo buffers in a fixed library
 * array of 32 MiB per device (held until the process ends) instead of
 * library-allocated scratch; the call makes no hipMalloc / hipFree.
 *   Arguments as for perks_stencil_run (no tuning).
 *   The first call on a device looks the array up and clears it (a fill
 *   kernel on `stream`); later calls continue from the epochs it holds.
 *   Calls that overlap in time on one device share the array and race.
 * Returns PERKS_OK, PERKS_E_UNSUPPORTED for other patterns, 3D grids or a
 * grid whose halo buffers do not fit the array (e.g. FP64 beyond about
 * 3500 x 3500), or another error as perks_stencil_run. */
int perks_stencil_run_noalloc(void *grid, const double *coeffs, perks_shape shape, int64_t steps, perks_dtype dt,
                              void *stream);

/* Same computation, host-looped: one kernel launch per step over ping-pong
 * buffers (the per-step-launch baseline the paper compares against, Sec. 3,
 * fig:exemodel left).  Bitwise identical result to perks_stencil_run. */
int perks_stencil_run_baseline(void *grid, const double *coeffs, perks_shape shape,
                               int64_t steps, perks_dtype dt, void *stream);

/* Fill *plan (host) with the plan perks_stencil_run would use. */
int perks_stencil_plan_query(const double *coeffs, perks_shape shape, perks_dtype dt,
                             const perks_tuning *tune, perks_stencil_plan *plan);

/*
 * perks_stencil_run_batched -- `steps` Jacobi sweeps of every grid in ONE
 * persistent launch (an extension: the paper runs one grid per launch).
 *   grids   host array of `count` device pointers, each updated in place.
 *   shapes  host array of `count` extents (2D, radius 1 only; sizes may differ).
 *   coeffs  one weight box for all grids (as for perks_stencil_run).
 * The tiles of all grids (48 columns x 16 rows) share the launch's waves;
 * each wave takes 8 steps of a tile and its 8-wide ghost ring in registers
 * between device-wide barriers (the temporal blocking of perks_tuning.kernel
 * 3), each grid ping-ponging between itself and a second buffer from the
 * library's scratch.  Results are bitwise those of perks_stencil_run (and of
 * the per-step baseline) on each grid.  Synchronises `stream` before it
 * uploads the grid table (host memory is not retained).
 */
int perks_stencil_run_batched(void *const *grids, const perks_shape *shapes, int32_t count,
                              const double *coeffs, int64_t steps, perks_dtype dt, void *stream);

/*
 * Batched stencils as a reusable plan, launched without host synchronisation
 * (an extension, as perks_stencil_run_batched):
 * perks_stencil_batch_create   validates, allocates (device memory owned by
 *                              the plan: barrier words, grid table, second
 *                              buffers; synchronous) and builds the launch.
 *                              grids[i] (count device pointers) stay bound to
 *                              the plan: refill them between runs (ring
 *                              included), do not free them before destroy.
 * perks_stencil_batch_run      enqueues `steps` sweeps of every grid on
 *                              `stream`: one kernel launch (a one-node HIP
 *                              graph with the cooperative attribute when the
 *                              runtime accepts it); nothing else runs on the
 *                              host or the stream, so the call may be made
 *                              during stream capture.  Results as for
 *                              perks_stencil_run_batched.
 * perks_stencil_batch_graph    the plan's hipGraph_t (as void *), for use as a
 *                              child graph; PERKS_E_UNSUPPORTED without one.
 *                              Owned by the plan.
 * perks_stencil_batch_destroy  synchronises the device and frees the plan.
 * Runs of one plan must not overlap in time (they share its barrier words).
 */
typedef struct perks_stencil_batch perks_stencil_batch;

int perks_stencil_batch_create(void *const *grids, const perks_shape *shapes, int32_t count,
                               const double *coeffs, int64_t steps, perks_dtype dt,
                               perks_stencil_batch **plan);
int perks_stencil_batch_run(perks_stencil_batch *plan, void *stream);
int perks_stencil_batch_graph(perks_stencil_batch *plan, void **graph);
int perks_stencil_batch_destroy(perks_stencil_batch *plan);

/*
 * The tunings perks_stencil_autotune remembers (per pattern, dtype and
 * extents, per device) as a text file, so that a later process can use them
 * without measuring again (an extension: the paper tunes per run).
 * perks_tuning_save  writes the current device's entries to `path`.
 * perks_tuning_load  reads `path` and adds its entries to the current
 *                    device's table (replacing entries of the same key);
 *                    PERKS_E_INVAL, and nothing loaded, for a file that is not
 *                    a tuning file of this library.
 */
int perks_tuning_save(const char *path);
int perks_tuning_load(const char *path);

/*
 * perks_stencil_autotune -- pick the launch plan by measurement.
 *
 * Times `probe_steps` sweeps of each candidate plan (the planner's own choice
 * and every register tile depth, in each synchronisation mode; for 3D every
 * tile depth in z) on a scratch grid of the given extents (allocated and freed
 * here; synchronises `stream`), and returns the fastest as *best (host) with
 * its rate in interior cells per ns as *best_gcells (may be NULL).  With
 * remember != 0, later perks_stencil_run calls on this device for the same
 * pattern, dtype and extents that pass tune == NULL use it.  The paper tunes
 * thread blocks per SM and the cache split by hand (Sec. 5.4); this automates
 * that choice.
 */
int perks_stencil_autotune(const double *coeffs, perks_shape shape, perks_dtype dt, int64_t probe_steps,
                           int32_t remember, void *stream, perks_tuning *best, double *best_gcells);

/* Sparse matrix in CSR form (0-based, 32-bit indices, column indices of a row
 * in any order).  rowptr, colind, val are device pointers; val holds float or
 * double per `dt`.
 * spmv selects the SpMV layout of the persistent solvers (the per-matrix
 * choice of what to keep on chip, Sec. 4.3.2):
 *   0  the library's choice: sliced ELL when each 64-row chunk's padding to
 *      its longest row costs at most a quarter more entries, then the solver
 *      with each workgroup's r, p, q in registers (when its rows fit) and the
 *      first part of its slice of A in LDS; irregular rows: sliced ELL over
 *      the rows sorted by length, else CSR; A's slice prefix in LDS;
 *   1  the same without the register-resident solver;
 *   2  merge-path SpMV (Merrill and Garland's merge-based CSR SpMV, the one
 *      the paper's CG uses, Sec. 4.3.1): each workgroup's rows and nonzeros
 *      split into chunks of 8 path items, the chunk starts searched once and
 *      kept, A's slice prefix in LDS. */
typedef struct {
    int64_t n, nnz;
    const int32_t *rowptr;
    const int32_t *colind;
    const void *val;
    perks_dtype dt;
    int32_t spmv;
} perks_csr;

typedef struct {
    int32_t iters;            /* CG iterations performed (restarts included)          */
    int32_t status;           /* PERKS_OK / PERKS_NOT_CONVERGED / PERKS_BREAKDOWN     */
    int32_t restarts;         /* restarts after a true-residual check failed          */
    int32_t wgs;              /* persistent grid size used                            */
    double relres;            /* final recursive ||r|| / ||b||                        */
    double relres_true;       /* ||b - A x|| / ||b|| recomputed at exit               */
    double cached_nnz_frac;   /* share of A's nonzeros held on chip                   */
    int32_t fallbacks;        /* flexible CG: iterations whose network step was
                                 replaced by the Jacobi step (0 for plain CG)         */
    int32_t switched_at;      /* flexible CG: iteration at which the solve continued
                                 as Jacobi-PCG after the network stalled (-1: never;
                                 -1 for plain CG)                                     */
    int64_t barrier_cycles;   /* mean over the persistent grid's workgroups of the
                                 shader-clock cycles spent inside device barriers
                                 during the solve's last persistent launch (entry to
                                 release; s_memtime); 0 for the host-looped baseline */
} perks_cg_result;

enum { PERKS_PRECOND_NONE = 0, PERKS_PRECOND_JACOBI = 1 };

/* Arithmetic of a CG solve.
 *   PERKS_PREC_F64    FP64 throughout.
 *   PERKS_PREC_MIXED  one CG recurrence in FP32 (FP32 copy of A's values, FP32
 *                     vectors, SpMV and AXPYs; FP64 dot products, alpha and
 *                     beta) whose recursive residual is replaced, from time
 *                     to time, by the true residual r = b - A x computed in
 *                     FP64 from an FP64 iterate x (residual replacement, the
 *                     "reliable updates" of Sleijpen and van der Vorst).  A
 *                     replacement follows the iteration after which the FP32
 *                     residual has fallen to PERKS_MIXED_UPDATE_TOL times its
 *                     largest value since the last one, or claims
 *                     convergence, or the budget is spent; it adds the FP32
 *                     correction d to x, forms r, stops if ||r|| <= tol ||b||,
 *                     and restarts the recurrence's residual from float(s r)
 *                     (s an exact power of two near 1/||r||) while keeping
 *                     its search direction (rescaled by the same power of
 *                     two), so the Krylov space is not discarded.
 *                     PERKS_MIXED_STALL replacements in a row without a new
 *                     smallest ||r||, or PERKS_MIXED_MAX_OUTER replacements,
 *                     end the solve as PERKS_NOT_CONVERGED.  The paper's CG
 *                     runs in one precision; this mode is an extension. */
enum { PERKS_PREC_F64 = 0, PERKS_PREC_MIXED = 1 };
#define PERKS_MIXED_UPDATE_TOL 0.3
#define PERKS_MIXED_MAX_OUTER 100
#define PERKS_MIXED_STALL 3

/*
 * perks_cg_solve -- conjugate gradient for SPD A (Sec. 2.2.2, Sec. 4.3).
 *
 * Hestenes-Stiefel CG as in the paper's CG algorithm, with its stopping test
 * read as: iterate while ||r||_2 > tol * ||b||_2 and iterations < maxit.
 * PERKS_PREC_F64: at exit the true residual is recomputed; if it exceeds tol
 * and iterations remain, CG restarts from the current x.  The whole solve is
 * one persistent kernel launch per (re)start: SpMV, dot products (a
 * fixed-order all-reduce inside the kernel) and AXPYs are fused, the first
 * part of each workgroup's slice of the matrix is cached in LDS, and
 * workgroups synchronise with a device-wide barrier.
 * PERKS_PREC_MIXED: the replacement scheme above, every FP32 iteration and
 * every FP64 replacement in ONE persistent launch; the stopping test is on
 * the true FP64 residual.
 *   A         host struct describing device CSR arrays (values FP64).
 *   b         device, n doubles.      x  device, n doubles: initial guess in,
 *             solution out.
 *   maxit     CG iterations allowed (mixed: FP32 iterations).
 *   precond   PERKS_PRECOND_NONE or PERKS_PRECOND_JACOBI (z = D^{-1} r).
 *   precision PERKS_PREC_F64 or PERKS_PREC_MIXED.
 *   out       host, filled on return (may be NULL); `restarts` counts
 *             restarts (F64) or residual replacements after the first
 *             residual (MIXED).
 * Returns PERKS_OK, PERKS_NOT_CONVERGED, PERKS_BREAKDOWN or an error.
 */
int perks_cg_solve(const perks_csr *A, const void *b, void *x, double tol, int32_t maxit,
                   int32_t precond, int32_t precision, void *stream, perks_cg_result *out);

/* perks_cg_solve (FP64) that also records the iterate and its recursive
 * residual after each iteration count listed in cap_iters (device, ncap
 * ascending int32): cap_x[j][n] and cap_r[j][n] (device doubles) receive
 * x_k and r_k for k = cap_iters[j]; entries not reached are left untouched.
 * Used to harvest (residual, error) training pairs from the solver itself. */
int perks_cg_solve_capture(const perks_csr *A, const void *b, void *x, double tol, int32_t maxit,
                           int32_t precond, const int32_t *cap_iters, int32_t ncap, double *cap_x,
                           double *cap_r, void *stream, perks_cg_result *out);

/* Same solve, host-looped: separate kernels per step (SpMV, dot products,
 * AXPYs) launched every iteration, scalars kept on the device, and the host
 * reading the residual norm back every `check_every` iterations (>= 1) to
 * decide convergence -- the multi-kernel structure the paper fuses (Sec. 3.1,
 * "Practicality of PERKS").  MIXED: the host also decides every residual
 * replacement (the trigger test then runs every check_every iterations). */
int perks_cg_solve_baseline(const perks_csr *A, const void *b, void *x, double tol,
                            int32_t maxit, int32_t precond, int32_t precision,
                            int32_t check_every, void *stream, perks_cg_result *out);

/*
 * Batched CG -- many independent SPD systems in ONE persistent launch.
 *
 * The paper solves one system per launch; batching is an extension of its
 * CG.  Every problem is solved exactly as perks_cg_solve would solve it with
 * the same arithmetic (`precision`, `precond`, tol, maxit apply to each
 * problem), by a group of workgroups of the one launch: a problem predicted
 * to cost more than two workgroups' fair share (predicted work: nnz * sqrt(n))
 * gets a group of its own, synchronised by the group's own barrier; the
 * other problems are solved by one workgroup each, packed onto the
 * least-loaded workgroups.  A problem's result depends only on the problem
 * and the size of its group, not on the other problems or their order.
 *
 * perks_cg_batch_create  validates, schedules and allocates (device memory
 *                        owned by the plan; synchronous).  As[i], bs[i],
 *                        xs[i] (count of each, host arrays of device
 *                        pointers) stay bound to the plan: refill b or x
 *                        between runs, do not free them before destroy.
 * perks_cg_batch_run     enqueues the solve on `stream`: one kernel launch
 *                        (a one-node HIP graph with the cooperative
 *                        attribute when the runtime accepts one); no host
 *                        synchronisation; x holds the solutions when the
 *                        stream reaches that point.
 * perks_cg_batch_results synchronises `stream` and fills outs[count] (host;
 *                        may be NULL); returns PERKS_BREAKDOWN if any problem
 *                        broke down, else PERKS_NOT_CONVERGED if any did not
 *                        converge, else PERKS_OK.
 * perks_cg_batch_graph   the plan's hipGraph_t (as void *) for use as a child
 *                        graph in a caller's graph; PERKS_E_UNSUPPORTED when
 *                        the plan has none.  Owned by the plan.
 * perks_cg_batch_destroy synchronises the device and frees the plan.
 * perks_cg_solve_batched create + run + results + destroy.
 * Runs of one plan must not overlap in time (they share its barrier words).
 */
typedef struct perks_cg_batch perks_cg_batch;

int perks_cg_batch_create(const perks_csr *As, const void *const *bs, void *const *xs, int32_t count,
                          double tol, int32_t maxit, int32_t precond, int32_t precision,
                          perks_cg_batch **plan);
int perks_cg_batch_run(perks_cg_batch *plan, void *stream);
int perks_cg_batch_results(perks_cg_batch *plan, perks_cg_result *outs, void *stream);
int perks_cg_batch_graph(perks_cg_batch *plan, void **graph);
int perks_cg_batch_destroy(perks_cg_batch *plan);
int perks_cg_solve_batched(const perks_csr *As, const void *const *bs, void *const *xs, int32_t count,
                           double tol, int32_t maxit, int32_t precond, int32_t precision, void *stream,
                           perks_cg_result *outs);

/*
 * Learned preconditioner (an extension; the paper has no learned part).
 *
 * A six-layer 3x3 convolutional network, run in BF16 on the matrix cores
 * with FP32 accumulation: input channels [r / rms(r), log k] on the N x N
 * grid of unknowns, layers 2 -> 16 -> 16 -> 16 -> 16 -> 16 -> 1, zero 'same'
 * padding, a bias per layer, ReLU after every layer but the last.  Weight
 * W[o][i][1+dy][1+dx] multiplies input channel i at (y+dy, x+dx) for output
 * channel o at (y, x).  Every layer's input and weights are rounded to BF16.
 *
 * params: PERKS_NN_PARAMS floats (device), layer l at l * PERKS_NN_LAYER_PARAMS:
 *         W[16][16][3][3] then b[16], channels beyond a layer's real count
 *         (2 inputs of layer 0, 1 output of layer 5) held at zero.
 * x:      [B][H][W][2] floats (device): the two input channels per pixel.
 */
#define PERKS_NN_LAYERS 6
#define PERKS_NN_LAYER_PARAMS (16 * 16 * 9 + 16)
#define PERKS_NN_PARAMS (PERKS_NN_LAYERS * PERKS_NN_LAYER_PARAMS)

/* out[B][H][W] (device floats) = the network applied to x. */
int perks_nn_forward(const float *params, const float *x, int32_t B, int32_t H, int32_t W, float *out,
                     void *stream);

/* Mean squared error over all B*H*W outputs against target[B][H][W]
 * (device floats) and its gradient w.r.t. params: grad (device,
 * PERKS_NN_PARAMS floats, padded entries zero), *loss (host; may be NULL:
 * then the call does not synchronise).  Requires H even and W <= 512. */
int perks_nn_loss_grad(const float *params, const float *x, const float *target, int32_t B, int32_t H,
                       int32_t W, float *grad, double *loss, void *stream);

/* Energy-norm loss instead of the MSE: with r = x[..][0] (the scaled
 * residual input) and A the 5-point operator of each sample given per pixel
 * as five planes (device floats [B][5][H][W]: weights of (y-1), (x-1),
 * centre, (x+1), (y+1), zero for neighbours outside the grid), the loss is
 * sum (z'Az - 2 z'r) / (B*H*W) over the samples' vectors z: the A-norm error
 * ||z - e||_A^2 of z up to the constant e'r, for r = A e.  z is the network
 * output (jacobi = 0) or the output plus the Jacobi step r / centre
 * (jacobi = 1: the form perks_fcg_solve applies).  Same requirements and
 * outputs as perks_nn_loss_grad. */
int perks_nn_energy_grad(const float *params, const float *x, const float *planes, int32_t jacobi, int32_t B,
                         int32_t H, int32_t W, float *grad, double *loss, void *stream);

/* One Adam step with bias correction (step counts from 1) on the FP32
 * master weights; m and v (device, PERKS_NN_PARAMS floats) start at zero. */
int perks_nn_adam(float *params, const float *grad, float *m, float *v, int32_t step, float lr,
                  float beta1, float beta2, float eps, void *stream);

/* Training of the network on P samples, every pass on the device: `epochs`
 * passes over the samples in a fresh seeded order each (splitmix64 from
 * `seed`, Fisher-Yates shuffle), mini-batches of `batch` samples (the last
 * P % batch of an order are skipped), each one forward + backward pass and
 * one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, rate lr).
 *   params  device, PERKS_NN_PARAMS floats: the initial weights in, the
 *           trained ones out; m, v: device Adam moments (zero to start afresh)
 *   x       device [P][H][W][2] network inputs
 *   target  device [P][H][W] targets of the MSE loss, or NULL for the energy
 *           loss of perks_nn_energy_grad in its Jacobi form with
 *   planes  device [F][5][H][W] operators and field (device int32 [P]) the
 *           operator of each sample
 *   step    host in/out: Adam steps taken so far (0 to start)
 *   losses  host, `epochs` doubles (mean batch loss of each epoch) or NULL
 * Requires batch <= P, H even and W <= 512.  Synchronises the stream. */
int perks_nn_train(float *params, const float *x, const float *target, const float *planes, const int32_t *field,
                   int32_t P, int32_t H, int32_t W, int32_t epochs, int32_t batch, float lr, uint64_t seed,
                   float *m, float *v, int32_t *step, double *losses, void *stream);

/* perks_nn_make_pairs -- training pairs of the network from iterates that
 * perks_cg_solve_capture recorded (Jacobi-PCG on the problem A x = f).  For
 * capture j with iterate x_j and recursive residual r_j, rms_j =
 * sqrt(||r_j||^2 / n) (summed in a fixed order) and, at grid point i (row i
 * of A, pixel i of the H x W grid, row-major):
 *   inputs[j][i]  = { r_j[i] / rms_j, logk[i] }
 *   targets[j][i] = (xstar[i] - x_j[i] - r_j[i] / A_ii) / rms_j
 * computed in FP64 and rounded to FP32: the part of the error e_j = x* - x_j
 * that the Jacobi step D^-1 r_j leaves, which the network adds to that step
 * inside perks_fcg_solve.
 *   A         FP64 CSR (device arrays), n = H * W rows, diagonal present.
 *   xstar, logk          device, n doubles (converged solution; log k).
 *   cap_x, cap_r         device, ncap x n doubles (0 <= ncap <= 4096).
 *   inputs    device, ncap x n x 2 floats; targets device, ncap x n floats:
 *             written for j < *count.
 *   count     host, out: the number of leading captures that form pairs
 *             (the first capture whose residual has a non-finite entry or
 *             rms 0, i.e. one the solve did not reach, ends the list).
 * Synchronises `stream` (the count is read back). */
int perks_nn_make_pairs(const perks_csr *A, const double *xstar, const double *logk, const double *cap_x,
                        const double *cap_r, int32_t ncap, int32_t H, int32_t W, float *inputs, float *targets,
                        int32_t *count, void *stream);

/*
 * perks_fcg_solve -- flexible CG preconditioned by the network, one
 * persistent launch.  FCG(1): p = z - (<z, q_old> / <p_old, q_old>) p_old,
 * q = A p, alpha = <p, r> / <p, q>, with
 * z = D^{-1} r + rms(r) * net([r / rms(r), log k]) -- the network corrects
 * the Jacobi step, so a zero network is Jacobi-PCG -- computed inside the
 * kernel (16 x 16 tiles, all six layers per tile in LDS).
 * Safeguards: z = D^{-1} r for an iteration where <z, r> <= 0 or z is not
 * finite; after `stall` iterations without a new minimum of ||r|| the kernel
 * ends and the solve continues from the current iterate as
 * perks_cg_solve(..., PERKS_PRECOND_JACOBI, PERKS_PREC_F64, ...) with the
 * remaining iterations (a restart of the direction recurrence, which FCG with
 * a fixed Jacobi step would take too).  nn_params == NULL: Jacobi-PCG inside
 * the FCG kernel from the start.
 *   A       FP64 CSR on an H x W grid of unknowns (row y * W + x), n = H * W.
 *   logk    device, H * W doubles (the second network input).
 *   out     iters, status, fallbacks (iterations that took the Jacobi step),
 *           switched_at (iteration at which the solve continued as Jacobi-PCG,
 *           -1: never), relres / relres_true as for perks_cg_solve,
 *           barrier_cycles of the FCG launch; restarts = 0.
 * Returns PERKS_OK when the true relative residual meets tol.
 */
int perks_fcg_solve(const perks_csr *A, const void *b, void *x, double tol, int32_t maxit,
                    const float *nn_params, const double *logk, int32_t H, int32_t W, int32_t stall,
                    void *stream, perks_cg_result *out);

/* perks_fcg_precondition -- the preconditioner of perks_fcg_solve applied
 * once, by the same tile routine the FCG kernel runs in every iteration:
 * z = dinv * r + rms(r) * net([r / rms(r), log k]) on the H x W grid
 * (row y * W + x), rms(r) = sqrt(||r||^2 / (H W)); z = 0 when r = 0.
 *   nn_params device, PERKS_NN_PARAMS floats (layout as perks_nn_forward).
 *   r, logk, dinv  device, H * W doubles each (dinv: the Jacobi step's D^-1).
 *   z         device, H * W doubles, written.
 * Asynchronous on `stream`; uses the library's FCG scratch (calls that
 * overlap in time with perks_fcg_solve on one device race). */
int perks_fcg_precondition(const float *nn_params, const double *r, const double *logk, const double *dinv,
                           int32_t H, int32_t W, double *z, void *stream);

/* perks_barrier_stats -- in-kernel timing of the device-wide barrier (the
 * grid.sync() that replaces each relaunch, Sec. 3 / Listing 1) in the last
 * persistent launch made by this library on the current device (stencil,
 * CG, FCG or batched).  Every workgroup counts, with the scalar shader clock
 * (s_memtime), the cycles from entering a barrier to leaving it, and the
 * cycles from its start to its end; the kernel stores one record per
 * workgroup.  This call synchronises `stream` (which must be the launch's
 * stream or one ordered after it) and averages the records.
 *   out  host, filled: wgs (grid size of that launch; 0 when no persistent
 *        launch has been made), barriers (per workgroup), wait_cycles and
 *        total_cycles (means over workgroups), max_wait_cycles, wait_share
 *        (sum of waits / sum of totals: the share of the kernel's time spent
 *        waiting in barriers, independent of the clock rate).
 * Launches on the same device after the one of interest overwrite the
 * records.  Returns PERKS_OK or an error. */
typedef struct {
    int32_t wgs;
    int32_t reserved;
    int64_t barriers;
    double wait_cycles;
    double max_wait_cycles;
    double total_cycles;
    double wait_share;
} perks_barrier_stats_t;

int perks_barrier_stats(void *stream, perks_barrier_stats_t *out);

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
