"""PERKS on MI355X: persistent-kernel iterative solvers (Python binding).

Thin ctypes binding of ``libperks.so`` (HIP for gfx950, built from ``csrc/``
by ``build.py``).  Every computation runs in the library's kernels; this
module only checks tensors and marshals pointers, sizes and the current HIP
stream.  PyTorch is used for device memory and streams only.

The library must be built; importing works without it, but every call raises
``RuntimeError`` when ``libperks.so`` is missing (there is no CPU fallback).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libperks.so")

PERKS_F32, PERKS_F64 = 0, 1
PRECOND = {None: 0, "none": 0, "jacobi": 1}
PRECISION = {None: 0, "f64": 0, "float64": 0, "mixed": 1}
STATUS = {0: "converged", 1: "not_converged", 2: "breakdown"}


class PerksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"perks error {code}: {msg}")
        self.code = code


class Shape(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("waves_per_wg", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
                ("rows_per_lane", ctypes.c_int32), ("planes_per_lane", ctypes.c_int32),
                ("sync", ctypes.c_int32), ("max_cached_tiles", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("steps_per_sync", ctypes.c_int32)]


class StencilPlan(ctypes.Structure):
    _fields_ = [("wgs", ctypes.c_int32), ("waves_per_wg", ctypes.c_int32),
                ("rows_per_lane", ctypes.c_int32), ("planes_per_lane", ctypes.c_int32),
                ("tiles", ctypes.c_int64), ("cached_tiles", ctypes.c_int64),
                ("cached_cells", ctypes.c_int64), ("interior_cells", ctypes.c_int64),
                ("halo_bytes_per_step", ctypes.c_int64), ("sync", ctypes.c_int32),
                ("lds_rows_per_lane", ctypes.c_int32)]


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("colind", ctypes.c_void_p), ("val", ctypes.c_void_p), ("dt", ctypes.c_int32),
                ("spmv", ctypes.c_int32)]


class CgResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("wgs", ctypes.c_int32), ("relres", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("cached_nnz_frac", ctypes.c_double), ("fallbacks", ctypes.c_int32),
                ("switched_at", ctypes.c_int32), ("barrier_cycles", ctypes.c_int64)]


class BarrierStats(ctypes.Structure):
    _fields_ = [("wgs", ctypes.c_int32), ("reserved", ctypes.c_int32), ("barriers", ctypes.c_int64),
                ("wait_cycles", ctypes.c_double), ("max_wait_cycles", ctypes.c_double),
                ("total_cycles", ctypes.c_double), ("wait_share", ctypes.c_double)]


class DeviceInfo(ctypes.Structure):
    _fields_ = [("cus", ctypes.c_int32), ("lds_per_cu", ctypes.c_int32), ("regs_per_cu", ctypes.c_int32),
                ("l2_bytes", ctypes.c_int32), ("hbm_bytes", ctypes.c_int64), ("arch", ctypes.c_char * 64)]


_lib = None


def lib():
    """Load libperks.so (raises RuntimeError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2204_02064_amd/build.py "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    L.perks_stencil_run.argtypes = [vp, dp, Shape, i64, i32, vp, ctypes.POINTER(Tuning)]
    L.perks_stencil_run_baseline.argtypes = [vp, dp, Shape, i64, i32, vp]
    L.perks_stencil_run_noalloc.argtypes = [vp, dp, Shape, i64, i32, vp]
    L.perks_stencil_run_noalloc.restype = ctypes.c_int
    L.perks_stencil_plan_query.argtypes = [dp, Shape, i32, ctypes.POINTER(Tuning), ctypes.POINTER(StencilPlan)]
    L.perks_stencil_autotune.argtypes = [dp, Shape, i32, i64, i32, vp, ctypes.POINTER(Tuning),
                                         ctypes.POINTER(ctypes.c_double)]
    L.perks_stencil_autotune.restype = ctypes.c_int
    L.perks_stencil_run_batched.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Shape), i32, dp, i64,
                                            i32, vp]
    L.perks_stencil_run_batched.restype = ctypes.c_int
    L.perks_stencil_batch_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Shape), i32, dp, i64,
                                             i32, ctypes.POINTER(ctypes.c_void_p)]
    L.perks_stencil_batch_run.argtypes = [vp, vp]
    L.perks_stencil_batch_graph.argtypes = [vp, ctypes.POINTER(ctypes.c_void_p)]
    L.perks_stencil_batch_destroy.argtypes = [vp]
    L.perks_tuning_save.argtypes = [ctypes.c_char_p]
    L.perks_tuning_load.argtypes = [ctypes.c_char_p]
    for name in ("perks_stencil_batch_create", "perks_stencil_batch_run", "perks_stencil_batch_graph",
                 "perks_stencil_batch_destroy", "perks_tuning_save", "perks_tuning_load"):
        getattr(L, name).restype = ctypes.c_int
    L.perks_strerror.restype = ctypes.c_char_p
    L.perks_strerror.argtypes = [ctypes.c_int]
    L.perks_last_error.restype = ctypes.c_char_p
    L.perks_device_query.argtypes = [ctypes.POINTER(DeviceInfo)]
    L.perks_barrier_stats.argtypes = [vp, ctypes.POINTER(BarrierStats)]
    L.perks_barrier_stats.restype = ctypes.c_int
    L.perks_cg_solve.argtypes = [ctypes.POINTER(Csr), vp, vp, f64, i32, i32, i32, vp, ctypes.POINTER(CgResult)]
    L.perks_cg_solve_baseline.argtypes = [ctypes.POINTER(Csr), vp, vp, f64, i32, i32, i32, i32, vp,
                                          ctypes.POINTER(CgResult)]
    pp = ctypes.POINTER(ctypes.c_void_p)
    L.perks_cg_batch_create.argtypes = [ctypes.POINTER(Csr), pp, pp, i32, f64, i32, i32, i32, pp]
    L.perks_cg_batch_run.argtypes = [vp, vp]
    L.perks_cg_batch_results.argtypes = [vp, ctypes.POINTER(CgResult), vp]
    L.perks_cg_batch_graph.argtypes = [vp, pp]
    L.perks_cg_batch_destroy.argtypes = [vp]
    L.perks_cg_solve_batched.argtypes = [ctypes.POINTER(Csr), pp, pp, i32, f64, i32, i32, i32, vp,
                                         ctypes.POINTER(CgResult)]
    L.perks_cg_solve_capture.argtypes = [ctypes.POINTER(Csr), vp, vp, f64, i32, i32, vp, i32, vp, vp, vp,
                                         ctypes.POINTER(CgResult)]
    L.perks_fcg_solve.argtypes = [ctypes.POINTER(Csr), vp, vp, f64, i32, vp, vp, i32, i32, i32, vp,
                                  ctypes.POINTER(CgResult)]
    L.perks_fcg_precondition.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp]
    for name in ("perks_cg_solve_capture", "perks_fcg_solve", "perks_fcg_precondition"):
        getattr(L, name).restype = ctypes.c_int
    L.perks_nn_forward.argtypes = [vp, vp, i32, i32, i32, vp, vp]
    L.perks_nn_loss_grad.argtypes = [vp, vp, vp, i32, i32, i32, vp, ctypes.POINTER(ctypes.c_double), vp]
    L.perks_nn_adam.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, vp]
    L.perks_nn_energy_grad.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, ctypes.POINTER(ctypes.c_double), vp]
    L.perks_nn_train.argtypes = [vp, vp, vp, vp, vp, i32, i32, i32, i32, i32, ctypes.c_float, ctypes.c_uint64, vp, vp,
                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), vp]
    L.perks_nn_make_pairs.argtypes = [ctypes.POINTER(Csr), vp, vp, vp, vp, i32, i32, i32, vp, vp,
                                      ctypes.POINTER(ctypes.c_int32), vp]
    for name in ("perks_nn_forward", "perks_nn_loss_grad", "perks_nn_adam", "perks_nn_energy_grad", "perks_nn_train",
                 "perks_nn_make_pairs"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("perks_stencil_run", "perks_stencil_run_baseline", "perks_stencil_plan_query",
                 "perks_device_query", "perks_cg_solve", "perks_cg_solve_baseline", "perks_cg_batch_create",
                 "perks_cg_batch_run", "perks_cg_batch_results", "perks_cg_batch_graph", "perks_cg_batch_destroy",
                 "perks_cg_solve_batched"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc, allow_positive=False):
    if rc < 0 or (rc > 0 and not allow_positive):
        L = lib()
        raise PerksError(rc, f"{L.perks_strerror(rc).decode()}: {L.perks_last_error().decode()}")
    return rc


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return PERKS_F64
    if t.dtype == torch.float32:
        return PERKS_F32
    raise TypeError(f"unsupported dtype {t.dtype} (float32 or float64)")


def _shape_from(dims, r=1):
    """perks_shape of full extents ``dims`` ([ny, nx] or [nz, ny, nx]) for a
    stencil of radius ``r``."""
    dims = tuple(int(d) for d in dims)
    if len(dims) == 2:
        return Shape(2, r, dims[1], dims[0], 1)
    if len(dims) == 3:
        return Shape(3, r, dims[2], dims[1], dims[0])
    raise ValueError("grid must be 2D [ny, nx] or 3D [nz, ny, nx]")


def _shape_of(t, r=1):
    return _shape_from(tuple(t.shape), r)


def _coeff_array(weights, ndim):
    """The weight box as contiguous float64 and its radius: a (2r+1)^ndim box."""
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
    if w.ndim != ndim or len(set(w.shape)) != 1 or w.shape[0] % 2 != 1 or w.shape[0] < 3:
        raise ValueError(f"weights must be a (2r+1)^{ndim} box with r >= 1")
    return w, w.shape[0] // 2


def _tuning(tuning):
    if tuning is None:
        return None
    t = Tuning()
    for k, v in dict(tuning).items():
        setattr(t, k, int(v))
    return ctypes.byref(t)


def _check_grid(grid):
    if not grid.is_cuda or not grid.is_contiguous():
        raise ValueError("grid must be a contiguous device tensor")


def stencil_run(grid, weights, steps, tuning=None, stream=None):
    """Run ``steps`` Jacobi sweeps in place as ONE persistent kernel launch."""
    _check_grid(grid)
    w, r = _coeff_array(weights, grid.dim())
    rc = lib().perks_stencil_run(ctypes.c_void_p(grid.data_ptr()), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 _shape_of(grid, r), int(steps), _dtype_code(grid), _stream_handle(stream),
                                 _tuning(tuning))
    _check(rc)
    return grid


def stencil_run_noalloc(grid, weights, steps, stream=None):
    """stencil_run of a 2D radius-1 pattern with no device allocation
    (perks_stencil_run_noalloc: the library's fixed per-device array)."""
    _check_grid(grid)
    w, r = _coeff_array(weights, grid.dim())
    rc = lib().perks_stencil_run_noalloc(ctypes.c_void_p(grid.data_ptr()),
                                         w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _shape_of(grid, r),
                                         int(steps), _dtype_code(grid), _stream_handle(stream))
    _check(rc)
    return grid


def stencil_run_baseline(grid, weights, steps, stream=None):
    """Same sweeps with one kernel launch per step (the host-looped baseline)."""
    _check_grid(grid)
    w, r = _coeff_array(weights, grid.dim())
    rc = lib().perks_stencil_run_baseline(ctypes.c_void_p(grid.data_ptr()),
                                          w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _shape_of(grid, r),
                                          int(steps), _dtype_code(grid), _stream_handle(stream))
    _check(rc)
    return grid


def stencil_plan(shape, weights, dtype="float64", tuning=None):
    """The launch plan perks_stencil_run would use, as a dict."""
    shape = tuple(int(s) for s in shape)
    w, r = _coeff_array(weights, len(shape))
    sh = _shape_from(shape, r)
    pl = StencilPlan()
    dt = PERKS_F64 if str(dtype).endswith("64") else PERKS_F32
    rc = lib().perks_stencil_plan_query(w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), sh, dt,
                                        _tuning(tuning), ctypes.byref(pl))
    _check(rc)
    return {f: getattr(pl, f) for f, _ in StencilPlan._fields_ if f != "reserved"}


def stencil_run_batched(grids, weights, steps, stream=None):
    """Run ``steps`` Jacobi sweeps on every 2D grid of the list in ONE persistent launch."""
    m = len(grids)
    if m == 0:
        return grids
    for g in grids:
        _check_grid(g)
        if g.dim() != 2 or g.dtype != grids[0].dtype:
            raise ValueError("batched grids must be 2D and of one dtype")
    w, r = _coeff_array(weights, 2)
    ptrs = (ctypes.c_void_p * m)(*[g.data_ptr() for g in grids])
    shapes = (Shape * m)(*[_shape_of(g, r) for g in grids])
    _check(lib().perks_stencil_run_batched(ptrs, shapes, m, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           int(steps), _dtype_code(grids[0]), _stream_handle(stream)))
    return grids


class StencilBatch:
    """A batched-stencil plan: device memory and the launch made once, run many
    times.  ``run()`` enqueues one launch (a HIP graph node when available)
    without synchronising; refill the grids in place between runs."""

    def __init__(self, grids, weights, steps):
        self._keep = list(grids)
        m = len(grids)
        for g in grids:
            _check_grid(g)
            if g.dim() != 2 or g.dtype != grids[0].dtype:
                raise ValueError("batched grids must be 2D and of one dtype")
        w, r = _coeff_array(weights, 2)
        ptrs = (ctypes.c_void_p * max(m, 1))(*[g.data_ptr() for g in grids])
        shapes = (Shape * max(m, 1))(*[_shape_of(g, r) for g in grids])
        self._h = ctypes.c_void_p()
        dt = _dtype_code(grids[0]) if m else 1
        _check(lib().perks_stencil_batch_create(ptrs, shapes, m, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                int(steps), dt, ctypes.byref(self._h)))

    def run(self, stream=None):
        _check(lib().perks_stencil_batch_run(self._h, _stream_handle(stream)))

    def has_graph(self):
        g = ctypes.c_void_p()
        return lib().perks_stencil_batch_graph(self._h, ctypes.byref(g)) == 0

    def close(self):
        if self._h:
            lib().perks_stencil_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tuning_save(path):
    """Write the remembered autotuner choices of the current device to ``path``."""
    _check(lib().perks_tuning_save(os.fsencode(path)))


def tuning_load(path):
    """Add the tunings in ``path`` (written by tuning_save) to the current device's table."""
    _check(lib().perks_tuning_load(os.fsencode(path)))


def stencil_autotune(shape, weights, dtype="float64", probe_steps=50, remember=True, stream=None):
    """Time the candidate plans for this stencil and shape; returns (tuning dict,
    GCells/s).  With ``remember``, later untuned stencil_run calls on this shape
    use the winner."""
    shape = tuple(int(s) for s in shape)
    w, r = _coeff_array(weights, len(shape))
    sh = _shape_from(shape, r)
    t = Tuning()
    rate = ctypes.c_double()
    dt = PERKS_F64 if str(dtype).endswith("64") else PERKS_F32
    _check(lib().perks_stencil_autotune(w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), sh, dt, int(probe_steps),
                                        1 if remember else 0, _stream_handle(stream), ctypes.byref(t),
                                        ctypes.byref(rate)))
    return {f: getattr(t, f) for f, _ in Tuning._fields_}, rate.value


def device_info():
    d = DeviceInfo()
    _check(lib().perks_device_query(ctypes.byref(d)))
    return {"cus": d.cus, "lds_per_cu": d.lds_per_cu, "regs_per_cu": d.regs_per_cu, "l2_bytes": d.l2_bytes,
            "hbm_bytes": d.hbm_bytes, "arch": d.arch.decode()}


SPMV = {None: 0, "auto": 0, "sell": 1, "merge": 2}


class CsrMatrix:
    """Device CSR matrix (int32 rowptr/colind, float64 values) as torch tensors.
    ``spmv`` picks the persistent solvers' SpMV layout (perks_csr.spmv):
    "auto" (the library's choice), "sell" (sliced ELL / CSR, vectors in
    memory) or "merge" (merge-path SpMV)."""

    def __init__(self, rowptr, colind, values, device="cuda", spmv="auto"):
        import torch

        def dev(a, npt, tt):
            if isinstance(a, torch.Tensor):
                return a.to(device=device, dtype=tt).contiguous()
            return torch.as_tensor(np.asarray(a, dtype=npt), device=device).contiguous()
        self.rowptr = dev(rowptr, np.int32, torch.int32)
        self.colind = dev(colind, np.int32, torch.int32)
        self.values = dev(values, np.float64, torch.float64)
        self.n = self.rowptr.numel() - 1
        self.nnz = self.colind.numel()
        if spmv not in SPMV:
            raise ValueError(f"spmv must be one of {sorted(k for k in SPMV if k)}")
        self.spmv = spmv

    def _struct(self):
        return Csr(self.n, self.nnz, self.rowptr.data_ptr(), self.colind.data_ptr(), self.values.data_ptr(),
                   PERKS_F64 if self.values.dtype.itemsize == 8 else PERKS_F32, SPMV[self.spmv])


def _cg_result(r, precision):
    d = {"iters": r.iters, "status": STATUS.get(r.status, str(r.status)), "wgs": r.wgs, "relres": r.relres,
         "relres_true": r.relres_true, "cached_nnz_frac": r.cached_nnz_frac, "barrier_cycles": r.barrier_cycles}
    d["outer" if PRECISION[precision] == 1 else "restarts"] = r.restarts
    return d


def barrier_stats(stream=None):
    """Barrier clock of the last persistent launch on the current device
    (perks_barrier_stats): mean cycles per workgroup waiting in device barriers,
    barriers per workgroup, and the share of the kernel's time spent waiting."""
    st = BarrierStats()
    _check(lib().perks_barrier_stats(_stream_handle(stream), ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in BarrierStats._fields_ if f != "reserved"}


def _check_vec(v, n, name):
    import torch
    if not v.is_cuda or not v.is_contiguous() or v.dtype != torch.float64 or v.numel() != n:
        raise ValueError(f"{name} must be a contiguous float64 device vector of length {n}")


def cg_solve(A, b, x, tol=1e-10, maxit=5000, precond=None, precision=None, stream=None):
    """Persistent-kernel CG: solves A x = b in place in ``x``; returns an info dict.

    ``precision``: None / "f64" (FP64 throughout) or "mixed" (one FP32 CG
    recurrence with FP64 residual replacement, one launch; ``outer`` counts
    the replacements).
    """
    _check_vec(b, A.n, "b")
    _check_vec(x, A.n, "x")
    res = CgResult()
    st = A._struct()
    rc = lib().perks_cg_solve(ctypes.byref(st), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                              float(tol), int(maxit), PRECOND[precond], PRECISION[precision],
                              _stream_handle(stream), ctypes.byref(res))
    _check(rc, allow_positive=True)
    return _cg_result(res, precision)


def cg_solve_baseline(A, b, x, tol=1e-10, maxit=5000, precond=None, precision=None, check_every=1, stream=None):
    """Host-looped multi-kernel CG (the baseline); same interface as cg_solve."""
    _check_vec(b, A.n, "b")
    _check_vec(x, A.n, "x")
    res = CgResult()
    st = A._struct()
    rc = lib().perks_cg_solve_baseline(ctypes.byref(st), ctypes.c_void_p(b.data_ptr()),
                                       ctypes.c_void_p(x.data_ptr()), float(tol), int(maxit), PRECOND[precond],
                                       PRECISION[precision], int(check_every), _stream_handle(stream),
                                       ctypes.byref(res))
    _check(rc, allow_positive=True)
    return _cg_result(res, precision)


def _batch_args(As, bs, xs):
    m = len(As)
    if len(bs) != m or len(xs) != m:
        raise ValueError("As, bs and xs must have the same length")
    for A, b, x in zip(As, bs, xs):
        _check_vec(b, A.n, "b")
        _check_vec(x, A.n, "x")
    arr = (Csr * max(m, 1))(*[A._struct() for A in As])
    bp = (ctypes.c_void_p * max(m, 1))(*[b.data_ptr() for b in bs])
    xp = (ctypes.c_void_p * max(m, 1))(*[x.data_ptr() for x in xs])
    return m, arr, bp, xp


def cg_solve_batched(As, bs, xs, tol=1e-10, maxit=5000, precond=None, precision=None, stream=None):
    """Solve every A_i x_i = b_i in ONE persistent launch; returns a list of info dicts."""
    m, arr, bp, xp = _batch_args(As, bs, xs)
    res = (CgResult * max(m, 1))()
    rc = lib().perks_cg_solve_batched(arr, bp, xp, m, float(tol), int(maxit), PRECOND[precond],
                                      PRECISION[precision], _stream_handle(stream), res)
    _check(rc, allow_positive=True)
    return [_cg_result(res[i], precision) for i in range(m)]


class CgBatch:
    """A batched CG plan: schedule and device memory made once, run many times.

    ``run()`` enqueues one launch (a HIP graph node when available) on the
    stream without synchronising; ``results()`` synchronises and returns the
    per-problem info dicts.  The plan keeps references to the matrices and
    vectors it was built from; refill ``bs`` / ``xs`` in place between runs.
    """

    def __init__(self, As, bs, xs, tol=1e-10, maxit=5000, precond=None, precision=None):
        self._keep = (list(As), list(bs), list(xs))
        self.count, arr, bp, xp = _batch_args(As, bs, xs)
        self.precision = precision
        self._h = ctypes.c_void_p()
        rc = lib().perks_cg_batch_create(arr, bp, xp, self.count, float(tol), int(maxit), PRECOND[precond],
                                         PRECISION[precision], ctypes.byref(self._h))
        _check(rc)

    def run(self, stream=None):
        _check(lib().perks_cg_batch_run(self._h, _stream_handle(stream)))

    def results(self, stream=None):
        res = (CgResult * max(self.count, 1))()
        rc = lib().perks_cg_batch_results(self._h, res, _stream_handle(stream))
        _check(rc, allow_positive=True)
        return [_cg_result(res[i], self.precision) for i in range(self.count)]

    def has_graph(self):
        g = ctypes.c_void_p()
        return lib().perks_cg_batch_graph(self._h, ctypes.byref(g)) == 0

    def close(self):
        if self._h:
            lib().perks_cg_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Learned preconditioner network (six 3x3 conv layers, BF16 on the matrix cores).
NN_LAYERS = [(2, 16), (16, 16), (16, 16), (16, 16), (16, 16), (16, 1)]
NN_LAYER_PARAMS = 16 * 16 * 9 + 16
NN_PARAMS = len(NN_LAYERS) * NN_LAYER_PARAMS


def nn_pack_params(layers):
    """[(W [co, ci, 3, 3], b [co]) per layer] -> padded float32 vector (host)."""
    out = np.zeros(NN_PARAMS, dtype=np.float32)
    for l, ((ci, co), (w, b)) in enumerate(zip(NN_LAYERS, layers)):
        blk = np.zeros((16, 16, 3, 3), dtype=np.float32)
        blk[:co, :ci] = np.asarray(w, dtype=np.float32).reshape(co, ci, 3, 3)
        bias = np.zeros(16, dtype=np.float32)
        bias[:co] = np.asarray(b, dtype=np.float32)
        base = l * NN_LAYER_PARAMS
        out[base:base + 16 * 16 * 9] = blk.ravel()
        out[base + 16 * 16 * 9:base + NN_LAYER_PARAMS] = bias
    return out


def nn_unpack_params(vec):
    """Inverse of nn_pack_params (real channels only), float32 arrays."""
    vec = np.asarray(vec, dtype=np.float32)
    layers = []
    for l, (ci, co) in enumerate(NN_LAYERS):
        base = l * NN_LAYER_PARAMS
        blk = vec[base:base + 16 * 16 * 9].reshape(16, 16, 3, 3)
        layers.append((blk[:co, :ci].copy(), vec[base + 16 * 16 * 9:base + 16 * 16 * 9 + co].copy()))
    return layers


def _check_f32(t, n, name):
    import torch
    if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float32 or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous float32 device tensor of {n} elements")


def nn_forward(params, x, out=None, stream=None):
    """Network output [B, H, W] for x [B, H, W, 2] (float32 device tensors)."""
    import torch
    B, H, W, C = x.shape
    if C != 2:
        raise ValueError("x must be [B, H, W, 2]")
    _check_f32(params, NN_PARAMS, "params")
    _check_f32(x, B * H * W * 2, "x")
    if out is None:
        out = torch.empty((B, H, W), dtype=torch.float32, device=x.device)
    _check_f32(out, B * H * W, "out")
    _check(lib().perks_nn_forward(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(x.data_ptr()), B, H, W,
                                  ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def nn_loss_grad(params, x, target, grad=None, stream=None):
    """(loss, grad): mean squared error of the network on (x, target) and its gradient."""
    import torch
    B, H, W, _ = x.shape
    _check_f32(params, NN_PARAMS, "params")
    _check_f32(x, B * H * W * 2, "x")
    _check_f32(target, B * H * W, "target")
    if grad is None:
        grad = torch.empty(NN_PARAMS, dtype=torch.float32, device=x.device)
    loss = ctypes.c_double()
    _check(lib().perks_nn_loss_grad(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(target.data_ptr()), B, H, W, ctypes.c_void_p(grad.data_ptr()),
                                    ctypes.byref(loss), _stream_handle(stream)))
    return loss.value, grad


def nn_energy_grad(params, x, planes, grad=None, stream=None, jacobi=True):
    """(loss, grad) of the energy-norm loss: planes [B, 5, H, W] float32 hold
    each sample's 5-point operator, x[..., 0] the scaled residual; with
    ``jacobi`` the loss is taken on the Jacobi step plus the network output
    (the preconditioner fcg_solve applies), else on the output alone."""
    import torch
    B, H, W, _ = x.shape
    _check_f32(params, NN_PARAMS, "params")
    _check_f32(x, B * H * W * 2, "x")
    _check_f32(planes, B * 5 * H * W, "planes")
    if grad is None:
        grad = torch.empty(NN_PARAMS, dtype=torch.float32, device=x.device)
    loss = ctypes.c_double()
    _check(lib().perks_nn_energy_grad(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(planes.data_ptr()), int(bool(jacobi)), B, H, W,
                                      ctypes.c_void_p(grad.data_ptr()),
                                      ctypes.byref(loss), _stream_handle(stream)))
    return loss.value, grad


def nn_train(params, x, epochs, batch, lr=1e-3, seed=0, target=None, planes=None, field=None, m=None, v=None,
             step=0, stream=None):
    """Adam training on the device (perks_nn_train): params is updated in place.
    Give ``target`` ([P, H, W], MSE loss) or ``planes`` ([F, 5, H, W]) with
    ``field`` ([P] int32, operator of each sample: energy loss, Jacobi form).
    Returns (per-epoch mean losses, Adam step count, m, v)."""
    import torch
    P, H, W, _ = x.shape
    _check_f32(params, NN_PARAMS, "params")
    _check_f32(x, P * H * W * 2, "x")
    if (target is None) == (planes is None):
        raise ValueError("give target or planes")
    if target is not None:
        _check_f32(target, P * H * W, "target")
    else:
        _check_f32(planes, planes.shape[0] * 5 * H * W, "planes")
        if field is None or field.dtype != torch.int32 or field.numel() != P or not field.is_contiguous():
            raise ValueError("field must be a contiguous int32 tensor of P entries")
    m = torch.zeros(NN_PARAMS, dtype=torch.float32, device=x.device) if m is None else m
    v = torch.zeros_like(m) if v is None else v
    st = ctypes.c_int32(int(step))
    losses = (ctypes.c_double * max(1, int(epochs)))()
    ptr = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else 0)
    _check(lib().perks_nn_train(ptr(params), ptr(x), ptr(target), ptr(planes), ptr(field), P, H, W, int(epochs),
                                int(batch), float(lr), int(seed) & ((1 << 64) - 1), ptr(m), ptr(v), ctypes.byref(st),
                                losses, _stream_handle(stream)))
    return [losses[i] for i in range(int(epochs))], st.value, m, v


def nn_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    for t, nm in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
        _check_f32(t, NN_PARAMS, nm)
    _check(lib().perks_nn_adam(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                               ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), int(step),
                               float(lr), float(beta1), float(beta2), float(eps), _stream_handle(stream)))


def nn_make_pairs(A, xstar, logk, xcap, rcap, H, W, stream=None):
    """Training pairs from captured iterates (perks_nn_make_pairs): returns
    (inputs [m, H, W, 2] float32, targets [m, H, W] float32) device tensors for
    the m leading captures the solve reached."""
    import torch
    n = int(H) * int(W)
    if A.n != n:
        raise ValueError("H * W must equal the matrix order")
    _check_vec(xstar, n, "xstar")
    _check_vec(logk.reshape(-1), n, "logk")
    for t, nm in ((xcap, "xcap"), (rcap, "rcap")):
        if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float64 or t.dim() != 2 or t.shape[1] != n:
            raise ValueError(f"{nm} must be a contiguous float64 device tensor [ncap, {n}]")
    if xcap.shape != rcap.shape:
        raise ValueError("xcap and rcap must have the same shape")
    ncap = int(rcap.shape[0])
    inputs = torch.empty((ncap, int(H), int(W), 2), dtype=torch.float32, device=rcap.device)
    targets = torch.empty((ncap, int(H), int(W)), dtype=torch.float32, device=rcap.device)
    cnt = ctypes.c_int32(0)
    st = A._struct()
    _check(lib().perks_nn_make_pairs(ctypes.byref(st), ctypes.c_void_p(xstar.data_ptr()),
                                     ctypes.c_void_p(logk.data_ptr()), ctypes.c_void_p(xcap.data_ptr()),
                                     ctypes.c_void_p(rcap.data_ptr()), ncap, int(H), int(W),
                                     ctypes.c_void_p(inputs.data_ptr()), ctypes.c_void_p(targets.data_ptr()),
                                     ctypes.byref(cnt), _stream_handle(stream)))
    return inputs[:cnt.value], targets[:cnt.value]


def cg_solve_capture(A, b, x, iters, tol=1e-10, maxit=5000, precond=None, stream=None):
    """Persistent FP64 CG that also returns x_k and r_k after each k in ``iters``.

    Returns (info, xcap [m, n], rcap [m, n]) with device tensors; rows for
    iteration counts the solve did not reach hold NaN.
    """
    import torch
    _check_vec(b, A.n, "b")
    _check_vec(x, A.n, "x")
    its = sorted(int(k) for k in iters)
    m = len(its)
    it_dev = torch.tensor(its if m else [0], dtype=torch.int32, device=b.device)
    xcap = torch.full((max(m, 1), A.n), float("nan"), dtype=torch.float64, device=b.device)
    rcap = torch.full((max(m, 1), A.n), float("nan"), dtype=torch.float64, device=b.device)
    res = CgResult()
    st = A._struct()
    rc = lib().perks_cg_solve_capture(ctypes.byref(st), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                      float(tol), int(maxit), PRECOND[precond], ctypes.c_void_p(it_dev.data_ptr()), m,
                                      ctypes.c_void_p(xcap.data_ptr()), ctypes.c_void_p(rcap.data_ptr()),
                                      _stream_handle(stream), ctypes.byref(res))
    _check(rc, allow_positive=True)
    return _cg_result(res, None), xcap[:m], rcap[:m]


def fcg_solve(A, b, x, H, W, params=None, logk=None, tol=1e-8, maxit=5000, stall=20, stream=None):
    """Flexible CG preconditioned by the network (``params`` None: Jacobi-PCG),
    one persistent launch.  Returns an info dict with ``fallbacks`` (iterations
    that used the Jacobi step) and ``switched_at`` (iteration at which the solve
    continued as Jacobi-PCG, or None)."""
    _check_vec(b, A.n, "b")
    _check_vec(x, A.n, "x")
    if params is not None:
        _check_f32(params, NN_PARAMS, "params")
        _check_vec(logk.reshape(-1), A.n, "logk")
    res = CgResult()
    st = A._struct()
    rc = lib().perks_fcg_solve(ctypes.byref(st), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                               float(tol), int(maxit),
                               ctypes.c_void_p(params.data_ptr() if params is not None else 0),
                               ctypes.c_void_p(logk.data_ptr() if params is not None else 0), int(H), int(W),
                               int(stall), _stream_handle(stream), ctypes.byref(res))
    _check(rc, allow_positive=True)
    d = _cg_result(res, None)
    d.pop("restarts")
    d["fallbacks"] = res.fallbacks
    d["switched_at"] = None if res.switched_at < 0 else int(res.switched_at)
    return d


def fcg_precondition(params, r, logk, dinv, H, W, z=None, stream=None):
    """z = dinv * r + rms(r) * net([r / rms(r), log k]) on the H x W grid, by the
    tile routine the FCG kernel applies (float64 device vectors of H * W)."""
    import torch
    n = int(H) * int(W)
    _check_f32(params, NN_PARAMS, "params")
    for t, nm in ((r, "r"), (logk, "logk"), (dinv, "dinv")):
        _check_vec(t.reshape(-1), n, nm)
    if z is None:
        z = torch.empty(n, dtype=torch.float64, device=r.device)
    _check_vec(z, n, "z")
    _check(lib().perks_fcg_precondition(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(r.data_ptr()),
                                        ctypes.c_void_p(logk.data_ptr()), ctypes.c_void_p(dinv.data_ptr()), int(H),
                                        int(W), ctypes.c_void_p(z.data_ptr()), _stream_handle(stream)))
    return z
