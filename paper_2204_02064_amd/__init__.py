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
STATUS = {0: "converged", 1: "not_converged", 2: "breakdown"}


class PerksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"perks error {code}: {msg}")
        self.code = code


class Shape(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("waves_per_wg", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
                ("rows_per_lane", ctypes.c_int32), ("planes_per_lane", ctypes.c_int32),
                ("sync", ctypes.c_int32), ("max_cached_tiles", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


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
                ("reserved", ctypes.c_int32)]


class CgResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("wgs", ctypes.c_int32), ("relres", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("cached_nnz_frac", ctypes.c_double), ("reserved", ctypes.c_double)]


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
    L.perks_stencil_plan_query.argtypes = [dp, Shape, i32, ctypes.POINTER(Tuning), ctypes.POINTER(StencilPlan)]
    L.perks_strerror.restype = ctypes.c_char_p
    L.perks_strerror.argtypes = [ctypes.c_int]
    L.perks_last_error.restype = ctypes.c_char_p
    L.perks_device_query.argtypes = [ctypes.POINTER(DeviceInfo)]
    if hasattr(L, "perks_cg_solve"):
        L.perks_cg_solve.argtypes = [ctypes.POINTER(Csr), vp, vp, f64, i32, i32, vp, ctypes.POINTER(CgResult)]
        L.perks_cg_solve_baseline.argtypes = [ctypes.POINTER(Csr), vp, vp, f64, i32, i32, i32, vp,
                                              ctypes.POINTER(CgResult)]
    for name in ("perks_stencil_run", "perks_stencil_run_baseline", "perks_stencil_plan_query",
                 "perks_device_query", "perks_cg_solve", "perks_cg_solve_baseline"):
        if hasattr(L, name):
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


def _shape_of(t):
    if t.dim() == 2:
        return Shape(2, 0, t.shape[1], t.shape[0], 1)
    if t.dim() == 3:
        return Shape(3, 0, t.shape[2], t.shape[1], t.shape[0])
    raise ValueError("grid must be 2D [ny, nx] or 3D [nz, ny, nx]")


def _coeff_array(weights, ndim):
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
    if w.shape != (3,) * ndim:
        raise ValueError(f"weights must be a {'x'.join(['3'] * ndim)} box")
    return w


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
    w = _coeff_array(weights, grid.dim())
    rc = lib().perks_stencil_run(ctypes.c_void_p(grid.data_ptr()), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 _shape_of(grid), int(steps), _dtype_code(grid), _stream_handle(stream),
                                 _tuning(tuning))
    _check(rc)
    return grid


def stencil_run_baseline(grid, weights, steps, stream=None):
    """Same sweeps with one kernel launch per step (the host-looped baseline)."""
    _check_grid(grid)
    w = _coeff_array(weights, grid.dim())
    rc = lib().perks_stencil_run_baseline(ctypes.c_void_p(grid.data_ptr()),
                                          w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _shape_of(grid),
                                          int(steps), _dtype_code(grid), _stream_handle(stream))
    _check(rc)
    return grid


def stencil_plan(shape, weights, dtype="float64", tuning=None):
    """The launch plan perks_stencil_run would use, as a dict."""
    shape = tuple(int(s) for s in shape)
    nd = len(shape)
    sh = Shape(2, 0, shape[1], shape[0], 1) if nd == 2 else Shape(3, 0, shape[2], shape[1], shape[0])
    w = _coeff_array(weights, nd)
    pl = StencilPlan()
    dt = PERKS_F64 if str(dtype).endswith("64") else PERKS_F32
    rc = lib().perks_stencil_plan_query(w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), sh, dt,
                                        _tuning(tuning), ctypes.byref(pl))
    _check(rc)
    return {f: getattr(pl, f) for f, _ in StencilPlan._fields_ if f != "reserved"}


def device_info():
    d = DeviceInfo()
    _check(lib().perks_device_query(ctypes.byref(d)))
    return {"cus": d.cus, "lds_per_cu": d.lds_per_cu, "regs_per_cu": d.regs_per_cu, "l2_bytes": d.l2_bytes,
            "hbm_bytes": d.hbm_bytes, "arch": d.arch.decode()}


class CsrMatrix:
    """Device CSR matrix (int32 rowptr/colind, float64 values) as torch tensors."""

    def __init__(self, rowptr, colind, values, device="cuda"):
        import torch
        self.rowptr = torch.as_tensor(np.asarray(rowptr, dtype=np.int32), device=device).contiguous()
        self.colind = torch.as_tensor(np.asarray(colind, dtype=np.int32), device=device).contiguous()
        self.values = torch.as_tensor(np.asarray(values, dtype=np.float64), device=device).contiguous()
        self.n = self.rowptr.numel() - 1
        self.nnz = self.colind.numel()

    def _struct(self):
        return Csr(self.n, self.nnz, self.rowptr.data_ptr(), self.colind.data_ptr(), self.values.data_ptr(),
                   PERKS_F64 if self.values.dtype.itemsize == 8 else PERKS_F32, 0)


def _cg_result(r):
    return {"iters": r.iters, "status": STATUS.get(r.status, str(r.status)), "restarts": r.restarts,
            "wgs": r.wgs, "relres": r.relres, "relres_true": r.relres_true, "cached_nnz_frac": r.cached_nnz_frac}


def cg_solve(A, b, x, tol=1e-10, maxit=5000, precond=None, stream=None):
    """Persistent-kernel CG: solves A x = b in place in ``x``; returns an info dict."""
    L = lib()
    if not hasattr(L, "perks_cg_solve"):
        raise RuntimeError("this libperks.so has no CG entry points")
    res = CgResult()
    st = A._struct()
    rc = L.perks_cg_solve(ctypes.byref(st), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                          float(tol), int(maxit), PRECOND[precond], _stream_handle(stream), ctypes.byref(res))
    _check(rc, allow_positive=True)
    return _cg_result(res)


def cg_solve_baseline(A, b, x, tol=1e-10, maxit=5000, precond=None, check_every=1, stream=None):
    """Host-looped multi-kernel CG (the baseline); same interface as cg_solve."""
    L = lib()
    res = CgResult()
    st = A._struct()
    rc = L.perks_cg_solve_baseline(ctypes.byref(st), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                   float(tol), int(maxit), PRECOND[precond], int(check_every),
                                   _stream_handle(stream), ctypes.byref(res))
    _check(rc, allow_positive=True)
    return _cg_result(res)
