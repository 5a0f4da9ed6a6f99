"""CPU oracle for the PERKS hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, float64 reference implementations written from the paper
("PERKS: a Locality-Optimized Execution Model for Iterative Memory-bound GPU
Applications", ICS '23).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2204_02064_amd``) and neither imports the
other; the only common inputs come from the seeded generators in
``workloads``.

The arithmetic lives in ``perks_oracle.c`` (gcc -O2 -ffp-contract=off, so no
fused multiply-add) and ``perf_model.py``; this file only marshals arrays.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "perks_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_f64p = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build_oracle():
    """Compile the oracle's C library in place (gcc, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build_oracle()
    lib = ctypes.CDLL(_LIB)
    lib.oracle_stencil.argtypes = [_f64p, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int64, _f64p, ctypes.c_int, ctypes.c_int64]
    lib.oracle_stencil.restype = ctypes.c_int
    lib.oracle_stencil_threads.argtypes = lib.oracle_stencil.argtypes + [ctypes.c_int]
    lib.oracle_stencil_threads.restype = ctypes.c_int
    lib.oracle_dot.argtypes = [_f64p, _f64p, ctypes.c_int64]
    lib.oracle_dot.restype = ctypes.c_double
    lib.oracle_spmv.argtypes = [ctypes.c_int64, _i32p, _i32p, _f64p, _f64p, _f64p]
    lib.oracle_spmv.restype = None
    lib.oracle_cg.argtypes = [ctypes.c_int64, _i32p, _i32p, _f64p, _f64p, _f64p,
                              ctypes.c_double, ctypes.c_int, ctypes.c_int, _f64p]
    lib.oracle_cg.restype = ctypes.c_int
    lib.oracle_cg_mixed.argtypes = [ctypes.c_int64, _i32p, _i32p, _f64p, _f64p, _f64p,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, _f64p, _f64p]
    lib.oracle_cg_mixed.restype = ctypes.c_int
    lib.oracle_chol_solve.argtypes = [ctypes.c_int64, _f64p, _f64p, _f64p]
    lib.oracle_chol_solve.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_f64p):
    return a.ctypes.data_as(t)


def stencil(grid, weights, steps, threads=1):
    """Return ``grid`` after ``steps`` Jacobi sweeps of the weight box.

    ``grid`` is 2D (ny, nx) or 3D (nz, ny, nx); ``weights`` is the dense
    (2r+1)^d box; the ring of width r stays fixed.  Computed in float64 on a
    float64 copy of ``grid`` (an FP32 input is first widened exactly).
    ``threads`` host threads share each sweep's rows (same result).
    """
    g = _f64(grid).copy()
    w = _f64(weights)
    nd = g.ndim
    if w.ndim != nd or len(set(w.shape)) != 1 or w.shape[0] % 2 != 1:
        raise ValueError("weights must be a (2r+1)^d box matching the grid's rank")
    r = w.shape[0] // 2
    nz, ny, nx = (g.shape if nd == 3 else (1,) + g.shape)
    rc = _load().oracle_stencil_threads(_ptr(g), nd, nx, ny, nz, _ptr(w), r, int(steps), int(threads))
    if rc != 0:
        raise ValueError("oracle_stencil rejected its arguments")
    return g


def dot(x, y):
    x, y = _f64(x), _f64(y)
    return _load().oracle_dot(_ptr(x), _ptr(y), x.size)


def spmv(rowptr, colind, values, x):
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(colind, dtype=np.int32)
    v, x = _f64(values), _f64(x)
    n = rp.size - 1
    y = np.empty(n)
    _load().oracle_spmv(n, _ptr(rp, _i32p), _ptr(ci, _i32p), _ptr(v), _ptr(x), _ptr(y))
    return y


CG_STATUS = {0: "converged", 1: "not_converged", 2: "breakdown"}


def cg(rowptr, colind, values, b, x0=None, tol=1e-10, maxit=5000, precond=None):
    """Conjugate gradient (Jacobi-preconditioned if ``precond == 'jacobi'``).

    Returns ``(x, info)`` with ``info = {iters, relres, relres_true,
    restarts, status}``.
    """
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(colind, dtype=np.int32)
    v, b = _f64(values), _f64(b)
    n = rp.size - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    out = np.zeros(4)
    pc = {None: 0, "none": 0, "jacobi": 1}[precond]
    st = _load().oracle_cg(n, _ptr(rp, _i32p), _ptr(ci, _i32p), _ptr(v), _ptr(b), _ptr(x),
                           float(tol), int(maxit), pc, _ptr(out))
    if st < 0:
        raise ValueError("oracle_cg rejected its arguments")
    return x, {"iters": int(out[0]), "relres": float(out[1]), "relres_true": float(out[2]),
               "restarts": int(out[3]), "status": CG_STATUS[st]}


MIXED_UPDATE_TOL = 0.3   # fall of the FP32 recursive residual that triggers an FP64 replacement
MIXED_MAX_OUTER = 100    # replacements allowed (after the first residual)
MIXED_STALL = 3          # replacements in a row without a new smallest true residual


def cg_mixed(rowptr, colind, values, b, x0=None, tol=1e-8, maxit=5000, precond=None,
             update_tol=MIXED_UPDATE_TOL, max_outer=MIXED_MAX_OUTER):
    """Mixed-precision CG: one FP32 CG recurrence whose residual is replaced
    by the true FP64 residual of an FP64 iterate whenever it has fallen by
    ``update_tol`` (the direction is kept across replacements).

    Returns ``(x, info)`` with ``info = {iters (FP32 iterations),
    relres_true, outer (replacements after the first residual), status,
    history}``; ``history[j]`` is the true relative residual at the j-th
    residual computation (``history[0]`` that of x0).
    """
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(colind, dtype=np.int32)
    v, b = _f64(values), _f64(b)
    n = rp.size - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    out = np.zeros(4)
    hist = np.full(max_outer + 1, np.nan)
    pc = {None: 0, "none": 0, "jacobi": 1}[precond]
    st = _load().oracle_cg_mixed(n, _ptr(rp, _i32p), _ptr(ci, _i32p), _ptr(v), _ptr(b), _ptr(x),
                                 float(tol), int(maxit), pc, float(update_tol), int(max_outer),
                                 _ptr(out), _ptr(hist))
    if st < 0:
        raise ValueError("oracle_cg_mixed rejected its arguments")
    outer = int(out[3])
    return x, {"iters": int(out[0]), "relres": float(out[1]), "relres_true": float(out[2]), "outer": outer,
               "status": CG_STATUS[st], "history": hist[:outer + 1][~np.isnan(hist[:outer + 1])]}


def chol_solve(A, b):
    """Dense Cholesky solve; raises ValueError if A is not positive definite."""
    A, b = _f64(A), _f64(b)
    n = b.size
    x = np.empty(n)
    rc = _load().oracle_chol_solve(n, _ptr(A), _ptr(b), _ptr(x))
    if rc != 0:
        raise ValueError("matrix is not positive definite")
    return x
