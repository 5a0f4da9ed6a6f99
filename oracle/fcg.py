"""Flexible CG reference (numpy, float64) -- TEST INFRASTRUCTURE ONLY.

Flexible conjugate gradient in Notay's truncated form with one previous
direction (FCG(1)): the new direction is the preconditioned residual made
A-orthogonal to the previous direction explicitly,
    p_k = z_k - (<z_k, q_{k-1}> / <p_{k-1}, q_{k-1}>) p_{k-1},  q = A p,
    alpha_k = <p_k, r_k> / <p_k, q_k>,
which tolerates a preconditioner that is not a fixed linear operator (a
network).  With a fixed SPD preconditioner it is preconditioned CG in exact
arithmetic.  The paper's CG is unpreconditioned; this method and its
safeguards are the learned-preconditioner extension's, and the readings are:

* fallback: when the preconditioner fails (returns None or a non-finite z)
  or <z, r> <= 0, the Jacobi step z = D^{-1} r is used for that iteration;
* switch: when the residual norm has not reached a new minimum for `stall`
  iterations, the solve continues as Jacobi-preconditioned CG for good,
  restarting the direction recurrence;
* stop: iterate while ||r|| > tol ||b|| and k < maxit; the true residual is
  recomputed at the end.
"""
import numpy as np

import oracle


def fcg(rowptr, colind, values, b, precond, x0=None, tol=1e-8, maxit=5000, stall=20):
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(colind, dtype=np.int32)
    v = np.ascontiguousarray(values, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = rp.size - 1
    diag = np.zeros(n)
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            if ci[k] == i:
                diag[i] += v[k]
    dinv = 1.0 / diag
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    r = b - oracle.spmv(rp, ci, v, x)
    bnorm = np.sqrt(oracle.dot(b, b))
    info = {"iters": 0, "fallbacks": 0, "switched_at": None, "status": "not_converged"}
    if bnorm == 0.0:
        x[:] = 0.0
        info.update(status="converged", relres_true=0.0)
        return x, info
    use_net = precond is not None
    p_prev = q_prev = None
    pq_prev = 0.0
    best, since = np.inf, 0
    k = 0
    rn = np.sqrt(oracle.dot(r, r))
    while k < maxit and rn > tol * bnorm:
        z = None
        if use_net:
            z = precond(r)
            if z is None or not np.all(np.isfinite(z)) or not oracle.dot(z, r) > 0.0:
                z = None
                info["fallbacks"] += 1
        if z is None:
            z = dinv * r
        if p_prev is None:
            p = z.copy()
        else:
            p = z - (oracle.dot(z, q_prev) / pq_prev) * p_prev
        q = oracle.spmv(rp, ci, v, p)
        pq = oracle.dot(p, q)
        if not (pq > 0.0) or not np.isfinite(pq):
            info["status"] = "breakdown"
            break
        alpha = oracle.dot(p, r) / pq
        x = x + alpha * p
        r = r - alpha * q
        p_prev, q_prev, pq_prev = p, q, pq
        k += 1
        rn = np.sqrt(oracle.dot(r, r))
        if rn < best:
            best, since = rn, 0
        else:
            since += 1
        if use_net and since >= stall:
            use_net = False
            info["switched_at"] = k
            p_prev = None
    rt = b - oracle.spmv(rp, ci, v, x)
    info["iters"] = k
    info["relres_true"] = float(np.sqrt(oracle.dot(rt, rt)) / bnorm)
    if info["status"] != "breakdown":
        info["status"] = "converged" if info["relres_true"] <= tol else "not_converged"
    return x, info
