"""Pins of the mixed-precision CG oracle (one FP32 CG recurrence with FP64
residual replacement; no GPU).

The mixed solver is pinned to a dense Cholesky solve on small SPD systems, to
the FP32 accuracy floor of a single FP32 segment (which an all-FP64 recurrence
would beat by orders of magnitude), to the FP64 CG oracle's iteration count
(a recurrence that keeps its direction across replacements follows FP64 CG;
one restarted at every replacement, or with a wrongly scaled beta, needs far
more iterations), to a true residual that falls at every replacement on
Poisson systems, to one step on a Poisson eigenvector, to exact invariance
under power-of-two scaling of b, to the stagnation rule, and to its edge
cases.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

U32 = 2.0 ** -24


def _dense_to_csr(A):
    n = A.shape[0]
    rowptr = [0]; cols = []; vals = []
    for i in range(n):
        nz = np.nonzero(A[i])[0]
        cols.extend(nz.tolist()); vals.extend(A[i, nz].tolist())
        rowptr.append(len(cols))
    return np.array(rowptr, np.int32), np.array(cols, np.int32), np.array(vals)


def _spd(n, kappa, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * np.geomspace(1.0, kappa, n)) @ Q.T
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("n,kappa,seed,precond", [(16, 10.0, 0, None), (48, 100.0, 1, None),
                                                  (64, 100.0, 2, "jacobi")])
def test_mixed_matches_direct_solution(n, kappa, seed, precond):
    A = _spd(n, kappa, seed)
    rp, ci, v = _dense_to_csr(A)
    b = np.random.default_rng(seed).uniform(-1, 1, n)
    x, info = oracle.cg_mixed(rp, ci, v, b, tol=1e-12, maxit=50 * n, precond=precond)
    assert info["status"] == "converged"
    assert info["relres_true"] <= 1e-12
    # the true residual is recomputed in FP64 from scratch
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 2e-12
    xs = oracle.chol_solve(A, b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-12


def test_single_step_stops_at_the_fp32_floor():
    """One refinement step cannot beat FP32 (kappa * u32 level); refinement can."""
    rp, ci, v = workloads.poisson_csr(64, 2)
    b = workloads.rhs_uniform(rp.size - 1, seed=3)
    _, one = oracle.cg_mixed(rp, ci, v, b, tol=1e-14, maxit=3000, update_tol=1e-14, max_outer=1)
    assert one["outer"] == 1 and one["status"] == "not_converged"
    assert 1e-9 < one["relres_true"] < 1e-4
    _, full = oracle.cg_mixed(rp, ci, v, b, tol=1e-12, maxit=3000)
    assert full["status"] == "converged" and full["relres_true"] <= 1e-12


@pytest.mark.parametrize("case", ["poisson2d", "poisson3d", "random_jacobi"])
def test_replacements_keep_the_krylov_space(case):
    """Total FP32 iterations within 15% (+2) of FP64 CG's on the same system.

    FP32 recurrences lose orthogonality a little faster than FP64 ones (on 2D
    Poisson the count ranges from equal to about 9% more, depending on where
    the replacements fall); restarting the recurrence at every replacement
    costs 1.5-2x."""
    precond = None
    if case == "poisson2d":
        rp, ci, v = workloads.poisson_csr(48, 2)
    elif case == "poisson3d":
        rp, ci, v = workloads.poisson_csr(16, 3)
    else:
        rp, ci, v = workloads.random_spd_csr(3000, seed=4)
        precond = "jacobi"
    b = workloads.rhs_uniform(rp.size - 1, seed=2)
    _, ref = oracle.cg(rp, ci, v, b, tol=1e-10, maxit=5000, precond=precond)
    _, mix = oracle.cg_mixed(rp, ci, v, b, tol=1e-10, maxit=5000, precond=precond)
    assert ref["status"] == "converged" and mix["status"] == "converged"
    assert abs(mix["iters"] - ref["iters"]) <= 0.15 * ref["iters"] + 2, (mix["iters"], ref["iters"])
    # replacements happen: the FP32 recursion alone would stop at the FP32 floor
    assert mix["outer"] >= 2


@pytest.mark.parametrize("side,dim", [(40, 2), (12, 3)])
def test_true_residual_falls_at_every_replacement(side, dim):
    rp, ci, v = workloads.poisson_csr(side, dim)
    n = rp.size - 1
    b = workloads.rhs_uniform(n, seed=side)
    x, info = oracle.cg_mixed(rp, ci, v, b, tol=1e-12, maxit=5000)
    h = info["history"]
    assert info["status"] == "converged" and h.size == info["outer"] + 1
    assert np.all(np.diff(h) < 0), h
    # the last entry is the true residual of the returned x
    import scipy.sparse as sp
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert abs(h[-1] - true) <= 1e-6 * true
    assert h[-1] <= 1e-12


def test_one_inner_step_on_poisson_eigenvector():
    side = 31
    rp, ci, v = workloads.poisson_csr(side, 2)
    i = np.arange(1, side + 1)
    th1, th2 = math.pi * 1 / (side + 1), math.pi * 3 / (side + 1)
    b = np.outer(np.sin(th2 * i), np.sin(th1 * i)).ravel()
    mu = (2 - 2 * math.cos(th1)) + (2 - 2 * math.cos(th2))
    x, info = oracle.cg_mixed(rp, ci, v, b, tol=1e-14, maxit=100, max_outer=1)
    assert info["iters"] == 1 and info["outer"] == 1
    # FP32 inner step: exact up to float rounding of b, A and the AXPY
    np.testing.assert_allclose(x, b / mu, rtol=0, atol=1e-6 * np.abs(b / mu).max())


def test_power_of_two_scaling_of_b_is_exact():
    rp, ci, v = workloads.poisson_csr(24, 2)
    b = workloads.rhs_normal(rp.size - 1, seed=7)
    x1, i1 = oracle.cg_mixed(rp, ci, v, b, tol=1e-10)
    x2, i2 = oracle.cg_mixed(rp, ci, v, b * 2.0 ** 40, tol=1e-10)
    assert i1["iters"] == i2["iters"] and i1["outer"] == i2["outer"]
    np.testing.assert_array_equal(x2, x1 * 2.0 ** 40)


def test_inner_solve_uses_fp32_matrix():
    """A matrix entry that FP32 cannot hold changes the inner iterates but not the answer."""
    A = np.diag([1.0, 2.0, 3.0]) + 1e-9 * np.ones((3, 3))
    rp, ci, v = _dense_to_csr(A)
    b = np.array([1.0, -2.0, 0.5])
    x, info = oracle.cg_mixed(rp, ci, v, b, tol=1e-14, maxit=100, update_tol=1e-6)
    assert info["status"] == "converged"
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-13)
    # the first FP32 segment solves float(A) (the 1e-9 part rounds away in
    # sum with the diagonal only at FP32 precision): history[1] ~ 1e-9 level
    assert 1e-11 < info["history"][1] < 1e-6


def test_mixed_edge_cases():
    rp, ci, v = workloads.poisson_csr(8, 2)
    n = rp.size - 1
    x, info = oracle.cg_mixed(rp, ci, v, np.zeros(n))
    assert info["status"] == "converged" and info["iters"] == 0 and np.all(x == 0)
    b = workloads.rhs_uniform(n, seed=1)
    xs, _ = oracle.cg(rp, ci, v, b, tol=1e-14)
    x, info = oracle.cg_mixed(rp, ci, v, b, x0=xs, tol=1e-8)
    assert info["iters"] == 0 and info["outer"] == 0 and info["status"] == "converged"
    x, info = oracle.cg_mixed(rp, ci, v, b, tol=1e-8, maxit=0)
    assert info["status"] == "not_converged" and info["iters"] == 0
    x, info = oracle.cg_mixed(rp, ci, v, b, tol=1e-12, maxit=1000, max_outer=1)
    assert info["status"] == "not_converged" and info["outer"] == 1


def test_mixed_reports_stagnation_when_fp32_cannot_resolve():
    A = _spd(32, 1e10, 11)
    rp, ci, v = _dense_to_csr(A)
    b = np.random.default_rng(11).uniform(-1, 1, 32)
    _, info = oracle.cg_mixed(rp, ci, v, b, tol=1e-10, maxit=20000)
    assert info["status"] in ("not_converged", "breakdown")
    assert info["outer"] < oracle.MIXED_MAX_OUTER
    if info["status"] == "not_converged":
        # ended by the stagnation rule: the last MIXED_STALL replacements set
        # no new smallest true residual
        h = info["history"]
        k = oracle.MIXED_STALL
        assert h.size > k and np.all(h[-k:] >= h[:-k].min())
