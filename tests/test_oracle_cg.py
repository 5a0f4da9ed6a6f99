"""Pins of the conjugate-gradient oracle (no GPU).

CG is pinned to a dense Cholesky solve on tiny SPD systems (Cholesky itself is
checked against numpy's LAPACK solve), to the finite-termination property on
matrices with few distinct eigenvalues, to one-step convergence on a Poisson
eigenvector, to the classical A-norm error bound, and to its edge cases.
"""
import math

import numpy as np
import pytest

import oracle
import workloads


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
    lam = np.geomspace(1.0, kappa, n)
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("n,kappa,seed", [(5, 3.0, 0), (16, 50.0, 1), (64, 100.0, 2)])
def test_cholesky_matches_lapack(n, kappa, seed):
    A = _spd(n, kappa, seed)
    b = np.random.default_rng(seed + 10).standard_normal(n)
    np.testing.assert_allclose(oracle.chol_solve(A, b), np.linalg.solve(A, b), rtol=1e-11, atol=1e-12)


def test_cholesky_rejects_indefinite():
    with pytest.raises(ValueError):
        oracle.chol_solve(np.array([[1.0, 2.0], [2.0, 1.0]]), np.ones(2))


@pytest.mark.parametrize("n,kappa,seed", [(8, 10.0, 3), (32, 100.0, 4), (64, 100.0, 5)])
def test_cg_matches_direct_solution(n, kappa, seed):
    A = _spd(n, kappa, seed)
    rp, ci, v = _dense_to_csr(A)
    b = np.random.default_rng(seed).uniform(-1, 1, n)
    x, info = oracle.cg(rp, ci, v, b, tol=1e-12, maxit=4 * n)
    assert info["status"] == "converged"
    assert info["relres_true"] <= 1e-12
    xs = oracle.chol_solve(A, b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-12


@pytest.mark.parametrize("n,kappa,seed", [(8, 10.0, 3), (24, 3.0, 6), (64, 2.0, 7)])
def test_cg_converges_within_n_steps_when_well_conditioned(n, kappa, seed):
    # finite termination in n steps holds in exact arithmetic; with rounding it
    # survives on well-conditioned systems, where the loss of orthogonality is mild
    A = _spd(n, kappa, seed)
    rp, ci, v = _dense_to_csr(A)
    b = np.random.default_rng(seed).uniform(-1, 1, n)
    x, info = oracle.cg(rp, ci, v, b, tol=1e-12, maxit=n)
    assert info["status"] == "converged" and info["iters"] <= n


@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_cg_terminates_in_m_steps_for_m_distinct_eigenvalues(m):
    n = 40
    eig = np.array([1.0 + 3.0 * (i % m) for i in range(n)])
    A = np.diag(eig)
    rp, ci, v = _dense_to_csr(A)
    b = np.random.default_rng(m).uniform(0.5, 1.5, n)
    x, info = oracle.cg(rp, ci, v, b, tol=1e-13, maxit=100)
    assert info["status"] == "converged"
    assert info["iters"] == m
    np.testing.assert_allclose(x, b / eig, rtol=1e-13)


def test_cg_one_step_on_poisson_eigenvector():
    side = 12
    rp, ci, v = workloads.poisson_csr(side, 2)
    th_x, th_y = math.pi * 2 / (side + 1), math.pi * 3 / (side + 1)
    i = np.arange(1, side + 1)
    b = np.outer(np.sin(3 * math.pi * i / (side + 1)), np.sin(2 * math.pi * i / (side + 1))).ravel()
    mu = (2 - 2 * math.cos(th_x)) + (2 - 2 * math.cos(th_y))
    x, info = oracle.cg(rp, ci, v, b, tol=1e-12, maxit=10)
    assert info["iters"] == 1
    np.testing.assert_allclose(x, b / mu, rtol=0, atol=1e-14)


def test_cg_a_norm_error_bound():
    n, kappa = 48, 400.0
    A = _spd(n, kappa, 9)
    rp, ci, v = _dense_to_csr(A)
    b = np.random.default_rng(9).standard_normal(n)
    xs = np.linalg.solve(A, b)
    e0 = math.sqrt(xs @ A @ xs)
    rate = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
    for k in range(1, 25):
        xk, info = oracle.cg(rp, ci, v, b, tol=0.0, maxit=k)
        assert info["iters"] == k
        ek = xk - xs
        assert math.sqrt(ek @ A @ ek) <= 2 * rate ** k * e0 * (1 + 1e-9)


def test_cg_residuals_mutually_orthogonal():
    n = 30
    A = _spd(n, 30.0, 11)
    rp, ci, v = _dense_to_csr(A)
    b = np.random.default_rng(11).standard_normal(n)
    rs = []
    for k in range(6):
        xk, _ = oracle.cg(rp, ci, v, b, tol=0.0, maxit=k)
        rs.append(b - A @ xk)
    for a in range(6):
        for c in range(a + 1, 6):
            cosang = abs(rs[a] @ rs[c]) / (np.linalg.norm(rs[a]) * np.linalg.norm(rs[c]))
            assert cosang < 1e-9


def test_jacobi_pcg_on_diagonal_is_one_step():
    d = np.linspace(1.0, 1000.0, 25)
    rp, ci, v = _dense_to_csr(np.diag(d))
    b = np.random.default_rng(1).standard_normal(25)
    x, info = oracle.cg(rp, ci, v, b, tol=1e-14, maxit=10, precond="jacobi")
    assert info["iters"] == 1
    np.testing.assert_allclose(x, b / d, rtol=1e-15)


def test_jacobi_pcg_matches_direct_on_random_spd():
    rp, ci, v = workloads.random_spd_csr(300, seed=3)
    A = workloads.csr_to_dense(rp, ci, v, 300)
    assert np.allclose(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0
    b = workloads.rhs_uniform(300, seed=3)
    x, info = oracle.cg(rp, ci, v, b, tol=1e-12, maxit=500, precond="jacobi")
    assert info["status"] == "converged"
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-11)


def test_spmv_and_dot_against_dense():
    rp, ci, v = workloads.random_spd_csr(200, seed=4)
    A = workloads.csr_to_dense(rp, ci, v, 200)
    x = np.random.default_rng(4).standard_normal(200)
    np.testing.assert_allclose(oracle.spmv(rp, ci, v, x), A @ x, rtol=1e-13, atol=1e-12)
    assert abs(oracle.dot(x, x) - math.fsum(x * x)) < 1e-12


def test_cg_edge_cases():
    rp, ci, v = workloads.poisson_csr(6, 2)
    x, info = oracle.cg(rp, ci, v, np.zeros(36))
    assert info["status"] == "converged" and info["iters"] == 0 and not x.any()
    b = np.ones(36)
    x, info = oracle.cg(rp, ci, v, b, maxit=0)
    assert info["status"] == "not_converged" and not x.any()
    A = np.diag([1.0, -2.0, 3.0])
    rp2, ci2, v2 = _dense_to_csr(A)
    _, info = oracle.cg(rp2, ci2, v2, np.array([0.0, 1.0, 0.0]))
    assert info["status"] == "breakdown"


def test_poisson_generator_matches_benchmark_sizes():
    rp, ci, v = workloads.poisson_csr(128, 3)
    assert rp.size - 1 == 2_097_152 and ci.size == 14_581_760
    small = workloads.poisson_csr(5, 3)
    A = workloads.csr_to_dense(*small, 125)
    assert np.allclose(A, A.T) and np.all(np.diag(A) == 6.0)
    assert np.allclose(A.sum(axis=1)[62], 0.0)          # interior row: 6 - 6 neighbours
