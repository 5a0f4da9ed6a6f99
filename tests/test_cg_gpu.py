"""GPU parity of the persistent and host-looped CG solvers against the oracle.

Several iterates are correct when the rounding order differs, so parity is:
the true relative residual ||b - A x|| / ||b|| (recomputed on the host from
the returned x) meets tol, the returned x agrees with the oracle's solution
within kappa * tol, and the iteration count is within max(2, 2%) of the
oracle's.
"""
import functools
import math

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    import paper_2204_02064_amd as pk
    pk.lib()
    return pk


def _dense_to_csr(A):
    rowptr = [0]; cols = []; vals = []
    for i in range(A.shape[0]):
        nz = np.nonzero(A[i])[0]
        cols.extend(nz.tolist()); vals.extend(A[i, nz].tolist())
        rowptr.append(len(cols))
    return np.array(rowptr, np.int32), np.array(cols, np.int32), np.array(vals)


def _spd(n, kappa, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * np.geomspace(1.0, kappa, n)) @ Q.T
    return 0.5 * (A + A.T)


def _true_relres(rp, ci, v, b, x):
    import scipy.sparse as sp
    n = rp.size - 1
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    return float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))


def _solve(pk, rp, ci, v, b, tol, maxit=5000, precond=None, baseline=False, x0=None, spmv="auto"):
    A = pk.CsrMatrix(rp, ci, v, spmv=spmv)
    bd = to_dev(b)
    xd = to_dev(np.zeros_like(b) if x0 is None else x0)
    fn = pk.cg_solve_baseline if baseline else pk.cg_solve
    info = fn(A, bd, xd, tol=tol, maxit=maxit, precond=precond)
    torch.cuda.synchronize()
    return xd.cpu().numpy(), info


def _iters_close(a, b):
    return abs(a - b) <= max(2, math.ceil(0.02 * b))


@pytest.mark.parametrize("baseline", [False, True])
@pytest.mark.parametrize("n,kappa,seed", [(8, 10.0, 1), (40, 50.0, 2), (64, 100.0, 3)])
def test_tiny_spd_matches_direct_solve(pk, baseline, n, kappa, seed):
    A = _spd(n, kappa, seed)
    rp, ci, v = _dense_to_csr(A)
    b = np.random.default_rng(seed).uniform(-1, 1, n)
    x, info = _solve(pk, rp, ci, v, b, 1e-12, maxit=500, baseline=baseline)
    assert info["status"] == "converged"
    xs = oracle.chol_solve(A, b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-11
    _, oinfo = oracle.cg(rp, ci, v, b, tol=1e-12, maxit=500)
    assert _iters_close(info["iters"], oinfo["iters"])


@pytest.mark.parametrize("baseline", [False, True])
@pytest.mark.parametrize("precond", [None, "jacobi"])
@pytest.mark.parametrize("case", ["poisson2d", "poisson3d", "random"])
def test_matches_oracle(pk, baseline, precond, case):
    if case == "poisson2d":
        rp, ci, v = workloads.poisson_csr(90, 2)
    elif case == "poisson3d":
        rp, ci, v = workloads.poisson_csr(24, 3)
    else:
        rp, ci, v = workloads.random_spd_csr(30000, seed=1)
    n = rp.size - 1
    b = workloads.rhs_uniform(n, seed=0)
    x, info = _solve(pk, rp, ci, v, b, 1e-10, precond=precond, baseline=baseline)
    xo, oinfo = oracle.cg(rp, ci, v, b, tol=1e-10, maxit=5000, precond=precond)
    assert info["status"] == "converged" and oinfo["status"] == "converged"
    assert _true_relres(rp, ci, v, b, x) <= 1e-10
    assert abs(info["relres_true"] - _true_relres(rp, ci, v, b, x)) <= 1e-12
    assert _iters_close(info["iters"], oinfo["iters"]), (info["iters"], oinfo["iters"])
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-6


def test_m_distinct_eigenvalues_take_m_steps(pk):
    m, n = 4, 3000
    eig = np.array([1.0 + 2.5 * (i % m) for i in range(n)])
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    b = np.random.default_rng(0).uniform(0.5, 1.5, n)
    x, info = _solve(pk, rp, ci, eig, b, 1e-13)
    assert info["iters"] == m
    np.testing.assert_allclose(x, b / eig, rtol=1e-12)


def test_edge_cases(pk):
    rp, ci, v = workloads.poisson_csr(30, 2)
    n = rp.size - 1
    x, info = _solve(pk, rp, ci, v, np.zeros(n), 1e-10)
    assert info["status"] == "converged" and info["iters"] == 0 and not x.any()
    x, info = _solve(pk, rp, ci, v, np.ones(n), 1e-10, maxit=0)
    assert info["status"] == "not_converged" and not x.any()
    d = np.tile(np.array([1.0, -2.0, 3.0]), 700)
    rpd = np.arange(d.size + 1, dtype=np.int32)
    b = np.zeros(d.size); b[1] = 1.0
    _, info = _solve(pk, rpd, rpd[:-1].copy(), d, b, 1e-10)
    assert info["status"] == "breakdown"


def test_warm_start_continues(pk):
    rp, ci, v = workloads.poisson_csr(60, 2)
    b = workloads.rhs_uniform(rp.size - 1, seed=4)
    x1, i1 = _solve(pk, rp, ci, v, b, 1e-10, maxit=40)
    assert i1["status"] == "not_converged" and i1["iters"] == 40
    x2, i2 = _solve(pk, rp, ci, v, b, 1e-10, x0=x1)
    assert i2["status"] == "converged"
    assert _true_relres(rp, ci, v, b, x2) <= 1e-10


def test_full_size_poisson_128(pk):
    # the 128^3 benchmark system: n = 2,097,152, nnz = 14,581,760
    rp, ci, v = workloads.poisson_csr(128, 3)
    b = workloads.rhs_uniform(rp.size - 1, seed=0)
    x, info = _solve(pk, rp, ci, v, b, 1e-10)
    assert info["status"] == "converged"
    assert _true_relres(rp, ci, v, b, x) <= 1e-10
    # CG on this system needs at most the sqrt(kappa) bound: ~975 iterations
    assert info["iters"] <= 1000
    xb, ib = _solve(pk, rp, ci, v, b, 1e-10, baseline=True)
    assert ib["status"] == "converged" and _iters_close(info["iters"], ib["iters"])
    # the oracle's CG on the same system (about 540 iterations of a 14.6M
    # nonzero SpMV in plain C: some seconds on the host)
    xo, oi = oracle.cg(rp, ci, v, b, tol=1e-10, maxit=5000)
    assert oi["status"] == "converged"
    assert _iters_close(info["iters"], oi["iters"]), (info["iters"], oi["iters"])
    # both iterates have relative residual <= 1e-10, so each is within
    # kappa * 1e-10 of the solution (kappa = 12 / (12 sin^2(pi / 258)) ~ 6.7e3)
    kappa = 1.0 / math.sin(math.pi / 258) ** 2
    assert np.linalg.norm(x - xo) <= 2 * kappa * 1e-10 * np.linalg.norm(xo)


def test_baseline_check_every_delays_stop_by_less_than_the_interval(pk):
    rp, ci, v = workloads.poisson_csr(20, 3)
    b = workloads.rhs_uniform(rp.size - 1, seed=4)
    A = pk.CsrMatrix(rp, ci, v)
    bd = to_dev(b)
    its = {}
    for ce in (1, 8):
        x = to_dev(np.zeros_like(b))
        info = pk.cg_solve_baseline(A, bd, x, tol=1e-10, maxit=5000, check_every=ce)
        assert info["status"] == "converged"
        its[ce] = info["iters"]
    assert its[1] <= its[8] <= its[1] + 7


@functools.lru_cache(maxsize=1)
def _random_million():
    rp, ci, v = workloads.random_spd_csr(1 << 20, seed=0)
    b = workloads.rhs_uniform(rp.size - 1, seed=0)
    _, oinfo = oracle.cg(rp, ci, v, b, tol=1e-10, maxit=5000, precond="jacobi")
    return rp, ci, v, b, oinfo


@pytest.mark.parametrize("baseline", [False, True])
def test_random_spd_one_million_rows_jacobi(pk, baseline):
    """n = 2^20, mean row length 20.6: the baseline SpMV then runs 32 lanes per
    row and more blocks than the vector kernels, and its partial sums must be
    sized for those (they once overran into the solver's vectors here)."""
    rp, ci, v, b, oinfo = _random_million()
    x, info = _solve(pk, rp, ci, v, b, 1e-10, precond="jacobi", baseline=baseline)
    assert info["status"] == "converged" and oinfo["status"] == "converged"
    assert _true_relres(rp, ci, v, b, x) <= 1e-10
    assert _iters_close(info["iters"], oinfo["iters"]), (info["iters"], oinfo["iters"])


# ---------------------------------------------------------------------------
# Merge-path SpMV (perks_csr.spmv = 2) and the vectors-in-memory sliced ELL
# (spmv = 1): the same parity bar.  Sizes give every workgroup several tiles of
# merge-path chunks (the random matrix: about 1,000 rows and 21,000 nonzeros
# per workgroup, 1024 threads x 8 items per tile) and rows that span chunks,
# threads and tiles (the longest random rows have up to 200 entries).

@pytest.mark.parametrize("spmv", ["merge", "sell"])
@pytest.mark.parametrize("precond", [None, "jacobi"])
@pytest.mark.parametrize("case", ["poisson2d", "poisson3d", "random", "random_big"])
def test_spmv_layouts_match_oracle(pk, spmv, precond, case):
    if case == "poisson2d":
        rp, ci, v = workloads.poisson_csr(90, 2)
    elif case == "poisson3d":
        rp, ci, v = workloads.poisson_csr(24, 3)
    elif case == "random":
        rp, ci, v = workloads.random_spd_csr(30000, seed=1)
    else:
        rp, ci, v = workloads.random_spd_csr(100000, seed=2)
    if case == "random_big" and precond is None:
        precond = "jacobi"   # unpreconditioned CG needs thousands of iterations here
    n = rp.size - 1
    b = workloads.rhs_uniform(n, seed=0)
    print(f"spmv {spmv} {case} precond {precond}", flush=True)
    x, info = _solve(pk, rp, ci, v, b, 1e-10, precond=precond, spmv=spmv)
    xo, oinfo = oracle.cg(rp, ci, v, b, tol=1e-10, maxit=5000, precond=precond)
    assert info["status"] == "converged" and oinfo["status"] == "converged"
    assert _true_relres(rp, ci, v, b, x) <= 1e-10
    assert _iters_close(info["iters"], oinfo["iters"]), (info["iters"], oinfo["iters"])
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-6


def test_merge_path_spmv_single_iteration_is_the_product(pk):
    """One CG iteration from x0 = 0 on a diagonal-dominant random matrix
    gives x1 = alpha r0 with alpha = (r.r) / (r.Ar): the merge-path SpMV's A r
    enters only through alpha, so x1 matches the oracle's product-based value
    to rounding; the rows include ones longer than a chunk and a tile."""
    rp, ci, v = workloads.random_spd_csr(50000, seed=3, max_degree=200)
    n = rp.size - 1
    b = workloads.rhs_uniform(n, seed=1)
    x, info = _solve(pk, rp, ci, v, b, 1e-30, maxit=1, spmv="merge")
    assert info["iters"] == 1
    Ab = oracle.spmv(rp, ci, v, b)
    alpha = float(np.dot(b, b) / np.dot(b, Ab))
    np.testing.assert_allclose(x, alpha * b, rtol=1e-13, atol=0)


@pytest.mark.parametrize("precond", [None, "jacobi"])
def test_merge_path_mixed_precision(pk, precond):
    rp, ci, v = workloads.random_spd_csr(30000, seed=1)
    n = rp.size - 1
    b = workloads.rhs_uniform(n, seed=0)
    A = pk.CsrMatrix(rp, ci, v, spmv="merge")
    bd, xd = to_dev(b), to_dev(np.zeros(n))
    info = pk.cg_solve(A, bd, xd, tol=1e-8, maxit=5000, precond=precond, precision="mixed")
    torch.cuda.synchronize()
    assert info["status"] == "converged"
    assert _true_relres(rp, ci, v, b, xd.cpu().numpy()) <= 1e-8
