"""GPU tests of the batched CG (many systems in one persistent launch).

Each problem of a batch must be solved as the single-system solver solves
it: parity with the oracle per problem (same bar as the single solves; for
mixed precision an FP32 iteration count within max(5, 15%) and a replacement
count within max(2, 20%), as the FP32
recurrences round differently on the GPU, which fuses multiply-adds), the
result of a problem independent of the rest of the batch and of the order of
the problems (bitwise, for the same workgroup count), bitwise equality with
the single-system persistent solver where both use one workgroup, and a plan
that re-runs (as a HIP graph launch) with refilled right-hand sides.
"""
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


def _true_relres(rp, ci, v, b, x):
    import scipy.sparse as sp
    n = rp.size - 1
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    return float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))


def _problems(sides, seed=0, extra_random=0):
    probs = []
    for j, s in enumerate(sides):
        rp, ci, v = workloads.poisson_csr(int(s), 2)
        probs.append((rp, ci, v, workloads.rhs_normal(rp.size - 1, seed=seed + j)))
    for j in range(extra_random):
        rp, ci, v = workloads.random_spd_csr(3000 + 1000 * j, seed=40 + j)
        probs.append((rp, ci, v, workloads.rhs_uniform(rp.size - 1, seed=60 + j)))
    return probs


def _to_dev(pk, probs):
    As = [pk.CsrMatrix(rp, ci, v) for rp, ci, v, _ in probs]
    bs = [to_dev(b) for *_, b in probs]
    xs = [to_dev(np.zeros_like(b)) for *_, b in probs]
    return As, bs, xs


@pytest.mark.parametrize("precision", [None, "mixed"])
@pytest.mark.parametrize("precond", [None, "jacobi"])
def test_batched_matches_oracle(pk, precision, precond):
    sides = workloads.lognormal_sides(10, lo=8, hi=72, seed=1)
    probs = _problems(sides, extra_random=2)
    As, bs, xs = _to_dev(pk, probs)
    tol = 1e-9
    print(f"batched CG {len(probs)} problems precision={precision} precond={precond}", flush=True)
    infos = pk.cg_solve_batched(As, bs, xs, tol=tol, maxit=5000, precond=precond, precision=precision)
    torch.cuda.synchronize()
    for (rp, ci, v, b), x, info in zip(probs, xs, infos):
        xh = x.cpu().numpy()
        assert info["status"] == "converged"
        assert _true_relres(rp, ci, v, b, xh) <= tol * 1.001
        if precision == "mixed":
            _, oi = oracle.cg_mixed(rp, ci, v, b, tol=tol, maxit=5000, precond=precond)
            assert abs(info["outer"] - oi["outer"]) <= max(2, math.ceil(0.2 * oi["outer"]))
            assert abs(info["iters"] - oi["iters"]) <= max(5, math.ceil(0.15 * oi["iters"]))
        else:
            _, oi = oracle.cg(rp, ci, v, b, tol=tol, maxit=5000, precond=precond)
            assert abs(info["iters"] - oi["iters"]) <= max(2, math.ceil(0.02 * oi["iters"]))
        xs_ref, _ = oracle.cg(rp, ci, v, b, tol=1e-13, maxit=20000, precond=precond)
        kappa = 4.0 * (int(round(math.sqrt(rp.size - 1))) + 1) ** 2 / math.pi ** 2 if rp.size > 1 else 1.0
        assert np.linalg.norm(xh - xs_ref) / np.linalg.norm(xs_ref) <= max(kappa, 1e3) * tol


@pytest.mark.parametrize("precision", [None, "mixed"])
def test_problem_results_independent_of_batch_and_order(pk, precision):
    sides = [40, 9, 63, 17, 30, 52, 12]
    probs = _problems(sides, seed=5)
    As, bs, xs = _to_dev(pk, probs)
    finfo = pk.cg_solve_batched(As, bs, xs, tol=1e-10, precision=precision)
    full = [x.cpu().numpy() for x in xs]
    perm = [3, 0, 6, 2, 5, 1, 4]
    As2, bs2, xs2 = _to_dev(pk, [probs[i] for i in perm])
    pk.cg_solve_batched(As2, bs2, xs2, tol=1e-10, precision=precision)
    for j, i in enumerate(perm):
        np.testing.assert_array_equal(xs2[j].cpu().numpy(), full[i])
    # alone in a batch, and through the single-system solver (one workgroup each)
    for i in (0, 2):
        A1, b1, x1 = _to_dev(pk, [probs[i]])
        pk.cg_solve_batched(A1, b1, x1, tol=1e-10, precision=precision)
        np.testing.assert_array_equal(x1[0].cpu().numpy(), full[i])
        xs1 = to_dev(np.zeros(probs[i][3].size))
        info = pk.cg_solve(A1[0], b1[0], xs1, tol=1e-10, precision=precision)
        if info["wgs"] == finfo[i]["wgs"]:
            np.testing.assert_array_equal(xs1.cpu().numpy(), full[i])


def test_grouped_problem_in_batch(pk):
    """A problem big enough to get several workgroups of its own."""
    probs = _problems([256, 12, 20, 16], seed=7)
    As, bs, xs = _to_dev(pk, probs)
    infos = pk.cg_solve_batched(As, bs, xs, tol=1e-10, precision="mixed")
    assert infos[0]["wgs"] >= 2
    for (rp, ci, v, b), x, info in zip(probs, xs, infos):
        assert info["status"] == "converged"
        assert _true_relres(rp, ci, v, b, x.cpu().numpy()) <= 1e-10 * 1.001


def test_plan_reruns_with_new_rhs(pk):
    probs = _problems([24, 33, 15, 48], seed=11)
    As, bs, xs = _to_dev(pk, probs)
    plan = pk.CgBatch(As, bs, xs, tol=1e-10, precision="mixed")
    print(f"batch plan graph={plan.has_graph()}", flush=True)
    for rep in range(3):
        rhs = [workloads.rhs_normal(b.numel(), seed=100 * rep + j) for j, b in enumerate(bs)]
        for b, r in zip(bs, rhs):
            b.copy_(torch.from_numpy(r))
        for x in xs:
            x.zero_()
        plan.run()
        infos = plan.results()
        torch.cuda.synchronize()
        for (rp, ci, v, _), r, x, info in zip(probs, rhs, xs, infos):
            assert info["status"] == "converged"
            assert _true_relres(rp, ci, v, r, x.cpu().numpy()) <= 1e-10 * 1.001
        # eager work on the same stream between replays
        torch.cuda.synchronize()
        _ = (bs[0] * 2).sum().item()
    plan.close()


def test_batched_edge_cases(pk):
    assert pk.cg_solve_batched([], [], []) == []
    rp, ci, v = workloads.poisson_csr(10, 2)
    n = rp.size - 1
    A = pk.CsrMatrix(rp, ci, v)
    z = pk.CsrMatrix(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    b0 = to_dev(np.zeros(n))
    b1 = to_dev(workloads.rhs_normal(n, seed=2))
    e = to_dev(np.zeros(0))
    xs = [to_dev(np.ones(n)), to_dev(np.zeros(n)), to_dev(np.zeros(0))]
    infos = pk.cg_solve_batched([A, A, z], [b0, b1, e], xs, tol=1e-12)
    assert infos[0]["status"] == "converged" and infos[0]["iters"] == 0
    assert np.all(xs[0].cpu().numpy() == 0)
    assert infos[1]["status"] == "converged"
    assert infos[2]["status"] == "converged" and infos[2]["iters"] == 0
    with pytest.raises(pk.PerksError):
        pk.cg_solve_batched([A], [b1], [xs[1]], tol=-1.0)
