"""Training of the learned preconditioner on the GPU (small end-to-end run).

Pairs harvested from the persistent PCG on seeded diffusion problems; Adam
through the library's kernels must reduce the loss substantially; the
trained network inside FCG must still reach the tolerance.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    import paper_2204_02064_amd as pk
    pk.lib()
    return pk


def test_harvest_train_and_apply(pk):
    from paper_2204_02064_amd import learned
    n = 32
    probs = [workloads.diffusion_problem_torch(n, seed=s) for s in range(8)]
    X, T = learned.harvest_pairs(probs, iters=(1, 2, 4, 8, 16, 32))
    assert X.shape[1:] == (n, n, 2) and T.shape[1:] == (n, n) and X.shape[0] >= 40
    assert torch.isfinite(X).all() and torch.isfinite(T).all()
    # input channel 0 has unit rms by construction
    rms = torch.sqrt(torch.mean(X[..., 0] ** 2, dim=(1, 2)))
    assert torch.allclose(rms, torch.ones_like(rms), atol=1e-5)
    params, losses = learned.train(X, T, epochs=30, batch=8, lr=2e-3, seed=0)
    first, last = np.mean(losses[:5]), np.mean(losses[-5:])
    print(f"loss {first:.4f} -> {last:.4f} over {len(losses)} epochs", flush=True)
    assert last < 0.6 * first
    rp, ci, v, lk, f = workloads.diffusion_problem_torch(n, seed=1000)
    A = pk.CsrMatrix(rp, ci, v)
    x = torch.zeros_like(f)
    info = pk.fcg_solve(A, f, x, n, n, params=params, logk=lk, tol=1e-8, stall=20)
    assert info["status"] == "converged"


def test_energy_loss_training_reduces_the_a_norm_error(pk):
    from paper_2204_02064_amd import learned
    n = 32
    seeds = range(6)
    probs = [workloads.diffusion_problem_torch(n, seed=s) for s in seeds]
    planes = torch.stack([workloads.diffusion_planes_torch(torch.exp(workloads.grf_log_k_torch(n, seed=s)))
                          for s in seeds]).to(torch.float32)
    X, T, field = learned.harvest_pairs(probs, iters=(1, 2, 4, 8, 16, 32), with_field=True)
    assert field.shape[0] == X.shape[0] and int(field.max()) == len(seeds) - 1
    params, losses = learned.train(X, T, epochs=30, batch=8, lr=2e-3, seed=1, planes=planes, field=field)
    first, last = np.mean(losses[:5]), np.mean(losses[-5:])
    print(f"energy loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < first


def test_pairs_match_the_oracle(pk):
    """perks_nn_make_pairs against oracle.nn.make_pairs on the same captured
    iterates (copied to the host): FP64 arithmetic rounded to FP32 on both
    sides, rms summed in different orders (a relative difference of a few
    FP64 ulps), so FP32 values agree to one FP32 rounding step."""
    import oracle.nn as onn
    n = 48
    rp, ci, v, lk, f = workloads.diffusion_problem_torch(n, seed=5)
    A = pk.CsrMatrix(rp, ci, v)
    xstar = torch.zeros_like(f)
    pk.cg_solve(A, f, xstar, tol=1e-12, maxit=20000, precond="jacobi")
    x = torch.zeros_like(f)
    iters = (1, 2, 4, 8, 16, 32, 64, 128, 100000)   # the last one is never reached
    _, xc, rc = pk.cg_solve_capture(A, f, x, iters, tol=1e-12, maxit=20000, precond="jacobi")
    X, T = pk.nn_make_pairs(A, xstar, lk.contiguous(), xc, rc, n, n)
    rph, cih, vh = rp.cpu().numpy(), ci.cpu().numpy(), v.cpu().numpy()
    diag = np.zeros(n * n)
    for i in range(n * n):
        for k in range(rph[i], rph[i + 1]):
            if cih[k] == i:
                diag[i] += vh[k]
    xs = [a.reshape(n, n) for a in xc.cpu().numpy()]
    rs = [a.reshape(n, n) for a in rc.cpu().numpy()]
    oin, otg = onn.make_pairs(diag.reshape(n, n), xstar.cpu().numpy().reshape(n, n), lk.cpu().numpy(), xs, rs)
    assert X.shape[0] == oin.shape[0] == len(iters) - 1
    np.testing.assert_allclose(X.cpu().numpy(), oin.astype(np.float32), rtol=2 ** -22, atol=0)
    np.testing.assert_allclose(T.cpu().numpy(), otg.astype(np.float32), rtol=2 ** -22, atol=1e-30)


def test_trained_network_against_jacobi_pcg(pk):
    """The measured effect of the learned preconditioner: a network trained
    with the energy loss on pairs from 48 seeded 64^2 fields, applied inside
    FCG on three held-out 64^2 fields, against Jacobi-PCG at the same
    tolerance.  It is not a reliable gain: on one field it needs about half
    of Jacobi-PCG's iterations, on the other two it falls back to the Jacobi
    step often and needs 1.6-2.4 times as many, until the stall rule hands
    the solve to Jacobi-PCG (the ratios are printed).  Pinned here: every
    held-out solve reaches the tolerance, and the fallback and the stall rule
    bound the loss to three times Jacobi-PCG's iterations."""
    from paper_2204_02064_amd import learned
    n = 64
    seeds = range(48)
    probs = [workloads.diffusion_problem_torch(n, seed=s) for s in seeds]
    planes = torch.stack([workloads.diffusion_planes_torch(torch.exp(workloads.grf_log_k_torch(n, seed=s)))
                          for s in seeds]).to(torch.float32)
    X, T, field = learned.harvest_pairs(probs, with_field=True)
    params, _ = learned.train(X, T, epochs=3, batch=16, lr=1e-3, seed=0, planes=planes, field=field)
    ratios = []
    for s in (10000, 10001, 10002):
        rp, ci, v, lk, f = workloads.diffusion_problem_torch(n, seed=s)
        A = pk.CsrMatrix(rp, ci, v)
        x = torch.zeros_like(f)
        ij = pk.cg_solve(A, f, x, tol=1e-8, maxit=20000, precond="jacobi")
        x.zero_()
        inet = pk.fcg_solve(A, f, x, n, n, params=params, logk=lk, tol=1e-8, maxit=20000, stall=20)
        assert ij["status"] == "converged" and inet["status"] == "converged"
        assert inet["relres_true"] <= 1e-8 * 1.001
        ratios.append(inet["iters"] / ij["iters"])
        print(f"seed {s}: Jacobi-PCG {ij['iters']} it, FCG+net {inet['iters']} it (fallbacks "
              f"{inet['fallbacks']}, switched at {inet['switched_at']})", flush=True)
    print("FCG+net / Jacobi-PCG iterations:", [round(r, 3) for r in ratios], flush=True)
    assert max(ratios) <= 3.0, ratios
