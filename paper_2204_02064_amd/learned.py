"""Training of the learned preconditioner from pairs the persistent CG produces.

Pairs: for a diffusion problem A x = f with log-permeability log k, the
persistent Jacobi-preconditioned CG is run to a tight tolerance, with
snapshots of its iterate x_k and residual r_k after k = 1, 2, 4, 8, ...
iterations; its final iterate is x*; each snapshot gives the network input
[r_k / rms(r_k), log k] and the target (x* - x_k - D^-1 r_k) / rms(r_k): the
preconditioner returns D^-1 r + rms(r) net(...), so the network's part of the
error e_k = x* - x_k is what the Jacobi step leaves of it.

Training: Adam over mini-batches of pairs, the whole loop in the library
(perks_nn_train: seeded shuffles, batch gathers, forward and backward passes,
Adam steps).  Two losses: the mean squared error against that target
(perks_nn_loss_grad), or the error of the preconditioned residual
z = D^-1 r + rms(r) net(...) in the energy norm of the problem's operator,
||z - e||_A^2 up to a constant (perks_nn_energy_grad, Jacobi form):
the quantity a CG step minimises, dominated neither by the smooth error
components a local network cannot represent nor by the scale of e.
"""
import numpy as np

from . import CsrMatrix, cg_solve_capture, nn_make_pairs, nn_pack_params, nn_train

CAPTURE_ITERS = (1, 2, 4, 8, 16, 32, 64, 128, 256, 512)


def harvest_pairs(problems, iters=CAPTURE_ITERS, tol=1e-12, maxit=20000, with_field=False):
    """problems: iterable of (rowptr, colind, values, log_k [n, n], f) torch
    tensors on the device.  Returns (inputs [P, n, n, 2] float32, targets
    [P, n, n] float32) device tensors, and with ``with_field`` also the index
    of each pair's problem (int64 [P]).  Every step runs in the library: the
    Jacobi-PCG solve with captured iterates (its final iterate is x*) and the
    pair formation (perks_nn_make_pairs); here only allocation and
    concatenation."""
    import torch
    xs, ts, fi = [], [], []
    for pid, (rp, ci, v, lk, f) in enumerate(problems):
        n = lk.shape[0]
        A = CsrMatrix(rp, ci, v)
        xstar = torch.zeros_like(f)
        info, xc, rc = cg_solve_capture(A, f, xstar, iters, tol=tol, maxit=maxit, precond="jacobi")
        X, T = nn_make_pairs(A, xstar, lk.contiguous(), xc, rc, n, n)
        xs.append(X)
        ts.append(T)
        fi.extend([pid] * X.shape[0])
    X, T = torch.cat(xs), torch.cat(ts)
    if with_field:
        return X, T, torch.tensor(fi, dtype=torch.int64, device=X.device)
    return X, T


def init_params(seed=0):
    """He-uniform weights (fan-in 9 * inputs), zero biases, padded float32 vector."""
    rng = np.random.default_rng(seed)
    layers = []
    for ci, co in [(2, 16), (16, 16), (16, 16), (16, 16), (16, 16), (16, 1)]:
        bound = np.sqrt(6.0 / (9 * ci))
        layers.append((rng.uniform(-bound, bound, (co, ci, 3, 3)).astype(np.float32), np.zeros(co, np.float32)))
    return nn_pack_params(layers)


def train(inputs, targets, epochs=4, batch=16, lr=1e-3, seed=0, params=None, log=None, planes=None, field=None):
    """Adam over (inputs, targets) in the library (perks_nn_train); returns
    (params, mean loss per epoch).  With ``planes`` ([F, 5, n, n] float32, the
    operator of each problem) and ``field`` (problem index per pair) the
    energy-norm loss is used."""
    import torch
    dev = inputs.device
    p = torch.from_numpy(init_params(seed)).to(dev) if params is None else params.clone()
    fld = field.to(torch.int32).contiguous() if field is not None else None
    losses, _, _, _ = nn_train(p, inputs.contiguous(), epochs, batch, lr=lr, seed=seed,
                               target=None if planes is not None else targets.contiguous(),
                               planes=planes.contiguous() if planes is not None else None, field=fld)
    if log:
        for ep, l in enumerate(losses):
            log(f"epoch {ep}: loss {l:.4e}")
    return p, losses
