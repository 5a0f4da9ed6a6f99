"""Pins of the learned-preconditioner oracle: network, training step, FCG,
and the diffusion inputs (no GPU).

The convolution is pinned to brute-force loops and to an impulse response
with asymmetric weights; the backward pass to float64 central finite
differences and to the adjoint identity of the convolution; bf16 rounding to
hand-computed values; the Adam step to its closed form on the first step;
FCG to preconditioned CG (fixed Jacobi preconditioner), to one-step
convergence with the exact inverse, to CG with a network that is the
identity, and to its fallback and switch rules; the diffusion matrix to the
5-point Laplacian for k = 1.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import fcg as ofcg
from oracle import nn
import workloads


def _rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return [(rng.uniform(-scale, scale, (co, ci, 3, 3)), rng.uniform(-0.1, 0.1, co))
            for ci, co, _ in nn.LAYERS]


def test_flops_per_pixel():
    assert nn.FLOPS_PER_PIXEL == 19296


def test_conv_matches_brute_force_loops():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 5, 4))
    w = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    y = nn.conv3x3(x, w, b)
    ref = np.zeros((2, 5, 4))
    for o in range(2):
        for yy in range(5):
            for xx in range(4):
                s = b[o]
                for i in range(3):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            if 0 <= yy + dy < 5 and 0 <= xx + dx < 4:
                                s += w[o, i, 1 + dy, 1 + dx] * x[i, yy + dy, xx + dx]
                ref[o, yy, xx] = s
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)


def test_conv_impulse_response_orientation():
    x = np.zeros((1, 5, 5))
    x[0, 2, 2] = 1.0
    w = np.arange(9, dtype=np.float64).reshape(1, 1, 3, 3)
    y = nn.conv3x3(x, w, [0.0])[0]
    # output at (2 - dy, 2 - dx) sees the impulse through tap (dy, dx)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            assert y[2 - dy, 2 - dx] == w[0, 0, 1 + dy, 1 + dx]
    assert y.sum() == w.sum()


def test_conv_backward_is_the_adjoint():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 6, 7))
    w = rng.standard_normal((3, 4, 3, 3))
    dy = rng.standard_normal((3, 6, 7))
    dx, _, _ = nn.conv3x3_backward(x, w, dy)
    lhs = np.sum(nn.conv3x3(x, w, np.zeros(3)) * dy)
    assert abs(lhs - np.sum(x * dx)) <= 1e-12 * abs(lhs) + 1e-12


def test_network_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    params = _rand_params(3)
    x = rng.standard_normal((2, 5, 6))
    t = rng.standard_normal((1, 5, 6))
    loss, grads = nn.loss_and_grads(params, [x], [t])
    h = 1e-6
    for layer, (o, i, ty, tx) in [(0, (3, 1, 0, 2)), (2, (7, 11, 1, 1)), (5, (0, 9, 2, 0))]:
        w, b = params[layer]
        wp, wm = w.copy(), w.copy()
        wp[o, i, ty, tx] += h
        wm[o, i, ty, tx] -= h
        lp, _ = nn.loss_and_grads([(wp, b) if j == layer else params[j] for j in range(6)], [x], [t])
        lm, _ = nn.loss_and_grads([(wm, b) if j == layer else params[j] for j in range(6)], [x], [t])
        fd = (lp - lm) / (2 * h)
        g = grads[layer][0][o, i, ty, tx]
        assert abs(fd - g) <= 1e-6 * max(abs(fd), 1e-3), (layer, fd, g)
    # a bias
    w, b = params[4]
    bp, bm = b.copy(), b.copy()
    bp[5] += h
    bm[5] -= h
    lp, _ = nn.loss_and_grads([(w, bp) if j == 4 else params[j] for j in range(6)], [x], [t])
    lm, _ = nn.loss_and_grads([(w, bm) if j == 4 else params[j] for j in range(6)], [x], [t])
    fd = (lp - lm) / (2 * h)
    assert abs(fd - grads[4][1][5]) <= 1e-6 * max(abs(fd), 1e-3)


def test_input_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    params = _rand_params(5)
    x = rng.standard_normal((2, 4, 4))
    out, cache = nn.forward(params, x)
    dout = rng.standard_normal(out.shape)
    _, dx = nn.backward(cache, dout)
    h = 1e-6
    for idx in [(0, 1, 2), (1, 3, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (np.sum(nn.forward(params, xp)[0] * dout) - np.sum(nn.forward(params, xm)[0] * dout)) / (2 * h)
        assert abs(fd - dx[idx]) <= 1e-6 * max(abs(fd), 1e-3)


def test_bf16_rounding_values():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20, -2.5, 0.0, 65504.0])
    exp = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -2.5, 0.0, 65536.0])
    np.testing.assert_array_equal(nn.bf16_round(vals), exp)
    assert np.isnan(nn.bf16_round(np.array([np.nan]))[0])


def test_adam_first_step_closed_form():
    params = [(np.full((2, 2, 3, 3), 0.5, np.float32), np.zeros(2, np.float32))]
    g = np.linspace(-1, 1, 36).reshape(2, 2, 3, 3)
    grads = [(g, np.array([0.25, -4.0]))]
    out, state = nn.adam_step(params, grads, nn.adam_init(params), lr=1e-3)
    exp = 0.5 - 1e-3 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(out[0][0], exp.astype(np.float32), rtol=1e-6)
    np.testing.assert_allclose(out[0][1], [-1e-3, 1e-3], rtol=1e-5)
    assert state[0] == 1


def _identity_params():
    """Layer 1: (r, -r) from centre taps +-1; hidden layers pass channels 0, 1;
    last: ch0 - ch1 = relu(r) - relu(-r) = r."""
    ps = []
    for li, (ci, co, _) in enumerate(nn.LAYERS):
        w = np.zeros((co, ci, 3, 3))
        if li == 0:
            w[0, 0, 1, 1], w[1, 0, 1, 1] = 1.0, -1.0
        elif li < 5:
            w[0, 0, 1, 1], w[1, 1, 1, 1] = 1.0, 1.0
        else:
            w[0, 0, 1, 1], w[0, 1, 1, 1] = 1.0, -1.0
        ps.append((w, np.zeros(co)))
    return ps


def test_identity_network_returns_r():
    rng = np.random.default_rng(6)
    r = rng.standard_normal((7, 9))
    z = nn.apply_preconditioner(_identity_params(), r, rng.standard_normal((7, 9)))
    np.testing.assert_allclose(z, r, rtol=1e-15, atol=1e-15)


def test_fcg_with_jacobi_equals_pcg():
    rp, ci, v, lk, f = workloads.diffusion_problem(24, seed=1)
    n = rp.size - 1
    dinv = 1.0 / np.array([v[rp[i]:rp[i + 1]][ci[rp[i]:rp[i + 1]] == i].sum() for i in range(n)])
    x, info = ofcg.fcg(rp, ci, v, f, lambda r: dinv * r, tol=1e-10)
    xp, ip = oracle.cg(rp, ci, v, f, tol=1e-10, precond="jacobi")
    assert info["status"] == "converged" and info["fallbacks"] == 0
    assert abs(info["iters"] - ip["iters"]) <= 1
    assert np.linalg.norm(x - xp) / np.linalg.norm(xp) <= 1e-8


def test_fcg_with_identity_network_equals_cg():
    rp, ci, v = workloads.poisson_csr(12, 2)
    b = workloads.rhs_normal(rp.size - 1, seed=3)
    lk = np.zeros((12, 12))
    params = _identity_params()
    x, info = ofcg.fcg(rp, ci, v, b, lambda r: nn.apply_preconditioner(params, r.reshape(12, 12), lk).ravel(),
                       tol=1e-10)
    xc, ic = oracle.cg(rp, ci, v, b, tol=1e-10)
    assert info["status"] == "converged" and info["fallbacks"] == 0
    assert abs(info["iters"] - ic["iters"]) <= 1
    assert np.linalg.norm(x - xc) / np.linalg.norm(xc) <= 1e-8


def test_fcg_with_exact_inverse_takes_one_step():
    rp, ci, v, _, f = workloads.diffusion_problem(6, seed=2)
    n = rp.size - 1
    A = workloads.csr_to_dense(rp, ci, v, n)
    Ainv = np.linalg.inv(A)
    x, info = ofcg.fcg(rp, ci, v, f, lambda r: Ainv @ r, tol=1e-10)
    assert info["iters"] == 1 and info["status"] == "converged"


def test_fcg_fallback_and_switch_rules():
    rp, ci, v, _, f = workloads.diffusion_problem(16, seed=4)
    # a preconditioner that always fails falls back to Jacobi on every step: PCG
    x1, i1 = ofcg.fcg(rp, ci, v, f, lambda r: -r, tol=1e-10)
    _, ip = oracle.cg(rp, ci, v, f, tol=1e-10, precond="jacobi")
    assert i1["fallbacks"] == i1["iters"] and abs(i1["iters"] - ip["iters"]) <= 1
    x2, i2 = ofcg.fcg(rp, ci, v, f, lambda r: None, tol=1e-10)
    assert i2["fallbacks"] == i2["iters"] and i2["status"] == "converged"
    # a useless preconditioner (random directions, sign chosen so <z, r> > 0)
    # makes no steady progress: the solve switches to Jacobi-PCG and converges
    rng = np.random.default_rng(0)

    def noise(r):
        z = rng.standard_normal(r.size)
        return z if z @ r > 0 else -z
    x3, i3 = ofcg.fcg(rp, ci, v, f, noise, tol=1e-10, maxit=4000, stall=10)
    assert i3["status"] == "converged" and i3["switched_at"] is not None


def test_diffusion_with_unit_k_is_poisson():
    n = 9
    rp, ci, v = workloads.diffusion_csr(np.ones((n + 2, n + 2)))
    prp, pci, pv = workloads.poisson_csr(n, 2)
    np.testing.assert_array_equal(rp, prp)
    np.testing.assert_array_equal(ci, pci)
    np.testing.assert_array_equal(v, pv)


def test_diffusion_matrix_symmetric_and_dominant():
    rp, ci, v, lk, _ = workloads.diffusion_problem(20, seed=7)
    n = rp.size - 1
    A = workloads.csr_to_dense(rp, ci, v, n)
    np.testing.assert_array_equal(A, A.T)
    off = np.abs(A).sum(1) - np.abs(np.diag(A))
    assert np.all(np.diag(A) >= off - 1e-12) and np.any(np.diag(A) > off + 1e-6)
    assert lk.shape == (20, 20)


def test_grf_pointwise_variance_is_sigma_squared():
    vals = np.array([workloads.grf_log_k(16, seed=s)[5, 7] for s in range(400)])
    assert abs(vals.var() - 1.0) < 0.2 and abs(vals.mean()) < 0.15
    assert abs(workloads.grf_log_k(16, seed=1, sigma=2.0)[3, 3] - 2 * workloads.grf_log_k(16, seed=1)[3, 3]) < 1e-12


def test_five_point_planes_apply_equals_csr_spmv():
    g = workloads.grf_log_k(9, seed=3)
    k = np.exp(g)
    rp, ci, v = workloads.diffusion_csr(k)
    planes = workloads.diffusion_planes(k)
    z = np.random.default_rng(0).standard_normal((9, 9))
    np.testing.assert_allclose(nn.apply_5pt(planes, z).ravel(), oracle.spmv(rp, ci, v, z.ravel()), rtol=1e-14,
                               atol=1e-13)


def test_energy_loss_is_the_a_norm_error_up_to_a_constant():
    """(z - e)'A(z - e) = L(z) * pixels + e'r for r = A e."""
    rng = np.random.default_rng(1)
    k = np.exp(workloads.grf_log_k(6, seed=2))
    planes = workloads.diffusion_planes(k)
    e = rng.standard_normal((6, 6))
    r = nn.apply_5pt(planes, e)
    params = _rand_params(8, scale=0.2)
    x = np.stack([r, rng.standard_normal((6, 6))])
    L, _ = nn.energy_loss_and_grads(params, [x], [planes])
    z = nn.forward(params, x)[0][0]
    d = z - e
    anorm = float(np.sum(d * nn.apply_5pt(planes, d)))
    assert abs(L * 36 + float(np.sum(e * r)) - anorm) <= 1e-10 * max(1.0, abs(anorm))


def test_energy_loss_gradients_match_finite_differences():
    rng = np.random.default_rng(5)
    params = _rand_params(9)
    k = np.exp(workloads.grf_log_k(5, seed=4))
    planes = [workloads.diffusion_planes(k)]
    x = [rng.standard_normal((2, 5, 5))]
    _, grads = nn.energy_loss_and_grads(params, x, planes)
    h = 1e-6
    for layer, idx in [(0, (2, 1, 1, 0)), (3, (5, 9, 2, 2)), (5, (0, 3, 1, 1))]:
        w, b = params[layer]
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        lp, _ = nn.energy_loss_and_grads([(wp, b) if j == layer else params[j] for j in range(6)], x, planes)
        lm, _ = nn.energy_loss_and_grads([(wm, b) if j == layer else params[j] for j in range(6)], x, planes)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grads[layer][0][idx]) <= 1e-6 * max(abs(fd), 1e-3)


def test_energy_loss_with_jacobi_term():
    """With the Jacobi term a zero network gives z = D^-1 r exactly; the loss
    then equals the energy functional of the Jacobi step."""
    rng = np.random.default_rng(2)
    k = np.exp(workloads.grf_log_k(7, seed=9))
    planes = workloads.diffusion_planes(k)
    zero = [(np.zeros_like(w), np.zeros_like(b)) for w, b in _rand_params(0)]
    x = rng.standard_normal((2, 7, 7))
    L, grads = nn.energy_loss_and_grads(zero, [x], [planes], jacobi=True)
    zj = x[0] / planes[2]
    ref = (np.sum(zj * nn.apply_5pt(planes, zj)) - 2 * np.sum(zj * x[0])) / 49
    assert abs(L - ref) <= 1e-13 * max(1.0, abs(ref))
    # and the preconditioner applies the same step
    z = nn.apply_preconditioner(zero, x[0], x[1], dinv=1.0 / planes[2])
    np.testing.assert_allclose(z, zj, rtol=1e-15)


# ---------------------------------------------------------------------------
# Training pairs (the error the Jacobi step leaves, scaled by rms(r)).

def test_pairs_of_a_diagonal_operator_have_zero_target():
    """For a diagonal operator the Jacobi step is the exact correction
    (e = D^-1 r), so every target vanishes; the input's first channel has
    unit rms and the second is log k unchanged."""
    rng = np.random.default_rng(3)
    n = 9
    diag = rng.uniform(0.5, 3.0, (n, n))
    lk = rng.standard_normal((n, n))
    xstar = rng.standard_normal((n, n))
    xs = [rng.standard_normal((n, n)) for _ in range(3)]
    rs = [diag * (xstar - x) for x in xs]
    ins, tg = nn.make_pairs(diag, xstar, lk, xs, rs)
    assert ins.shape == (3, n, n, 2) and tg.shape == (3, n, n)
    assert np.max(np.abs(tg)) <= 1e-14 * max(1.0, np.max(np.abs(xstar)))
    for j in range(3):
        assert abs(np.sqrt(np.mean(ins[j, ..., 0] ** 2)) - 1.0) <= 1e-14
        np.testing.assert_array_equal(ins[j, ..., 1], lk)


def test_pairs_are_scale_invariant_and_stop_at_unreached_captures():
    """Scaling residual and error together by c leaves every pair unchanged
    (both are divided by rms(r)); a NaN or zero residual ends the list."""
    rng = np.random.default_rng(4)
    n = 7
    diag = rng.uniform(1.0, 2.0, (n, n))
    lk = rng.standard_normal((n, n))
    xstar = rng.standard_normal((n, n))
    x = rng.standard_normal((n, n))
    r = rng.standard_normal((n, n))
    a_in, a_t = nn.make_pairs(diag, xstar, lk, [x], [r])
    c = 2.0 ** -7
    b_in, b_t = nn.make_pairs(diag, c * xstar, lk, [c * x], [c * r])
    np.testing.assert_allclose(b_in, a_in, rtol=0, atol=1e-14)
    np.testing.assert_allclose(b_t, a_t, rtol=1e-13, atol=1e-15)
    # the second capture was not reached (NaN) -> one pair; a zero residual too
    nan = np.full((n, n), np.nan)
    assert nn.make_pairs(diag, xstar, lk, [x, x, x], [r, nan, r])[0].shape[0] == 1
    assert nn.make_pairs(diag, xstar, lk, [x, x], [np.zeros((n, n)), r])[0].shape[0] == 0
    # direct evaluation at one pixel
    s = np.sqrt(np.mean(r ** 2))
    assert a_t[0, 2, 3] == pytest.approx((xstar[2, 3] - x[2, 3] - r[2, 3] / diag[2, 3]) / s, rel=1e-14)
