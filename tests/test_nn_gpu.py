"""GPU parity of the learned-preconditioner network kernels with the oracle.

The oracle emulates the GPU's reduced precision (every layer input and
weight rounded to bfloat16; it then sums in float64 where the GPU sums in
float32), so the forward pass agrees to float32 summation error, except
where that error flips a bfloat16 rounding of an intermediate activation:
the bar is relative L2 error <= 2e-3 and max error <= 2e-2 of the output
scale.  Gradients (bf16 gradients flowing backward on the GPU, float64 in the
oracle, same bf16-rounded weights and forward activations): cosine >= 0.999
and relative L2 <= 2e-2 per layer.  Adam is elementwise float32: <= 1e-6.
"""
import numpy as np
import pytest

from oracle import nn as onn
from gpu_util import to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    import paper_2204_02064_amd as pk
    pk.lib()
    return pk


def _inputs(B, H, W, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, H, W, 2)).astype(np.float32)
    t = rng.standard_normal((B, H, W)).astype(np.float32)
    return x, t


def _oracle_params(pk, seed):
    return pk.nn_unpack_params(pk.nn_pack_params(onn.init_params(seed)))


@pytest.mark.parametrize("B,H,W", [(1, 8, 16), (2, 13, 37), (1, 64, 64), (3, 32, 50)])
def test_forward_matches_oracle(pk, B, H, W):
    layers = onn.init_params(seed=B + H)
    layers = [(w, np.random.default_rng(7).uniform(-0.2, 0.2, b.shape).astype(np.float32)) for w, b in layers]
    params = to_dev(pk.nn_pack_params(layers))
    x, _ = _inputs(B, H, W, seed=H)
    out = pk.nn_forward(params, to_dev(x)).cpu().numpy()
    for bi in range(B):
        ref, _ = onn.forward(layers, np.moveaxis(x[bi], -1, 0).astype(np.float64), bf16=True)
        ref = ref[0]
        err = out[bi] - ref
        scale = np.abs(ref).max()
        assert np.linalg.norm(err) <= 2e-3 * np.linalg.norm(ref)
        assert np.abs(err).max() <= 2e-2 * scale


def test_forward_single_tap_layers_are_exact(pk):
    """Centre-tap-only weights with small integer values: every product and
    sum is exact in bf16/fp32, so GPU and oracle agree bit for bit; an
    off-centre tap checks the orientation of the taps."""
    layers = []
    for li, (ci, co) in enumerate(pk.NN_LAYERS):
        w = np.zeros((co, ci, 3, 3), np.float32)
        for o in range(co):
            w[o, o % ci, 1, 1] = 1.0 if li % 2 == 0 else 2.0
        if li == 2:
            w[0, 0, 0, 2] = 1.0   # dy = -1, dx = +1
        layers.append((w, np.zeros(co, np.float32)))
    params = to_dev(pk.nn_pack_params(layers))
    rng = np.random.default_rng(3)
    x = rng.integers(-4, 5, (1, 9, 20, 2)).astype(np.float32)
    out = pk.nn_forward(params, to_dev(x)).cpu().numpy()[0]
    ref, _ = onn.forward(layers, np.moveaxis(x[0], -1, 0).astype(np.float64), bf16=True)
    np.testing.assert_array_equal(out, ref[0].astype(np.float32))


@pytest.mark.parametrize("B,H,W", [(1, 8, 16), (2, 12, 24), (2, 32, 32)])
def test_gradients_match_oracle(pk, B, H, W):
    layers = _oracle_params(pk, seed=11)
    params = to_dev(pk.nn_pack_params(layers))
    x, t = _inputs(B, H, W, seed=5 + W)
    loss, grad = pk.nn_loss_grad(params, to_dev(x), to_dev(t))
    g = pk.nn_unpack_params(grad.cpu().numpy())
    xs = [np.moveaxis(x[b], -1, 0).astype(np.float64) for b in range(B)]
    ts = [t[b][None].astype(np.float64) for b in range(B)]
    oloss, ograds = onn.loss_and_grads(layers, xs, ts, bf16=True)
    assert abs(loss - oloss) <= 1e-3 * oloss
    for l, ((gw, gb), (ow, ob)) in enumerate(zip(g, ograds)):
        a = np.concatenate([gw.ravel(), gb.ravel()]).astype(np.float64)
        o = np.concatenate([ow.ravel(), ob.ravel()])
        cos = a @ o / (np.linalg.norm(a) * np.linalg.norm(o))
        rel = np.linalg.norm(a - o) / np.linalg.norm(o)
        assert cos >= 0.999 and rel <= 2e-2, (l, cos, rel)
    # padded entries stay zero
    full = grad.cpu().numpy()
    assert np.all(full[pk.nn_pack_params(g) == 0] == 0)


def test_adam_matches_oracle(pk):
    layers = _oracle_params(pk, seed=2)
    rng = np.random.default_rng(9)
    grads = [(rng.standard_normal(w.shape), rng.standard_normal(b.shape)) for w, b in layers]
    state = onn.adam_init(layers)
    p = to_dev(pk.nn_pack_params(layers))
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    ol = layers
    for step in (1, 2, 3):
        g = to_dev(pk.nn_pack_params(grads))
        pk.nn_adam(p, g, m, v, step, lr=1e-3)
        ol, state = onn.adam_step(ol, grads, state, lr=1e-3)
        grads = [(gw * 0.5 + 0.1, gb * 0.5 - 0.1) for gw, gb in grads]
    got = pk.nn_unpack_params(p.cpu().numpy())
    for (gw, gb), (ow, ob) in zip(got, ol):
        np.testing.assert_allclose(gw, ow, rtol=0, atol=2e-6)
        np.testing.assert_allclose(gb, ob, rtol=0, atol=2e-6)


@pytest.mark.parametrize("B,H,W,jacobi", [(1, 8, 16, False), (2, 12, 24, False), (2, 12, 24, True)])
def test_energy_gradients_match_oracle(pk, B, H, W, jacobi):
    import workloads
    layers = _oracle_params(pk, seed=13)
    params = to_dev(pk.nn_pack_params(layers))
    x, _ = _inputs(B, H, W, seed=3 + H)
    planes = []
    for b in range(B):
        gk = workloads.grf_log_k(max(H, W), seed=b)[:H + 2, :W + 2]
        planes.append(workloads.diffusion_planes(np.exp(gk)).astype(np.float32))
    pl = np.stack(planes)
    loss, grad = pk.nn_energy_grad(params, to_dev(x), to_dev(pl), jacobi=jacobi)
    xs = [np.moveaxis(x[b], -1, 0).astype(np.float64) for b in range(B)]
    oloss, ograds = onn.energy_loss_and_grads(layers, xs, [p.astype(np.float64) for p in planes], bf16=True,
                                              jacobi=jacobi)
    assert abs(loss - oloss) <= 2e-3 * max(abs(oloss), 1e-3)
    g = pk.nn_unpack_params(grad.cpu().numpy())
    for l, ((gw, gb), (ow, ob)) in enumerate(zip(g, ograds)):
        a = np.concatenate([gw.ravel(), gb.ravel()]).astype(np.float64)
        o = np.concatenate([ow.ravel(), ob.ravel()])
        cos = a @ o / (np.linalg.norm(a) * np.linalg.norm(o))
        rel = np.linalg.norm(a - o) / np.linalg.norm(o)
        assert cos >= 0.999 and rel <= 2e-2, (l, cos, rel)


def _splitmix_orders(seed, P, epochs):
    """The sample orders perks_nn_train draws: splitmix64 (Steele, Lea and
    Flood) feeding a Fisher-Yates shuffle per epoch."""
    state = seed
    M = (1 << 64) - 1
    orders = []
    for _ in range(epochs):
        perm = list(range(P))
        for i in range(P - 1, 0, -1):
            state = (state + 0x9E3779B97F4A7C15) & M
            z = state
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
            z ^= z >> 31
            j = z % (i + 1)
            perm[i], perm[j] = perm[j], perm[i]
        orders.append(perm)
    return orders


@pytest.mark.parametrize("energy", [False, True])
def test_native_training_loop_equals_the_step_by_step_loop(pk, energy):
    """perks_nn_train gives the bits of the same batches taken one call at a
    time (gather, loss and gradient, Adam), and reports each epoch's mean
    batch loss."""
    import workloads
    P, H, W, batch, epochs, seed = 7, 8, 16, 3, 2, 12345
    layers = _oracle_params(pk, seed=21)
    x, t = _inputs(P, H, W, seed=4)
    X, T = to_dev(x), to_dev(t)
    planes = np.stack([workloads.diffusion_planes(np.exp(workloads.grf_log_k(16, seed=f)[:H + 2, :W + 2]))
                       for f in range(3)]).astype(np.float32)
    field = np.array([0, 1, 2, 0, 1, 2, 0], np.int32)
    PL, F = to_dev(planes), torch.from_numpy(field).cuda()
    p0 = to_dev(pk.nn_pack_params(layers))
    pa = p0.clone()
    if energy:
        losses, steps, _, _ = pk.nn_train(pa, X, epochs, batch, lr=2e-3, seed=seed, planes=PL, field=F)
    else:
        losses, steps, _, _ = pk.nn_train(pa, X, epochs, batch, lr=2e-3, seed=seed, target=T)
    assert steps == epochs * (P // batch) and len(losses) == epochs
    pb = p0.clone()
    m = torch.zeros_like(pb)
    v = torch.zeros_like(pb)
    k = 0
    for order in _splitmix_orders(seed, P, epochs):
        tot = 0.0
        for b in range(P // batch):
            idx = torch.tensor(order[b * batch:(b + 1) * batch], device="cuda")
            xb = X.index_select(0, idx).contiguous()
            if energy:
                pl = PL.index_select(0, F.long().index_select(0, idx)).contiguous()
                loss, g = pk.nn_energy_grad(pb, xb, pl, jacobi=True)
            else:
                loss, g = pk.nn_loss_grad(pb, xb, T.index_select(0, idx).contiguous())
            k += 1
            pk.nn_adam(pb, g, m, v, k, lr=2e-3)
            tot += loss
        assert abs(losses.pop(0) - tot / (P // batch)) <= 1e-9 * max(1.0, abs(tot))
    assert torch.equal(pa, pb)
