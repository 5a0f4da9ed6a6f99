"""Learned-preconditioner reference (numpy, float64) -- TEST INFRASTRUCTURE ONLY.

The paper has no learned component; this is the CPU reference of the
extension that applies a small convolutional network as the preconditioner
of flexible CG.  Readings (the choices are ours, stated once here):

* Network: input channels [r / rms(r), log k] on the N x N grid of unknowns;
  six 3x3 convolutions with zero 'same' padding and a bias each,
  2 -> 16 -> 16 -> 16 -> 16 -> 16 -> 1 channels, ReLU after every layer but
  the last; rms(v) = sqrt(mean(v^2)).
* Preconditioner: z = D^-1 r + rms(r) * net(...) -- the network learns a
  correction to the Jacobi step, so an untrained (zero) network is exactly
  Jacobi preconditioning and training can only move away from it where the
  loss improves; the plain form z = rms(r) * net(...) is kept for the pins.
* Weights W[o, i, 1 + dy, 1 + dx] multiply input channel i at (y + dy, x + dx)
  for output channel o at (y, x); arrays are [C, H, W] with x fastest.
* Reduced precision: with ``bf16=True`` every layer input and every weight is
  rounded to bfloat16 (round to nearest, ties to even) before the layer, the
  products and sums then run in float64 (the GPU sums in float32); biases and
  the final output stay unrounded.
* Loss: mean over all output elements of (net output - target)^2, the target
  being the scaled error e / rms(r) for a residual r of an iterate x with
  error e = x* - x.
* Adam with bias correction (lr, beta1, beta2, eps) on float32 master
  weights.
"""
import numpy as np

LAYERS = [(2, 16, True), (16, 16, True), (16, 16, True), (16, 16, True), (16, 16, True), (16, 1, False)]
FLOPS_PER_PIXEL = sum(2 * 9 * ci * co for ci, co, _ in LAYERS)   # 19,296


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def init_params(seed=0):
    """He-uniform weights, zero biases, float32 master copies."""
    rng = np.random.default_rng(seed)
    params = []
    for ci, co, _ in LAYERS:
        bound = np.sqrt(6.0 / (9 * ci))
        params.append((rng.uniform(-bound, bound, (co, ci, 3, 3)).astype(np.float32),
                       np.zeros(co, dtype=np.float32)))
    return params


def conv3x3(x, w, b):
    """y[o] = b[o] + sum_{i,dy,dx} w[o,i,1+dy,1+dx] * x[i, y+dy, x+dx], zero padding."""
    c, h, wd = x.shape
    xp = np.zeros((c, h + 2, wd + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((w.shape[0], h, wd)) + np.asarray(b, dtype=np.float64)[:, None, None]
    for ty in range(3):
        for tx in range(3):
            y += np.einsum("oi,ihw->ohw", w[:, :, ty, tx].astype(np.float64), xp[:, ty:ty + h, tx:tx + wd])
    return y


def conv3x3_backward(x, w, dy):
    """Gradients of sum(dy * conv3x3(x, w, b)) w.r.t. x, w and b."""
    c, h, wd = x.shape
    xp = np.zeros((c, h + 2, wd + 2))
    xp[:, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros(w.shape)
    w64 = w.astype(np.float64)
    for ty in range(3):
        for tx in range(3):
            dw[:, :, ty, tx] = np.einsum("ohw,ihw->oi", dy, xp[:, ty:ty + h, tx:tx + wd])
            dxp[:, ty:ty + h, tx:tx + wd] += np.einsum("oi,ohw->ihw", w64[:, :, ty, tx], dy)
    return dxp[:, 1:-1, 1:-1], dw, dy.sum(axis=(1, 2))


def forward(params, x, bf16=False):
    """Network output [1, H, W] and the per-layer cache (inputs, pre-activations)."""
    cache = []
    a = np.asarray(x, dtype=np.float64)
    for (w, b), (_, _, relu) in zip(params, LAYERS):
        xin = bf16_round(a) if bf16 else a
        wl = bf16_round(w) if bf16 else np.asarray(w, dtype=np.float64)
        pre = conv3x3(xin, wl, b)
        cache.append((xin, wl, pre))
        a = np.maximum(pre, 0.0) if relu else pre
    return a, cache


def backward(cache, dout):
    """Gradients (list of (dW, db)) and d input, for upstream gradient dout."""
    grads = []
    g = np.asarray(dout, dtype=np.float64)
    for (xin, wl, pre), (_, _, relu) in zip(reversed(cache), reversed(LAYERS)):
        if relu:
            g = g * (pre > 0.0)
        gx, gw, gb = conv3x3_backward(xin, wl, g)
        grads.append((gw, gb))
        g = gx
    return grads[::-1], g


def loss_and_grads(params, inputs, targets, bf16=False):
    """Mean squared error over all samples and pixels, and its gradients."""
    total = 0.0
    count = sum(t.size for t in targets)
    acc = [(np.zeros(w.shape), np.zeros(b.shape)) for w, b in params]
    for x, t in zip(inputs, targets):
        out, cache = forward(params, x, bf16)
        d = out - t.reshape(out.shape)
        total += float((d * d).sum())
        grads, _ = backward(cache, 2.0 * d / count)
        acc = [(aw + gw, ab + gb) for (aw, ab), (gw, gb) in zip(acc, grads)]
    return total / count, acc


def adam_step(params, grads, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on float32 master weights; state = (t, m list, v list)."""
    t, ms, vs = state
    t += 1
    out, nm, nv = [], [], []
    for (p, pb), (g, gb), (m, mb), (v, vb) in zip(params, grads, ms, vs):
        res = []
        for x, gx, mx, vx in ((p, g, m, v), (pb, gb, mb, vb)):
            mx = beta1 * mx + (1 - beta1) * gx
            vx = beta2 * vx + (1 - beta2) * gx * gx
            mh = mx / (1 - beta1 ** t)
            vh = vx / (1 - beta2 ** t)
            res.append(((x - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32), mx, vx))
        out.append((res[0][0], res[1][0]))
        nm.append((res[0][1], res[1][1]))
        nv.append((res[0][2], res[1][2]))
    return out, (t, nm, nv)


def adam_init(params):
    return (0, [(np.zeros(w.shape), np.zeros(b.shape)) for w, b in params],
            [(np.zeros(w.shape), np.zeros(b.shape)) for w, b in params])


def rms(v):
    return float(np.sqrt(np.mean(np.square(v))))


def make_pairs(diag, xstar, log_k, xs, rs):
    """Training pairs from iterates x_j with residuals r_j of a problem with
    solution xstar (arrays of shape (N, N); diag: the operator's diagonal).
    The preconditioner adds rms(r) * net(...) to the Jacobi step r / diag, so
    the network's target is the rest of the error, scaled like its input:
        input_j  = [r_j / rms(r_j), log k]
        target_j = (xstar - x_j - r_j / diag) / rms(r_j).
    Pairs stop at the first residual that is not finite or is zero.  Returns
    (inputs [P, N, N, 2], targets [P, N, N]) in float64."""
    ins, tgts = [], []
    for x, r in zip(xs, rs):
        r = np.asarray(r, dtype=np.float64)
        if not np.all(np.isfinite(r)):
            break
        s = rms(r)
        if s == 0.0:
            break
        ins.append(np.stack([r / s, np.asarray(log_k, dtype=np.float64)], axis=-1))
        tgts.append((np.asarray(xstar, dtype=np.float64) - np.asarray(x, dtype=np.float64) - r / diag) / s)
    n = np.shape(log_k)
    if not ins:
        return np.zeros((0,) + n + (2,)), np.zeros((0,) + n)
    return np.stack(ins), np.stack(tgts)


def apply_preconditioner(params, r, log_k, bf16=False, dinv=None):
    """z = rms(r) * net([r / rms(r), log k]) (+ dinv * r when dinv is given)
    for r, log_k (and dinv) of shape (N, N)."""
    r = np.asarray(r, dtype=np.float64)
    s = rms(r)
    jac = np.zeros_like(r) if dinv is None else np.asarray(dinv, dtype=np.float64) * r
    if s == 0.0:
        return jac
    x = np.stack([r / s, np.asarray(log_k, dtype=np.float64)])
    out, _ = forward(params, x, bf16)
    return s * out[0] + jac


# ---------------------------------------------------------------------------
# Energy-norm training loss.  For a residual r = A e (e the error of an
# iterate), the preconditioner output z is judged by its error in the A-norm,
#     ||z - e||_A^2 = z'Az - 2 z'r + e'r,
# the quantity a CG step minimises.  Dropping the constant e'r gives the
# functional  L(z) = (z'Az - 2 z'r) / (pixels), with gradient 2 (Az - r) /
# (pixels); it needs A and r but not e.  r here is the network's first input
# channel (the scaled residual), so L is scale-consistent with the output.
# A is the 5-point operator of the diffusion problem, given per pixel as five
# planes [S, W, C, E, N] (weights of (y-1), (x-1), centre, (x+1), (y+1); zero
# where the neighbour is outside the grid).

def apply_5pt(planes, z):
    """y = A z for A given as five coefficient planes [5, H, W]."""
    s, w, c, e, n = (np.asarray(p, dtype=np.float64) for p in planes)
    z = np.asarray(z, dtype=np.float64)
    y = c * z
    y[1:, :] += s[1:, :] * z[:-1, :]
    y[:, 1:] += w[:, 1:] * z[:, :-1]
    y[:, :-1] += e[:, :-1] * z[:, 1:]
    y[:-1, :] += n[:-1, :] * z[1:, :]
    return y


def energy_loss_and_grads(params, inputs, planes, bf16=False, jacobi=False):
    """sum over samples of (z'Az - 2 z'r), divided by the total pixel count,
    and its gradients; r = inputs[j][0], z the network output (plus the
    Jacobi step r / C, C the centre plane, when ``jacobi``)."""
    count = sum(x.shape[1] * x.shape[2] for x in inputs)
    total = 0.0
    acc = [(np.zeros(w.shape), np.zeros(b.shape)) for w, b in params]
    for x, pl in zip(inputs, planes):
        out, cache = forward(params, x, bf16)
        r = np.asarray(x[0], dtype=np.float64)
        z = out[0] + (r / np.asarray(pl[2], dtype=np.float64) if jacobi else 0.0)
        az = apply_5pt(pl, z)
        total += float(np.sum(z * az) - 2.0 * np.sum(z * r))
        grads, _ = backward(cache, (2.0 * (az - r) / count)[None])
        acc = [(aw + gw, ab + gb) for (aw, ab), (gw, gb) in zip(acc, grads)]
    return total / count, acc
