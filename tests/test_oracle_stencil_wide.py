"""Pins of the stencil oracle for the radius-2..4 patterns (no GPU).

The oracle's sweep is checked against things other than itself: the impulse
response (one step spreads a unit cell into the mirrored weight box, which
fixes orientation and offsets), several steps of it against scipy's 2D
convolution, the radius-2 box against exact pentanomial coefficients, whole
sweeps against scipy.ndimage's correlation on the interior, conservation of
constants, linearity and composition of runs.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import ndimage, signal

import oracle
import workloads


def _random_pattern_weights(kind, seed):
    """Asymmetric weights on the footprint of `kind` (zeros elsewhere)."""
    base = workloads.stencil_weights(kind)
    rng = np.random.default_rng(seed)
    return np.where(base != 0.0, rng.uniform(-1.0, 1.0, base.shape), 0.0)


@pytest.mark.parametrize("kind", workloads.WIDE_KINDS)
def test_weights_cover_the_named_footprint(kind):
    w = workloads.stencil_weights(kind)
    r = workloads.stencil_radius(kind)
    assert w.shape == (2 * r + 1, 2 * r + 1)
    pts = {"2ds9pt": 9, "2d13pt": 13, "2d17pt": 17, "2d25pt": 25}[kind]
    assert (w != 0).sum() == pts
    assert abs(w.sum() - 1.0) < 1e-15


@pytest.mark.parametrize("kind", workloads.WIDE_KINDS)
def test_impulse_one_step_is_the_mirrored_weight_box(kind):
    r = workloads.stencil_radius(kind)
    w = _random_pattern_weights(kind, 3)
    n = 4 * r + 5
    g = np.zeros((n, n + 2))
    cy, cx = n // 2, (n + 2) // 2
    g[cy, cx] = 1.0
    got = oracle.stencil(g, w, 1)
    exp = np.zeros_like(g)
    exp[cy - r:cy + r + 1, cx - r:cx + r + 1] = w[::-1, ::-1]
    np.testing.assert_array_equal(got, exp)


@pytest.mark.parametrize("kind", workloads.WIDE_KINDS)
@pytest.mark.parametrize("k", [2, 3])
def test_impulse_k_steps_is_the_k_fold_convolution(kind, k):
    r = workloads.stencil_radius(kind)
    w = _random_pattern_weights(kind, 5)
    n = 2 * k * r + 2 * r + 7
    g = np.zeros((n, n))
    c = n // 2
    g[c, c] = 1.0
    got = oracle.stencil(g, w, k)
    ker = w[::-1, ::-1]
    acc = np.ones((1, 1))
    for _ in range(k):
        acc = signal.convolve2d(acc, ker)
    exp = np.zeros_like(g)
    exp[c - k * r:c + k * r + 1, c - k * r:c + k * r + 1] = acc
    np.testing.assert_allclose(got, exp, rtol=0, atol=1e-14 * np.abs(exp).max())


def _pentanomial_row(k):
    t = [Fraction(1)]
    for _ in range(k):
        nxt = [Fraction(0)] * (len(t) + 4)
        for i, v in enumerate(t):
            for d in range(5):
                nxt[i + d] += v / 5
        t = nxt
    return np.array([float(v) for v in t])


@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_25pt_box_impulse_is_pentanomial_outer_product(k):
    n = 4 * k + 9
    g = np.zeros((n, n))
    c = n // 2
    g[c, c] = 1.0
    got = oracle.stencil(g, workloads.stencil_weights("2d25pt"), k)
    t = _pentanomial_row(k)
    exp = np.zeros_like(g)
    exp[c - 2 * k:c + 2 * k + 1, c - 2 * k:c + 2 * k + 1] = np.outer(t, t)
    np.testing.assert_allclose(got, exp, rtol=0, atol=1e-16)


@pytest.mark.parametrize("kind", workloads.WIDE_KINDS)
def test_sweeps_match_scipy_correlation_on_the_interior(kind):
    r = workloads.stencil_radius(kind)
    w = _random_pattern_weights(kind, 11)
    g = workloads.stencil_grid((13 + 2 * r, 17 + 2 * r), seed=4, r=r, ring_value=0.75)
    inner = workloads.interior_slices(2, r)
    ref = g.copy()
    for _ in range(4):
        nxt = ndimage.correlate(ref, w, mode="constant", cval=0.0)
        ref[inner] = nxt[inner]
    got = oracle.stencil(g, w, 4)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("kind", workloads.WIDE_KINDS)
def test_constant_preserved_ring_fixed_linear_and_composable(kind):
    r = workloads.stencil_radius(kind)
    w = workloads.stencil_weights(kind)
    shape = (15 + 2 * r, 19 + 2 * r)
    c = np.full(shape, 0.3725)
    np.testing.assert_allclose(oracle.stencil(c, w, 40), c, rtol=0, atol=40 * 4e-16)
    u = workloads.stencil_grid(shape, seed=1, r=r, ring_value=0.5)
    v = workloads.stencil_grid(shape, seed=2, r=r, ring_value=-0.25)
    su, sv = oracle.stencil(u, w, 6), oracle.stencil(v, w, 6)
    np.testing.assert_allclose(oracle.stencil(2.0 * u - 3.0 * v, w, 6), 2.0 * su - 3.0 * sv, rtol=0, atol=1e-13)
    ring = np.ones(shape, dtype=bool)
    ring[workloads.interior_slices(2, r)] = False
    np.testing.assert_array_equal(su[ring], u[ring])
    np.testing.assert_array_equal(oracle.stencil(oracle.stencil(u, w, 2), w, 4), su)


# ---------------------------------------------------------------------------
# 3D patterns beyond the 7-point star (3d13pt, 3d17pt, 3d27pt, poisson)

@pytest.mark.parametrize("kind", workloads.WIDE3_KINDS)
def test_3d_weights_cover_the_named_footprint(kind):
    w = workloads.stencil_weights(kind)
    r = workloads.stencil_radius(kind)
    assert w.shape == (2 * r + 1,) * 3
    assert (w != 0).sum() == {"3d13pt": 13, "3d17pt": 17, "3d27pt": 27, "poisson": 19}[kind]
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_array_equal(w, w[::-1, ::-1, ::-1])   # centrally symmetric


@pytest.mark.parametrize("kind", workloads.WIDE3_KINDS)
def test_3d_impulse_one_step_is_the_mirrored_weight_box(kind):
    r = workloads.stencil_radius(kind)
    w = _random_pattern_weights(kind, 13)
    n = 2 * r + 5
    g = np.zeros((n, n + 1, n + 2))
    c = (n // 2, (n + 1) // 2, (n + 2) // 2)
    g[c] = 1.0
    got = oracle.stencil(g, w, 1)
    exp = np.zeros_like(g)
    exp[c[0] - r:c[0] + r + 1, c[1] - r:c[1] + r + 1, c[2] - r:c[2] + r + 1] = w[::-1, ::-1, ::-1]
    np.testing.assert_array_equal(got, exp)


@pytest.mark.parametrize("kind", workloads.WIDE3_KINDS)
def test_3d_impulse_two_steps_is_the_convolution(kind):
    r = workloads.stencil_radius(kind)
    w = _random_pattern_weights(kind, 17)
    n = 4 * r + 5
    g = np.zeros((n, n, n))
    c = n // 2
    g[c, c, c] = 1.0
    got = oracle.stencil(g, w, 2)
    ker = w[::-1, ::-1, ::-1]
    acc = signal.convolve(ker, ker, method="direct")
    exp = np.zeros_like(g)
    exp[c - 2 * r:c + 2 * r + 1, c - 2 * r:c + 2 * r + 1, c - 2 * r:c + 2 * r + 1] = acc
    np.testing.assert_allclose(got, exp, rtol=0, atol=1e-14 * np.abs(exp).max())


@pytest.mark.parametrize("k", [1, 3])
def test_27pt_box_impulse_is_trinomial_outer_product(k):
    n = 2 * k + 5
    g = np.zeros((n, n, n))
    c = n // 2
    g[c, c, c] = 1.0
    got = oracle.stencil(g, workloads.stencil_weights("3d27pt"), k)
    t = [Fraction(1)]
    for _ in range(k):
        nxt = [Fraction(0)] * (len(t) + 2)
        for i, v in enumerate(t):
            for d in range(3):
                nxt[i + d] += v / 3
        t = nxt
    t = np.array([float(v) for v in t])
    exp = np.zeros_like(g)
    exp[c - k:c + k + 1, c - k:c + k + 1, c - k:c + k + 1] = t[:, None, None] * t[None, :, None] * t[None, None, :]
    np.testing.assert_allclose(got, exp, rtol=0, atol=1e-16)


@pytest.mark.parametrize("kind", workloads.WIDE3_KINDS)
def test_3d_sweeps_match_scipy_correlation_and_keep_constants(kind):
    r = workloads.stencil_radius(kind)
    w = _random_pattern_weights(kind, 19)
    shape = (5 + 2 * r, 7 + 2 * r, 9 + 2 * r)
    g = workloads.stencil_grid(shape, seed=6, r=r, ring_value=-0.5)
    inner = workloads.interior_slices(3, r)
    ref = g.copy()
    for _ in range(3):
        nxt = ndimage.correlate(ref, w, mode="constant", cval=0.0)
        ref[inner] = nxt[inner]
    np.testing.assert_allclose(oracle.stencil(g, w, 3), ref, rtol=0, atol=1e-13)
    c = np.full(shape, 0.3725)
    np.testing.assert_allclose(oracle.stencil(c, workloads.stencil_weights(kind), 20), c, rtol=0, atol=20 * 4e-16)
