"""Pins of the stencil oracle against closed forms (no GPU).

Each test fixes the oracle to something other than itself: Laplace eigenmodes
decaying by their known factor, exact translations that fix the orientation of
Eq. 2, the trinomial impulse response of the 9-point box, conservation of
constants, linearity, and composition of runs.
"""
import math

import numpy as np
import pytest

import oracle
import workloads


def _mode_2d(ny, nx, p, q):
    """sin(pi p i/(Nx+1)) sin(pi q j/(Ny+1)) on the interior, zero ring."""
    Nx, Ny = nx - 2, ny - 2
    i = np.arange(nx)
    j = np.arange(ny)
    ux = np.sin(np.pi * p * i / (Nx + 1))
    uy = np.sin(np.pi * q * j / (Ny + 1))
    u = np.outer(uy, ux)
    u[0, :] = u[-1, :] = 0.0
    u[:, 0] = u[:, -1] = 0.0
    return u, np.pi * p / (Nx + 1), np.pi * q / (Ny + 1)


@pytest.mark.parametrize("p,q", [(1, 1), (3, 2), (17, 5), (30, 29)])
def test_2d5pt_eigenmode_decay(p, q):
    ny, nx, k = 33, 32, 20
    u, tx, ty = _mode_2d(ny, nx, p, q)
    lam = 0.2 + 0.4 * math.cos(tx) + 0.4 * math.cos(ty)
    got = oracle.stencil(u, workloads.stencil_weights("2d5pt"), k)
    np.testing.assert_allclose(got, lam ** k * u, rtol=0, atol=1e-13)


@pytest.mark.parametrize("p,q", [(1, 1), (2, 7), (25, 3)])
def test_2d9pt_box_eigenmode_decay(p, q):
    ny, nx, k = 31, 28, 15
    u, tx, ty = _mode_2d(ny, nx, p, q)
    lam = (1 + 2 * math.cos(tx)) * (1 + 2 * math.cos(ty)) / 9.0
    got = oracle.stencil(u, workloads.stencil_weights("2d9pt"), k)
    np.testing.assert_allclose(got, lam ** k * u, rtol=0, atol=1e-13)


@pytest.mark.parametrize("p,q,s", [(1, 1, 1), (2, 5, 3), (9, 1, 7)])
def test_3d7pt_eigenmode_decay(p, q, s):
    nz, ny, nx, k = 12, 11, 13, 10
    i, j, l = np.arange(nx), np.arange(ny), np.arange(nz)
    tx, ty, tz = np.pi * p / (nx - 1), np.pi * q / (ny - 1), np.pi * s / (nz - 1)
    u = np.einsum("k,j,i->kji", np.sin(tz * l), np.sin(ty * j), np.sin(tx * i))
    u[0], u[-1], u[:, 0], u[:, -1], u[:, :, 0], u[:, :, -1] = 0, 0, 0, 0, 0, 0
    lam = 0.4 + 0.2 * (math.cos(tx) + math.cos(ty) + math.cos(tz))
    got = oracle.stencil(u, workloads.stencil_weights("3d7pt"), k)
    np.testing.assert_allclose(got, lam ** k * u, rtol=0, atol=1e-13)


def test_config0_low_mode_factor():
    # 256^2 grid (254^2 interior), mode (1,1): lambda = 0.2 + 0.8 cos(pi/255)
    lam = 0.2 + 0.8 * math.cos(math.pi / 255)
    assert abs(lam - 0.99994) < 5e-6
    assert abs(lam ** 100 - 0.99395) < 5e-6


def test_orientation_east_is_x_plus_one():
    # Eq. 2: E multiplies x(i+1, j) with i along x.  A box holding only E = 1
    # makes each interior cell copy its x+1 neighbour: a shift towards -x.
    g = workloads.stencil_grid((9, 14), seed=3)
    w = np.zeros((3, 3)); w[1, 2] = 1.0
    k = 4
    got = oracle.stencil(g, w, k)
    exp = g.copy()
    for y in range(1, 8):
        for x in range(1, 13):
            exp[y, x] = g[y, x + k] if x + k <= 12 else 0.0
    np.testing.assert_array_equal(got, exp)


def test_orientation_north_is_y_plus_one():
    g = workloads.stencil_grid((13, 9), seed=4)
    w = np.zeros((3, 3)); w[2, 1] = 1.0
    k = 3
    got = oracle.stencil(g, w, k)
    exp = g.copy()
    for y in range(1, 12):
        exp[y, 1:8] = g[y + k, 1:8] if y + k <= 11 else 0.0
    np.testing.assert_array_equal(got, exp)


def test_orientation_3d_z_plus_one_and_west():
    g = workloads.stencil_grid((8, 6, 7), seed=5)
    w = np.zeros((3, 3, 3)); w[2, 1, 1] = 1.0      # out(z) = in(z+1)
    got = oracle.stencil(g, w, 2)
    exp = g.copy()
    for z in range(1, 7):
        exp[z, 1:5, 1:6] = g[z + 2, 1:5, 1:6] if z + 2 <= 6 else 0.0
    np.testing.assert_array_equal(got, exp)
    w = np.zeros((3, 3, 3)); w[1, 1, 0] = 1.0      # out(x) = in(x-1)
    got = oracle.stencil(g, w, 1)
    exp = g.copy()
    exp[1:7, 1:5, 2:6] = g[1:7, 1:5, 1:5]
    exp[1:7, 1:5, 1] = 0.0
    np.testing.assert_array_equal(got, exp)


def _trinomial_row(k):
    t = np.array([1], dtype=object)
    for _ in range(k):
        t = np.convolve(t, np.array([1, 1, 1], dtype=object))
    return np.array([float(v) for v in t]) / 3.0 ** k


@pytest.mark.parametrize("k", [1, 2, 5, 12])
def test_9pt_box_impulse_is_trinomial_outer_product(k):
    n = 2 * k + 9
    g = np.zeros((n, n)); c = n // 2
    g[c, c] = 1.0
    got = oracle.stencil(g, workloads.stencil_weights("2d9pt"), k)
    t = _trinomial_row(k)
    exp = np.zeros_like(g)
    exp[c - k:c + k + 1, c - k:c + k + 1] = np.outer(t, t)
    np.testing.assert_allclose(got, exp, rtol=0, atol=1e-15)


@pytest.mark.parametrize("kind", workloads.STENCIL_KINDS)
def test_constant_field_preserved(kind):
    shape = (17, 23) if kind.startswith("2d") else (9, 10, 11)
    g = np.full(shape, 0.3725)
    got = oracle.stencil(g, workloads.stencil_weights(kind), 50)
    np.testing.assert_allclose(got, g, rtol=0, atol=50 * 4e-16)


@pytest.mark.parametrize("kind", workloads.STENCIL_KINDS)
def test_ring_fixed_linearity_and_split_runs(kind):
    shape = (15, 19) if kind.startswith("2d") else (7, 9, 10)
    w = workloads.stencil_weights(kind)
    u = workloads.stencil_grid(shape, seed=1, ring_value=0.5)
    v = workloads.stencil_grid(shape, seed=2, ring_value=-0.25)
    su, sv = oracle.stencil(u, w, 6), oracle.stencil(v, w, 6)
    sl = oracle.stencil(2.0 * u - 3.0 * v, w, 6)
    np.testing.assert_allclose(sl, 2.0 * su - 3.0 * sv, rtol=0, atol=1e-13)
    ring = np.ones(shape, dtype=bool); ring[workloads.interior_slices(len(shape))] = False
    np.testing.assert_array_equal(su[ring], u[ring])
    np.testing.assert_array_equal(oracle.stencil(oracle.stencil(u, w, 2), w, 4), su)
    np.testing.assert_array_equal(oracle.stencil(u, w, 0), u)


def test_reflection_symmetry():
    g = workloads.stencil_grid((12, 16), seed=7)
    w = workloads.stencil_weights("2d9pt")
    a = oracle.stencil(g[:, ::-1], w, 5)
    b = oracle.stencil(g, w, 5)[:, ::-1]
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


def test_bad_arguments_raise():
    with pytest.raises(ValueError):
        oracle.stencil(np.zeros((2, 5)), workloads.stencil_weights("2d5pt"), 1)


@pytest.mark.parametrize("kind,shape", [("2d9pt", (67, 130)), ("3d7pt", (9, 14, 33))])
def test_threaded_sweeps_give_the_same_bits(kind, shape):
    """Rows of one sweep are independent: sharing them among threads changes
    no cell's sum (the CPU baseline's all-core leg)."""
    g = workloads.stencil_grid(shape, seed=3)
    w = workloads.stencil_weights(kind)
    np.testing.assert_array_equal(oracle.stencil(g, w, 7, threads=4), oracle.stencil(g, w, 7))
