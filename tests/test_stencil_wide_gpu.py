"""GPU parity of the radius-2..4 2D stencils (the 2ds9pt, 2d13pt, 2d17pt stars
and the 2d25pt box) against the oracle.

Bars as for the radius-1 kernels: FP64 relative error <= 1e-12, FP32 <= 1e-5
against the FP64 oracle on the same FP32-rounded grid and weights.  The
persistent kernel (register-cached tiles of 24, 32, 48 or 80 rows, or every tile
streamed) and the per-step baseline share one tile routine, so all of them
must agree bitwise.  Weights are random and asymmetric on each footprint, so
a transposed or mirrored offset cannot pass.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    import paper_2204_02064_amd as pk
    pk.lib()
    return pk


def _weights(kind, seed, dtype):
    base = workloads.stencil_weights(kind)
    rng = np.random.default_rng(seed)
    w = np.where(base != 0.0, rng.uniform(0.0, 2.0 / (base != 0).sum(), base.shape), 0.0)
    return w.astype(np.float32).astype(np.float64) if dtype == "float32" else w


def _grid(shape, r, seed, dtype):
    g = workloads.stencil_grid(shape, seed=seed, r=r, ring_value=0.25)
    return g.astype(np.float32).astype(np.float64) if dtype == "float32" else g


def _run(pk, g, w, steps, dtype, baseline=False, tuning=None):
    t = to_dev(g, getattr(torch, dtype))
    if baseline:
        pk.stencil_run_baseline(t, w, steps)
    else:
        pk.stencil_run(t, w, steps, tuning=tuning)
    torch.cuda.synchronize()
    return t.cpu().double().numpy()


def _tol(dtype):
    return 1e-12 if dtype == "float64" else 1e-5


# (extra rows, extra columns) beyond the ring: a single cell, a tile and a
# ragged tail in x, several 32-row tiles with a ragged last one
SHAPES = [(1, 2), (23, 141), (97, 70)]


@pytest.mark.parametrize("kind", workloads.WIDE_KINDS)
@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("inner", SHAPES)
def test_wide_stencils_match_oracle_and_baseline(pk, kind, dtype, inner):
    r = workloads.stencil_radius(kind)
    shape = (inner[0] + 2 * r, inner[1] + 2 * r)
    g = _grid(shape, r, 7, dtype)
    w = _weights(kind, 3, dtype)
    for steps in (1, 6, 9):
        ref = oracle.stencil(g, w, steps)
        base = _run(pk, g, w, steps, dtype, baseline=True)
        assert rel_err(base, ref) <= _tol(dtype), (steps, "baseline")
        for tu in (None, {"rows_per_lane": 32}, {"rows_per_lane": 48}, {"rows_per_lane": 80}, {"max_cached_tiles": -1}):
            got = _run(pk, g, w, steps, dtype, tuning=tu)
            np.testing.assert_array_equal(got, base, err_msg=f"steps {steps} tuning {tu}")


@pytest.mark.parametrize("kind", workloads.WIDE_KINDS)
def test_wide_plan_caches_every_tile_at_3072(pk, kind):
    r = workloads.stencil_radius(kind)
    w = workloads.stencil_weights(kind)
    for dtype in ("float64", "float32"):
        pl = pk.stencil_plan((3072, 3072), w, dtype)
        assert pl["cached_tiles"] == pl["tiles"] > 0, (dtype, pl)
        assert pl["interior_cells"] == (3072 - 2 * r) ** 2
        assert pl["rows_per_lane"] in (24, 32, 48, 80)
    pl = pk.stencil_plan((3072, 3072), w, "float64", tuning={"max_cached_tiles": -1})
    assert pl["cached_tiles"] == 0


@pytest.mark.parametrize("kind", workloads.WIDE_KINDS)
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_full_size_wide_matches_oracle_for_a_few_steps(pk, kind, dtype):
    """3072^2 in the benchmark's launch configuration (every tile cached)."""
    r = workloads.stencil_radius(kind)
    g = _grid((3072, 3072), r, 0, dtype)
    w = workloads.stencil_weights(kind)
    w = w.astype(np.float32).astype(np.float64) if dtype == "float32" else w
    got = _run(pk, g, w, 3, dtype)
    assert rel_err(got, oracle.stencil(g, w, 3)) <= _tol(dtype)
    np.testing.assert_array_equal(got, _run(pk, g, w, 3, dtype, baseline=True))


def test_wide_stencil_steps_zero_is_identity(pk):
    g = _grid((40, 90), 3, 2, "float64")
    np.testing.assert_array_equal(_run(pk, g, workloads.stencil_weights("2d13pt"), 0, "float64"), g)


# ---------------------------------------------------------------------------
# 3D patterns beyond the 7-point star: any radius-1 pattern (3d27pt, poisson,
# 3d17pt) and the radius-2 star (3d13pt); streamed persistent kernel and
# per-step baseline on one tile routine.

SHAPES3 = [(1, 1, 2), (5, 23, 70), (9, 40, 131)]
_BOX3_OFF = ("the radius-1 3D box kernel is disabled: it hung once at 256^3 (four workgroups per CU) "
             "and the cause is not found")
KINDS3 = [k if workloads.stencil_radius(k) == 2 else pytest.param(k, marks=pytest.mark.skip(reason=_BOX3_OFF))
          for k in workloads.WIDE3_KINDS]


@pytest.mark.parametrize("kind", KINDS3)
@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("inner", SHAPES3)
def test_wide3_stencils_match_oracle_and_baseline(pk, kind, dtype, inner):
    r = workloads.stencil_radius(kind)
    shape = tuple(s + 2 * r for s in inner)
    g = _grid(shape, r, 9, dtype)
    w = _weights(kind, 5, dtype)
    for steps in (1, 4, 7):
        ref = oracle.stencil(g, w, steps)
        base = _run(pk, g, w, steps, dtype, baseline=True)
        assert rel_err(base, ref) <= _tol(dtype), (steps, "baseline")
        np.testing.assert_array_equal(_run(pk, g, w, steps, dtype), base, err_msg=f"steps {steps}")


@pytest.mark.parametrize("kind", KINDS3)
def test_full_size_wide3_matches_oracle_for_a_few_steps(pk, kind):
    """256^3 FP64 and FP32 in the benchmark's launch configuration."""
    r = workloads.stencil_radius(kind)
    for dtype in ("float64", "float32"):
        g = _grid((256, 256, 256), r, 0, dtype)
        w = workloads.stencil_weights(kind)
        w = w.astype(np.float32).astype(np.float64) if dtype == "float32" else w
        got = _run(pk, g, w, 2, dtype)
        assert rel_err(got, oracle.stencil(g, w, 2)) <= _tol(dtype), dtype
        np.testing.assert_array_equal(got, _run(pk, g, w, 2, dtype, baseline=True))
        pl = pk.stencil_plan((256, 256, 256), w, dtype)
        assert pl["interior_cells"] == (256 - 2 * r) ** 3 and pl["cached_tiles"] == 0
