"""GPU parity of the persistent and per-step stencil kernels against the oracle.

Bars: FP64 relative error <= 1e-12 (max|u - u_ref| / max|u_ref|); FP32 (FP32
storage and arithmetic) <= 1e-5 against the FP64 oracle run on the same
FP32-rounded inputs (grid and weights: an FP32 run multiplies by the FP32
weights, so the oracle is given those).  The persistent and per-step paths
apply the same per-cell arithmetic, so they must agree bitwise.
"""
import math

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


def _run(pk, g_np, w, steps, dtype, baseline=False, tuning=None):
    t = to_dev(g_np, dtype)
    if baseline:
        pk.stencil_run_baseline(t, w, steps)
    else:
        pk.stencil_run(t, w, steps, tuning=tuning)
    torch.cuda.synchronize()
    return t.cpu().double().numpy()


CASES = [
    ("2d5pt", (256, 256), 100),      # the 256^2 FP64 100-step configuration
    ("2d5pt", (5, 7), 3),
    ("2d5pt", (33, 65), 9),
    ("2d5pt", (130, 200), 17),
    ("2d9pt", (66, 130), 11),
    ("2d9pt", (301, 77), 6),
    ("3d7pt", (5, 6, 7), 4),
    ("3d7pt", (17, 9, 13), 5),
    ("3d7pt", (40, 37, 70), 8),
]


@pytest.mark.parametrize("kind,shape,steps", CASES)
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_persistent_matches_oracle(pk, kind, shape, steps, dtype):
    tdt = getattr(torch, dtype)
    g = workloads.stencil_grid(shape, seed=0, dtype=np.float64)
    g = g.astype(np.float32).astype(np.float64) if dtype == "float32" else g
    w = workloads.stencil_weights(kind)
    w = w.astype(np.float32).astype(np.float64) if dtype == "float32" else w
    ref = oracle.stencil(g, w, steps)
    got = _run(pk, g, w, steps, tdt)
    assert rel_err(got, ref) <= (1e-12 if dtype == "float64" else 1e-5)
    base = _run(pk, g, w, steps, tdt, baseline=True)
    np.testing.assert_array_equal(got, base)


@pytest.mark.parametrize("kind,shape", [("2d5pt", (45, 150)), ("2d9pt", (70, 99)), ("2d5pt", (3072, 300)),
                                        ("2d9pt", (5, 7))])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_radius1_on_the_wide_kernel_family_is_bitwise_the_same(pk, kind, shape, dtype):
    """tuning.kernel = 2 runs a radius-1 pattern on the radius-2..4 kernels
    (grid barrier, 32/48/80 register rows, cached or streamed); both families
    sum the same terms in the same order, so they agree bitwise with each
    other and with the per-step baseline, and match the oracle."""
    rng = np.random.default_rng(7)
    w = workloads.stencil_weights(kind)
    w = np.where(w != 0, rng.uniform(0.05, 0.3, w.shape), 0.0)
    tdt = getattr(torch, dtype)
    g = workloads.stencil_grid(shape, seed=8, ring_value=0.3)
    if dtype == "float32":
        g = g.astype(np.float32).astype(np.float64)
        w = w.astype(np.float32).astype(np.float64)
    ref = _run(pk, g, w, 9, tdt)
    assert rel_err(ref, oracle.stencil(g, w, 9)) <= (1e-12 if dtype == "float64" else 1e-5)
    np.testing.assert_array_equal(_run(pk, g, w, 9, tdt, baseline=True), ref)
    for tu in ({"kernel": 2}, {"kernel": 2, "rows_per_lane": 32}, {"kernel": 2, "rows_per_lane": 80},
               {"kernel": 2, "max_cached_tiles": -1}):
        np.testing.assert_array_equal(_run(pk, g, w, 9, tdt, tuning=tu), ref, err_msg=str(tu))
    assert pk.stencil_plan(shape, w, dtype, tuning={"kernel": 2})["sync"] == 1


@pytest.mark.parametrize("kind,shape", [("2d5pt", (45, 150)), ("2d9pt", (70, 99)), ("3d7pt", (11, 21, 67))])
def test_asymmetric_weights_fix_orientation(pk, kind, shape):
    rng = np.random.default_rng(42)
    w = workloads.stencil_weights(kind)
    w = np.where(w != 0, rng.uniform(0.05, 0.3, w.shape), 0.0)
    g = workloads.stencil_grid(shape, seed=5, ring_value=0.7)
    ref = oracle.stencil(g, w, 6)
    got = _run(pk, g, w, 6, torch.float64)
    assert rel_err(got, ref) <= 1e-12


@pytest.mark.parametrize("kind,shape", [("2d5pt", (200, 300)), ("2d9pt", (129, 257)), ("3d7pt", (30, 40, 130))])
def test_streamed_and_partially_cached_tiles_agree_bitwise(pk, kind, shape):
    g = workloads.stencil_grid(shape, seed=3)
    w = workloads.stencil_weights(kind)
    full = _run(pk, g, w, 13, torch.float64)
    none = _run(pk, g, w, 13, torch.float64, tuning={"max_cached_tiles": -1})
    part = _run(pk, g, w, 13, torch.float64, tuning={"max_cached_tiles": 3})
    np.testing.assert_array_equal(full, none)
    np.testing.assert_array_equal(full, part)
    assert rel_err(full, oracle.stencil(g, w, 13)) <= 1e-12


@pytest.mark.parametrize("kind,shape", [("2d5pt", (150, 333)), ("2d9pt", (211, 100)), ("3d7pt", (19, 23, 90))])
def test_grid_barrier_and_point_to_point_sync_agree_bitwise(pk, kind, shape):
    # sync=1: a device-wide barrier after every step (the paper's grid.sync);
    # sync=2: point-to-point halo words tagged with the step's epoch
    g = workloads.stencil_grid(shape, seed=11)
    w = workloads.stencil_weights(kind)
    a = _run(pk, g, w, 21, torch.float64, tuning={"sync": 1})
    b = _run(pk, g, w, 21, torch.float64, tuning={"sync": 2})
    c = _run(pk, g, w, 21, torch.float64, tuning={"sync": 2, "max_cached_tiles": 5})
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c)
    assert rel_err(a, oracle.stencil(g, w, 21)) <= 1e-12


_XCD_OFF = ("halo words within one XCD's L2 (sync 3) are not in the library: a build of that mode (8 workgroups "
            "launched per working one, words moved with L1-bypassing loads and stores) did not finish on 2d5pt "
            "256^2 FP64 with 16 working workgroups, twice; the cause was not found and the mode was taken out")


@pytest.mark.skip(reason=_XCD_OFF)
@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("kind,shape", [("2d5pt", (256, 256)), ("2d9pt", (130, 389)), ("2d5pt", (70, 1000)),
                                        ("2d9pt", (5, 3))])
def test_xcd_local_halo_words_agree_bitwise(pk, dtype, kind, shape):
    # sync=3: the point-to-point halo words kept in one XCD's L2 (8 workgroups
    # launched per working one); the same arithmetic as sync=2
    g = workloads.stencil_grid(shape, seed=12).astype(dtype)
    w = workloads.stencil_weights(kind)
    tt = getattr(torch, dtype)
    print(f"xcd-local {kind} {shape} {dtype}", flush=True)
    assert pk.stencil_plan(shape, w, dtype, tuning={"sync": 3})["sync"] == 3
    for steps in (1, 2, 37):
        a = _run(pk, g, w, steps, tt, tuning={"sync": 3})
        b = _run(pk, g, w, steps, tt, tuning={"sync": 2})
        np.testing.assert_array_equal(a, b, err_msg=f"steps {steps}")
    gd = g.astype(np.float64)
    wd = w.astype(np.float32).astype(np.float64) if dtype == "float32" else w
    assert rel_err(a, oracle.stencil(gd, wd, 37)) <= (1e-12 if dtype == "float64" else 1e-5)


def test_xcd_local_mode_is_refused(pk):
    # sync 3 is not a mode of this library: the plan must refuse it
    w = workloads.stencil_weights("2d5pt")
    with pytest.raises(RuntimeError):
        pk.stencil_plan((256, 256), w, "float64", tuning={"sync": 3})


@pytest.mark.parametrize("k,h,resident", [(2, 8, True), (4, 16, True), (8, 8, True), (8, 16, True),
                                          (2, 32, True), (4, 56, True),
                                          (2, 8, False), (4, 16, False), (8, 8, False), (8, 16, False)])
@pytest.mark.parametrize("shape", [(256, 256), (130, 389), (70, 1000), (5, 3)])
@pytest.mark.parametrize("kind", ["2d5pt", "2d9pt"])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_temporally_blocked_kernel_is_bitwise_the_per_step_baseline(pk, dtype, kind, shape, k, h, resident):
    """kernel 3: K steps per exchange on tiles of 64 - 2K columns x h rows with
    a K-wide ghost ring; step counts below, at and past K, ragged tiles and a
    grid smaller than one tile.  Resident: every block stays in registers and
    only the bands move; otherwise (max_cached_tiles -1) every block is loaded
    and stored whole."""
    g = workloads.stencil_grid(shape, seed=21).astype(dtype)
    w = workloads.stencil_weights(kind)
    tt = getattr(torch, dtype)
    tu = {"kernel": 3, "steps_per_sync": k, "rows_per_lane": h}
    if not resident:
        tu["max_cached_tiles"] = -1
    print(f"temporal blocking {kind} {shape} {dtype} K={k} H={h} resident={resident}", flush=True)
    plan = pk.stencil_plan(shape, w, dtype, tuning=tu)
    assert plan["sync"] == 3 and plan["rows_per_lane"] == h
    assert plan["cached_tiles"] == (plan["tiles"] if resident else 0)
    for steps in sorted({1, k - 1, k, 2 * k + 1, 37} - {0}):
        a = _run(pk, g, w, steps, tt, tuning=tu)
        b = _run(pk, g, w, steps, tt, baseline=True)
        np.testing.assert_array_equal(a, b, err_msg=f"steps {steps}")
    gd = g.astype(np.float64)
    wd = w.astype(np.float32).astype(np.float64) if dtype == "float32" else w
    assert rel_err(a, oracle.stencil(gd, wd, 37)) <= (1e-12 if dtype == "float64" else 1e-5)


def test_temporally_blocked_kernel_rejects_other_shapes(pk):
    w = workloads.stencil_weights("2d5pt")
    for tu in ({"kernel": 3, "steps_per_sync": 3}, {"kernel": 3, "rows_per_lane": 12}, {"steps_per_sync": 4},
               {"kernel": 3, "rows_per_lane": 56, "max_cached_tiles": -1}):
        with pytest.raises(RuntimeError):
            pk.stencil_plan((256, 256), w, "float64", tuning=tu)
    # 56-row tiles exist only register resident: FP64 4096^2 has too many
    with pytest.raises(RuntimeError):
        pk.stencil_plan((4096, 4096), w, "float64", tuning={"kernel": 3, "steps_per_sync": 4, "rows_per_lane": 56})


def test_repeated_launches_reuse_epochs_safely(pk):
    # consecutive persistent launches on different shapes share the face
    # buffers; stale words must never be taken for current ones
    w = workloads.stencil_weights("2d9pt")
    for shape, steps in [((77, 300), 5), ((300, 77), 7), ((77, 300), 1), ((129, 129), 12)]:
        g = workloads.stencil_grid(shape, seed=steps)
        got = _run(pk, g, w, steps, torch.float64)
        assert rel_err(got, oracle.stencil(g, w, steps)) <= 1e-12


@pytest.mark.parametrize("rows", [8, 16, 32, 48])
def test_tile_depth_does_not_change_bits(pk, rows):
    g = workloads.stencil_grid((190, 260), seed=8)
    w = workloads.stencil_weights("2d5pt")
    a = _run(pk, g, w, 10, torch.float64, tuning={"rows_per_lane": rows})
    b = _run(pk, g, w, 10, torch.float64, baseline=True)
    np.testing.assert_array_equal(a, b)


def test_split_runs_compose_bitwise_and_zero_steps_is_identity(pk):
    g = workloads.stencil_grid((97, 131), seed=2)
    w = workloads.stencil_weights("2d9pt")
    t = to_dev(g)
    pk.stencil_run(t, w, 4)
    pk.stencil_run(t, w, 9)
    torch.cuda.synchronize()
    whole = _run(pk, g, w, 13, torch.float64)
    np.testing.assert_array_equal(t.cpu().numpy(), whole)
    np.testing.assert_array_equal(_run(pk, g, w, 0, torch.float64), g)


# The plans the benchmark times at 3072^2 (the radius-2..4 kernel family at
# radius 1: 48 register rows per lane in FP64, 24 in FP32, every tile cached;
# also the untuned default there) and the radius-1 kernel family.
BENCH_TUNING = {"float64": {"kernel": 3, "steps_per_sync": 4, "rows_per_lane": 56},
                "float32": {"kernel": 3, "steps_per_sync": 4, "rows_per_lane": 56}}
WIDE_TUNING = {"float64": {"kernel": 2, "rows_per_lane": 48}, "float32": {"kernel": 2, "rows_per_lane": 24}}
EIGEN_CASES = [("2d5pt", (3072, 3072), "float64", {"kernel": 1}), ("2d9pt", (3072, 3072), "float32", {"kernel": 1}),
               ("3d7pt", (256, 256, 256), "float64", None)]
EIGEN_CASES += [(k, (3072, 3072), dt, BENCH_TUNING[dt]) for k in ("2d5pt", "2d9pt") for dt in ("float64", "float32")]
EIGEN_CASES += [(k, (3072, 3072), dt, WIDE_TUNING[dt]) for k in ("2d5pt", "2d9pt") for dt in ("float64", "float32")]


@pytest.mark.parametrize("kind,shape,dtype,tuning", EIGEN_CASES)
def test_full_size_eigenmode_decay(pk, kind, shape, dtype, tuning):
    # At the benchmark sizes the oracle cannot follow 1000 steps cell by cell;
    # a discrete sine mode must decay by its closed-form factor instead.  The
    # factor is evaluated with the weights the kernel multiplies by (FP32
    # weights for an FP32 grid), so only the arithmetic's rounding remains.
    steps = 1000
    wk = workloads.stencil_weights(kind)
    if dtype == "float32":
        wk = wk.astype(np.float32).astype(np.float64)
    c = wk[(1,) * len(shape)]
    off = wk[(1,) * (len(shape) - 1) + (2,)]
    axes = [np.sin(np.pi * (2 if d == 0 else 1) * np.arange(n) / (n - 1)) for d, n in enumerate(shape)]
    thetas = [np.pi * (2 if d == 0 else 1) / (n - 1) for d, n in enumerate(shape)]
    if len(shape) == 2:
        u = np.outer(axes[0], axes[1])
        if kind == "2d5pt":
            lam = c + 2 * off * (math.cos(thetas[0]) + math.cos(thetas[1]))
        else:
            lam = c * (1 + 2 * math.cos(thetas[0])) * (1 + 2 * math.cos(thetas[1]))
    else:
        u = np.einsum("k,j,i->kji", *axes)
        lam = c + 2 * off * sum(math.cos(t) for t in thetas)
    for d in range(len(shape)):
        idx = [slice(None)] * len(shape)
        idx[d] = 0
        u[tuple(idx)] = 0
        idx[d] = -1
        u[tuple(idx)] = 0
    tdt = getattr(torch, dtype)
    u = u.astype(np.float32).astype(np.float64) if dtype == "float32" else u
    got = _run(pk, u, workloads.stencil_weights(kind), steps, tdt, tuning=tuning)
    err = rel_err(got, lam ** steps * u)
    print(f"{kind} {dtype} {shape}: relative error after {steps} steps {err:.2e}")
    # FP32: each step rounds npts partial sums, each bounded by max|u| (the
    # weights are non-negative and sum to ~1), so the error after `steps`
    # steps is at most steps * npts * eps32 / 2 relative to max|u| (5.4e-5 per
    # 100 steps for the 9-point box).  The 1e-5 bar of the FP32 form holds
    # for runs of up to ~100 steps (checked against the oracle above); this
    # 1000-step run is held to the derived bound.
    npts = int(np.count_nonzero(wk))
    tol = 1e-12 if dtype == "float64" else steps * npts * 2.0 ** -24 / 2
    assert err <= tol


@pytest.mark.parametrize("kind", ["2d5pt", "2d9pt"])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_full_size_bench_plans_match_oracle(pk, kind, dtype):
    """3072^2 on exactly the plans the benchmark times: a few steps against
    the oracle and bitwise against the per-step baseline; the untuned default
    is the same plan, and it caches every tile."""
    tu = BENCH_TUNING[dtype]
    tdt = getattr(torch, dtype)
    g = workloads.stencil_grid((3072, 3072), seed=0)
    w = workloads.stencil_weights(kind)
    if dtype == "float32":
        g = g.astype(np.float32).astype(np.float64)
        w = w.astype(np.float32).astype(np.float64)
    # six steps: with K = 4 one block exchanges its bands, the second is short
    got = _run(pk, g, w, 6, tdt, tuning=tu)
    assert rel_err(got, oracle.stencil(g, w, 6)) <= (1e-12 if dtype == "float64" else 1e-5)
    np.testing.assert_array_equal(got, _run(pk, g, w, 6, tdt, baseline=True))
    np.testing.assert_array_equal(got, _run(pk, g, w, 6, tdt))
    plan, default = pk.stencil_plan((3072, 3072), w, dtype, tuning=tu), pk.stencil_plan((3072, 3072), w, dtype)
    assert plan == default
    assert plan["rows_per_lane"] == tu["rows_per_lane"] and plan["cached_tiles"] == plan["tiles"] > 0


def test_untuned_small_grids_take_temporal_blocking(pk):
    """Below 2^20 interior cells the untuned plan is the temporally blocked
    kernel (8 steps per exchange on 8-row tiles up to 2^18 cells, on 16-row
    tiles above), every tile in registers; above 2^20 it is too when 56-row
    tiles all fit (3072^2), else not (FP64 4096^2: the radius-2..4 family
    when it caches every tile, else the radius-1 kernel).
    The 256^2 100-step configuration runs on it, and matches the oracle."""
    w = workloads.stencil_weights("2d5pt")
    pl = pk.stencil_plan((256, 256), w, "float64")
    assert pl["sync"] == 3 and pl["rows_per_lane"] == 8 and pl["cached_tiles"] == pl["tiles"]
    pl = pk.stencil_plan((1024, 1024), w, "float32")
    assert pl["sync"] == 3 and pl["rows_per_lane"] == 16 and pl["cached_tiles"] == pl["tiles"]
    pl = pk.stencil_plan((3072, 3072), w, "float32")
    assert pl["sync"] == 3 and pl["rows_per_lane"] == 56 and pl["cached_tiles"] == pl["tiles"]
    pl = pk.stencil_plan((3072, 3072), w, "float64")
    assert pl["sync"] == 3 and pl["rows_per_lane"] == 56 and pl["cached_tiles"] == pl["tiles"]
    assert pk.stencil_plan((4096, 4096), w, "float64")["sync"] != 3
    assert pk.stencil_plan((256, 256), w, "float64", tuning={"sync": 2})["sync"] == 2
    assert pk.stencil_plan((256, 256), w, "float64", tuning={"kernel": 2})["sync"] == 1
    g = workloads.stencil_grid((256, 256), seed=0)
    got = _run(pk, g, w, 100, torch.float64)
    assert rel_err(got, oracle.stencil(g, w, 100)) <= 1e-12
    np.testing.assert_array_equal(got, _run(pk, g, w, 100, torch.float64, baseline=True))


def test_full_size_matches_oracle_for_a_few_steps(pk):
    g = workloads.stencil_grid((3072, 3072), seed=0)
    w = workloads.stencil_weights("2d5pt")
    got = _run(pk, g, w, 6, torch.float64, tuning={"kernel": 1})
    assert rel_err(got, oracle.stencil(g, w, 6)) <= 1e-12
    base = _run(pk, g, w, 6, torch.float64, baseline=True)
    np.testing.assert_array_equal(got, base)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_full_size_3d_matches_oracle_for_a_few_steps(pk, dtype):
    """256^3 in the benchmark's launch configuration (columns 64 x 32 x 32,
    streamed, LDS and register planes in FP64; every plane in registers in
    FP32), five steps against the oracle, and bitwise against the per-step
    baseline."""
    g = workloads.stencil_grid((256, 256, 256), seed=0)
    w = workloads.stencil_weights("3d7pt")
    tdt = torch.float64 if dtype == "float64" else torch.float32
    if dtype == "float32":
        g = g.astype(np.float32).astype(np.float64)
        w = w.astype(np.float32).astype(np.float64)
    got = _run(pk, g, w, 5, tdt)
    assert rel_err(got, oracle.stencil(g, w, 5)) <= (1e-12 if dtype == "float64" else 1e-5)
    np.testing.assert_array_equal(got, _run(pk, g, w, 5, tdt, baseline=True))
    plan = pk.stencil_plan((256, 256, 256), w, dtype)
    assert plan["planes_per_lane"] == 32 and plan["tiles"] == 256 and plan["cached_tiles"] == 256


def test_plan_reports_cached_share(pk):
    pl = pk.stencil_plan((3072, 3072), workloads.stencil_weights("2d5pt"), "float64")
    assert pl["tiles"] >= pl["cached_tiles"] > 0
    assert pl["interior_cells"] == 3070 * 3070


@pytest.mark.parametrize("dtype,planes", [("float64", 1), ("float64", 5), ("float64", 13), ("float64", 32),
                                          ("float32", 3), ("float32", 8), ("float32", 32)])
def test_3d_column_depths_match_baseline_bitwise(pk, dtype, planes):
    """Every 3D column depth (ragged in x, y and z; all planes in registers,
    and deeper than the register cache so that the bottom planes stream;
    several columns per workgroup when the depth is small) gives the
    baseline's bits and the oracle's values."""
    shape = (37, 23, 131)     # interior 35 x 21 x 129: x tiles 64 + 64 + 1
    g = workloads.stencil_grid(shape, seed=21)
    w = workloads.stencil_weights("3d7pt")
    tdt = torch.float64 if dtype == "float64" else torch.float32
    if dtype == "float32":
        g = g.astype(np.float32).astype(np.float64)
        w = w.astype(np.float32).astype(np.float64)
    tu = {"planes_per_lane": planes}
    a = _run(pk, g, w, 9, tdt, tuning=tu)
    c = _run(pk, g, w, 9, tdt, tuning=dict(tu, max_cached_tiles=7))
    n = _run(pk, g, w, 9, tdt, tuning=dict(tu, max_cached_tiles=-1))
    b = _run(pk, g, w, 9, tdt, baseline=True)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(c, b)
    np.testing.assert_array_equal(n, b)
    assert rel_err(a, oracle.stencil(g, w, 9)) <= (1e-12 if dtype == "float64" else 1e-5)
    plan = pk.stencil_plan(shape, w, dtype, tuning=tu)
    assert plan["planes_per_lane"] == planes
    assert plan["tiles"] == 3 * 1 * -(-35 // planes)     # columns: 3 along x, 1 along y


@pytest.mark.parametrize("kind,shape,dtype", [("2d5pt", (300, 520), "float64"), ("2d9pt", (257, 190), "float32"),
                                              ("3d7pt", (40, 45, 130), "float32"), ("2d13pt", (210, 333), "float64"),
                                              ("2d25pt", (99, 150), "float32"), ("3d13pt", (20, 37, 90), "float64")])
def test_autotune_returns_a_valid_plan_and_untuned_runs_use_it(pk, kind, shape, dtype):
    w = workloads.stencil_weights(kind)
    tuning, rate = pk.stencil_autotune(shape, w, dtype, probe_steps=8, remember=True)
    assert rate > 0
    plan = pk.stencil_plan(shape, w, dtype, tuning=tuning)
    assert plan["tiles"] > 0
    g = workloads.stencil_grid(shape, seed=31, r=workloads.stencil_radius(kind))
    tdt = torch.float64 if dtype == "float64" else torch.float32
    if dtype == "float32":
        g = g.astype(np.float32).astype(np.float64)
    remembered = _run(pk, g, w, 7, tdt)                  # untuned: uses the remembered plan
    explicit = _run(pk, g, w, 7, tdt, tuning=tuning)
    base = _run(pk, g, w, 7, tdt, baseline=True)
    np.testing.assert_array_equal(remembered, explicit)
    np.testing.assert_array_equal(remembered, base)


@pytest.mark.parametrize("kind,dtype", [("2d5pt", "float64"), ("2d9pt", "float32"), ("2d5pt", "float32")])
def test_batched_grids_equal_single_runs_bitwise(pk, kind, dtype):
    """Uneven grids (including a one-tile grid and ragged tiles) in one launch
    give exactly the bits of one launch per grid and the oracle's values."""
    shapes = [(66, 130), (5, 7), (257, 190), (40, 64), (129, 300), (18, 33)]
    w = workloads.stencil_weights(kind)
    tdt = torch.float64 if dtype == "float64" else torch.float32
    if dtype == "float32":
        w = w.astype(np.float32).astype(np.float64)
    grids_np = []
    for j, sh in enumerate(shapes):
        g = workloads.stencil_grid(sh, seed=40 + j, ring_value=0.25 * j)
        grids_np.append(g.astype(np.float32).astype(np.float64) if dtype == "float32" else g)
    devs = [to_dev(g, tdt) for g in grids_np]
    pk.stencil_run_batched(devs, w, 17)
    torch.cuda.synchronize()
    for g, d in zip(grids_np, devs):
        single = _run(pk, g, w, 17, tdt)
        got = d.cpu().double().numpy()
        np.testing.assert_array_equal(got, single)
        assert rel_err(got, oracle.stencil(g, w, 17)) <= (1e-12 if dtype == "float64" else 1e-5)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_batched_plan_reruns_bitwise(pk, dtype):
    """perks_stencil_batch_*: one plan, three runs (its HIP graph when the
    runtime gives one), the grids refilled in place between runs (new values,
    new rings); every run bitwise the single-grid runs of the same input."""
    shapes = [(66, 130), (5, 7), (257, 190), (129, 300)]
    w = workloads.stencil_weights("2d9pt")
    tdt = getattr(torch, dtype)
    devs = [to_dev(np.zeros(sh), tdt) for sh in shapes]
    plan = pk.StencilBatch(devs, w, 19)
    print(f"batched plan {dtype}: graph {plan.has_graph()}", flush=True)
    for rep in range(3):
        inputs = [workloads.stencil_grid(sh, seed=100 * rep + j, ring_value=0.1 * (j + rep)).astype(dtype)
                  for j, sh in enumerate(shapes)]
        for d, g in zip(devs, inputs):
            d.copy_(torch.from_numpy(g))
        plan.run()
        torch.cuda.synchronize()
        for d, g in zip(devs, inputs):
            np.testing.assert_array_equal(d.cpu().double().numpy(), _run(pk, g, w, 19, tdt, baseline=True))
    plan.close()


def test_batched_many_small_grids(pk):
    sides = workloads.lognormal_sides(64, lo=16, hi=96, seed=5)
    w = workloads.stencil_weights("2d5pt")
    grids_np = [workloads.stencil_grid((int(s), int(s) + 3), seed=int(s)) for s in sides]
    devs = [to_dev(g) for g in grids_np]
    pk.stencil_run_batched(devs, w, 25)
    torch.cuda.synchronize()
    for g, d in zip(grids_np[:8], devs[:8]):
        assert rel_err(d.cpu().numpy(), oracle.stencil(g, w, 25)) <= 1e-12
