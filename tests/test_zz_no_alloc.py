"""perks_stencil_run_noalloc (the entry point for callers that cannot
allocate device memory) against perks_stencil_run with the same plan
(tuning.kernel = 1: the radius-1 kernel with point-to-point halo words):
bitwise equal, on two calls in a row, the second with a smaller grid, called
through the C ABI; a grid too large for the fixed array is refused before
any GPU work."""
import ctypes

import numpy as np
import pytest

import workloads
from gpu_util import to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    import paper_2204_02064_amd as pk
    pk.lib()
    return pk


def _noalloc(pk, t, w, steps):
    wa, r = pk._coeff_array(w, t.dim())
    rc = pk.lib().perks_stencil_run_noalloc(ctypes.c_void_p(t.data_ptr()),
                                            wa.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), pk._shape_of(t, r),
                                            int(steps), pk._dtype_code(t), None)
    torch.cuda.synchronize()
    return rc


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_noalloc_matches_the_allocating_entry_point(pk, dtype):
    cases = [((517, 701), "2d5pt", 7, 3), ((130, 201), "2d9pt", 4, 8)]   # the second call is smaller
    for shape, kind, steps, seed in cases:
        g = workloads.stencil_grid(shape, seed=seed, ring_value=0.5).astype(dtype)
        rng = np.random.default_rng(seed)
        w = np.where(workloads.stencil_weights(kind) != 0, rng.uniform(0.0, 0.25, (3, 3)), 0.0)
        if dtype == "float32":
            w = w.astype(np.float32).astype(np.float64)
        a = to_dev(g, getattr(torch, dtype))
        b = a.clone()
        print(f"noalloc {dtype} {kind} {shape} {steps} steps", flush=True)
        assert _noalloc(pk, a, w, steps) == 0, pk.lib().perks_last_error()
        pk.stencil_run(b, w, steps, tuning={"kernel": 1})
        torch.cuda.synchronize()
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
        assert not np.array_equal(a.cpu().numpy(), g)


def test_noalloc_refuses_what_does_not_fit(pk):
    # FP64 6000 x 6000: its halo buffers exceed the fixed array (refused on
    # the host, before any kernel); a 3D grid and a radius-2 pattern too
    big = torch.zeros((6000, 6000), dtype=torch.float64, device="cuda")
    assert _noalloc(pk, big, workloads.stencil_weights("2d5pt"), 1) == -5
    del big
    g3 = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    assert _noalloc(pk, g3, workloads.stencil_weights("3d7pt"), 1) == -5
    g2 = torch.zeros((40, 40), dtype=torch.float64, device="cuda")
    assert _noalloc(pk, g2, workloads.stencil_weights("2d13pt"), 1) == -5
    assert _noalloc(pk, g2, workloads.stencil_weights("2d5pt"), 0) == 0
