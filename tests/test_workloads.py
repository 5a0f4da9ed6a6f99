"""Checks of the seeded input generators (no GPU)."""
import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("side", [1, 2, 3, 17])
def test_torch_poisson2d_equals_numpy(side):
    torch = pytest.importorskip("torch")
    rp, ci, v = workloads.poisson_csr(side, 2)
    trp, tci, tv = workloads.poisson2d_csr_torch(side, device="cpu")
    np.testing.assert_array_equal(trp.numpy(), rp)
    np.testing.assert_array_equal(tci.numpy(), ci)
    np.testing.assert_array_equal(tv.numpy(), v)


def test_poisson_rows_are_sorted_and_symmetric():
    rp, ci, v = workloads.poisson_csr(6, 3)
    n = rp.size - 1
    A = workloads.csr_to_dense(rp, ci, v, n)
    np.testing.assert_array_equal(A, A.T)
    for i in range(n):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)


def test_lognormal_sides_range_and_seed():
    s = workloads.lognormal_sides(512, seed=0)
    assert s.min() >= 64 and s.max() <= 1024
    np.testing.assert_array_equal(s, workloads.lognormal_sides(512, seed=0))
    # log-uniform: the median side is near sqrt(64 * 1024) = 256
    assert 200 < np.median(s) < 330


def test_torch_diffusion_assembly_equals_numpy():
    torch = pytest.importorskip("torch")
    g = workloads.grf_log_k(13, seed=4)
    rp, ci, v = workloads.diffusion_csr(np.exp(g))
    trp, tci, tv = workloads.diffusion_csr_torch(torch.exp(torch.from_numpy(g)))
    np.testing.assert_array_equal(trp.numpy(), rp)
    np.testing.assert_array_equal(tci.numpy(), ci)
    np.testing.assert_allclose(tv.numpy(), v, rtol=1e-15, atol=0)


def test_torch_grf_statistics():
    torch = pytest.importorskip("torch")
    vals = torch.stack([workloads.grf_log_k_torch(16, seed=s, device="cpu")[5, 7] for s in range(400)])
    assert abs(float(vals.var()) - 1.0) < 0.2 and abs(float(vals.mean())) < 0.15


def test_torch_planes_equal_numpy():
    torch = pytest.importorskip("torch")
    g = workloads.grf_log_k(11, seed=2)
    np.testing.assert_allclose(workloads.diffusion_planes_torch(torch.exp(torch.from_numpy(g))).numpy(),
                               workloads.diffusion_planes(np.exp(g)), rtol=1e-15, atol=0)
