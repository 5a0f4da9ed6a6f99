"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only builds inputs (grids, weights, sparse matrices, right-hand
sides).  It holds none of the solver arithmetic: no stencil sweep, no
matrix-vector product, no Krylov step.  Both the CPU oracle and the GPU path
receive the arrays produced here, so parity never depends on a random number
generator being reimplemented twice.

Every random generator draws from ``numpy.random.default_rng(seed)``
(PCG64) in row-major order.
"""
from .stencil import (stencil_grid, stencil_weights, stencil_radius, interior_slices, STENCIL_KINDS,
                      WIDE_KINDS, WIDE3_KINDS)
from .diffusion import (grf_log_k, diffusion_csr, diffusion_problem, grf_log_k_torch, diffusion_csr_torch,
                        diffusion_problem_torch, diffusion_planes, diffusion_planes_torch)
from .sparse import (poisson_csr, poisson2d_csr_torch, random_spd_csr, rhs_uniform, rhs_normal,
                     csr_to_dense, lognormal_sides)

__all__ = [
    "stencil_grid", "stencil_weights", "stencil_radius", "interior_slices", "STENCIL_KINDS", "WIDE_KINDS",
    "WIDE3_KINDS",
    "poisson_csr", "poisson2d_csr_torch", "random_spd_csr", "rhs_uniform", "rhs_normal", "csr_to_dense",
    "lognormal_sides", "grf_log_k", "diffusion_csr", "diffusion_problem", "grf_log_k_torch",
    "diffusion_csr_torch", "diffusion_problem_torch", "diffusion_planes", "diffusion_planes_torch",
]
