"""PERKS performance model (Sec. 5.2, Eq. 5-10) -- TEST INFRASTRUCTURE ONLY.

All byte counts are in elements times the element size S(type), as in the
paper.  One reading is needed: Eq. 9 prints T_PERKS = max(T_gm(D), T_sm), but
the worked example (FP32 2d5pt, 3072^2, N = 1000, A100) arrives at 876.09
GCells/s only when the halo time of the cached part is added to T_gm(D):
3072^2 * 1000 / (9900.70 us + 871.22 us).  The model below therefore uses
the global-memory side T_gm(D) + T_gm(halo).

The shared-memory side of Eq. 9 (Eq. 7 for A_sm and Eq. 8 for T_sm) is not
part of this model: the paper prints no value that would pin it (its worked
example is global-memory bound), and Eq. 7 is garbled (N (L_sm + S_sm) is
set equal to 2 (N - 1) D^sm_cache).
"""


def global_accesses(n_steps, d_uncache, d_cache):
    """Eq. 5: A_gm(D) = 2 N D_uncache + 2 D_cache (elements)."""
    return 2 * n_steps * d_uncache + 2 * d_cache


def t_gm(accesses, elem_bytes, bw_bytes_per_s):
    """Eq. 6: T_gm = A_gm * S(type) / B_gm (seconds)."""
    return accesses * elem_bytes / bw_bytes_per_s


def t_perks(t_gm_domain, t_gm_halo=0.0):
    """Eq. 9, global-memory side, with the halo term (see module docstring)."""
    return t_gm_domain + t_gm_halo


def projected_cells_per_s(domain_cells, n_steps, t):
    """Eq. 10: P = D * N / T_PERKS (cells updated per second)."""
    return domain_cells * n_steps / t
