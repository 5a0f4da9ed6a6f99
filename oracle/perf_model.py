"""PERKS performance model (Sec. 5.2, Eq. 5-10) -- TEST INFRASTRUCTURE ONLY.

All byte counts are in elements times the element size S(type), as in the
paper.  One reading is needed: Eq. 9 prints T_PERKS = max(T_gm(D), T_sm), but
the worked example (FP32 2d5pt, 3072^2, N = 1000, A100) arrives at 876.09
GCells/s only when the halo time of the cached part is added to T_gm(D):
3072^2 * 1000 / (9900.70 us + 871.22 us).  The model below therefore uses
T_PERKS = max(T_gm(D) + T_gm(halo), T_sm).
"""


def global_accesses(n_steps, d_uncache, d_cache):
    """Eq. 5: A_gm(D) = 2 N D_uncache + 2 D_cache (elements)."""
    return 2 * n_steps * d_uncache + 2 * d_cache


def t_gm(accesses, elem_bytes, bw_bytes_per_s):
    """Eq. 6: T_gm = A_gm * S(type) / B_gm (seconds)."""
    return accesses * elem_bytes / bw_bytes_per_s


def shared_accesses(n_steps, d_cache_sm):
    """Eq. 7: A_sm = 2 (N - 1) D^sm_cache (elements)."""
    return 2 * (n_steps - 1) * d_cache_sm


def t_sm(a_sm_cache, a_sm_kernel, elem_bytes, bw_sm_bytes_per_s):
    """Eq. 8: T_sm = (A_sm(D^sm_cache) + A_sm(KERNEL)) * S(type) / B_sm."""
    return (a_sm_cache + a_sm_kernel) * elem_bytes / bw_sm_bytes_per_s


def t_perks(t_gm_domain, t_gm_halo=0.0, t_sm_total=0.0):
    """Eq. 9 with the halo term (see module docstring)."""
    return max(t_gm_domain + t_gm_halo, t_sm_total)


def projected_cells_per_s(domain_cells, n_steps, t):
    """Eq. 10: P = D * N / T_PERKS (cells updated per second)."""
    return domain_cells * n_steps / t
