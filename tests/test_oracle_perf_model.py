"""The performance model reproduces the paper's worked example (Sec. 5.2)."""
import json
import os

import pytest

from oracle import perf_model as pm

GOLD = os.path.join(os.path.dirname(__file__), "golden", "perf_model_worked_example.json")


def test_worked_example():
    g = json.load(open(GOLD))
    i, p = g["inputs"], g["printed"]
    assert i["tiles"] * i["tile_shape"][0] * i["tile_shape"][1] == 3072 * 2448 == i["d_cache_cells"]
    assert 1000 * 2 * 216 * (136 * 2 + 256 * 2) == i["halo_elements"]
    a = pm.global_accesses(i["n_steps"], i["domain_cells"] - i["d_cache_cells"], i["d_cache_cells"])
    t_dom = pm.t_gm(a, i["elem_bytes"], i["bw_bytes_per_s"])
    t_halo = pm.t_gm(i["halo_elements"], i["elem_bytes"], i["bw_bytes_per_s"])
    assert t_dom * 1e6 == pytest.approx(p["t_gm_domain_us"], abs=0.005)
    assert t_halo * 1e6 == pytest.approx(p["t_gm_halo_us"], abs=0.005)
    P = pm.projected_cells_per_s(i["domain_cells"], i["n_steps"], pm.t_perks(t_dom, t_halo))
    assert P / 1e9 == pytest.approx(p["gcells_per_s"], abs=0.005)
    # Eq. 9 read literally (max without the halo term) does not give the printed value
    P_literal = pm.projected_cells_per_s(i["domain_cells"], i["n_steps"], pm.t_perks(t_dom))
    assert abs(P_literal / 1e9 - p["gcells_per_s"]) > 50
