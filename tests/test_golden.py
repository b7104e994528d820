"""Fixtures under tests/golden/: the parameters the paper prints (Table 1,
Sec. 6) against the defaults of the oracle and of the library's binding, and
the oracle against the values that tests/golden/make_golden.py stored from it
(a change of the oracle's arithmetic shows up as a changed fixture)."""
import json
import os

import numpy as np

import paper_1912_09240_amd as pr
from oracle import chem as CH

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_table1_defaults():
    t = _load("table1_parameters.json")
    for c in (CH.Chem(), pr.Chem()):
        assert c.tau_x == t["tau_x"] and c.eps == t["eps"]
        k = list(t["k"])
        k[3] = t["reading_k3"]  # the one reading of the table (see the fixture's note)
        assert np.allclose(c.k, k, rtol=0, atol=0)
        assert tuple(c.x0) == tuple(t["x0_mean_sd"]) and tuple(c.y0) == tuple(t["y0_mean_sd"])
    assert (t["grid"][1] - t["grid"][0]) / t["dx"] == 600
    assert round(40.0 / t["dt_fine"]) == 40_000 and 40.0 / t["n_intervals"] == t["reporting_dt"]


def test_oracle_reproduces_its_stored_values(oracle_lib):
    import sys
    sys.path.insert(0, GOLDEN)
    import make_golden
    got = make_golden.values()
    ref = _load("oracle_values.json")
    assert got["philox_blocks_seed7_tag0_m3_p0to3"] == ref["philox_blocks_seed7_tag0_m3_p0to3"]
    assert np.array_equal(np.array(got["normals_seed7_tag1_m0_p0to3"]), np.array(ref["normals_seed7_tag1_m0_p0to3"]))
    a = np.array(got["small_workload_knots_after_one_iteration_t10"])
    b = np.array(ref["small_workload_knots_after_one_iteration_t10"])
    assert np.abs(a - b).max() < 1e-12
    assert abs(got["chem_fast_mean_table1_reading"] - ref["chem_fast_mean_table1_reading"]) < 1e-10
    for m, row in ref["advection_error_at_T_after_one_iteration"].items():
        for it, v in row.items():
            assert abs(got["advection_error_at_T_after_one_iteration"][m][it] - v) < 1e-12 * max(1.0, v)
