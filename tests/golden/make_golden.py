"""Writes tests/golden/oracle_values.json from the oracle alone (no library
code): a few Philox blocks and normals, the small workload's quantile knots
after one micro-macro iteration, the chemical system's fast mean, and the
linear-advection errors after one iteration.  The CPU tests compare the
oracle against these stored values, so that a change of the oracle's
arithmetic shows up as a changed fixture in review.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import advection as AD  # noqa: E402
from oracle import chem as CH  # noqa: E402
from oracle import coarse as OC  # noqa: E402
from oracle import histogram as H  # noqa: E402
from oracle import iterate as OI  # noqa: E402
from oracle import particles as OP  # noqa: E402


def values():
    out = {}
    out["philox_blocks_seed7_tag0_m3_p0to3"] = OP.blocks(7, 0, 0, 3, 0, 4).astype(int).tolist()
    out["normals_seed7_tag1_m0_p0to3"] = OP.normals(7, 0, 1, 0, 0, 4, 2).tolist()
    sde = OP.Sde(lam=1.0, eps=0.1, beta=2.0)
    g = OC.Grid(200)
    pr, hp = OI.micmac_parareal(sde, 0, 0, 10_000, 1.0, 1e-3, 10, g, 100)
    pr.iterate()
    out["small_workload_knots_after_one_iteration_t10"] = [float(v) for v in pr.rho[10]]
    out["chem_fast_mean_table1_reading"] = CH.mean_fast(CH.Chem())
    ga = OC.Grid(800, -8.0, 8.0)
    rho0 = AD.gaussian_cells(ga, 2.0, 0.5)
    errs = {}
    for name, (e, b) in dict(underdiffusive=(1.0, 2.0), advection=(2.0, 1.0), overdiffusive=(1.0, 0.5)).items():
        row = {}
        for it, kind in dict(add=H.J_ADD, quantile=H.J_QUANTILE).items():
            p, serial, _, _ = AD.fp_parareal(AD.Advection(), AD.Advection(e, b), ga, rho0, 1.0, 10, kind)
            p.iterate()
            row[it] = H.hist_error(p.rho[10], serial[10])
        errs[name] = row
    out["advection_error_at_T_after_one_iteration"] = errs
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "oracle_values.json"), "w") as f:
        json.dump(values(), f, indent=1)
    print("written")
