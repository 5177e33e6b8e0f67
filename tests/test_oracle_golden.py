"""Regression lock of the oracle on the small sessile-drop case.

The stored file is written by tests/golden/make_golden.py, which calls only the
oracle; it guards against accidental changes of the oracle's arithmetic.
"""
import json
import os

import numpy as np

from paper_1202_6130_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden", "drop_64x32_fp64.json")


def test_oracle_matches_golden(orc):
    with open(GOLD) as fh:
        g = json.load(fh)
    nx, ny = 64, 32
    p = orc.make_params(nx, ny, tau=1.0, G=-5.0, G_R=0.5, G_A=0.3, eps=1.0)
    w = orc.Walls.flat_slab(nx, ny, 8, 2.0, 1.0, 3.0)
    f = orc.run(p, w, orc.init(p, I.drop_field(nx, ny, 12.0)), 2000)
    rho, ux, uy, tot = orc.macros(p, w, f)
    assert np.allclose(tot, g["totals"], rtol=1e-12, atol=1e-12)
    ang = orc.contact_angle(p, w, f, 1.07, 0.0)
    assert np.allclose(ang, g["contact_angle"], rtol=1e-10, atol=1e-10)
    for s in g["samples"]:
        y, x = s["y"], s["x"]
        assert abs(rho[y, x] - s["rho"]) < 1e-12
        assert abs(ux[y, x] - s["ux"]) < 1e-13
        assert abs(uy[y, x] - s["uy"]) < 1e-13
