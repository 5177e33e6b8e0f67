"""Write tests/golden/drop_64x32_fp64.json from the FP64 oracle only.

Workload: the small sessile-drop case -- 64x32 D2Q9, tau = 1, G = -5,
psi = 1 - exp(-rho), flat solid band of 8 rows with tanh wall functions
(width 2, core range 1 amplitude 0.5, tail range 3 amplitude 0.3, eps = 1),
half-disc drop of radius 12 on the wall (rho_l = 2.0, rho_g = 0.15), 2000 steps.
The stored values lock the oracle: a change to its arithmetic must regenerate
this file in a commit that names the passage of the paper justifying it.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1202_6130_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "drop_64x32_fp64.json")
SAMPLES = [(0, 32), (1, 32), (5, 20), (10, 32), (12, 40), (20, 10), (27, 0), (31, 63)]


def main():
    nx, ny = 64, 32
    p = O.make_params(nx, ny, tau=1.0, G=-5.0, G_R=0.5, G_A=0.3, eps=1.0)
    w = O.Walls.flat_slab(nx, ny, 8, 2.0, 1.0, 3.0)
    f = O.run(p, w, O.init(p, I.drop_field(nx, ny, 12.0)), 2000)
    rho, ux, uy, tot = O.macros(p, w, f)
    ang = O.contact_angle(p, w, f, 1.07, 0.0)
    data = {
        "workload": "sessile drop 64x32, 2000 steps, FP64 oracle",
        "totals": tot.tolist(),
        "contact_angle": ang.tolist(),
        "samples": [{"y": y, "x": x, "rho": rho[y, x], "ux": ux[y, x], "uy": uy[y, x]}
                    for y, x in SAMPLES],
    }
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
