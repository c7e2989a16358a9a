"""Writes config2_serial_oracle.json: the FP64 oracle's serial fine solve of
the 128^2 Galloway-Proctor workload (Rm = 100, kz = 0.57, T = 64 over 64
slices of length 1, fine SBDF2 dt = 2e-3 restarted every slice, seeded
initial field 200000), its slice-boundary norms |U_n| and its amplitude
growth rate.  Calls only ``oracle`` and ``synthetic``.  Takes a few minutes:

    python tests/golden/make_config2_growth.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import parareal as opr, stepper  # noqa: E402
from synthetic import initial_field  # noqa: E402

N, KZ, RM, T, P, DTF, SEED = 128, 0.57, 100.0, 64.0, 64, 2e-3, 200000


def main():
    t0 = time.time()
    F = stepper.SliceSolver("gp", RM, KZ, N, T / P, DTF)
    U = opr.serial_fine(initial_field(N, KZ, SEED), P, T / P, F)
    norms = [opr.norm2(u) for u in U]
    gamma = opr.growth_rate(norms, np.arange(P + 1) * (T / P))
    out = {"workload": "gp Rm=100 kz=0.57 N=128 T=64 P=64 dt_fine=2e-3 sbdf2, "
                       "initial field synthetic.initial_field(128, 0.57, 200000)",
           "writer": "tests/golden/make_config2_growth.py (oracle serial fine solve)",
           "norms": norms, "growth_rate": gamma}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_serial_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"growth {gamma:.12f} in {time.time() - t0:.0f} s -> {path}")


if __name__ == "__main__":
    main()
