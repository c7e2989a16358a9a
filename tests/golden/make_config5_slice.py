"""Writes config5_slice_oracle.json: the FP64 oracle's fine propagator F over
one whole slice of the 512^2 Galloway-Proctor workload (Rm = 2000,
kz = 0.57, fine SBDF2 dt = 5e-4, 2000 steps from the slice start t0 = n,
slice length 1), for four seeded fields over the whole 2/3 box (amplitude 1)
at slice starts n = 0, 37, 128, 255.  Stored per field: the seed, t0, the
two-norm of the result (all three components of the box coefficients), the
norm of each component, and the coefficients of every mode with
|kx|, |ky| <= 4 plus 240 seeded box positions.  Calls only ``oracle`` and
``synthetic``; about 6 minutes on 4 cores:

    python tests/golden/make_config5_slice.py
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import stepper  # noqa: E402
from synthetic import initial_field  # noqa: E402

N, KZ, RM, DTF, NSTEPS = 512, 0.57, 2000.0, 5e-4, 2000
CASES = ((520000, 0), (520001, 37), (520002, 128), (520003, 255))  # (seed, slice index n)
K = (N - 1) // 3


def sample_positions():
    """(c, ky, kx) triples: every mode with |kx|, |ky| <= 4 in each component,
    then 240 positions drawn uniformly over the 2/3 box (seeded)."""
    pos = [(c, ky, kx) for c in range(3) for ky in range(-4, 5) for kx in range(-4, 5)]
    rng = np.random.default_rng(5120)
    for _ in range(240):
        pos.append((int(rng.integers(0, 3)), int(rng.integers(-K, K + 1)),
                    int(rng.integers(-K, K + 1))))
    return pos


def run(case):
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    seed, n = case
    b0 = initial_field(N, KZ, seed, amp=1.0, kmax=1000.0)
    t = time.time()
    y = stepper.propagate(b0, "gp", RM, KZ, float(n), DTF, NSTEPS)
    samples = [[c, ky, kx, float(y[c, ky % N, kx % N].real), float(y[c, ky % N, kx % N].imag)]
               for c, ky, kx in sample_positions()]
    return {"seed": seed, "t0": float(n), "norm": float(np.linalg.norm(y)),
            "component_norms": [float(np.linalg.norm(y[c])) for c in range(3)],
            "samples": samples, "seconds": time.time() - t}


def main():
    t0 = time.time()
    with mp.get_context("fork").Pool(len(CASES)) as pool:
        fields = pool.map(run, CASES)
    out = {"workload": "gp Rm=2000 kz=0.57 N=512, F over one slice: sbdf2 dt=5e-4, 2000 steps "
                       "from t0 = n; inputs synthetic.initial_field(512, 0.57, seed, amp=1, "
                       "kmax=1000) (the whole 2/3 box)",
           "writer": "tests/golden/make_config5_slice.py (oracle fine propagator)",
           "layout": "samples: [component, ky, kx, re, im] of the result b_hat (b = sum "
                     "b_hat e^{ik.x})",
           "fields": fields}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config5_slice_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"{len(fields)} fields in {time.time() - t0:.0f} s -> {path}")


if __name__ == "__main__":
    main()
