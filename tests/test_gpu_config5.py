"""The largest single-GPU workload at its full size: Galloway-Proctor flow,
Rm = 2000, kz = 0.57, 512^2 grid, T = 256 over 256 slices, fine SBDF2 with
dt = 5e-4.  The batched fine propagator runs over all 256 slices in the
launch configuration the benchmark times; the oracle recomputes sampled
slices step by step (a whole 2000-step slice costs the oracle minutes, so
the samples take a few steps).  Bar: 1e-12 relative L2."""
import ctypes
import json
import os

import numpy as np
import pytest

from oracle import stepper

pytestmark = pytest.mark.gpu

TOL = 1e-12
N, KZ, RM, T, P, DTF = 512, 0.57, 2000.0, 256.0, 256, 5e-4


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def seeded(lib, seed, kmax=1000.0, amp=1.0):
    """A field over the whole 2/3 box from the library's host generator
    (bitwise the reference generator's, see tests/test_synthetic.py)."""
    out = np.empty((3, N, N), np.complex128)
    assert lib.lib.pd_seed_field(N, KZ, ctypes.c_uint64(seed), amp, kmax,
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == lib.OK
    return out


def test_config5_batched_fine_steps_sampled(lib):
    """256 fields over the whole box (16 distinct seeded fields at 16 start
    times each), three fine steps in one batch, for every launch variant."""
    import torch
    distinct = np.stack([seeded(lib, 510000 + i) for i in range(16)])
    t0 = np.arange(P, dtype=np.float64) * (T / P)
    x = torch.from_numpy(distinct).cuda().repeat(16, 1, 1, 1)       # field f = distinct[f % 16]
    samples = (0, 17, 130, 255)
    refs = {f: stepper.propagate(distinct[f % 16], "gp", RM, KZ, t0[f], DTF, 3) for f in samples}
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", RM, KZ, N)
        ctx.set_path(0)
        try:
            for rv in range(len(lib.variants(N, 0))):
                for cv in range(len(lib.variants(N, 1))):
                    lib.select_variant(N, rv, cv)
                    print(f"config5 batch of {P}, variants rows {rv} cols {cv}", flush=True)
                    y = ctx.steps(t0, DTF, 3, x)
                    for f in samples:
                        e = rel(y[f].cpu().numpy(), refs[f])
                        assert e <= TOL, (rv, cv, f, e)
                    del y
        finally:
            lib.select_variant(N, 0, 0)


def test_config5_stepwise_sweep_matches_oracle(lib):
    """The benchmark's step: pd_fine_sweep_steps over the context's 256
    slice states (the initial coarse run from the library's seeded field),
    after autotuning; sampled slices against the oracle."""
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", RM, KZ, N)
        ctx.set_time(T, P, DTF, 2.5e-3, 64)
        ctx.seed_initial(500000, 1e-3, 4.0)
        ctx.parareal(0.0, 0)
        print("config5 stepwise sweep: autotune", flush=True)
        ctx.autotune(2)
        samples = (0, 1, 200)
        U = ctx.get_slices_dev()
        start = {n: U[n].cpu().numpy() for n in samples}
        del U
        ctx.set_fine_blocking(4, 3)             # the blocked order (groups of 4 on 3 streams)
        ctx.fine_sweep_steps(0, 2)
        ms = ctx.fine_sweep_steps(2, 1, timed=True)
        assert ms[0] == ms[1] == -1.0 and ms[2] > 0
        for n in samples:
            y = ctx.get_fine_states_dev(n, 1)[0].cpu().numpy()
            ref = stepper.propagate(start[n], "gp", RM, KZ, n * (T / P), DTF, 3)
            assert rel(y, ref) <= TOL, (n, rel(y, ref))
        with pytest.raises(lib.PitdynError):
            ctx.fine_sweep_steps(5, 1)          # the sweep stands at step 3
        # the same sweep continued with whole-batch launches, kernel by kernel
        ctx.set_fine_blocking(0)
        ms = ctx.fine_sweep_steps(3, 1, timed=True)
        assert all(m > 0 for m in ms)
        y = ctx.get_fine_states_dev(200, 1)[0].cpu().numpy()
        ref = stepper.propagate(start[200], "gp", RM, KZ, 200 * (T / P), DTF, 4)
        assert rel(y, ref) <= TOL, rel(y, ref)


GOLD5 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config5_slice_oracle.json")


def test_config5_whole_slice_matches_oracle(lib):
    """F over one whole slice (2000 fine steps) of the 512^2 workload, for four
    seeded whole-box fields starting at slices 0, 37, 128, 255, in one batch
    (blocked as the library does by default), against the oracle's results
    stored by tests/golden/make_config5_slice.py: the norm of each result and
    of its components, and 483 sampled coefficients, each within 1e-12 of the
    result's norm."""
    import torch
    with open(GOLD5) as fh:
        gold = json.load(fh)
    fields = gold["fields"]
    x = torch.from_numpy(np.stack([seeded(lib, f["seed"]) for f in fields])).cuda()
    t0 = np.array([f["t0"] for f in fields])
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", RM, KZ, N)
        ctx.set_time(T, P, DTF, 2.5e-3, 64)
        print(f"config5 whole slice: {len(fields)} fields, blocking {ctx.fine_blocking()}", flush=True)
        y = ctx.fine(t0, x).cpu().numpy()
    worst = 0.0
    for f, yi in zip(fields, y):
        nrm = f["norm"]
        assert abs(np.linalg.norm(yi) - nrm) <= TOL * nrm, (f["seed"], np.linalg.norm(yi), nrm)
        for c in range(3):
            cn = f["component_norms"][c]
            assert abs(np.linalg.norm(yi[c]) - cn) <= TOL * nrm
        for c, ky, kx, re, im in f["samples"]:
            e = abs(yi[c, ky % N, kx % N] - complex(re, im)) / nrm
            worst = max(worst, e)
            assert e <= TOL, (f["seed"], c, ky, kx, e)
    print(f"worst sampled coefficient difference / norm: {worst:.2e}", flush=True)

