"""The 128^2 Galloway-Proctor workload's own coarse path against the FP64
oracle: the 64^2 coarse grid with dt = 1e-2 (the one-workgroup convolution
sweep at box width 43 with its table of flow phases), pipelined as the
benchmark runs it, every slice state and defect at a fixed iteration count;
and the full workload's growth rate against the oracle's serial fine solve.
Bars: states 1e-12 relative L2, defects 2e-12 absolute, growth rate 1e-6."""
import json
import os

import numpy as np
import pytest

from oracle import parareal as opr, stepper
from synthetic import initial_field

pytestmark = pytest.mark.gpu

TOL = 1e-12
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def oracle_run():
    """Oracle Parareal: Rm = 100, kz = 0.57, 128^2 fine (dt = 2e-3), 64^2
    coarse (dt = 1e-2), 8 slices of length 0.5 (start times off the integer
    grid), two iterations."""
    N, Nc, kz, Rm, T, P, dtf, dtc, iters = 128, 64, 0.57, 100.0, 4.0, 8, 2e-3, 1e-2, 2
    b0 = initial_field(N, kz, 200000)
    F = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtf)
    G = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtc, Nc)
    ref = opr.parareal(b0, P, T / P, F, G, tol=0.0, max_iter=iters)
    return dict(N=N, Nc=Nc, kz=kz, Rm=Rm, T=T, P=P, dtf=dtf, dtc=dtc, iters=iters, b0=b0, ref=ref)


@pytest.mark.parametrize("chunks", [0, 2, 4])
def test_headline_coarse_sweep_matches_oracle(lib, oracle_run, chunks):
    w = oracle_run
    print(f"headline coarse path: chunks={chunks}", flush=True)
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", w["Rm"], w["kz"], w["N"])
        ctx.set_time(w["T"], w["P"], w["dtf"], w["dtc"], w["Nc"])
        ctx.set_pipeline(chunks, 2)
        ctx.set_initial(w["b0"])
        rep = ctx.parareal(0.0, w["iters"])
        U = ctx.get_slices()
    ref = w["ref"]
    assert rep["iters"] == w["iters"]
    for n in range(w["P"] + 1):
        assert rel(U[n], ref.U[n]) <= TOL, (n, rel(U[n], ref.U[n]))
    assert np.allclose(rep["sigma"], ref.sigma, rtol=0, atol=2 * TOL), (rep["sigma"], ref.sigma)


def test_config2_growth_rate_matches_oracle_serial_solve(lib):
    """The full 128^2 workload (T = 64 over 64 slices, coarse 64^2 with dt =
    1e-2, tol 1e-8, pipelined) solved by Parareal on the GPU: its growth rate
    equals the oracle's serial fine solve's to 1e-6 and every slice norm the
    oracle's to 1e-7 relative (the stopping tolerance is 1e-8); the oracle
    values come from tests/golden/make_config2_growth.py."""
    with open(os.path.join(GOLDEN, "config2_serial_oracle.json")) as fh:
        gold = json.load(fh)
    N, kz, Rm, T, P = 128, 0.57, 100.0, 64.0, 64
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", Rm, kz, N)
        ctx.set_time(T, P, 2e-3, 1e-2, 64)
        ctx.set_initial(initial_field(N, kz, 200000))
        rep = ctx.parareal(1e-8, P)
        gam = ctx.growth_rate()
        norms = ctx.slice_norms()
    print(f"k_con {rep['k_con']} growth {gam:.10f} oracle {gold['growth_rate']:.10f}", flush=True)
    assert 0 < rep["k_con"] <= P
    assert abs(gam - gold["growth_rate"]) <= 1e-6
    nr = np.asarray(gold["norms"])
    assert np.max(np.abs(np.asarray(norms) - nr) / nr) <= 1e-7
