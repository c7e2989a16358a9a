"""GPU parity of the batched-instances path (pd_batch_*): uneven instances
(grid 32..256, both flows, per-instance Rm and kz, coarse boxes held in LDS
and in global memory) against the FP64 oracle, graph replay against eager
launches (bitwise), and per-instance convergence against single-instance
contexts."""
import numpy as np
import pytest

from oracle import parareal as opr, stepper
from synthetic import initial_field

pytestmark = pytest.mark.gpu

TOL = 1e-12

# flow, Rm, kz, N, T, P, dt_fine, dt_coarse, N_coarse
INSTANCES = [
    ("gp", 50.0, 0.57, 32, 1.0, 4, 5e-3, 2.5e-2, 16),
    ("gp", 200.0, 0.9, 64, 1.2, 3, 4e-3, 2e-2, 32),
    ("roberts", 20.0, 1.0, 64, 2.0, 4, 5e-3, 2.5e-2, 64),
    ("gp", 80.0, 0.4, 128, 0.4, 2, 4e-3, 2e-2, 128),
    ("gp", 500.0, 0.3, 32, 1.0, 4, 5e-3, 2.5e-2, 32),
    # a 256^2 instance (the largest class of the mixed workload) with its
    # 128^2 coarse box stepped from global memory
    ("gp", 300.0, 0.7, 256, 0.05, 2, 2.5e-3, 2.5e-3, 128),
]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def fields():
    return [initial_field(p[3], p[2], 300000 + i) for i, p in enumerate(INSTANCES)]


def make_batch(lib, b0s):
    b = lib.Batch(0)
    for p, b0 in zip(INSTANCES, b0s):
        b.add(*p, b0)
    return b


def test_batch_matches_oracle_and_graph_matches_eager(lib):
    b0s = fields()
    iters = 2
    with make_batch(lib, b0s) as bg, make_batch(lib, b0s) as be:
        print("batch graph run", flush=True)
        bg.run(0.0, iters, use_graph=True)
        print("batch eager run", flush=True)
        be.run(0.0, iters, use_graph=False)
        for i, (flow, Rm, kz, N, T, P, dtf, dtc, Nc) in enumerate(INSTANCES):
            Ug, Ue = bg.slices(i), be.slices(i)
            assert np.array_equal(Ug, Ue), i
            F = stepper.SliceSolver(flow, Rm, kz, N, T / P, dtf)
            G = stepper.SliceSolver(flow, Rm, kz, N, T / P, dtc, Nc)
            ref = opr.parareal(b0s[i], P, T / P, F, G, tol=0.0, max_iter=iters)
            for n in range(P + 1):
                assert rel(Ug[n], ref.U[n]) <= TOL, (i, n, rel(Ug[n], ref.U[n]))
            rg = bg.result(i)
            assert rg["iters"] == iters
            assert np.allclose(rg["sigma"], ref.sigma, rtol=0, atol=2 * TOL)


def test_batch_convergence_matches_single_contexts(lib):
    """Each instance stops at its own k_con, the one a context alone reaches,
    with the same final states (to the parity bar) and growth rate."""
    b0s = fields()
    with make_batch(lib, b0s) as b:
        b.run(1e-9, 12)
        for i, (flow, Rm, kz, N, T, P, dtf, dtc, Nc) in enumerate(INSTANCES):
            with lib.Context(0) as ctx:
                ctx.set_problem(flow, Rm, kz, N)
                ctx.set_time(T, P, dtf, dtc, Nc)
                ctx.set_initial(b0s[i])
                rep = ctx.parareal(1e-9, 12)
                U = ctx.get_slices()
                g = ctx.growth_rate() if P >= 2 else None
            rb = b.result(i)
            assert rb["k_con"] == rep["k_con"], (i, rb["k_con"], rep["k_con"])
            Ub = b.slices(i)
            for n in range(P + 1):
                assert rel(Ub[n], U[n]) <= TOL, (i, n)
            if g is not None:
                assert abs(rb["growth_rate"] - g) <= 1e-9


def test_batch_rejects_bad_instances(lib):
    with lib.Batch(0) as b:
        with pytest.raises(lib.PitdynError):
            b.add("gp", 10.0, 1.0, 48, 1.0, 2, 1e-2, 5e-2, 0, np.zeros((3, 48, 48)))
        bad = np.zeros((3, 32, 32), complex)
        bad[1, 0, 16] = 1.0
        with pytest.raises(lib.PitdynError):
            b.add("gp", 10.0, 1.0, 32, 1.0, 2, 1e-2, 5e-2, 0, bad)
        with pytest.raises(lib.PitdynError):
            b.run(1e-8, 3)   # no instances
