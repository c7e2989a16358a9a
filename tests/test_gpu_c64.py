"""The complex64 variant (FP32 kernels; fields enter and leave as complex128)
against the FP64 oracle.  Bar: 1e-4 relative L2 for states (FP32 rounding,
unit 6e-8, grows with the transform length and the steps), defects to 1e-5
absolute.  The Parareal tolerance of this variant is 1e-4: 1e-8 lies far
below the FP32 rounding floor of the defect, and so, on the 128^2 workload,
does 1e-5."""
import json
import os

import numpy as np
import pytest

from oracle import parareal as opr, spectral as osp, stepper
from synthetic import initial_field

pytestmark = pytest.mark.gpu

TOL64 = 1e-4
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rand_box(N, seed, batch):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((batch, 3, N, N)) + 1j * rng.standard_normal((batch, 3, N, N))
    return b * osp.box_mask(N)


@pytest.mark.parametrize("flow", ["roberts", "gp"])
@pytest.mark.parametrize("N", [16, 32, 64, 128, 256, 512])
def test_c64_steps_match_oracle(lib, N, flow):
    """Three SBDF steps of a ragged batch with different start times."""
    kz, Rm, dt, batch = 0.57, 30.0, 2e-3, 3
    x = rand_box(N, 900 + N, batch)
    t0 = np.array([0.0, 1.7, 5.3])
    print(f"c64 steps N={N} flow={flow}", flush=True)
    with lib.Context(0) as ctx:
        ctx.set_problem(flow, Rm, kz, N)
        ctx.set_precision("c64")
        y = ctx.steps(t0, dt, 3, dev(x)).cpu().numpy()
    for f in range(batch):
        ref = stepper.propagate(x[f], flow, Rm, kz, t0[f], dt, 3)
        e = rel(y[f], ref)
        assert 1e-9 < e <= TOL64, (f, e)   # FP32 (not FP64) and within the bar


@pytest.mark.parametrize("chunks", [0, 2])
def test_c64_headline_coarse_path_matches_oracle(lib, chunks):
    """The 128^2 workload's coarse path (64^2 convolution sweep with dt =
    1e-2), 8 slices of length 0.5, two iterations, plain and pipelined."""
    N, Nc, kz, Rm, T, P, dtf, dtc, iters = 128, 64, 0.57, 100.0, 4.0, 8, 2e-3, 1e-2, 2
    b0 = initial_field(N, kz, 200000)
    F = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtf)
    G = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtc, Nc)
    ref = opr.parareal(b0, P, T / P, F, G, tol=0.0, max_iter=iters)
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", Rm, kz, N)
        ctx.set_precision("c64")
        ctx.set_time(T, P, dtf, dtc, Nc)
        ctx.set_pipeline(chunks, 2)
        ctx.set_initial(b0)
        rep = ctx.parareal(0.0, iters)
        U = ctx.get_slices()
    for n in range(P + 1):
        assert rel(U[n], ref.U[n]) <= TOL64, (n, rel(U[n], ref.U[n]))
    assert np.allclose(rep["sigma"], ref.sigma, rtol=0, atol=1e-5), (rep["sigma"], ref.sigma)


def test_c64_multi_launch_coarse_sweep(lib):
    """The multi-launch coarse sweep (N_C above 64) in complex64."""
    N, Nc, kz, Rm, T, P, dtf, dtc, iters = 256, 128, 0.57, 200.0, 0.5, 4, 2.5e-3, 2.5e-3, 2
    b0 = initial_field(N, kz, 31)
    F = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtf)
    G = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtc, Nc)
    ref = opr.parareal(b0, P, T / P, F, G, tol=0.0, max_iter=iters)
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", Rm, kz, N)
        ctx.set_precision("c64")
        ctx.set_time(T, P, dtf, dtc, Nc)
        ctx.set_pipeline(0)
        ctx.set_initial(b0)
        rep = ctx.parareal(0.0, iters)
        U = ctx.get_slices()
    for n in range(P + 1):
        assert rel(U[n], ref.U[n]) <= TOL64, (n, rel(U[n], ref.U[n]))
    assert np.allclose(rep["sigma"], ref.sigma, rtol=0, atol=1e-5)


def test_c64_config2_solve(lib):
    """The full 128^2 workload (T = 64 over 64 slices) in complex64.  FP32
    rounding gives the defect a floor near 2e-5 on this workload (measured:
    sigma_k wanders between 1e-5 and 3e-5 from k = 3 on), so the variant's
    tolerance is 1e-4; Parareal then stops at k_con = 3 like complex128 and
    its last state matches the complex64 serial fine solve (slice after slice
    on the GPU) to 1e-4.  Against the FP64 oracle's serial solve
    (tests/golden/make_config2_growth.py) complex64 carries a systematic
    drift: the growth rate comes out about 1.2e-5 low, so the slice norms
    part by about 1.2e-5 per unit time (7.7e-4 at t = 64); bars 5e-5 on the
    growth rate and 2e-3 on the norms."""
    import torch
    with open(os.path.join(GOLDEN, "config2_serial_oracle.json")) as fh:
        gold = json.load(fh)
    N, kz, Rm, T, P = 128, 0.57, 100.0, 64.0, 64
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", Rm, kz, N)
        ctx.set_precision("c64")
        ctx.set_time(T, P, 2e-3, 1e-2, 64)
        b0 = initial_field(N, kz, 200000)
        u = dev(b0[None])
        for n in range(P):
            u = ctx.fine([float(n)], u)
        ctx.set_initial(b0)
        rep = ctx.parareal(1e-4, P)
        gam = ctx.growth_rate()
        norms = ctx.slice_norms()
        UP = ctx.get_slices_dev()[P]
    d = float(torch.linalg.vector_norm(UP - u[0]) / torch.linalg.vector_norm(u[0]))
    nr = np.asarray(gold["norms"])
    en = float(np.max(np.abs(np.asarray(norms) - nr) / nr))
    print(f"c64 k_con {rep['k_con']} vs own serial {d:.2e}, norms vs oracle {en:.2e}, "
          f"growth {gam:.8f} oracle {gold['growth_rate']:.8f}", flush=True)
    assert rep["k_con"] == 3
    assert d <= 1e-4
    assert en <= 2e-3
    assert abs(gam - gold["growth_rate"]) <= 5e-5


def test_c64_unsupported_calls_are_rejected(lib):
    import torch
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", 50.0, 0.57, 32)
        ctx.set_precision("c64")
        with pytest.raises(lib.PitdynError):
            ctx.set_scheme("rk443", "sbdf2")
        ctx.set_time(1.0, 4, 1e-2, 5e-2, 16)
        with pytest.raises(lib.PitdynError):
            ctx.lg_init(2, 1)
        with pytest.raises(lib.PitdynError):
            ctx.autotune(2)
        with pytest.raises(lib.PitdynError):
            ctx.set_coarse_form(1)
        x = torch.zeros((1, 3, 32, 32), dtype=torch.complex128, device="cuda")
        with pytest.raises(lib.PitdynError):
            ctx.steps_noalloc([0.0], 1e-2, 1, x, torch.empty_like(x))
        ctx.set_initial(initial_field(32, 0.57, 1))
        ctx.parareal(0.0, 1)
        with pytest.raises(lib.PitdynError):
            ctx.get_coarse_values()
        # back to complex128: the same context runs RK443 again
        ctx.set_precision("c128")
        ctx.set_scheme("rk443", "sbdf2")
        ctx.set_time(1.0, 4, 1e-2, 5e-2, 16)
