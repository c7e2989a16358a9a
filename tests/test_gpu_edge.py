"""GPU edge cases: a single slice, no iterations, the two-dimensional limit
kz = 0 without flow, the largest grid with many slices, a run that does not
converge and one that blows up."""
import numpy as np
import pytest

from oracle import parareal as opr, stepper
from synthetic import initial_field

pytestmark = pytest.mark.gpu

TOL = 1e-12


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def dev(a):
    import torch
    assert torch.cuda.is_available()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture()
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def test_single_slice(ctx):
    """P = 1: iteration 1 gives F(b0) bitwise (G_new = G_old), iteration 2
    has defect 0."""
    import torch
    N = 32
    b0 = initial_field(N, 0.57, 41)
    ctx.set_problem("gp", 30.0, 0.57, N)
    ctx.set_time(0.5, 1, 5e-3, 2.5e-2, 16)
    ctx.set_initial(b0)
    rep = ctx.parareal(0.0, 2)
    U = ctx.get_slices_dev()
    f = ctx.fine([0.0], dev(b0[None]))
    assert torch.equal(U[1], f[0])
    assert rep["sigma"][0] > 0.0 and rep["sigma"][1] == 0.0


def test_no_iterations_is_the_coarse_run(ctx):
    N, P, T = 32, 5, 1.25
    b0 = initial_field(N, 0.57, 42)
    ctx.set_problem("gp", 30.0, 0.57, N)
    ctx.set_time(T, P, 5e-3, 2.5e-2, 16)
    ctx.set_initial(b0)
    rep = ctx.parareal(0.0, 0)
    assert rep["iters"] == 0 and rep["status"] == 0
    U = ctx.get_slices()
    G = stepper.SliceSolver("gp", 30.0, 0.57, N, T / P, 2.5e-2, 16)
    u = b0
    for n in range(P):
        u = G(u, n * T / P)
        assert rel(U[n + 1], u) <= TOL, n


def test_two_dimensional_pure_diffusion(ctx):
    """kz = 0 and no flow: every mode decays by the SBDF recurrence, the mean
    field (k = 0) is kept to rounding."""
    N = 16
    x = np.stack([initial_field(N, 0.0, 43, amp=1.0)])
    x[0, :, 0, 0] = [0.3 + 0.1j, -0.2j, 0.0]  # mean field (allowed with kz = 0)
    ctx.set_problem("none", 7.0, 0.0, N)
    y = ctx.steps([0.0], 0.05, 9, dev(x)).cpu().numpy()
    ref = stepper.propagate(x[0], "none", 7.0, 0.0, 0.0, 0.05, 9)
    assert rel(y[0], ref) <= TOL
    assert np.allclose(y[0, :, 0, 0], x[0, :, 0, 0], rtol=1e-14, atol=0.0)


def test_largest_grid_many_slices(ctx):
    """512^2 with 256 fields batched (the largest grid, many slices): two
    steps of every field, sampled fields against the oracle."""
    N, P = 512, 256
    kz, Rm, dt = 0.57, 2000.0, 5e-4
    rng = np.random.default_rng(8)
    x = np.stack([initial_field(N, kz, 900 + (n % 4)) * (1.0 + 0.1 * n) for n in range(P)])
    t0 = rng.uniform(0.0, 256.0, P)
    ctx.set_problem("gp", Rm, kz, N)
    print("512^2 x 256 fields", flush=True)
    y = ctx.steps(t0, dt, 2, dev(x)).cpu().numpy()
    for n in (0, 129, 255):
        ref = stepper.propagate(x[n], "gp", Rm, kz, t0[n], dt, 2)
        assert rel(y[n], ref) <= TOL, n


def test_not_converged_report(ctx, lib):
    N, P = 32, 6
    ctx.set_problem("gp", 30.0, 0.57, N)
    ctx.set_time(1.5, P, 5e-3, 2.5e-2, 16)
    ctx.set_initial(initial_field(N, 0.57, 44))
    rep = ctx.parareal(1e-300, 2)
    assert rep["status"] == lib.NOT_CONVERGED and rep["iters"] == 2 and rep["k_con"] < 0
    assert rep["sigma"][0] > 0 and rep["sigma"][1] > 0


def test_blow_up_is_reported(ctx, lib):
    """A step far beyond stability overflows to non-finite values; the
    defect check reports it (no fault, no hang)."""
    N = 64
    ctx.set_problem("gp", 100.0, 0.57, N)
    ctx.set_time(300.0, 2, 0.25, 0.5, 32)
    ctx.set_initial(initial_field(N, 0.57, 45))
    with pytest.raises(lib.PitdynError) as e:
        ctx.parareal(1e-8, 3)
    assert e.value.status == lib.EUNSTABLE
