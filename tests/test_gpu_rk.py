"""GPU parity of the IMEX Runge-Kutta steppers -- ARS(4,4,3) (the paper's
RK443), ARS(2,2,2), ARS(1,1,1) -- against the FP64 oracle: steps on every
grid, both flows, both launch paths; F and G over a slice with coarsening;
Parareal with Runge-Kutta F and G; bitwise finite termination; argument
errors.  Bar: relative L2 <= 1e-12."""
import numpy as np
import pytest

from oracle import parareal as opr, spectral as osp, stepper
from synthetic import initial_field

pytestmark = pytest.mark.gpu

TOL = 1e-12


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def rand_box(N, seed, batch):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((batch, 3, N, N)) + 1j * rng.standard_normal((batch, 3, N, N))
    return b * osp.box_mask(N)


def dev(a):
    import torch
    assert torch.cuda.is_available()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture()
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("scheme", ["rk443", "rk222", "rk111"])
@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("flow", ["roberts", "gp"])
@pytest.mark.parametrize("N", [16, 32, 64, 128, 256, 512])
def test_rk_steps_match_oracle(ctx, N, flow, path, scheme):
    kz, Rm, dt, batch = 0.57, 30.0, 4e-3, 3
    nsteps = 2 if N <= 256 else 1
    x = rand_box(N, 7 * N + path, batch)
    t0 = np.array([0.0, 1.7, 5.3])
    ctx.set_problem(flow, Rm, kz, N)
    ctx.set_scheme(scheme, scheme)
    ctx.set_path(path)
    print(f"{scheme} steps N={N} flow={flow} path={path}", flush=True)
    y = ctx.steps(t0, dt, nsteps, dev(x)).cpu().numpy()
    for f in range(batch):
        ref = stepper.propagate_imex_rk(x[f], flow, Rm, kz, t0[f], dt, nsteps, scheme)
        assert rel(y[f], ref) <= TOL, (f, rel(y[f], ref))


@pytest.mark.parametrize("Nc", [32, 16])
def test_rk443_fine_and_coarse_slice(ctx, Nc):
    N, kz, Rm, T, P, dtf, dtc = 32, 0.57, 50.0, 1.0, 4, 5e-3, 2.5e-2
    x = rand_box(N, 11, 2)
    t0 = np.array([0.25, 0.75])
    ctx.set_problem("gp", Rm, kz, N)
    ctx.set_time(T, P, dtf, dtc, Nc)
    ctx.set_scheme("rk443", "rk443")
    F = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtf, scheme="rk443")
    G = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtc, Nc, scheme="rk443")
    yf = ctx.fine(t0, dev(x)).cpu().numpy()
    yg = ctx.coarse(t0, dev(x)).cpu().numpy()
    for f in range(2):
        assert rel(yf[f], F(x[f], t0[f])) <= TOL
        assert rel(yg[f], G(x[f], t0[f])) <= TOL


@pytest.mark.parametrize("schemes", [("rk443", "rk443"), ("rk443", "sbdf2"), ("sbdf2", "rk443"),
                                     ("rk222", "rk111")])
def test_rk443_parareal_matches_oracle(ctx, schemes):
    """Galloway-Proctor, Rm = 50, 32^2, T = 2 over 8 slices, fine dt = 5e-3,
    coarse dt = 5e-2 on 16^2 (FFT form of the coarse sweep for a Runge-Kutta
    G): every slice state and defect of three iterations, and k_con."""
    sf, sc = schemes
    N, Nc, kz, Rm, T, P, dtf, dtc = 32, 16, 0.57, 50.0, 2.0, 8, 5e-3, 5e-2
    b0 = initial_field(N, kz, 31)
    ctx.set_problem("gp", Rm, kz, N)
    ctx.set_time(T, P, dtf, dtc, Nc)
    ctx.set_scheme(sf, sc)
    ctx.set_initial(b0)
    rep = ctx.parareal(0.0, 3)
    U = ctx.get_slices()
    F = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtf, scheme=sf)
    G = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtc, Nc, scheme=sc)
    ref = opr.parareal(b0, P, T / P, F, G, tol=0.0, max_iter=3)
    for n in range(P + 1):
        assert rel(U[n], ref.U[n]) <= TOL, (n, rel(U[n], ref.U[n]))
    assert np.allclose(rep["sigma"], ref.sigma, rtol=0, atol=2 * TOL)
    ctx.set_initial(b0)
    rep2 = ctx.parareal(1e-9, P + 1)
    ref2 = opr.parareal(b0, P, T / P, F, G, tol=1e-9, max_iter=P + 1)
    assert rep2["k_con"] == ref2.k_con > 0


def test_rk443_finite_termination_bitwise(ctx):
    import torch
    N, P = 32, 5
    b0 = initial_field(N, 0.57, 9)
    ctx.set_problem("gp", 40.0, 0.57, N)
    ctx.set_time(1.0, P, 1e-2, 5e-2, 16)
    ctx.set_scheme("rk443", "rk443")
    ctx.set_initial(b0)
    rep = ctx.parareal(0.0, P + 1)
    U = ctx.get_slices_dev()
    u = dev(b0[None])
    for n in range(P):
        u = ctx.fine([n * 0.2], u)
        assert torch.equal(U[n + 1], u[0]), n
    assert rep["sigma"][-1] == 0.0


def test_rk443_scheme_errors(ctx, lib):
    ctx.set_problem("gp", 40.0, 0.57, 32)
    ctx.set_time(1.0, 4, 1e-2, 5e-2, 16)
    ctx.set_coarse_form(2)  # convolution form: SBDF2 only
    with pytest.raises(lib.PitdynError):
        ctx.set_scheme("sbdf2", "rk443")
    ctx.set_coarse_form(0)
    ctx.set_scheme("sbdf2", "rk443")
    with pytest.raises(lib.PitdynError):
        ctx.set_coarse_form(2)
    assert lib.lib.pd_set_scheme(ctx._h, 4, 0) == lib.EINVAL
