"""GPU parity: the HIP library against the FP64 CPU oracle, element by element
on the same seeded inputs.  Bar: relative L2 <= 1e-12 for states, 1e-6
absolute for growth rates; bitwise for the Parareal finite-termination
property, determinism and batch invariance."""
import math

import numpy as np
import pytest

from oracle import parareal as opr, spectral as osp, stepper
from synthetic import initial_field

pytestmark = pytest.mark.gpu

TOL = 1e-12


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def rand_box(N, seed, batch=None):
    rng = np.random.default_rng(seed)
    shape = (3, N, N) if batch is None else (batch, 3, N, N)
    b = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return b * osp.box_mask(N)


def dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture()
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("path", [0, 1, 2])
@pytest.mark.parametrize("flow", ["roberts", "gp"])
@pytest.mark.parametrize("N", [16, 32, 64, 128, 256, 512])
def test_steps_match_oracle(ctx, lib, N, flow, path):
    """n SBDF steps for a ragged batch of fields with different start times."""
    kz, Rm = 0.57, 30.0
    nsteps = 3 if N <= 256 else 2
    dt = 2e-3
    batch = 3
    x = rand_box(N, N + path, batch)
    t0 = np.array([0.0, 1.7, 5.3])
    ctx.set_problem(flow, Rm, kz, N)
    ctx.set_path(path)
    print(f"steps N={N} flow={flow} path={path}", flush=True)
    y = ctx.steps(t0, dt, nsteps, dev(x)).cpu().numpy()
    for f in range(batch):
        ref = stepper.propagate(x[f], flow, Rm, kz, t0[f], dt, nsteps)
        assert rel(y[f], ref) <= TOL, (f, rel(y[f], ref))


def test_pure_diffusion_closed_form(ctx):
    """u = 0 against the per-mode SBDF closed form (independent of the oracle's
    stepper)."""
    from tests import pins
    N, kz, Rm, dt, n = 64, 0.8, 3.0, 0.05, 17
    x = rand_box(N, 1)
    ctx.set_problem("none", Rm, kz, N)
    y = ctx.steps([0.0], dt, n, dev(x[None])).cpu().numpy()[0]
    ref = pins.sbdf_diffusion_factor(dt * osp.k_squared(N, kz) / Rm, n)[None] * x
    assert rel(y, ref) <= TOL


@pytest.mark.parametrize("N,Nc", [(64, 64), (64, 32), (128, 64)])
def test_fine_and_coarse_slice_match_oracle(ctx, N, Nc):
    kz, Rm, T, P, dtf, dtc = 0.57, 100.0, 2.0, 4, 5e-3, 2.5e-2
    ctx.set_problem("gp", Rm, kz, N)
    ctx.set_time(T, P, dtf, dtc, Nc)
    x = np.stack([initial_field(N, kz, s, amp=1.0, kmax=N / 4) for s in (3, 4)])
    t0 = np.array([0.5, 1.0])
    print(f"slice N={N} Nc={Nc}", flush=True)
    yf = ctx.fine(t0, dev(x)).cpu().numpy()
    yc = ctx.coarse(t0, dev(x)).cpu().numpy()
    F = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtf)
    G = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtc, Nc)
    for f in range(2):
        assert rel(yf[f], F(x[f], t0[f])) <= TOL
        assert rel(yc[f], G(x[f], t0[f])) <= TOL


def test_batch_invariance_and_determinism(ctx):
    """A field's result does not depend on its batch neighbours or on the run
    (bitwise), on both launch paths."""
    N = 64
    ctx.set_problem("gp", 50.0, 0.57, N)
    x = rand_box(N, 5, 4)
    t0 = np.array([0.3, 0.3, 0.3, 0.3])
    outs = []
    for path in (0, 1, 2):
        ctx.set_path(path)
        a = ctx.steps(t0, 1e-2, 5, dev(x)).cpu().numpy()
        b = ctx.steps(t0, 1e-2, 5, dev(x)).cpu().numpy()
        c = ctx.steps(t0[:1], 1e-2, 5, dev(x[2:3])).cpu().numpy()
        assert np.array_equal(a, b)
        assert np.array_equal(a[2], c[0])
        outs.append(a)
    assert rel(outs[0], outs[1]) <= TOL
    assert np.array_equal(outs[0], outs[2])


def test_config1_parareal_matches_oracle(ctx):
    """Roberts flow, Rm = 10, kz = 1, 32^2, T = 8 over 8 slices, dt = 1e-3,
    coarse dt = 1e-2 on the same grid: three iterations, every slice state,
    every defect and the growth rate."""
    N, kz, Rm, T, P, dtf, dtc, iters = 32, 1.0, 10.0, 8.0, 8, 1e-3, 1e-2, 3
    b0 = initial_field(N, kz, 100000)
    ctx.set_problem("roberts", Rm, kz, N)
    ctx.set_time(T, P, dtf, dtc, 0)
    ctx.set_initial(b0)
    rep = ctx.parareal(0.0, iters)
    U = ctx.get_slices()
    F = stepper.SliceSolver("roberts", Rm, kz, N, T / P, dtf)
    G = stepper.SliceSolver("roberts", Rm, kz, N, T / P, dtc)
    ref = opr.parareal(b0, P, T / P, F, G, tol=0.0, max_iter=iters)
    for n in range(P + 1):
        assert rel(U[n], ref.U[n]) <= TOL, (n, rel(U[n], ref.U[n]))
    # sigma is a relative difference of two states, each within TOL of the
    # oracle, so it can differ by at most about 2 TOL in absolute terms
    assert np.allclose(rep["sigma"], ref.sigma, rtol=0, atol=2 * TOL)
    gam_ref = opr.growth_rate([opr.norm2(u) for u in ref.U], np.arange(P + 1) * T / P)
    assert abs(ctx.growth_rate() - gam_ref) <= 1e-6
    # the defect reaches the tolerance at the same iteration as the oracle
    ctx.set_initial(b0)
    rep2 = ctx.parareal(1e-8, 8)
    ref2 = opr.parareal(b0, P, T / P, F, G, tol=1e-8, max_iter=8)
    assert rep2["k_con"] == ref2.k_con == 3


def test_parareal_finite_termination_bitwise(ctx):
    """After P iterations every slice equals the serial fine solution
    (restarted per slice) bitwise, computed with the library's own F."""
    torch = _torch()
    N, kz, Rm, P = 32, 0.57, 40.0, 5
    b0 = initial_field(N, kz, 9)
    ctx.set_problem("gp", Rm, kz, N)
    ctx.set_time(1.0, P, 1e-2, 5e-2, 16)
    ctx.set_initial(b0)
    rep = ctx.parareal(0.0, P + 1)
    U = ctx.get_slices_dev()
    u = dev(b0[None])
    for n in range(P):
        u = ctx.fine([n * 0.2], u)
        assert torch.equal(U[n + 1], u[0]), n
    assert rep["sigma"][-1] == 0.0


def test_growth_rate_gp_table1(ctx):
    """Table 1 (Section 5.3): Galloway-Proctor Rm = 3, wavenumber 0.57, N = 16,
    dt = 5e-3 grows at 0.15; the GPU's rate equals the oracle's to 1e-6."""
    N, kz, Rm, T, P, dt = 16, 0.57, 3.0, 50.0, 50, 5e-3
    b0 = initial_field(N, kz, 3)
    ctx.set_problem("gp", Rm, kz, N)
    ctx.set_time(T, P, dt, 0.1, 0)
    ctx.set_initial(b0)
    ctx.parareal(0.0, P)
    g = ctx.growth_rate()
    F = stepper.SliceSolver("gp", Rm, kz, N, 1.0, dt)
    ref = opr.serial_fine(b0, P, 1.0, F)
    gref = opr.growth_rate([opr.norm2(u) for u in ref], np.arange(P + 1.0))
    assert abs(g - gref) <= 1e-6
    assert abs(g - 0.15) <= 0.005


def test_config2_sampled_fine_sweep(ctx):
    """Galloway-Proctor Rm = 100, kz = 0.57, 128^2, 64 slices of length 1 with
    dt = 2e-3 (500 steps), batched in one fine sweep as the benchmark runs it:
    sampled slices against the oracle."""
    torch = _torch()
    N, kz, Rm, P = 128, 0.57, 100.0, 64
    ctx.set_problem("gp", Rm, kz, N)
    ctx.set_time(64.0, P, 2e-3, 1e-2, 64)
    x = np.stack([initial_field(N, kz, 200000 + n) for n in range(P)])
    y = ctx.fine(np.arange(P, dtype=float), dev(x)).cpu().numpy()
    F = stepper.SliceSolver("gp", Rm, kz, N, 1.0, 2e-3)
    for n in (0, 37, 63):
        assert rel(y[n], F(x[n], float(n))) <= TOL, n


def test_config2_parareal_full_size(ctx):
    """The Galloway-Proctor 128^2 workload at its full size (Rm = 100, kz =
    0.57, T = 64 over 64 slices, fine dt = 2e-3, coarse dt = 1e-2 on 64^2,
    tol 1e-8, pipelined as the benchmark runs it): properties that hold at
    any size.  The converged iterate agrees with the serial fine solve (the
    library's own F, slice after slice) and, on sampled slices, the oracle's
    F maps U_n to U_{n+1}, both to 1e-7 (Parareal stops once the relative
    change of U_P between iterations is <= 1e-8); the growth rate equals the
    serial solve's to 1e-6, and the defects fall monotonically."""
    N, kz, Rm, T, P, dtf = 128, 0.57, 100.0, 64.0, 64, 2e-3
    b0 = initial_field(N, kz, 1)
    ctx.set_problem("gp", Rm, kz, N)
    ctx.set_time(T, P, dtf, 1e-2, 64)
    ctx.set_initial(b0)
    print("full-size parareal", flush=True)
    rep = ctx.parareal(1e-8, P)
    assert 0 < rep["k_con"] <= P
    sig = rep["sigma"][:rep["iters"]]
    assert sig[-1] <= 1e-8 and all(b < a for a, b in zip(sig, sig[1:]))
    U = ctx.get_slices()
    gam = ctx.growth_rate()
    # serial fine solve on the GPU, slice after slice
    u = dev(b0[None])
    serial = [b0]
    for n in range(P):
        u = ctx.fine([float(n)], u)
        serial.append(u[0].cpu().numpy())
    d_serial = max(rel(U[n], serial[n]) for n in (1, 17, 40, 64))
    gs = opr.growth_rate([opr.norm2(x) for x in serial], np.arange(P + 1.0))
    F = stepper.SliceSolver("gp", Rm, kz, N, 1.0, dtf)
    d_oracle = max(rel(U[n + 1], F(U[n], float(n))) for n in (0, 51))
    print(f"k_con {rep['k_con']}: vs serial {d_serial:.1e}, vs oracle F {d_oracle:.1e}, "
          f"growth {abs(gam - gs):.1e}", flush=True)
    assert d_serial <= 1e-7 and d_oracle <= 1e-7
    assert abs(gam - gs) <= 1e-6


def test_invalid_arguments(ctx, lib):
    torch = _torch()
    with pytest.raises(lib.PitdynError) as e:
        ctx.set_problem("gp", 10.0, 1.0, 48)
    assert e.value.status == lib.EINVAL
    ctx.set_problem("gp", 10.0, 1.0, 32)
    with pytest.raises(lib.PitdynError):
        ctx.set_time(1.0, 4, 0.3, 0.1, 0)       # 0.25 / 0.3 not an integer
    with pytest.raises(lib.PitdynError):
        ctx.set_time(1.0, 4, 1e-2, 5e-2, 64)    # coarse grid finer than N
    ctx.set_time(1.0, 4, 1e-2, 5e-2, 16)
    bad = np.zeros((1, 3, 32, 32), complex)
    bad[0, 0, 16, 0] = 1.0                       # Nyquist row: outside the box
    with pytest.raises(lib.PitdynError) as e:
        ctx.fine([0.0], dev(bad))
    assert e.value.status == lib.EINVAL
    # empty batch is a no-op
    empty = torch.zeros((0, 3, 32, 32), dtype=torch.complex128, device="cuda")
    assert ctx.fine(np.zeros(0), empty).shape[0] == 0


@pytest.mark.parametrize("form", [1, 2, 3])
def test_parareal_coarse_forms_match_oracle(ctx, lib, form):
    """The serial coarse sweep in one-workgroup pseudo-spectral (FFT) form,
    in exact spectral-convolution form and in host-driven multi-launch form
    reproduces the oracle's Parareal iterates (Galloway-Proctor, 64^2 fine,
    32^2 coarse, 6 slices, 2 iterations)."""
    N, Nc, kz, Rm, T, P, dtf, dtc, iters = 64, 32, 0.57, 50.0, 1.5, 6, 5e-3, 2.5e-2, 2
    b0 = initial_field(N, kz, 77)
    ctx.set_problem("gp", Rm, kz, N)
    ctx.set_time(T, P, dtf, dtc, Nc)
    ctx.set_coarse_form(form)
    ctx.set_initial(b0)
    rep = ctx.parareal(0.0, iters)
    U = ctx.get_slices()
    F = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtf)
    G = stepper.SliceSolver("gp", Rm, kz, N, T / P, dtc, Nc)
    ref = opr.parareal(b0, P, T / P, F, G, tol=0.0, max_iter=iters)
    for n in range(P + 1):
        assert rel(U[n], ref.U[n]) <= TOL, (form, n, rel(U[n], ref.U[n]))
    assert np.allclose(rep["sigma"], ref.sigma, rtol=0, atol=2 * TOL)


@pytest.mark.parametrize("N", [64, 128, 256, 512])
def test_every_launch_variant_matches_oracle(ctx, lib, N):
    """Each launch-shape variant of the row and column kernels reproduces the
    oracle (the autotuner may pick any of them)."""
    kz, Rm, dt, nsteps = 0.57, 40.0, 2e-3, 2
    x = rand_box(N, 11 + N, 2)
    t0 = np.array([0.4, 3.3])
    refs = [stepper.propagate(x[f], "gp", Rm, kz, t0[f], dt, nsteps) for f in range(2)]
    ctx.set_problem("gp", Rm, kz, N)
    ctx.set_path(0)
    try:
        for kind in (0, 1):
            for v in range(len(lib.variants(N, kind))):
                lib.select_variant(N, v if kind == 0 else 0, v if kind == 1 else 0)
                print(f"variant N={N} kind={kind} v={v}", flush=True)
                y = ctx.steps(t0, dt, nsteps, dev(x)).cpu().numpy()
                for f in range(2):
                    assert rel(y[f], refs[f]) <= TOL, (kind, v, f)
    finally:
        lib.select_variant(N, 0, 0)


def test_autotune_selects_and_caches(ctx, lib, tmp_path):
    N = 64
    ctx.set_problem("gp", 50.0, 0.57, N)
    ctx.set_time(4.0, 8, 1e-2, 5e-2, 32)
    ctx.set_initial(initial_field(N, 0.57, 5))
    ctx.parareal(0.0, 0)
    cache = str(tmp_path / "tune.json")
    try:
        (rv, cv), (mr, mc) = ctx.autotune(5, cache)
        assert 0 <= rv < len(lib.variants(N, 0)) and 0 <= cv < len(lib.variants(N, 1))
        assert mr > 0 and mc > 0
        text = open(cache).read()
        assert f"|{N}|8" in text
        blk = ctx.fine_blocking()                       # tuned with the launch shapes
        assert blk[0] in (0, 1, 2, 3, 4) and 1 <= blk[1] <= 3
        ctx.set_fine_blocking(-1)
        (rv2, cv2), (mr2, mc2) = ctx.autotune(5, cache)   # cache hit
        assert (rv2, cv2) == (rv, cv) and mr2 == 0.0
        assert ctx.fine_blocking() == blk               # the cached blocking
        # Parareal after tuning still matches an untuned context (the choice
        # is this context's; another context keeps the defaults) to the bar
        ctx.set_initial(initial_field(N, 0.57, 5))
        ctx.parareal(0.0, 2)
        U1 = ctx.get_slices()
        with lib.Context(0) as other:
            other.set_problem("gp", 50.0, 0.57, N)
            other.set_time(4.0, 8, 1e-2, 5e-2, 32)
            other.set_initial(initial_field(N, 0.57, 5))
            other.parareal(0.0, 2)
            U0 = other.get_slices()
        for n in range(9):
            assert rel(U1[n], U0[n]) <= TOL
    finally:
        lib.select_variant(N, 0, 0)
