"""GPU tests of pipelined Parareal: the overlapped schedule (coarse sweep on
its own stream in runs of slices, fine sweeps of the next iteration started
early) gives bitwise the iterates, defects and k_con of the plain order."""
import numpy as np
import pytest

from synthetic import initial_field

pytestmark = pytest.mark.gpu


def run(lib, chunks, P=10, N=32, tol=1e-10, max_iter=None, flow="gp", Nc=16, resume=None, form=0,
        spec=2, scheme=None):
    with lib.Context(0) as ctx:
        ctx.set_problem(flow, 60.0, 0.57, N)
        ctx.set_time(0.25 * P, P, 5e-3, 2.5e-2, Nc)
        if scheme is not None:
            ctx.set_scheme(*scheme)
        ctx.set_coarse_form(form)
        ctx.set_pipeline(chunks, spec)
        b0 = initial_field(N, 0.57, 77)
        if resume is None:
            ctx.set_initial(b0)
        else:
            ctx.set_initial(b0)
            ctx.set_pipeline(0)
            ctx.parareal(0.0, resume)
            U, G = ctx.get_slices(), ctx.get_coarse_values()
            ctx.set_pipeline(chunks, spec)
            ctx.set_slices(U, G, resume)
        rep = ctx.parareal(tol, P + 1 if max_iter is None else max_iter)
        return rep, ctx.get_slices(), ctx.get_coarse_values()


@pytest.mark.parametrize("chunks,spec", [(2, 1), (3, 2), (4, 0), (7, 1), (10, 2), (64, 1)])
def test_pipelined_equals_plain_order_bitwise(lib, chunks, spec):
    r0, U0, G0 = run(lib, 0)
    r1, U1, G1 = run(lib, chunks, spec=spec)
    assert r0["k_con"] == r1["k_con"] and r0["iters"] == r1["iters"]
    assert r0["sigma"][:r0["iters"]] == r1["sigma"][:r1["iters"]]
    assert np.array_equal(U0, U1)
    assert np.array_equal(G0, G1)


def test_pipelined_fixed_iterations_and_no_iterations(lib):
    for it in (0, 1, 3):
        r0, U0, _ = run(lib, 0, tol=0.0, max_iter=it)
        r1, U1, _ = run(lib, 4, tol=0.0, max_iter=it)
        assert r0["iters"] == r1["iters"] == it
        assert np.array_equal(U0, U1)


def test_pipelined_resume_and_fft_coarse_form(lib):
    r0, U0, _ = run(lib, 0, resume=2)
    r1, U1, _ = run(lib, 3, resume=2)
    assert r0["k_con"] == r1["k_con"]
    assert np.array_equal(U0, U1)
    # the pseudo-spectral (FFT) form of the coarse sweep
    r0, U0, _ = run(lib, 0, P=6, tol=1e-8, form=1)
    r1, U1, _ = run(lib, 4, P=6, tol=1e-8, form=1)
    assert r0["k_con"] == r1["k_con"] > 0
    assert np.array_equal(U0, U1)


@pytest.mark.parametrize("scheme,form", [(("rk443", "rk443"), 3), (("sbdf2", "rk222"), 1),
                                         (("rk443", "sbdf2"), 0)])
def test_pipelined_runge_kutta_and_coarse_forms_bitwise(lib, scheme, form):
    """Runge-Kutta fine or coarse steppers with the multi-launch (3), FFT (1)
    and automatic (0) coarse forms: pipelined = plain order, bitwise."""
    r0, U0, G0 = run(lib, 0, P=8, tol=1e-9, scheme=scheme, form=form)
    r1, U1, G1 = run(lib, 3, P=8, tol=1e-9, scheme=scheme, form=form)
    assert r0["k_con"] == r1["k_con"] > 0 and r0["iters"] == r1["iters"]
    assert r0["sigma"][:r0["iters"]] == r1["sigma"][:r1["iters"]]
    assert np.array_equal(U0, U1)
    assert np.array_equal(G0, G1)


def test_pipelined_with_autotuned_launch_shapes_is_bitwise(lib):
    """After the autotuner has picked the launch shapes (among them the row
    variant that loads state and history with the row), the pipelined order
    stays bitwise equal to the plain order."""
    N, P = 64, 8
    b0 = initial_field(N, 0.57, 12)
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", 60.0, 0.57, N)
        ctx.set_time(0.25 * P, P, 5e-3, 2.5e-2, 32)
        ctx.set_initial(b0)
        ctx.parareal(0.0, 0)
        try:
            ctx.autotune(3)
            ctx.set_initial(b0)
            r1 = ctx.parareal(1e-9, P + 1)
            U1 = ctx.get_slices()
            ctx.set_pipeline(0)
            ctx.set_initial(b0)
            r0 = ctx.parareal(1e-9, P + 1)
            U0 = ctx.get_slices()
        finally:
            lib.select_variant(N, 0, 0)
    assert r0["k_con"] == r1["k_con"] > 0
    assert r0["sigma"][:r0["iters"]] == r1["sigma"][:r1["iters"]]
    assert np.array_equal(U0, U1)


def test_pipelined_learned_coarse_is_bitwise(lib):
    """The learned coarse propagator (difference form) run by run in the
    pipelined schedule gives bitwise the iterates, defects and k_con of the
    plain order."""
    N, P = 32, 8
    b0 = initial_field(N, 0.57, 14)
    res = []
    for chunks in (0, 2, 3):
        with lib.Context(0) as ctx:
            ctx.set_problem("gp", 40.0, 0.57, N)
            ctx.set_time(0.25 * P, P, 5e-3, 2.5e-2, 16)
            ctx.lg_init(2, 7)
            p = ctx.lg_params()
            rng = np.random.default_rng(3)
            p[-32 * 6:] = (rng.standard_normal(32 * 6) * 0.05).astype(np.float32)
            ctx.lg_set_params(p)
            ctx.set_coarse(True)
            ctx.set_pipeline(chunks, 2)
            ctx.set_initial(b0)
            r = ctx.parareal(1e-10, P + 1)
            res.append((r, ctx.get_slices()))
    for r, U in res[1:]:
        assert r["k_con"] == res[0][0]["k_con"] > 0
        assert r["sigma"][:r["iters"]] == res[0][0]["sigma"][:res[0][0]["iters"]]
        assert np.array_equal(U, res[0][1])
