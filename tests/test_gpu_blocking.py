"""GPU tests of the blocked fine sweep: groups of fields that run all their
fine steps back to back, dealt to up to three streams, give bitwise the
results of stepping the whole batch one step at a time (the fine solves of
the slices are independent, Section 3)."""
import numpy as np
import pytest

from synthetic import initial_field

pytestmark = pytest.mark.gpu

OFF = (0, 1)


def sweep_states(lib, blocking, N=64, P=7, prec="c128", steps=((0, 3), (3, 2))):
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", 80.0, 0.57, N)
        if prec != "c128":
            ctx.set_precision(prec)
        ctx.set_time(0.1 * P, P, 5e-3, 2.5e-2, N // 2)
        ctx.set_fine_blocking(*blocking)
        ctx.seed_initial(4242, 1.0, N / 3.0)     # the whole 2/3 box
        ctx.parareal(0.0, 0)                      # slice states from the initial coarse run
        print(f"blocked sweep N={N} P={P} {prec} blocking={blocking}", flush=True)
        for a, n in steps:
            ctx.fine_sweep_steps(a, n)
        return ctx.fine_blocking(), ctx.get_fine_states_dev(0, P).cpu().numpy()


@pytest.mark.parametrize("blocking", [(2, 3), (3, 2), (4, 1), (1, 3), (6, 2)])
def test_blocked_stepwise_sweep_is_bitwise(lib, blocking):
    eff0, y0 = sweep_states(lib, OFF)
    eff1, y1 = sweep_states(lib, blocking)
    assert eff0 == OFF and eff1 == blocking
    assert np.abs(y0).max() > 0
    assert np.array_equal(y0, y1)


def test_blocked_stepwise_sweep_complex64_is_bitwise(lib):
    _, y0 = sweep_states(lib, OFF, prec="c64")
    _, y1 = sweep_states(lib, (2, 3), prec="c64")
    assert np.array_equal(y0, y1)


def test_blocked_timed_sweep_reports_the_whole(lib):
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", 80.0, 0.57, 64)
        ctx.set_time(0.7, 7, 5e-3, 2.5e-2, 32)
        ctx.set_fine_blocking(2, 3)
        ctx.seed_initial(4242, 1.0, 21.0)
        ctx.parareal(0.0, 0)
        ctx.fine_sweep_steps(0, 1)
        ms = ctx.fine_sweep_steps(1, 3, timed=True)
        assert ms[0] == -1.0 and ms[1] == -1.0 and ms[2] > 0


def parareal_run(lib, blocking, chunks, scheme=None, P=9, N=32):
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", 60.0, 0.57, N)
        ctx.set_time(0.25 * P, P, 5e-3, 2.5e-2, 16)
        if scheme is not None:
            ctx.set_scheme(*scheme)
        ctx.set_pipeline(chunks, 2)
        ctx.set_fine_blocking(*blocking)
        ctx.set_initial(initial_field(N, 0.57, 77))
        print(f"blocked parareal chunks={chunks} blocking={blocking} scheme={scheme}", flush=True)
        rep = ctx.parareal(1e-10, P + 1)
        return rep, ctx.get_slices(), ctx.get_coarse_values()


@pytest.mark.parametrize("chunks,blocking,scheme", [
    (0, (2, 3), None), (0, (4, 2), ("rk443", "sbdf2")), (3, (2, 3), None), (2, (1, 1), None)])
def test_blocked_parareal_is_bitwise(lib, chunks, blocking, scheme):
    r0, U0, G0 = parareal_run(lib, OFF, 0, scheme)
    r1, U1, G1 = parareal_run(lib, blocking, chunks, scheme)
    assert r0["k_con"] == r1["k_con"] > 0 and r0["iters"] == r1["iters"]
    assert r0["sigma"][:r0["iters"]] == r1["sigma"][:r1["iters"]]
    assert np.array_equal(U0, U1)
    assert np.array_equal(G0, G1)


def test_blocked_batch_steps_are_bitwise(lib):
    """pd_steps_dev on a ragged batch of 5 fields with different start times."""
    import torch
    N = 64
    x = torch.from_numpy(np.stack([initial_field(N, 0.57, 900 + f) for f in range(5)])).cuda()
    t0 = np.array([0.0, 0.3, 1.1, 2.9, 7.0])
    out = []
    for blocking in (OFF, (2, 3), (3, 1)):
        with lib.Context(0) as ctx:
            ctx.set_problem("gp", 80.0, 0.57, N)
            ctx.set_fine_blocking(*blocking)
            out.append(ctx.steps(t0, 5e-3, 4, x).cpu().numpy())
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_default_blocking_and_argument_errors(lib):
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", 2000.0, 0.57, 512)
        with pytest.raises(lib.PitdynError):
            ctx.fine_blocking()                   # before pd_set_time
        ctx.set_time(8.0, 8, 5e-4, 2.5e-3, 64)
        assert ctx.fine_blocking() == (4, 3)      # default at 512^2
        ctx.set_fine_blocking(0)
        assert ctx.fine_blocking() == OFF
        ctx.set_fine_blocking(8, 2)
        assert ctx.fine_blocking() == OFF         # a group as large as the batch: unblocked
        for bad in ((-2, 1), (2, 0), (2, 4)):
            with pytest.raises(lib.PitdynError):
                ctx.set_fine_blocking(*bad)
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", 500.0, 0.57, 256)
        ctx.set_time(16.0, 32, 1e-3, 5e-3, 64)
        assert ctx.fine_blocking() == (16, 3)     # default at 256^2
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", 100.0, 0.57, 128)
        ctx.set_time(4.0, 4, 2e-3, 1e-2, 64)
        assert ctx.fine_blocking() == OFF         # default below 256^2
