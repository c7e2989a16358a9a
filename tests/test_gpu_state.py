"""GPU tests of the host-array propagator calls, Parareal checkpoint and
resume, and the parameter file of the learned coarse propagator."""
import numpy as np
import pytest

from oracle import stepper
from synthetic import initial_field

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def problem(ctx, N=32, P=6, flow="gp"):
    ctx.set_problem(flow, 50.0, 0.57, N)
    ctx.set_time(1.5, P, 5e-3, 2.5e-2, N // 2)


def test_host_steps_equal_device_steps_and_oracle(lib):
    torch = _torch()
    N = 32
    with lib.Context(0) as ctx:
        problem(ctx, N=N)
        b = np.stack([initial_field(N, 0.57, s) for s in (1, 2, 3)])
        t0 = np.array([0.0, 0.25, 0.75])
        for fine in (True, False):
            h = ctx.step_host(t0, b, fine=fine)
            d = (ctx.fine if fine else ctx.coarse)(t0, torch.from_numpy(b).cuda()).cpu().numpy()
            assert np.array_equal(h, d)
        ref = stepper.SliceSolver("gp", 50.0, 0.57, N, 0.25, 5e-3)(b[1], 0.25)
        got = ctx.step_host(t0[1:2], b[1:2])[0]
        assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("learned", [False, True])
def test_checkpoint_resume_is_bitwise(lib, learned):
    N, P, tol = 32, 6, 1e-10
    b0 = initial_field(N, 0.57, 31)
    with lib.Context(0) as ctx:
        problem(ctx, N=N, P=P)
        if learned:
            ctx.lg_init(2, 7)
            p = ctx.lg_params()
            p[-32 * 6:] = np.random.default_rng(3).standard_normal(32 * 6).astype(np.float32) * 0.05
            ctx.lg_set_params(p)
            ctx.set_coarse(True)
        ctx.set_initial(b0)
        full = ctx.parareal(tol, P + 1)
        U_full = ctx.get_slices()
        assert full["k_con"] > 3
        ctx.set_initial(b0)
        part = ctx.parareal(0.0, 3)
        U3 = ctx.get_slices()
        G3 = None if learned else ctx.get_coarse_values()
        assert part["sigma"][:3] == full["sigma"][:3]
        # a second context stands for a restarted process
        with lib.Context(0) as c2:
            problem(c2, N=N, P=P)
            if learned:
                c2.lg_init(2, 7)
                c2.lg_set_params(ctx.lg_params())
                c2.set_coarse(True)
            c2.set_slices(U3, G3, 3)
            rest = c2.parareal(tol, P + 1)
            assert rest["k_con"] == full["k_con"]
            assert rest["sigma"][3:rest["iters"]] == full["sigma"][3:full["iters"]]
            assert np.array_equal(c2.get_slices(), U_full)


def test_resume_argument_errors(lib):
    N, P = 32, 6
    with lib.Context(0) as ctx:
        problem(ctx, N=N, P=P)
        ctx.set_initial(initial_field(N, 0.57, 5))
        ctx.parareal(0.0, 2)
        U = ctx.get_slices()
        G = ctx.get_coarse_values()
        ctx.set_slices(U, None, 2)
        with pytest.raises(lib.PitdynError):
            ctx.parareal(0.0, 4)  # plain G needs the coarse values
        ctx.set_slices(U, G, 2)
        with pytest.raises(lib.PitdynError):
            ctx.parareal(0.0, 2)  # nothing after iteration 2
        bad = U.copy()
        bad[1, 0, N // 2, 0] = 1.0  # outside the 2/3 box
        with pytest.raises(lib.PitdynError):
            ctx.set_slices(bad, G, 2)
        ctx.set_slices(U, G, 2)
        ctx.set_initial(U[0])  # cancels the resume
        r = ctx.parareal(0.0, 2)
        assert r["iters"] == 2


def test_learned_parameter_file_round_trip(lib, tmp_path):
    N = 32
    path = tmp_path / "net.bin"
    with lib.Context(0) as ctx:
        problem(ctx, N=N)
        ctx.lg_init(3, 11)
        p = ctx.lg_params()
        p += np.random.default_rng(0).standard_normal(p.size).astype(np.float32) * 0.01
        ctx.lg_set_params(p)
        ctx.lg_save(path)
        with lib.Context(0) as c2:
            problem(c2, N=N)
            c2.lg_load(path)
            assert np.array_equal(c2.lg_params(), p)
        with lib.Context(0) as c3:
            problem(c3, N=64)
            with pytest.raises(lib.PitdynError):
                c3.lg_load(path)  # other grid
        raw = path.read_bytes()
        (tmp_path / "short.bin").write_bytes(raw[:-4])
        (tmp_path / "magic.bin").write_bytes(b"XXXXXXXX" + raw[8:])
        with lib.Context(0) as c4:
            problem(c4, N=N)
            for bad in ("short.bin", "magic.bin", "missing.bin"):
                with pytest.raises(lib.PitdynError):
                    c4.lg_load(tmp_path / bad)


@pytest.mark.parametrize("chunks", [0, 2])
def test_report_speedup_model_matches_its_times(lib, chunks):
    """R_f / R_c and the speed-up estimate in the report follow eq. speed_up
    from the report's own sweep times (oracle formula), stay under the
    bound of eq. speed_bound, and are zero when no iteration ran."""
    from oracle import parareal as pr
    N, P, tol = 32, 6, 1e-10
    with lib.Context(0) as ctx:
        problem(ctx, N=N, P=P)
        ctx.set_pipeline(chunks)
        ctx.set_initial(initial_field(N, 0.57, 41))
        r = ctx.parareal(tol, P + 1)
        k = r["k_con"] if r["k_con"] > 0 else r["iters"]
        Rf = r["t_fine_s"] / r["iters"]
        Rc = (r["t_coarse0_s"] + r["t_coarse_s"]) / (r["iters"] + 1) / P
        assert r["Rf_over_Rc"] == pytest.approx(Rf / Rc, rel=1e-12)
        s = pr.speedup_model(k, P, Rc / Rf)
        assert r["model_speedup"] == pytest.approx(s, rel=1e-12)
        assert 0.0 < r["model_speedup"] <= pr.speedup_bound(k, P, Rc / Rf) * (1 + 1e-12)
        ctx.set_initial(initial_field(N, 0.57, 41))
        r0 = ctx.parareal(tol, 0)
        assert r0["Rf_over_Rc"] == 0.0 and r0["model_speedup"] == 0.0


@pytest.mark.parametrize("N,kz,seed,kmax", [(32, 0.57, 7, 4.0), (256, 1.1, 300017, 30.0)])
def test_seed_initial_is_the_reference_field(lib, N, kz, seed, kmax):
    """pd_seed_initial puts the generator's field bitwise into U_0."""
    from synthetic import initial_field
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", 50.0, kz, N)
        ctx.set_time(1.0, 2, 0.05, 0.25, 0)
        ctx.seed_initial(seed, 1e-3, kmax)
        U0 = ctx.get_slices()[0]
    ref = initial_field(N, kz, seed, amp=1e-3, kmax=kmax)
    assert np.array_equal(U0.view(np.uint64), ref.view(np.uint64))


@pytest.mark.parametrize("chunks,learned", [(0, False), (3, False), (0, True), (2, True)])
def test_parareal_continue_is_bitwise_an_uninterrupted_run(lib, chunks, learned):
    """A solve run in pieces (pd_parareal to iteration 2, then
    pd_parareal_continue to 4 and to the end) gives the iterates, defects and
    k_con of one call, plain and pipelined, plain and learned coarse
    propagator."""
    N, P = 32, 8

    def make():
        ctx = lib.Context(0)
        ctx.set_problem("gp", 60.0, 0.57, N)
        ctx.set_time(0.25 * P, P, 5e-3, 2.5e-2, 16)
        ctx.set_pipeline(chunks, 2)
        if learned:
            ctx.lg_init(2, 11)
            ctx.set_coarse(True)
        ctx.set_initial(initial_field(N, 0.57, 77))
        return ctx

    with make() as a:
        ra = a.parareal(1e-10, P + 1)
        Ua = a.get_slices()
    with make() as b:
        r1 = b.parareal(1e-10, 2)
        assert r1["iters"] == 2 and r1["status"] == lib.NOT_CONVERGED
        r2 = b.parareal_continue(1e-10, 4)
        assert r2["iters"] == 4
        r3 = b.parareal_continue(1e-10, P + 1)
        Ub = b.get_slices()
        with pytest.raises(lib.PitdynError):
            b.parareal_continue(1e-10, r3["iters"])     # max_iter must exceed the last iteration
    assert r3["k_con"] == ra["k_con"] and r3["iters"] == ra["iters"]
    sig = r1["sigma"][:2] + r2["sigma"][2:4] + r3["sigma"][4:r3["iters"]]
    assert sig == ra["sigma"][:ra["iters"]]
    assert np.array_equal(Ua, Ub)


def test_parareal_continue_needs_a_run_on_the_current_state(lib):
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", 60.0, 0.57, 32)
        ctx.set_time(2.0, 8, 5e-3, 2.5e-2, 16)
        ctx.set_initial(initial_field(32, 0.57, 77))
        with pytest.raises(lib.PitdynError):
            ctx.parareal_continue(1e-10, 3)             # no run yet
        ctx.parareal(1e-10, 1)
        ctx.set_initial(initial_field(32, 0.57, 78))
        with pytest.raises(lib.PitdynError):
            ctx.parareal_continue(1e-10, 3)             # the state changed since
        ctx.parareal(0.0, 0)                            # the initial coarse run only
        r = ctx.parareal_continue(0.0, 2)
        assert r["iters"] == 2


def test_plain_then_learned_coarse_propagator(lib):
    """Iterations 1-2 with the plain coarse propagator, then the learned one
    (pd_set_coarse between pd_parareal and pd_parareal_continue): after P
    iterations the result is the serial fine solution, bitwise the plain
    run's (finite termination holds for any coarse propagator); switching
    back to the plain propagator cannot continue (no coarse values)."""
    N, P = 32, 6

    def make():
        ctx = lib.Context(0)
        ctx.set_problem("gp", 60.0, 0.57, N)
        ctx.set_time(0.25 * P, P, 5e-3, 2.5e-2, 16)
        ctx.lg_init(2, 11)
        ctx.set_initial(initial_field(N, 0.57, 77))
        return ctx

    with make() as a:
        a.parareal(0.0, P)
        Ua = a.get_slices()
    with make() as b:
        b.parareal(0.0, 2)
        b.set_coarse(True)
        r = b.parareal_continue(0.0, P)
        assert r["iters"] == P
        Ub = b.get_slices()
        b.set_coarse(False)
        with pytest.raises(lib.PitdynError):
            b.parareal_continue(0.0, P + 1)
    assert np.array_equal(Ua, Ub)
