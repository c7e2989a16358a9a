"""GPU tests of the learned coarse propagator: the matrix-core forward and
backward (FP32-operand test mode and BF16) against the FP64 reference network
on host-made inputs, bitwise finite termination of
learned-G Parareal, and the gain of the trained network over plain G."""
import numpy as np
import pytest

from oracle import network as onet
from synthetic import initial_field

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def relnorm(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def unflatten(p, Q, L, C=32):
    o = 0
    out = {}
    for name, shape in (("W_in", (12, C)), ("V", (L, 3, 5, C, C)), ("gamma", (L, Q, C)),
                        ("W_out", (C, 6))):
        n = int(np.prod(shape))
        out[name] = p[o:o + n].astype(np.float64).reshape(shape)
        o += n
    assert o == p.size
    return out


def small_ctx(lib, N=32, P=4, layers=2, seed=1):
    ctx = lib.Context(0)
    ctx.set_problem("gp", 50.0, 0.57, N)
    ctx.set_time(1.0, P, 5e-3, 2.5e-2, N // 2)
    ctx.lg_init(layers, seed)
    return ctx


def _network_case(lib, ctx, N, L, beta, seed):
    """Host-made network inputs (features, targets, slice times) and
    trained-like parameters, stored in ctx; returns the FP64 views."""
    Q = (2 * ((N - 1) // 3) + 1) ** 2
    rng = np.random.default_rng(seed)
    p = ctx.lg_params()
    n_in, n_v = 12 * 32, L * 15 * 32 * 32
    p[:n_in] = (rng.standard_normal(n_in) / np.sqrt(12.0)).astype(np.float32)
    p[n_in:n_in + n_v] = (rng.standard_normal(n_v) * 0.3 / np.sqrt(160.0)).astype(np.float32)
    p[n_in + n_v:-32 * 6] = (1.0 + 0.3 * rng.standard_normal(L * Q * 32)).astype(np.float32)
    p[-32 * 6:] = (rng.standard_normal(32 * 6) * 0.2).astype(np.float32)
    ctx.lg_set_params(p)
    B = 4
    x = rng.standard_normal((B, Q, 12)).astype(np.float32)
    r = rng.standard_normal((B, Q, 6)).astype(np.float32)
    t = np.array([0.0, 0.7, 2.1, 5.3])
    assert ctx.lg_add_feature_samples(x, r, t) == B
    K = (N - 1) // 3
    ky, kx = np.meshgrid(np.arange(-K, K + 1), np.arange(-K, K + 1), indexing="ij")
    dT, Rm, kz = 1.0 / 4, 50.0, 0.57
    w = np.exp(-beta * (kx ** 2 + ky ** 2 + kz ** 2) * dT / Rm).ravel() if beta > 0 else None
    return unflatten(p, Q, L), x.astype(np.float64), r.astype(np.float64), t, w, int(round(np.sqrt(Q)))


@pytest.mark.parametrize("beta", [0.0, 4.0])
def test_network_fp32_operands_match_fp64_reference(lib, beta):
    """FP32-operand mode of the matrix-core kernels: forward outputs and the
    gradients of the (uniform or per-mode weighted) loss against the FP64
    network on the same host inputs, to 1e-5 relative (FP32 accumulation)."""
    N, L = 32, 2
    with small_ctx(lib, N=N, layers=L) as ctx:
        ctx.lg_set_loss_decay(beta)
        ctx.lg_set_operands(True)
        prm, x, r, t, w, Mf = _network_case(lib, ctx, N, L, beta, 3)
        c_ref, _ = onet.forward(prm, x, t, Mf)
        for i in range(4):
            e = relnorm(ctx.lg_forward_sample(i), c_ref[i])
            assert e <= 1e-5, (i, e)
        g_gpu, loss_gpu = ctx.lg_gradients(0, 4)
        loss_ref, g_ref = onet.loss_and_grad(prm, x, t, r, Mf, w)
        assert abs(loss_gpu - loss_ref) <= 1e-6 * loss_ref
        gg = unflatten(g_gpu, (2 * ((N - 1) // 3) + 1) ** 2, L)
        for name in ("W_in", "V", "gamma", "W_out"):
            e = relnorm(gg[name], g_ref[name])
            print(f"fp32 operands, beta={beta}: {name} gradient rel. L2 {e:.2e}", flush=True)
            assert e <= 1e-5, (name, e)


@pytest.mark.parametrize("beta", [0.0, 4.0])
def test_network_bf16_matches_fp64_on_rounded_operands(lib, beta):
    """BF16 mode (the default) against the FP64 network evaluated with both
    operands of every channel-mixing product rounded to BF16 the way the
    kernels round them (FP32 value, nearest even); products and sums exact
    in FP64 there, FP32-accumulated on the matrix cores.  A shift, transpose
    or channel-tile mistake confined to a few modes moves the result by far
    more than the 1e-4 bar."""
    N, L = 32, 2
    with small_ctx(lib, N=N, layers=L) as ctx:
        ctx.lg_set_loss_decay(beta)
        prm, x, r, t, w, Mf = _network_case(lib, ctx, N, L, beta, 4)
        c_ref, _ = onet.forward(prm, x, t, Mf, rnd=onet.bf16)
        c_exact, _ = onet.forward(prm, x, t, Mf)
        for i in range(4):
            e = relnorm(ctx.lg_forward_sample(i), c_ref[i])
            # the rounding itself moves the output by far more than the bar
            assert relnorm(c_exact[i], c_ref[i]) > 10 * max(e, 1e-5)
            assert e <= 1e-4, (i, e)
        g_gpu, loss_gpu = ctx.lg_gradients(0, 4)
        loss_ref, g_ref = onet.loss_and_grad(prm, x, t, r, Mf, w, rnd=onet.bf16)
        assert abs(loss_gpu - loss_ref) <= 1e-5 * loss_ref
        gg = unflatten(g_gpu, (2 * ((N - 1) // 3) + 1) ** 2, L)
        for name in ("W_in", "V", "gamma", "W_out"):
            e = relnorm(gg[name], g_ref[name])
            print(f"bf16 operands, beta={beta}: {name} gradient rel. L2 {e:.2e}", flush=True)
            assert e <= 1e-4, (name, e)


def test_learned_parareal_finite_termination_bitwise(lib):
    torch = _torch()
    N, P = 32, 4
    with small_ctx(lib, N=N, P=P) as ctx:
        b0 = initial_field(N, 0.57, 9)
        ctx.set_coarse(True)
        ctx.set_initial(b0)
        rep = ctx.parareal(0.0, P + 1)
        U = ctx.get_slices_dev()
        u = dev(b0[None])
        for n in range(P):
            u = ctx.fine([n * 1.0 / P], u)
            assert torch.equal(U[n + 1], u[0]), n
        assert rep["sigma"][-1] == 0.0


def test_parareal_samples_are_the_coarse_inputs(lib):
    """The harvested samples of iteration 0 are U^0_n of the plain coarse run
    and those of iteration 1 are U^1_n - U^0_n (n >= 1); the stored feature
    x = D/|D| (FP32) reproduces them slice by slice, with the slice
    start times."""
    N, P = 32, 4
    with small_ctx(lib, N=N, P=P) as ctx:
        b0 = initial_field(N, 0.57, 21)
        ctx.set_coarse(False)
        ctx.set_initial(b0)
        ctx.parareal(0.0, 0)
        U0 = ctx.get_slices()
        ctx.set_initial(b0)
        ctx.parareal(0.0, 1)
        U1 = ctx.get_slices()
        ctx.set_initial(b0)
        assert ctx.lg_add_parareal_samples(1) == P + (P - 1)
        K = (N - 1) // 3
        idx = np.r_[N - K:N, 0:K + 1]  # box rows/columns run over k = -K..K
        expect = [U0[n] for n in range(P)] + [U1[n] - U0[n] for n in range(1, P)]
        times = [float(n) / P for n in range(P)] + [float(n) / P for n in range(1, P)]
        for i, (D, tn) in enumerate(zip(expect, times)):
            x, _, t = ctx.lg_sample(i)
            box = D[:, idx][:, :, idx]
            Dn = box / np.linalg.norm(box)
            xm = x.reshape(2 * K + 1, 2 * K + 1, 12)
            got = (xm[..., 0:6:2] + 1j * xm[..., 1:6:2]).transpose(2, 0, 1)
            assert relnorm(got, Dn) <= 1e-6, (i, relnorm(got, Dn))
            assert abs(t - tn) <= 1e-12


def test_trained_network_lowers_coarse_error_and_converges(lib):
    """Train on the coarse inputs of plain-G Parareal runs (Galloway-Proctor
    Rm = 100, 64^2, 16 slices of length 1, coarse 32^2 with dt = 1e-2) from
    four initial fields; on a fifth run the relative one-slice error
    |F - G_learned| / |F - G| drops, and learned-G Parareal from a sixth
    field reaches sigma <= 1e-8 at the plain-G solution."""
    N, Nc, P, Rm, kz = 64, 32, 16, 100.0, 0.57
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", Rm, kz, N)
        ctx.set_time(float(P), P, 2e-3, 1e-2, Nc)
        ctx.lg_init(4, 3)
        ctx.set_coarse(False)
        n = 0
        for r in range(5):
            ntr = n
            ctx.set_initial(initial_field(N, kz, 700 + r))
            n = ctx.lg_add_parareal_samples(8)
        val0 = ctx.lg_loss(ntr, n - ntr)
        losses = ctx.lg_train(0, ntr, 800, 16, 2e-3, seed=11)
        val1 = ctx.lg_loss(ntr, n - ntr)
        print(f"held-out loss {val0:.3f} -> {val1:.3f}; last batch {losses[-1]:.3f}", flush=True)
        assert abs(val0 - 1.0) < 0.05  # untrained output is ~1e-3 of the target
        assert val1 < 0.7 * val0
        b0 = initial_field(N, kz, 123)
        ctx.set_coarse(False)
        ctx.set_initial(b0)
        rp = ctx.parareal(1e-8, P + 1)
        Up = ctx.get_slices()
        ctx.set_coarse(True)
        ctx.set_initial(b0)
        rl = ctx.parareal(1e-8, P + 1)
        Ul = ctx.get_slices()
        print(f"k_con plain {rp['k_con']} learned {rl['k_con']}", flush=True)
        assert 0 < rl["k_con"] <= P + 1
        assert relnorm(Ul[P], Up[P]) <= 1e-7


def test_learned_coarse_propagator_needs_fewer_iterations(lib):
    """The learned workload (Galloway-Proctor Rm = 500, kz = 0.57, 256^2,
    T = 64 over 128 slices, fine SBDF2 dt = 1e-3, coarse 64^2 with dt =
    5e-3, tol 1e-8): a network trained on the coarse inputs of iterations
    k >= 4 of plain-G Parareal from one initial field (2000 Adam steps)
    reaches the defect tolerance from another field in fewer iterations than
    the plain coarse propagator, at the same solution."""
    N, Nc, P, T, Rm, kz = 256, 64, 128, 64.0, 500.0, 0.57
    with lib.Context(0) as ctx:
        ctx.set_problem("gp", Rm, kz, N)
        ctx.set_time(T, P, 1e-3, 5e-3, Nc)
        b0 = initial_field(N, kz, 400000)
        ctx.set_coarse(False)
        ctx.set_initial(b0)
        rp = ctx.parareal(1e-8, P + 1)
        Up = ctx.get_slices()
        print(f"plain G: k_con {rp['k_con']} in {rp['t_total_s']:.2f} s", flush=True)
        ctx.lg_init(4, 400000)
        H, K0 = 16, 4
        block = P * (H + 1) - H * (H + 1) // 2
        skip = P + (K0 - 1) * P - (K0 - 1) * K0 // 2
        ctx.set_initial(initial_field(N, kz, 401000))
        n = ctx.lg_add_parareal_samples(H)
        assert n == block
        ctx.lg_train(skip, block - skip, 2000, 8, 1e-3, seed=5)
        ctx.set_coarse(True)
        ctx.set_initial(b0)
        rl = ctx.parareal(1e-8, P + 1)
        Ul = ctx.get_slices()
        print(f"learned G: k_con {rl['k_con']} in {rl['t_total_s']:.2f} s", flush=True)
        # the schedule the network was trained for: plain G for iterations
        # 1-4, the learned propagator from iteration 5 on
        ctx.set_coarse(False)
        ctx.set_initial(b0)
        ctx.parareal(1e-8, K0)
        ctx.set_coarse(True)
        rh = ctx.parareal_continue(1e-8, P + 1)
        Uh = ctx.get_slices()
        print(f"plain then learned G: k_con {rh['k_con']}", flush=True)
    assert 0 < rl["k_con"] < rp["k_con"]
    assert 0 < rh["k_con"] < rp["k_con"]
    assert relnorm(Ul[P], Up[P]) <= 1e-7
    assert relnorm(Uh[P], Up[P]) <= 1e-7
