"""Pins of the FP64 reference network (learned coarse correction):
manual gradients against central differences, linearity, G(0) = 0."""
import numpy as np
import pytest

from oracle import network as net


def tiny(seed=0, Mf=5, C=4, L=2, B=2):
    rng = np.random.default_rng(seed)
    p = net.init_params(Mf, C=C, L=L, seed=seed)
    p["W_out"] = rng.standard_normal(p["W_out"].shape) * 0.3
    p["gamma"] = 1.0 + 0.3 * rng.standard_normal(p["gamma"].shape)
    x = rng.standard_normal((B, Mf * Mf, 12))
    t = rng.uniform(0, 6, B)
    r = rng.standard_normal((B, Mf * Mf, 6))
    return p, x, t, r, Mf


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("name", ["W_in", "V", "gamma", "W_out"])
def test_manual_gradients_match_central_differences(name, weighted):
    p, x, t, r, Mf = tiny()
    w = np.random.default_rng(4).uniform(0.1, 2.0, Mf * Mf) if weighted else None
    _, g = net.loss_and_grad(p, x, t, r, Mf, w)
    rng = np.random.default_rng(1)
    flat = p[name].reshape(-1)
    for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
        h = 1e-6
        old = flat[idx]
        flat[idx] = old + h
        lp, _ = net.loss_and_grad(p, x, t, r, Mf, w)
        flat[idx] = old - h
        lm, _ = net.loss_and_grad(p, x, t, r, Mf, w)
        flat[idx] = old
        fd = (lp - lm) / (2 * h)
        an = g[name].reshape(-1)[idx]
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)


def test_shift_convention():
    Mf = 4
    h = np.arange(Mf * Mf, dtype=float).reshape(1, Mf * Mf, 1)
    s = net.shift_rows(h, Mf, 0, 1)            # out[m] = h[m + (0, +1)]
    assert s[0, 0, 0] == 1 and s[0, Mf - 1, 0] == 0
    s = net.shift_rows(h, Mf, 1, 0)            # out[m] = h[m + (+1, 0)]
    assert s[0, 0, 0] == Mf and s[0, (Mf - 1) * Mf, 0] == 0


def test_learned_propagator_is_linear_and_zero_at_zero():
    rng = np.random.default_rng(3)
    Mf = 7
    p = net.init_params(Mf, C=4, L=2, seed=3)
    p["W_out"] = rng.standard_normal(p["W_out"].shape)
    D = rng.standard_normal((1, 3, Mf, Mf)) + 1j * rng.standard_normal((1, 3, Mf, Mf))
    g = rng.standard_normal((1, 3, Mf, Mf)) + 1j * rng.standard_normal((1, 3, Mf, Mf))
    t = np.array([1.3])
    a = net.apply(p, D, g, t)
    b = net.apply(p, 2.5 * D, 2.5 * g, t)
    assert np.allclose(b, 2.5 * a, rtol=1e-12, atol=1e-12)
    z = net.apply(p, 0 * D, 0 * g, t)
    assert np.all(z == 0)


def test_weighted_loss_closed_form():
    """With all weights equal the weighted loss is the plain one; with a
    weight on one mode only it is that mode's relative error."""
    p, x, t, r, Mf = tiny(seed=5)
    l1, _ = net.loss_and_grad(p, x, t, r, Mf)
    l2, _ = net.loss_and_grad(p, x, t, r, Mf, np.full(Mf * Mf, 3.0))
    assert abs(l1 - l2) <= 1e-14 * l1
    w = np.zeros(Mf * Mf)
    w[7] = 1.0
    c, _ = net.forward(p, x, t, Mf)
    ref = np.sum((c[:, 7] - r[:, 7]) ** 2) / np.sum(r[:, 7] ** 2)
    l3, _ = net.loss_and_grad(p, x, t, r, Mf, w)
    assert abs(l3 - ref) <= 1e-14 * ref


def test_bf16_rounding_pins():
    """BF16 keeps 8 significant bits, rounding to nearest with ties to even."""
    one = 1.0
    cases = [(1.0, 1.0), (1 + 2.0 ** -8, 1.0), (1 + 3 * 2.0 ** -8, 1 + 2.0 ** -6),
             (1 + 2.0 ** -7, 1 + 2.0 ** -7), (1 + 1.5 * 2.0 ** -7, 1 + 2.0 ** -6),
             (-3.0, -3.0), (0.0, 0.0), (2.0 ** -130, 2.0 ** -130), (65504.0, 65536.0)]
    for v, want in cases:
        assert net.bf16(np.array([v]))[0] == want, (v, net.bf16(np.array([v]))[0], want)
    rng = np.random.default_rng(0)
    a = rng.standard_normal(10000) * 10.0 ** rng.uniform(-5, 5, 10000)
    b = net.bf16(a)
    assert np.all(np.abs(b - a) <= (2.0 ** -8 + 2.0 ** -23) * np.abs(a))
    assert one == 1.0


def test_rounded_operands_change_only_the_products():
    """With rnd = identity the forward and gradients are the exact network;
    with BF16 rounding they move by about the BF16 unit."""
    p, x, t, r, Mf = tiny()
    c0, _ = net.forward(p, x, t, Mf)
    c1, _ = net.forward(p, x, t, Mf, rnd=lambda a: a)
    assert np.array_equal(c0, c1)
    c2, _ = net.forward(p, x, t, Mf, rnd=net.bf16)
    d = np.linalg.norm(c2 - c0) / np.linalg.norm(c0)
    assert 1e-5 < d < 2e-2
    l0, g0 = net.loss_and_grad(p, x, t, r, Mf)
    l2, g2 = net.loss_and_grad(p, x, t, r, Mf, rnd=net.bf16)
    assert abs(l2 - l0) <= 2e-2 * l0
