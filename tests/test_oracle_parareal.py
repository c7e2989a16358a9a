"""Pins of the oracle's Parareal iteration, defect, growth rate and
speed-up model."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import parareal as pr, spectral as sp, stepper
from synthetic import initial_field
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _setup(flow="roberts", N=16, Nc=16, P=6, Rm=10.0, kz=1.0, dt=1e-2, Dt=5e-2, dT=0.5):
    F = stepper.SliceSolver(flow, Rm, kz, N, dT, dt)
    G = stepper.SliceSolver(flow, Rm, kz, N, dT, Dt, Nc)
    b0 = initial_field(N, kz, 42)
    return F, G, b0, P, dT


@pytest.mark.parametrize("flow,Nc", [("roberts", 16), ("gp", 8)])
def test_finite_termination_is_bitwise(flow, Nc):
    """After k iterations U_n for n <= k equals the serial fine solution
    exactly (Section 3.1); k = P gives serial F everywhere; k = 0 is the
    serial coarse solution."""
    F, G, b0, P, dT = _setup(flow=flow, Nc=Nc)
    serial_f = pr.serial_fine(b0, P, dT, F)
    serial_g = pr.coarse_sweep(b0, P, dT, G)
    r = pr.parareal(b0, P, dT, F, G, tol=0.0, max_iter=P + 1, keep_history=True)
    for n in range(P + 1):
        assert np.array_equal(r.history[0][n], serial_g[n])
    for k in range(1, P + 2):
        for n in range(min(k, P) + 1):
            assert np.array_equal(r.history[k][n], serial_f[n]), (k, n)
    # iteration P + 1 changes nothing: zero defect, and the run stops there
    assert r.sigma[-1] == 0.0 and r.sigma[-2] > 0.0 and r.k_con == P + 1


def test_scalar_parareal_closed_form():
    """u = 0: every mode is a scalar linear problem, and Parareal's iterates
    follow the binomial closed form with the slice amplification factors of
    F and G (G on a coarser grid annihilates the modes outside its box)."""
    N, Nc, kz, Rm, dT, dt, Dt, P = 16, 8, 0.6, 2.0, 0.4, 0.02, 0.1, 5
    F = stepper.SliceSolver("none", Rm, kz, N, dT, dt)
    G = stepper.SliceSolver("none", Rm, kz, N, dT, Dt, Nc)
    rng = np.random.default_rng(9)
    b0 = (rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N)))
    b0 *= sp.box_mask(N)[None]
    k2 = sp.k_squared(N, kz)
    phiF = pins.sbdf_diffusion_factor(dt * k2 / Rm, int(round(dT / dt)))
    kc = sp.wavenumbers(N)
    in_coarse = (np.abs(kc)[None, :] <= sp.box_K(Nc)) & (np.abs(kc)[:, None] <= sp.box_K(Nc))
    phiG = np.where(in_coarse, pins.sbdf_diffusion_factor(Dt * k2 / Rm, int(round(dT / Dt))), 0.0)
    r = pr.parareal(b0, P, dT, F, G, tol=0.0, max_iter=3, keep_history=True)
    for k in range(4):
        for n in range(P + 1):
            ref = pins.scalar_parareal(phiF, phiG, n, k)[None] * b0
            assert np.max(np.abs(r.history[k][n] - ref)) <= 1e-13 * np.max(np.abs(b0)), (k, n)


def test_difference_form_equals_standard_for_linear_G():
    F, G, b0, P, dT = _setup(flow="gp", Nc=8, P=5)
    a = pr.parareal(b0, P, dT, F, G, tol=0.0, max_iter=3)
    b = pr.parareal(b0, P, dT, F, G, tol=0.0, max_iter=3, form="difference")
    for n in range(P + 1):
        assert np.linalg.norm(a.U[n] - b.U[n]) <= 1e-13 * np.linalg.norm(a.U[n])
    assert np.allclose(a.sigma, b.sigma, rtol=1e-6, atol=1e-15)


def test_fine_solves_in_any_order_or_processes_give_the_same_iterates():
    """The fine solves of one iteration are independent (Section 3): applied
    in reverse slice order, or in worker processes, they give bitwise the
    serial iterates."""
    import multiprocessing as mp
    F, G, b0, P, dT = _setup(flow="gp", Nc=8, P=5)
    a = pr.parareal(b0, P, dT, F, G, tol=0.0, max_iter=2)

    def reverse_map(fn, xs, ts):
        out = [fn(x, t) for x, t in reversed(list(zip(xs, ts)))]
        return list(reversed(out))
    b = pr.parareal(b0, P, dT, F, G, tol=0.0, max_iter=2, fmap=reverse_map)
    with mp.get_context("fork").Pool(2) as pool:
        c = pr.parareal(b0, P, dT, F, G, tol=0.0, max_iter=2,
                        fmap=lambda fn, xs, ts: pool.starmap(fn, zip(xs, ts)))
    for n in range(P + 1):
        assert np.array_equal(a.U[n], b.U[n]) and np.array_equal(a.U[n], c.U[n])
    assert a.sigma == b.sigma == c.sigma


def test_defect_and_k_con():
    F, G, b0, P, dT = _setup(flow="gp", Nc=16, P=6)
    r = pr.parareal(b0, P, dT, F, G, tol=1e-4, max_iter=6, keep_history=True)
    assert r.k_con == len(r.sigma) == 5 and r.sigma[-1] <= 1e-4
    assert all(s > 1e-4 for s in r.sigma[:-1])
    k = len(r.sigma)
    u1, u0 = r.history[k][P], r.history[k - 1][P]
    assert r.sigma[-1] == pytest.approx(np.sqrt(np.sum(np.abs(u1 - u0) ** 2) / np.sum(np.abs(u1) ** 2)), rel=1e-12)


def test_growth_rate_estimator_recovers_exact_exponential():
    t = np.arange(11) * 0.5
    norms = 3.0 * np.exp(0.137 * t)
    assert pr.growth_rate(norms, t) == pytest.approx(0.137, abs=1e-14)


def _direct_operator(flow, Rm, kz, N, t=0.0):
    """Dense matrix of the semi-discrete operator on the box coefficients,
    built column by column from the direct convolution."""
    mask = sp.box_mask(N)
    idx = np.argwhere(np.broadcast_to(mask, (3, N, N)))
    n = len(idx)
    k2 = sp.k_squared(N, kz)
    M = np.zeros((n, n), complex)
    for j, (c, y, x) in enumerate(idx):
        e = np.zeros((3, N, N), complex)
        e[c, y, x] = 1.0
        col = pins.direct_explicit(e, flow, kz, t) - (k2 / Rm)[None] * e
        M[:, j] = col[idx[:, 0], idx[:, 1], idx[:, 2]]
    return M


def test_roberts_growth_rate_matches_leading_eigenvalue():
    """Steady flow (Section 1: growth rate from an eigenvalue problem): the
    time-stepped amplitude growth rate tends to Re(lambda_max) of the
    discrete operator."""
    N, kz, Rm = 16, 1.0, 8.0
    lam = scipy.linalg.eigvals(_direct_operator("roberts", Rm, kz, N))
    lam_max = np.max(lam.real)
    P, dT, dt = 12, 2.5, 5e-3
    F = stepper.SliceSolver("roberts", Rm, kz, N, dT, dt)
    U = pr.serial_fine(initial_field(N, kz, 1), P, dT, F)
    gamma = pr.growth_rate([pr.norm2(u) for u in U], np.arange(P + 1) * dT)
    assert abs(gamma - lam_max) < 2e-3, (gamma, lam_max)


def test_table1_gp_growth_rate():
    """Table 1 (Section 5.3): Galloway-Proctor, Rm = 3, wavenumber 0.57,
    N_F = 16, dt = 5e-3 grows at 0.15 (two significant figures)."""
    with open(os.path.join(GOLDEN, "table1_growth_rates.json")) as fh:
        rows = json.load(fh)["rows"]
    row = next(r for r in rows if r["flow"] == "gp" and r["Rm"] == 3)
    N, kz, Rm, dt = row["N_F"], row["k"], row["Rm"], row["dt_fine"]
    P, dT = 50, 1.0
    F = stepper.SliceSolver("gp", Rm, kz, N, dT, dt)
    U = pr.serial_fine(initial_field(N, kz, 3), P, dT, F)
    gamma = pr.growth_rate([pr.norm2(u) for u in U], np.arange(P + 1) * dT)
    assert abs(gamma - row["growth_rate"]) <= 0.005 + 1e-9, gamma


def test_speedup_model_respects_bound_and_limits():
    rng = np.random.default_rng(0)
    for _ in range(200):
        P = int(rng.integers(2, 2000))
        k = int(rng.integers(1, P + 1))
        r = float(10 ** rng.uniform(-4, 0))
        s = pr.speedup_model(k, P, r)
        assert s <= pr.speedup_bound(k, P, r) * (1 + 1e-12)
    # free coarse solver: s = P / k exactly; k = P: s < 1
    assert pr.speedup_model(3, 48, 0.0) == pytest.approx(16.0)
    assert pr.speedup_model(10, 10, 1e-2) < 1.0
    assert pr.efficiency(pr.speedup_model(3, 48, 0.0), 48) == pytest.approx(1 / 3)


def test_speedup_model_hand_values_from_cost_decomposition():
    """Eq. speed_up (Section 3.1) is the ratio of the serial fine cost P R_f
    to the Parareal cost of one initial coarse run over all P slices plus k
    iterations of one fine slice and one coarse slice each:
    P R_c + k (R_f + R_c).  Hand-evaluated at nonzero R_c, so a swapped
    coefficient (1 + P/k in place of 1 + k/P) or a dropped term fails."""
    # P = 48, k = 3, R_f = 1, R_c = 0.01: 48 / (0.48 + 3 * 1.01) = 48 / 3.51
    assert pr.speedup_model(3, 48, 0.01) == pytest.approx(48.0 / 3.51, rel=1e-14)
    # P = 10, k = 4, R_f = 2, R_c = 0.5: 20 / (5 + 4 * 2.5) = 4/3
    assert pr.speedup_model(4, 10, 0.25) == pytest.approx(4.0 / 3.0, rel=1e-14)
    # P = 8, k = 8, R_c = R_f: 8 / (8 + 16) = 1/3 (Parareal with k = P loses)
    assert pr.speedup_model(8, 8, 1.0) == pytest.approx(1.0 / 3.0, rel=1e-14)


def test_speedup_model_reproduces_paper_gp_efficiency():
    """Section 5.3: Galloway-Proctor Parareal converges in k_con = 3 with an
    efficiency close to 0.3, near the 1/k_con bound.  The coarse solver there
    has half the resolution in each direction and a 50 times larger step
    (N_C = 256 vs N_F = 512, dt 5e-3 vs 1e-4), so R_c/R_f is about 1/200;
    with about 50 slices the model gives an efficiency of about 0.3."""
    s = pr.speedup_model(3, 50, 1.0 / 200.0)
    assert 0.28 <= pr.efficiency(s, 50) <= 1.0 / 3.0
