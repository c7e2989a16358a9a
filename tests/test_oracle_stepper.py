"""Pins of the oracle's SBDF slice propagator and Fourier resampling."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import spectral as sp, stepper
from synthetic import initial_field
from tests import pins


def test_pure_diffusion_matches_discrete_closed_form():
    """u = 0: each mode follows the SBDF1/SBDF2 recurrence exactly; its
    closed form (roots of (3/2 + a) r^2 - 2 r + 1/2) fixes every step."""
    N, kz, Rm, dt = 16, 0.8, 3.0, 0.05
    rng = np.random.default_rng(0)
    b0 = (rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N)))
    b0 *= sp.box_mask(N)[None]
    a = dt * sp.k_squared(N, kz) / Rm
    for n in (1, 2, 7, 40):
        got = stepper.propagate(b0, "none", Rm, kz, 0.0, dt, n)
        ref = pins.sbdf_diffusion_factor(a, n)[None] * b0
        assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(b0))


def test_pure_diffusion_is_second_order_against_exp_decay():
    """u = 0 against the exact decay exp(-|k|^2 t / Rm): error ~ dt^2."""
    N, kz, Rm, T = 16, 1.0, 5.0, 1.0
    b0 = initial_field(N, kz, 3)
    exact = b0 * np.exp(-sp.k_squared(N, kz) * T / Rm)[None]
    errs = []
    for n in (50, 100, 200):
        b = stepper.propagate(b0, "none", Rm, kz, 0.0, T / n, n)
        errs.append(np.linalg.norm(b - exact) / np.linalg.norm(exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


@pytest.mark.parametrize("flow", ["roberts", "gp"])
def test_time_order_two_with_flow(flow):
    """Self-convergence ratio near 4 when dt halves (second order)."""
    N, kz, Rm, T = 16, 0.57, 20.0, 0.5
    b0 = initial_field(N, kz, 4)
    sols = [stepper.propagate(b0, flow, Rm, kz, 0.7, T / n, n)
            for n in (50, 100, 200, 400)]
    d = [np.linalg.norm(sols[i] - sols[i + 1]) for i in range(3)]
    assert 3.6 < d[0] / d[1] < 4.4 and 3.6 < d[1] / d[2] < 4.4, d


def _direct_rhs(flow, Rm, kz, N):
    mask = sp.box_mask(N)
    k2 = sp.k_squared(N, kz)
    shape = (3, N, N)

    def f(t, y):
        bh = y.reshape(shape)
        return (pins.direct_explicit(bh, flow, kz, t) - (k2 / Rm)[None] * bh * mask).ravel()
    return f


def test_gp_trajectory_matches_independent_integrator():
    """The SBDF2 solution (dt = 1e-3) of the Galloway-Proctor dynamo over
    [0.4, 2.4] against DOP853 on the direct-convolution ODE (rtol 1e-11):
    agreement to the expected O(dt^2) level."""
    N, kz, Rm = 16, 0.57, 3.0
    b0 = initial_field(N, kz, 5, amp=1.0)
    t0, T = 0.4, 2.0
    ref = solve_ivp(_direct_rhs("gp", Rm, kz, N), (t0, t0 + T), b0.ravel(),
                    method="DOP853", rtol=1e-11, atol=1e-13).y[:, -1].reshape(b0.shape)
    errs = []
    for dt in (2e-3, 1e-3):
        got = stepper.propagate(b0, "gp", Rm, kz, t0, dt, int(round(T / dt)))
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert errs[1] < 1e-5, errs
    assert 3.3 < errs[0] / errs[1] < 4.7, errs


def test_restrict_prolong_roundtrip_and_interpolation():
    N, Nc, kz = 32, 16, 0.9
    rng = np.random.default_rng(1)
    bc = (rng.standard_normal((3, Nc, Nc)) + 1j * rng.standard_normal((3, Nc, Nc)))
    bc *= sp.box_mask(Nc)[None]
    bf = stepper.prolong(bc, N)
    assert np.array_equal(stepper.restrict(bf, Nc), bc)
    # spectral interpolation: the fine field sampled on the coarse points
    fine_phys = pins.brute_synthesis(bf)
    coarse_phys = pins.brute_synthesis(bc)
    assert np.max(np.abs(fine_phys[:, ::2, ::2] - coarse_phys)) <= 1e-12 * np.max(np.abs(coarse_phys))
    # restriction keeps exactly the coarse box
    b = initial_field(N, kz, 2, kmax=N / 3)
    r = stepper.restrict(b, Nc)
    Kc = sp.box_K(Nc)
    for (my, mx) in [(0, 0), (1, Kc), (Nc - Kc, 3)]:
        ky = my if my < Nc // 2 else my - Nc
        kx = mx if mx < Nc // 2 else mx - Nc
        assert r[0, my, mx] == b[0, ky % N, kx % N]
    assert np.all(r[:, :, Kc + 1:Nc - Kc] == 0)


def test_slice_solver_rejects_non_integer_step_count():
    with pytest.raises(ValueError):
        stepper.SliceSolver("gp", 10.0, 1.0, 16, 1.0, 0.3)


# ---- ARS(4,4,3) ------------------------------------------------------------

def test_rk443_tableau_order_conditions():
    """Both parts of the transcribed ARS(4,4,3) tableau satisfy the Runge-Kutta
    order conditions up to order 3 and the two coupling conditions of an
    order-3 IMEX pair (exact rational arithmetic); row sums equal the stage
    times; both parts are stiffly accurate."""
    from fractions import Fraction as Fr
    C = stepper.RK443_C
    A = [list(r) + [Fr(0)] * (5 - len(r)) for r in stepper.RK443_A]
    AT = [list(r) + [Fr(0)] * (5 - len(r)) for r in stepper.RK443_AT]
    b, bt = A[4], AT[4]  # stiffly accurate: the weights are the last rows
    assert b[4] == 0 and bt[4] == Fr(1, 2)
    for i in range(5):
        assert sum(A[i]) == C[i] and sum(AT[i]) == C[i]
        assert all(A[i][j] == 0 for j in range(i, 5))
        assert all(AT[i][j] == 0 for j in range(i + 1, 5))
        assert AT[i][0] == 0 and (i == 0 or AT[i][i] == Fr(1, 2))
    for w, M in ((b, A), (bt, AT)):
        assert sum(w) == 1
        assert sum(w[i] * C[i] for i in range(5)) == Fr(1, 2)
        assert sum(w[i] * C[i] ** 2 for i in range(5)) == Fr(1, 3)
        assert sum(w[i] * M[i][j] * C[j] for i in range(5) for j in range(5)) == Fr(1, 6)
    # coupling of the explicit and implicit parts
    assert sum(b[i] * AT[i][j] * C[j] for i in range(5) for j in range(5)) == Fr(1, 6)
    assert sum(bt[i] * A[i][j] * C[j] for i in range(5) for j in range(5)) == Fr(1, 6)


def test_rk443_pure_diffusion_third_order_and_l_stable():
    """u = 0 against exp(-|k|^2 t/Rm): error ~ dt^3; one huge step (|k|^2 dt/Rm
    ~ 1e6) damps every mode to nearly zero (L-stability)."""
    N, kz, Rm, T = 16, 1.0, 5.0, 1.0
    b0 = initial_field(N, kz, 3)
    exact = b0 * np.exp(-sp.k_squared(N, kz) * T / Rm)[None]
    errs = []
    for n in (10, 20, 40):
        b = stepper.propagate_rk443(b0, "none", Rm, kz, 0.0, T / n, n)
        errs.append(np.linalg.norm(b - exact) / np.linalg.norm(exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 6.5 < r1 < 9.5 and 6.5 < r2 < 9.5, errs
    big = stepper.propagate_rk443(b0, "none", 1e-6, kz, 0.0, 1.0, 1)
    assert np.linalg.norm(big) <= 1e-5 * np.linalg.norm(b0)


def test_rk443_gp_trajectory_third_order_against_independent_integrator():
    """The ARS(4,4,3) solution of the Galloway-Proctor dynamo over [0.4, 2.4]
    against DOP853 on the direct-convolution ODE: error ratio near 8 when dt
    halves."""
    N, kz, Rm = 16, 0.57, 3.0
    b0 = initial_field(N, kz, 5, amp=1.0)
    t0, T = 0.4, 2.0
    ref = solve_ivp(_direct_rhs("gp", Rm, kz, N), (t0, t0 + T), b0.ravel(),
                    method="DOP853", rtol=1e-12, atol=1e-14).y[:, -1].reshape(b0.shape)
    errs = []
    for dt in (4e-2, 2e-2, 1e-2):
        got = stepper.propagate_rk443(b0, "gp", Rm, kz, t0, dt, int(round(T / dt)))
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert errs[2] < 1e-5, errs
    assert 6.0 < errs[0] / errs[1] < 10.0 and 6.0 < errs[1] / errs[2] < 10.0, errs


def test_rk443_slice_solver_and_scheme_switch():
    N, kz = 16, 0.57
    b0 = initial_field(N, kz, 6)
    F = stepper.SliceSolver("roberts", 10.0, kz, N, 0.5, 0.05, scheme="rk443")
    assert np.array_equal(F(b0, 0.0), stepper.propagate_rk443(b0, "roberts", 10.0, kz, 0.0, 0.05, 10))
    with pytest.raises(ValueError):
        stepper.propagate_scheme(b0, "roberts", 10.0, kz, 0.0, 0.05, 1, "rk4")


def test_rk222_and_rk111_tableaus_and_orders():
    """ARS(2,2,2): order-2 conditions of both parts and their coupling (floats,
    gamma irrational); ARS(1,1,1): a single step is the SBDF1 step exactly in
    exact arithmetic (forward-backward Euler), and to rounding in floats.
    Self-convergence orders 2 and 1 with the Galloway-Proctor flow."""
    C, A, AT = stepper.RK222_C, stepper.RK222_A, stepper.RK222_AT
    A = [list(r) + [0.0] * (3 - len(r)) for r in A]
    AT = [list(r) + [0.0] * (3 - len(r)) for r in AT]
    b, bt = A[2], AT[2]
    for i in range(3):
        assert abs(sum(A[i]) - C[i]) < 1e-15 and abs(sum(AT[i]) - C[i]) < 1e-15
    for w in (b, bt):
        assert abs(sum(w) - 1.0) < 1e-15
        assert abs(sum(w[i] * C[i] for i in range(3)) - 0.5) < 1e-15
    assert abs(AT[1][1] - AT[2][2]) < 1e-15 and abs(AT[1][1] - (1 - 2 ** -0.5)) < 1e-15
    N, kz = 16, 0.57
    b0 = initial_field(N, kz, 12, amp=1.0)
    one = stepper.propagate_imex_rk(b0, "gp", 3.0, kz, 0.3, 0.02, 1, "rk111")
    sb1 = stepper.propagate(b0, "gp", 3.0, kz, 0.3, 0.02, 1)
    assert np.linalg.norm(one - sb1) <= 1e-15 * np.linalg.norm(sb1)
    for scheme, lo, hi in (("rk222", 3.5, 4.5), ("rk111", 1.8, 2.2)):
        sols = [stepper.propagate_imex_rk(b0, "gp", 3.0, kz, 0.3, 0.5 / n, n, scheme)
                for n in (40, 80, 160)]
        d = [np.linalg.norm(sols[i] - sols[i + 1]) for i in range(2)]
        assert lo < d[0] / d[1] < hi, (scheme, d)
