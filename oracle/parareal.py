"""Parareal iteration, defect, growth rate and speed-up model (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Follows Section 3 of the paper: the interval [0, T] is cut into P equal
slices of length dT = T/P with t_n = n dT; a coarse sweep gives U^0_n; then

  U^{k}_{n+1} = G(U^{k}_n) + F(U^{k-1}_n) - G(U^{k-1}_n)      (eq. parareal)

with U^k_0 = U_0.  The fine solves F(U^{k-1}_n) are independent across
slices; the coarse sweep with the correction is sequential in n.  The
correction is evaluated as F + (G_new - G_old), the order the paper's
pseudo-code uses (new coarse minus old coarse plus fine), so that a slice
whose input did not change returns F bitwise.  Convergence is the relative
two-norm defect at the last slice (eq. error); k_con is the first k with
sigma_k <= tol (k = 0 is the coarse-only sweep, k_con counts fine sweeps).

For a propagator G that is linear in the field, G(a) - G(b) = G(a - b); the
``difference`` form evaluates U^k_{n+1} = F_n + G(U^k_n - U^{k-1}_n), which
is the same iteration and is what a learned linear coarse operator uses.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def norm2(x: np.ndarray) -> float:
    """Two-norm over every coefficient of a field."""
    return float(np.sqrt(np.sum(np.abs(x) ** 2)))


def defect(u_new: np.ndarray, u_old: np.ndarray) -> float:
    """sigma = ||u_new - u_old||_2 / ||u_new||_2 (eq. error)."""
    return norm2(u_new - u_old) / norm2(u_new)


@dataclass
class PararealResult:
    U: list                      # U[n], n = 0..P, final iterate
    history: list = field(default_factory=list)   # U^k for every k (optional)
    sigma: list = field(default_factory=list)     # sigma_k, k = 1..
    k_con: int = -1              # first k with sigma_k <= tol, -1 if none


def coarse_sweep(U0: np.ndarray, P: int, dT: float, G) -> list:
    """Initial coarse run: U^0_{n+1} = G(U^0_n), n = 0..P-1."""
    U = [np.array(U0, dtype=np.complex128)]
    for n in range(P):
        U.append(G(U[n], n * dT))
    return U


def serial_fine(U0: np.ndarray, P: int, dT: float, F) -> list:
    """The solution Parareal converges to: F applied slice after slice,
    restarting the stepper at every slice boundary."""
    return coarse_sweep(U0, P, dT, F)


def parareal(U0: np.ndarray, P: int, dT: float, F, G, tol: float,
             max_iter: int, form: str = "standard",
             keep_history: bool = False, fmap=None) -> PararealResult:
    """Run Parareal until sigma_k <= tol or k = max_iter.

    ``form`` is ``"standard"`` (store G(U^{k-1}_n) and correct with
    F + (G_new - G_old)) or ``"difference"`` (F + G(U^k_n - U^{k-1}_n),
    valid for linear G).  ``fmap(F, states, times)`` applies F to the
    slices of one iteration and returns the results in slice order (default:
    the built-in ``map``, one slice after another); the fine solves of an
    iteration are independent (Section 3), so a process pool's ``map`` may
    run them concurrently.
    """
    fmap = map if fmap is None else fmap
    if form not in ("standard", "difference"):
        raise ValueError(form)
    U = coarse_sweep(U0, P, dT, G)
    g_old = [U[n + 1] for n in range(P)]
    res = PararealResult(U=U)
    if keep_history:
        res.history.append([u.copy() for u in U])
    for k in range(1, max_iter + 1):
        f = list(fmap(F, [U[n] for n in range(P)], [n * dT for n in range(P)]))
        V = [U[0]]
        for n in range(P):
            if form == "standard":
                g_new = G(V[n], n * dT)
                V.append(f[n] + (g_new - g_old[n]))
                g_old[n] = g_new
            else:
                V.append(f[n] + G(V[n] - U[n], n * dT))
        sigma = defect(V[P], U[P])
        U = V
        res.U = U
        res.sigma.append(sigma)
        if keep_history:
            res.history.append([u.copy() for u in U])
        if sigma <= tol:
            res.k_con = k
            break
    return res


def growth_rate(norms, times) -> float:
    """Amplitude growth rate: least-squares slope of ln||U_n|| against t_n
    over the second half of the slices, n = ceil(P/2) .. P.

    The paper reports growth rates (Table 1) without stating the estimator;
    this window skips the initial transient.
    """
    P = len(norms) - 1
    n0 = (P + 1) // 2
    t = np.asarray(times[n0:], dtype=np.float64)
    y = np.log(np.asarray(norms[n0:], dtype=np.float64))
    tm = t.mean()
    return float(np.sum((t - tm) * (y - y.mean())) / np.sum((t - tm) ** 2))


def speedup_model(k_con: int, P: int, Rc_over_Rf: float) -> float:
    """Estimated Parareal speed-up, eq. speed_up:
    s = [(1 + k/P) Rc/Rf + k/P]^-1."""
    return 1.0 / ((1.0 + k_con / P) * Rc_over_Rf + k_con / P)


def speedup_bound(k_con: int, P: int, Rc_over_Rf: float) -> float:
    """Upper bound, eq. speed_bound: min(P/k, Rf/Rc)."""
    return min(P / k_con, 1.0 / Rc_over_Rf)


def efficiency(s: float, P: int) -> float:
    """Parallel efficiency s / P (Section 3.1)."""
    return s / P
