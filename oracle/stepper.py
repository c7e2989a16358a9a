"""IMEX slice propagators (SBDF2, ARS(4,4,3)) and Fourier resampling (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The explicit operator (advection/stretching, curl(u x b)) is stepped
explicitly and the diffusion Rm^-1 (lap - kz^2) = -|k|^2/Rm implicitly
(Section 4: explicit (u.grad)B and (B.grad)u, implicit diffusion).  The
stepper is the second-order semi-implicit backward difference formula SBDF2
of the multistep IMEX family Section 4 cites.  Because a multistep method
must restart in every time slice (Section 4), each slice starts with one
SBDF1 (backward/forward Euler) step:

  SBDF1:  (1 + dt|k|^2/Rm) b1 = b0 + dt N(b0, t0)
  SBDF2:  (3/2 + dt|k|^2/Rm) b_{j+1} = 2 b_j - b_{j-1}/2
                                       + dt (2 N(b_j, t_j) - N(b_{j-1}, t_{j-1}))

with t_j = t0 + j dt evaluated as a product, never accumulated.

Coarse grids (Section 3.2 lists coarsening in space together with a larger
step as a coarse strategy, and Section 5.2 adopts it; Section 4 moves fields
between the two solvers by Fourier re-sampling): a field moves to an N_C grid
by keeping the coefficients inside the N_C 2/3 box, and back by zero
padding.
"""
from __future__ import annotations

import numpy as np

from . import spectral as sp


def propagate(bh: np.ndarray, flow: str, Rm: float, kz: float, t0: float,
              dt: float, nsteps: int) -> np.ndarray:
    """Advance one field ``[3][N][N]`` by ``nsteps`` steps of size ``dt``
    from time ``t0``: one SBDF1 start step, then SBDF2."""
    if nsteps < 1:
        raise ValueError("nsteps must be >= 1")
    N = bh.shape[-1]
    a = dt * sp.k_squared(N, kz) / Rm
    b_old = np.array(bh, dtype=np.complex128)
    n_old = sp.explicit_term(b_old, flow, kz, t0)
    b = (b_old + dt * n_old) / (1.0 + a)
    for j in range(1, nsteps):
        n_j = sp.explicit_term(b, flow, kz, t0 + j * dt)
        b_new = (2.0 * b - 0.5 * b_old + dt * (2.0 * n_j - n_old)) / (1.5 + a)
        b_old, b, n_old = b, b_new, n_j
    return b


# IMEX Runge-Kutta pairs of Ascher, Ruuth & Spiteri (1997): ARS(4,4,3) is
# the "RK443" the paper steps with (Section 4; Section 5.1 compares it with
# the lower-order RK111 = ARS(1,1,1) and RK222 = ARS(2,2,2)).  For a pair
# with s explicit stages, stage i = 1..s+1 (stage 1 = the step's start value)
# solves
#   X_i = b_n + dt sum_{j<i} A_ij N(X_j, t + C_j dt) + dt sum_{j<=i} AT_ij L X_j,
# L = -|k|^2/Rm diagonal; all three are stiffly accurate: b_{n+1} = X_{s+1}.
from fractions import Fraction as _Fr

RK443_C = (_Fr(0), _Fr(1, 2), _Fr(2, 3), _Fr(1, 2), _Fr(1))
RK443_A = (  # explicit part, strictly lower triangular
    (),
    (_Fr(1, 2),),
    (_Fr(11, 18), _Fr(1, 18)),
    (_Fr(5, 6), _Fr(-5, 6), _Fr(1, 2)),
    (_Fr(1, 4), _Fr(7, 4), _Fr(3, 4), _Fr(-7, 4)),
)
RK443_AT = (  # implicit part, lower triangular with diagonal 1/2 (first row and column zero)
    (_Fr(0),),
    (_Fr(0), _Fr(1, 2)),
    (_Fr(0), _Fr(1, 6), _Fr(1, 2)),
    (_Fr(0), _Fr(-1, 2), _Fr(1, 2), _Fr(1, 2)),
    (_Fr(0), _Fr(3, 2), _Fr(-3, 2), _Fr(1, 2), _Fr(1, 2)),
)

# ARS(2,2,2): gamma = 1 - 1/sqrt(2), delta = 1 - 1/(2 gamma) (irrational, so floats)
_G2 = 1.0 - 1.0 / np.sqrt(2.0)
_D2 = 1.0 - 1.0 / (2.0 * _G2)
RK222_C = (0.0, _G2, 1.0)
RK222_A = ((), (_G2,), (_D2, 1.0 - _D2))
RK222_AT = ((0.0,), (0.0, _G2), (0.0, 1.0 - _G2, _G2))

# ARS(1,1,1): forward-backward Euler
RK111_C = (_Fr(0), _Fr(1))
RK111_A = ((), (_Fr(1),))
RK111_AT = ((_Fr(0),), (_Fr(0), _Fr(1)))

RK_TABLEAUS = {
    "rk443": (RK443_C, RK443_A, RK443_AT),
    "rk222": (RK222_C, RK222_A, RK222_AT),
    "rk111": (RK111_C, RK111_A, RK111_AT),
}


def propagate_imex_rk(bh: np.ndarray, flow: str, Rm: float, kz: float, t0: float,
                      dt: float, nsteps: int, scheme: str = "rk443") -> np.ndarray:
    """Advance one field ``[3][N][N]`` by ``nsteps`` steps of the IMEX
    Runge-Kutta pair ``scheme`` with size ``dt`` from time ``t0`` (step j
    starts at t0 + j dt, a product; stage i of it evaluates the flow at
    t0 + j dt + C_i dt).  One-step methods: nothing restarts at slice
    boundaries."""
    if nsteps < 1:
        raise ValueError("nsteps must be >= 1")
    Ct, At, ATt = RK_TABLEAUS[scheme]
    S = len(Ct)  # stages including the start value
    N = bh.shape[-1]
    L = -sp.k_squared(N, kz) / Rm
    A = [[float(v) for v in row] for row in At]
    AT = [[float(v) for v in row] for row in ATt]
    C = [float(v) for v in Ct]
    b = np.array(bh, dtype=np.complex128)
    for j in range(nsteps):
        t = t0 + j * dt
        X, NX = [], []
        for i in range(S):
            rhs = b.copy()
            for m in range(i):
                rhs = rhs + dt * (A[i][m] * NX[m] + AT[i][m] * L * X[m])
            Xi = rhs / (1.0 - dt * AT[i][i] * L) if AT[i][i] != 0.0 else rhs
            X.append(Xi)
            if i < S - 1:
                NX.append(sp.explicit_term(Xi, flow, kz, t + C[i] * dt))
        b = X[S - 1]
    return b


def propagate_rk443(bh: np.ndarray, flow: str, Rm: float, kz: float, t0: float,
                    dt: float, nsteps: int) -> np.ndarray:
    """``propagate_imex_rk`` with ARS(4,4,3)."""
    return propagate_imex_rk(bh, flow, Rm, kz, t0, dt, nsteps, "rk443")


def propagate_scheme(bh: np.ndarray, flow: str, Rm: float, kz: float, t0: float,
                     dt: float, nsteps: int, scheme: str = "sbdf2") -> np.ndarray:
    """``propagate`` (scheme "sbdf2") or ``propagate_imex_rk`` ("rk443",
    "rk222", "rk111")."""
    if scheme == "sbdf2":
        return propagate(bh, flow, Rm, kz, t0, dt, nsteps)
    if scheme in RK_TABLEAUS:
        return propagate_imex_rk(bh, flow, Rm, kz, t0, dt, nsteps, scheme)
    raise ValueError(f"unknown scheme {scheme!r}")


def restrict(bh: np.ndarray, Nc: int) -> np.ndarray:
    """Fine ``[3][N][N]`` -> coarse ``[3][Nc][Nc]``: keep the modes with
    |kx|, |ky| <= floor((Nc - 1)/3), drop the rest."""
    N = bh.shape[-1]
    if Nc == N:
        return np.array(bh, dtype=np.complex128)
    Kc = sp.box_K(Nc)
    kc = sp.wavenumbers(Nc)
    out = np.zeros(bh.shape[:-2] + (Nc, Nc), dtype=np.complex128)
    for iy in range(Nc):
        for ix in range(Nc):
            ky, kx = int(kc[iy]), int(kc[ix])
            if abs(ky) <= Kc and abs(kx) <= Kc:
                out[..., iy, ix] = bh[..., ky % N, kx % N]
    return out


def prolong(bc: np.ndarray, N: int) -> np.ndarray:
    """Coarse ``[3][Nc][Nc]`` -> fine ``[3][N][N]`` by zero padding."""
    Nc = bc.shape[-1]
    if Nc == N:
        return np.array(bc, dtype=np.complex128)
    kc = sp.wavenumbers(Nc)
    out = np.zeros(bc.shape[:-2] + (N, N), dtype=np.complex128)
    for iy in range(Nc):
        for ix in range(Nc):
            ky, kx = int(kc[iy]), int(kc[ix])
            out[..., ky % N, kx % N] = bc[..., iy, ix]
    return out


class SliceSolver:
    """One propagator (F or G) over a Parareal time slice [t_n, t_n + dT].

    ``N_solver`` is the grid it steps on; fields come in and go out on the
    fine grid ``N`` (restricted on entry, prolonged on exit when the grids
    differ, as the Parareal pseudo-code of Section 4.1 re-samples around each
    coarse solve).
    """

    def __init__(self, flow: str, Rm: float, kz: float, N: int, dT: float,
                 dt: float, N_solver: int | None = None, scheme: str = "sbdf2"):
        steps = dT / dt
        n = int(round(steps))
        if n < 1 or abs(steps - n) > 1e-9 * max(1.0, steps):
            raise ValueError("slice length must be an integer number of steps")
        self.flow, self.Rm, self.kz, self.N = flow, Rm, kz, N
        self.dT, self.dt, self.nsteps = dT, dt, n
        self.N_solver = N if N_solver is None else N_solver
        self.scheme = scheme

    def __call__(self, bh: np.ndarray, t0: float) -> np.ndarray:
        x = restrict(bh, self.N_solver)
        y = propagate_scheme(x, self.flow, self.Rm, self.kz, t0, self.dt, self.nsteps,
                             self.scheme)
        return prolong(y, self.N)
