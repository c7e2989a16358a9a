"""Fourier collocation pieces of the 2.5D kinematic dynamo (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Model (paper Section 2, eq. induction-dimensionless-1): dB/dt =
curl(u x B) + Rm^-1 lap B with B = b(x, y, t) exp(i kz z) (2.5D monochromatic
ansatz, Section 1), so d/dz -> i kz and the problem is 2D and complex on the
2pi-periodic square (Section 4: Fourier bases, N x N modes).

Conventions (readings of the paper where it is silent or ambiguous):
  * coefficients: b(x, y) = sum_k bh[k] exp(i (kx x + ky y)); arrays are
    complex128 ``[3][N][N]`` = [component][ky index][kx index];
  * dealiasing: the explicit term is truncated to the square box
    |kx|, |ky| <= K, K = floor((N - 1) / 3) (the 2/3 rule);
  * the explicit term is evaluated in curl form, i k x FFT(u x b); for
    solenoidal b and u it equals the advective component equations of
    Section 2.1 (Roberts) and 2.2 (Galloway-Proctor).
"""
from __future__ import annotations

import math

import numpy as np

FLOWS = ("none", "roberts", "gp")

# Galloway-Proctor CP amplitude: B = C = sqrt(3/2) (Section 2.2).
GP_AMPLITUDE = math.sqrt(1.5)


def wavenumbers(N: int) -> np.ndarray:
    """Signed wavenumber of FFT index m: m if m < N/2 else m - N."""
    return np.array([m if m < N // 2 else m - N for m in range(N)],
                    dtype=np.float64)


def box_K(N: int) -> int:
    """Largest retained |wavenumber| under the 2/3 rule."""
    return (N - 1) // 3


def box_mask(N: int) -> np.ndarray:
    """Boolean ``[N][N]`` (ky, kx) mask of the retained square box."""
    k = np.abs(wavenumbers(N))
    K = box_K(N)
    return (k[:, None] <= K) & (k[None, :] <= K)


def grid(N: int) -> np.ndarray:
    """Collocation points x_j = 2 pi j / N on [0, 2pi)."""
    return 2.0 * np.pi * np.arange(N) / N


def k_squared(N: int, kz: float) -> np.ndarray:
    """|k|^2 = kx^2 + ky^2 + kz^2 on the ``[ky][kx]`` index grid."""
    k = wavenumbers(N)
    return k[None, :] ** 2 + k[:, None] ** 2 + kz * kz


def to_physical(bh: np.ndarray) -> np.ndarray:
    """Grid values b(x_j, y_i) = sum_k bh[k] e^{i k.x} (last two axes)."""
    N = bh.shape[-1]
    return np.fft.ifft2(bh, axes=(-2, -1)) * (N * N)


def to_spectral(f: np.ndarray) -> np.ndarray:
    """Inverse of :func:`to_physical`: coefficients = FFT2(grid values)/N^2."""
    N = f.shape[-1]
    return np.fft.fft2(f, axes=(-2, -1)) / (N * N)


def velocity(flow: str, N: int, t: float):
    """Prescribed flow (ux, uy, uz) on the ``[y][x]`` grid at time t.

    * ``roberts`` (Section 2.1, ABC flow with A = B = 1, C = 0):
      u = (cos y, sin x, sin y + cos x), steady.
    * ``gp`` (Section 2.2, Galloway-Proctor CP flow, omega = 1,
      B = C = sqrt(3/2)).  The paper writes it in the (y, z) plane with the
      field varying as exp(i k_x x); relabelling the paper's (y, z, x) as
      (x, y, z) here gives
      u = A (cos(y + sin t), sin(x + cos t), cos(x + cos t) + sin(y + sin t)),
      A = sqrt(3/2); t is absolute time from the start of the run.
    * ``none``: u = 0 (pure diffusion; used by the closed-form checks).
    """
    x = grid(N)
    X = np.broadcast_to(x[None, :], (N, N))
    Y = np.broadcast_to(x[:, None], (N, N))
    if flow == "roberts":
        ux = np.cos(Y)
        uy = np.sin(X)
        uz = np.sin(Y) + np.cos(X)
    elif flow == "gp":
        A = GP_AMPLITUDE
        ux = A * np.cos(Y + math.sin(t))
        uy = A * np.sin(X + math.cos(t))
        uz = A * (np.cos(X + math.cos(t)) + np.sin(Y + math.sin(t)))
    elif flow == "none":
        z = np.zeros((N, N))
        ux, uy, uz = z, z, z
    else:
        raise ValueError(f"unknown flow {flow!r}")
    return np.array(ux), np.array(uy), np.array(uz)


def explicit_term(bh: np.ndarray, flow: str, kz: float, t: float) -> np.ndarray:
    """Dealiased explicit operator Nh(bh, t) = M * (i k x FFT(u x b)).

    Pseudo-spectral evaluation (Section 4): transform b to the grid, form the
    electromotive force E = u x b pointwise, transform back, take the
    spectral curl with k = (kx, ky, kz), and keep the 2/3 box M.
    """
    N = bh.shape[-1]
    b = to_physical(bh)
    ux, uy, uz = velocity(flow, N, t)
    Ex = uy * b[2] - uz * b[1]
    Ey = uz * b[0] - ux * b[2]
    Ez = ux * b[1] - uy * b[0]
    Eh = to_spectral(np.stack([Ex, Ey, Ez]))
    k = wavenumbers(N)
    kx = k[None, :]
    ky = k[:, None]
    Nx = 1j * (ky * Eh[2] - kz * Eh[1])
    Ny = 1j * (kz * Eh[0] - kx * Eh[2])
    Nz = 1j * (kx * Eh[1] - ky * Eh[0])
    return np.stack([Nx, Ny, Nz]) * box_mask(N)[None]


def divergence(bh: np.ndarray, kz: float) -> np.ndarray:
    """Spectral divergence i k . bh (paper's solenoidal constraint)."""
    N = bh.shape[-1]
    k = wavenumbers(N)
    return 1j * (k[None, :] * bh[0] + k[:, None] * bh[1] + kz * bh[2])
