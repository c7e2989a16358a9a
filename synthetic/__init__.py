"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws and shapes inputs.  It holds none of the induction
equation's arithmetic (no transforms, flows, time stepping or Parareal); the
oracle under ``oracle/`` and the HIP library both receive its arrays as plain
inputs.

Initial field (stands in for the paper's random initial perturbation,
Section 4): for each of the three components and every Fourier mode with
kx^2 + ky^2 <= kmax^2, the real and imaginary parts are independent normal
deviates times ``amp``; every other mode is zero.  The field is then made
solenoidal for the 2.5D wavevector k = (kx, ky, kz):
b <- b - k (k . b) / |k|^2 (no complex conjugate; |k| = 0 is left alone).

Array layout: complex128 ``[3][N][N]`` of spectral coefficients with the ky
index on the middle axis and kx fastest; index m stands for wavenumber m when
m < N/2 and m - N otherwise.  The physical field is b(x, y) =
sum_k b_k exp(i (kx x + ky y)).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["mode_numbers", "initial_field", "initial_fields", "gp_instance_params"]


def mode_numbers(N: int) -> np.ndarray:
    """Signed wavenumber of each FFT index: m for m < N/2, m - N otherwise."""
    m = np.arange(N)
    return np.where(m < N // 2, m, m - N).astype(np.float64)


def initial_field(N: int, kz: float, seed: int, amp: float = 1e-3,
                  kmax: float = 4.0) -> np.ndarray:
    """One seeded solenoidal initial field, complex128 ``[3][N][N]``."""
    if N < 16 or (N & (N - 1)):
        raise ValueError("N must be a power of two >= 16")
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((3, N, N, 2))
    k = mode_numbers(N)
    kx = k[None, :]
    ky = k[:, None]
    keep = (kx * kx + ky * ky) <= kmax * kmax
    b = (z[..., 0] + 1j * z[..., 1]) * amp * keep[None]
    kk = kx * kx + ky * ky + kz * kz
    kdotb = kx * b[0] + ky * b[1] + kz * b[2]
    with np.errstate(invalid="ignore", divide="ignore"):
        f = np.where(kk > 0, kdotb / np.where(kk > 0, kk, 1.0), 0.0)
    b = np.stack([b[0] - kx * f, b[1] - ky * f, b[2] - kz * f])
    return np.ascontiguousarray(b.astype(np.complex128))


def initial_fields(N: int, kz: float, seeds, amp: float = 1e-3,
                   kmax: float = 4.0) -> np.ndarray:
    """A batch ``[B][3][N][N]`` of seeded fields, one per seed."""
    return np.stack([initial_field(N, kz, s, amp, kmax) for s in seeds])


def gp_instance_params(n_instances: int, seed: int,
                       rm_range=(10.0, 1000.0), kz_range=(0.2, 1.2)):
    """Seeded (Rm, kz) pairs for a batch of independent Galloway-Proctor
    problems: Rm log-uniform and kz uniform over the given ranges."""
    rng = np.random.default_rng(seed)
    lo, hi = math.log(rm_range[0]), math.log(rm_range[1])
    rm = np.exp(rng.uniform(lo, hi, n_instances))
    kz = rng.uniform(kz_range[0], kz_range[1], n_instances)
    return rm, kz
