"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws and shapes inputs.  It holds none of the induction
equation's arithmetic (no transforms, flows, time stepping or Parareal); the
oracle under ``oracle/`` and the HIP library both receive its arrays as plain
inputs.

Initial field (stands in for the paper's random initial perturbation,
Section 4): for each of the three components and every Fourier mode inside
the 2/3 box with kx^2 + ky^2 <= kmax^2, the real and imaginary parts are a
pair of independent normal deviates times ``amp``; every other mode is zero.
The field is then made solenoidal for the 2.5D wavevector k = (kx, ky, kz):
b <- b - k (k . b) / |k|^2 (no complex conjugate; |k| = 0 is left alone).

The deviates come from a counter-based generator written from its published
definitions, so that the C library (``pd_seed_initial``) reproduces the field
bit for bit: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC 2011) keyed by the 64-bit seed, counter
(kx mod 2^32, ky mod 2^32, component, 0); its four 32-bit words make two
53-bit uniforms u1 = (j1 + 1) 2^-53 in (0, 1] and u2 = j2 2^-53 in [0, 1),
j = (w_a >> 5) 2^26 + (w_b >> 6); the Box-Muller transform (Box & Muller,
1958) turns them into re = r cos(2 pi u2), im = r sin(2 pi u2) with
r = sqrt(-2 ln u1).  The logarithm, sine and cosine are the C library's
(Python's ``math`` module), evaluated one value at a time; every other
operation is a single IEEE double operation in a fixed order.

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


PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57   # round multipliers
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85   # Weyl key increments
MASK32 = 0xFFFFFFFF
TWO_PI = 6.283185307179586                      # the double nearest 2 pi


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on arrays of counters.

    ctr: four uint64 arrays holding 32-bit words; key: two 32-bit ints.
    Each round maps (c0, c1, c2, c3) to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2),
    hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key is bumped by the Weyl
    increments before every round after the first."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & np.uint64(MASK32) for c in ctr)
    k0, k1 = int(key[0]) & MASK32, int(key[1]) & MASK32
    m0, m1, m32 = np.uint64(PHILOX_M0), np.uint64(PHILOX_M1), np.uint64(MASK32)
    for r in range(10):
        if r:
            k0, k1 = (k0 + PHILOX_W0) & MASK32, (k1 + PHILOX_W1) & MASK32
        p0, p1 = c0 * m0, c2 * m1          # exact: 32 x 32 -> 64 bits
        c0, c1, c2, c3 = ((p1 >> np.uint64(32)) ^ c1 ^ np.uint64(k0), p1 & m32,
                          (p0 >> np.uint64(32)) ^ c3 ^ np.uint64(k1), p0 & m32)
    return c0, c1, c2, c3


def normal_pairs(seed: int, kx, ky, comp):
    """Two independent N(0, 1) deviates per (kx, ky, component) entry."""
    kx = np.asarray(kx, dtype=np.int64)
    ky = np.asarray(ky, dtype=np.int64)
    comp = np.asarray(comp, dtype=np.int64)
    w = philox4x32_10((kx & MASK32, ky & MASK32, comp, np.zeros_like(kx)),
                      (seed & MASK32, (seed >> 32) & MASK32))
    s5, s6 = np.uint64(5), np.uint64(6)
    j1 = (w[0] >> s5) * np.uint64(1 << 26) + (w[1] >> s6)
    j2 = (w[2] >> s5) * np.uint64(1 << 26) + (w[3] >> s6)
    u1 = (j1 + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = j2.astype(np.float64) * 2.0 ** -53
    r = np.sqrt(np.array([-2.0 * math.log(u) for u in u1.ravel()]).reshape(u1.shape))
    th = TWO_PI * u2
    re = r * np.array([math.cos(a) for a in th.ravel()]).reshape(th.shape)
    im = r * np.array([math.sin(a) for a in th.ravel()]).reshape(th.shape)
    return re, im


def initial_field(N: int, kz: float, seed: int, amp: float = 1e-3,
                  kmax: float = 4.0) -> np.ndarray:
    """One seeded solenoidal initial field, complex128 ``[3][N][N]``."""
    if N < 16 or (N & (N - 1)):
        raise ValueError("N must be a power of two >= 16")
    if seed < 0 or seed >= 1 << 64:
        raise ValueError("seed must fit 64 unsigned bits")
    K = (N - 1) // 3
    k = mode_numbers(N)
    KX, KY = np.meshgrid(k, k)                     # [ky index][kx index]
    keep = (np.abs(KX) <= K) & (np.abs(KY) <= K) & (KX * KX + KY * KY <= kmax * kmax)
    iy, ix = np.nonzero(keep)
    kx, ky = k[ix], k[iy]
    re = np.zeros((3, iy.size))
    im = np.zeros((3, iy.size))
    for c in range(3):
        re[c], im[c] = normal_pairs(seed, kx.astype(np.int64), ky.astype(np.int64),
                                    np.full(iy.size, c))
    re, im = re * amp, im * amp
    # solenoidal projection, real and imaginary parts separately
    kzf = float(kz)
    k2 = kx * kx + ky * ky + kzf * kzf
    pos = k2 > 0
    d = np.where(pos, k2, 1.0)
    sr = np.where(pos, (kx * re[0] + ky * re[1] + kzf * re[2]) / d, 0.0)
    si = np.where(pos, (kx * im[0] + ky * im[1] + kzf * im[2]) / d, 0.0)
    kv = (kx, ky, np.full_like(kx, kzf))
    b = np.zeros((3, N, N), dtype=np.complex128)
    for c in range(3):
        b[c, iy, ix] = (re[c] - kv[c] * sr) + 1j * (im[c] - kv[c] * si)
    return b


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
