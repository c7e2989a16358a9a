"""Independent reference computations used to pin the oracle.

Nothing here calls the oracle's transforms or operators: each routine is a
different route to the same mathematics (brute-force sums, the flows' own
Fourier coefficients, the paper's advective component equations, closed
forms of the discrete recurrences, a general-purpose ODE integrator).
"""
from __future__ import annotations

import cmath
import math

import numpy as np


def signed(N):
    return np.array([m if m < N // 2 else m - N for m in range(N)], float)


def brute_synthesis(bh):
    """b(x_j, y_i) = sum_k bh e^{i(kx x_j + ky y_i)} by an O(N^4) double sum."""
    N = bh.shape[-1]
    k = signed(N)
    x = 2 * np.pi * np.arange(N) / N
    out = np.zeros(bh.shape, complex)
    for iy in range(N):
        for ix in range(N):
            ph = np.exp(1j * (k[None, :] * x[ix] + k[:, None] * x[iy]))
            out[..., iy, ix] = np.sum(bh * ph, axis=(-2, -1))
    return out


def brute_analysis(f):
    """Coefficients bh[k] = N^-2 sum_x f(x) e^{-i k.x} by an O(N^4) sum."""
    N = f.shape[-1]
    k = signed(N)
    x = 2 * np.pi * np.arange(N) / N
    out = np.zeros(f.shape, complex)
    for my in range(N):
        for mx in range(N):
            ph = np.exp(-1j * (k[mx] * x[None, :] + k[my] * x[:, None]))
            out[..., my, mx] = np.sum(f * ph, axis=(-2, -1)) / (N * N)
    return out


def flow_modes(flow, t):
    """Fourier coefficients of the flow: {(ky, kx): (ux, uy, uz)}.

    Roberts u = (cos y, sin x, sin y + cos x); Galloway-Proctor (relabelled)
    u = A (cos(y + s), sin(x + c), cos(x + c) + sin(y + s)), s = sin t,
    c = cos t, A = sqrt(3/2).  cos(q + p) = (e^{i(q+p)} + e^{-i(q+p)})/2,
    sin(q + p) = (e^{i(q+p)} - e^{-i(q+p)})/(2i).
    """
    if flow == "roberts":
        A, s, c = 1.0, 0.0, 0.0
    elif flow == "gp":
        A, s, c = math.sqrt(1.5), math.sin(t), math.cos(t)
    else:
        return {}
    ey, ey_ = cmath.exp(1j * s), cmath.exp(-1j * s)
    ex, ex_ = cmath.exp(1j * c), cmath.exp(-1j * c)
    m = {}
    # modes in y: ux = A cos(y+s), uz += A sin(y+s)
    m[(1, 0)] = (A * ey / 2, 0.0, A * ey / 2j)
    m[(-1, 0)] = (A * ey_ / 2, 0.0, -A * ey_ / 2j)
    # modes in x: uy = A sin(x+c), uz += A cos(x+c)
    m[(0, 1)] = (0.0, A * ex / 2j, A * ex / 2)
    m[(0, -1)] = (0.0, -A * ex_ / 2j, A * ex_ / 2)
    return m


def direct_explicit(bh, flow, kz, t):
    """Dealiased curl(u x b) by direct convolution in spectral space.

    E_k = sum_q u_q x b_{k-q} over the flow's four Fourier modes q, then
    i k x E kept on the 2/3 box.  No transform is used.  A shift by q is a
    circular roll of the index arrays: b is zero outside the box and
    K + 1 < N/2, so no retained coefficient wraps around.
    """
    N = bh.shape[-1]
    K = (N - 1) // 3
    k = signed(N)
    KX, KY = k[None, :], k[:, None]
    mask = (np.abs(KX) <= K) & (np.abs(KY) <= K)
    b = bh * mask
    E = np.zeros(bh.shape, complex)
    for (qy, qx), u in flow_modes(flow, t).items():
        s = np.roll(b, shift=(qy, qx), axis=(-2, -1))   # s_k = b_{k-q}
        E[0] += u[1] * s[2] - u[2] * s[1]
        E[1] += u[2] * s[0] - u[0] * s[2]
        E[2] += u[0] * s[1] - u[1] * s[0]
    out = np.stack([1j * (KY * E[2] - kz * E[1]),
                    1j * (kz * E[0] - KX * E[2]),
                    1j * (KX * E[1] - KY * E[0])])
    return out * mask


def _grid_deriv(bh, axis_k):
    return np.fft.ifft2(1j * axis_k * bh, axes=(-2, -1)) * bh.shape[-1] ** 2


def advective_roberts(bh, kz):
    """Paper Section 2.1, equations for b_x and b_y (without diffusion),
    evaluated on the grid and returned as masked coefficients [2][N][N]."""
    N = bh.shape[-1]
    k = signed(N)
    KX, KY = k[None, :], k[:, None]
    x = 2 * np.pi * np.arange(N) / N
    X, Y = x[None, :], x[:, None]
    b = np.fft.ifft2(bh, axes=(-2, -1)) * N * N
    dxbx, dybx = _grid_deriv(bh[0], KX), _grid_deriv(bh[0], KY)
    dxby, dyby = _grid_deriv(bh[1], KX), _grid_deriv(bh[1], KY)
    w = np.sin(Y) + np.cos(X)
    rx = -b[1] * np.sin(Y) - np.cos(Y) * dxbx - np.sin(X) * dybx - w * 1j * kz * b[0]
    ry = b[0] * np.cos(X) - np.cos(Y) * dxby - np.sin(X) * dyby - w * 1j * kz * b[1]
    K = (N - 1) // 3
    mask = (np.abs(KX) <= K) & (np.abs(KY) <= K)
    return np.stack([np.fft.fft2(rx), np.fft.fft2(ry)]) / (N * N) * mask


def advective_gp(bh, kz, t):
    """Paper Section 2.2, equations gp-dynamo_y / gp-dynamo_z relabelled
    from the paper's (y, z, x) to (x, y, z): with u = (ux, uy, uz),
      d_t b_x = b_y d_y ux - uz i kz b_x - ux d_x b_x - uy d_y b_x
      d_t b_y = b_x d_x uy - uz i kz b_y - ux d_x b_y - uy d_y b_y
    (the paper's first equation carries k_z^2 in its diffusion where k_x^2
    is meant; diffusion is not part of this check)."""
    N = bh.shape[-1]
    k = signed(N)
    KX, KY = k[None, :], k[:, None]
    x = 2 * np.pi * np.arange(N) / N
    X, Y = x[None, :], x[:, None]
    A, s, c = math.sqrt(1.5), math.sin(t), math.cos(t)
    ux = A * np.cos(Y + s)
    uy = A * np.sin(X + c)
    uz = A * (np.cos(X + c) + np.sin(Y + s))
    dy_ux = -A * np.sin(Y + s)
    dx_uy = A * np.cos(X + c)
    b = np.fft.ifft2(bh, axes=(-2, -1)) * N * N
    dxbx, dybx = _grid_deriv(bh[0], KX), _grid_deriv(bh[0], KY)
    dxby, dyby = _grid_deriv(bh[1], KX), _grid_deriv(bh[1], KY)
    rx = b[1] * dy_ux - uz * 1j * kz * b[0] - ux * dxbx - uy * dybx
    ry = b[0] * dx_uy - uz * 1j * kz * b[1] - ux * dxby - uy * dyby
    K = (N - 1) // 3
    mask = (np.abs(KX) <= K) & (np.abs(KY) <= K)
    return np.stack([np.fft.fft2(rx), np.fft.fft2(ry)]) / (N * N) * mask


def sbdf_diffusion_factor(a, n):
    """Amplification of one mode after n steps of SBDF1-started SBDF2 for
    db/dt = -lam b with a = dt*lam, from the closed form of the recurrence
    (3/2 + a) r^2 - 2 r + 1/2 = 0: b_j = c1 r1^j + c2 r2^j, b_0 = 1,
    b_1 = 1/(1 + a)."""
    a = np.asarray(a, dtype=complex)
    disc = np.sqrt(1.0 - 2.0 * a + 0j)
    r1 = (2.0 + disc) / (3.0 + 2.0 * a)
    r2 = (2.0 - disc) / (3.0 + 2.0 * a)
    b1 = 1.0 / (1.0 + a)
    c2 = (b1 - r1) / (r2 - r1)
    c1 = 1.0 - c2
    if n == 0:
        return np.ones_like(a)
    return c1 * r1 ** n + c2 * r2 ** n


def scalar_parareal(phiF, phiG, n, k):
    """Closed form of linear scalar Parareal:
    U^k_n / U_0 = sum_{j<=k} C(n, j) (phiF - phiG)^j phiG^(n-j)."""
    d = phiF - phiG
    out = np.zeros(np.shape(phiF), complex)
    for j in range(0, min(k, n) + 1):
        out = out + math.comb(n, j) * d ** j * phiG ** (n - j)
    return out
