"""FP64 reference of the learned coarse-propagator correction (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The paper's coarse propagators are time steppers (Section 3.2); the build adds
a learned correction on top of the plain coarse step: for a slice starting at
time t and an input field D (a Parareal difference U^k_n - U^{k-1}_n, or any
field), with g = G(D) the plain coarse result on the fine 2/3 box,

    G_learned(D) = g + |D| * c,   c = Net(D/|D|, g/|D|; t)      (G(0) = 0)

Net is linear in its inputs (no activation), acting on the fine box of
Mf x Mf modes with C real channels per mode:

    h0[m]   = x[m] W_in                       x[m]: 12 reals (re/im of D, g)
    y_l[m]  = sum_s h_l[m + s] W_{l,s}(t)     s in {0, +kx, -kx, +ky, -ky}
    W_{l,s}(t) = V_{l,0,s} + cos t V_{l,1,s} + sin t V_{l,2,s}
    h_{l+1} = h_l + gamma_l * y_l             (per-mode, per-channel gains)
    c[m]    = h_L[m] W_out                    6 reals = 3 complex

with h = 0 outside the box.  Loss over a batch:
    L = sum_b |c_b - r_b|^2 / sum_b |r_b|^2,  r_b = (F(D_b) - g_b) / |D_b|.

Array conventions: fields [B][3][Mf][Mf] complex (compact box, row ky, column
kx), activations [B][Mf*Mf][C], modes m = (ky + K) * Mf + (kx + K).
Pinned by central finite differences in ``tests/test_oracle_network.py``.
"""
from __future__ import annotations

import numpy as np

SHIFTS = ((0, 0), (0, 1), (0, -1), (1, 0), (-1, 0))   # (dky, dkx)


def init_params(Mf: int, C: int = 32, L: int = 4, seed: int = 0) -> dict:
    rng = np.random.default_rng(seed)
    return {
        "W_in": rng.standard_normal((12, C)) / np.sqrt(12.0),
        "V": rng.standard_normal((L, 3, 5, C, C)) * (0.3 / np.sqrt(5 * C)),
        "gamma": np.ones((L, Mf * Mf, C)),
        "W_out": rng.standard_normal((C, 6)) * (1e-3 / np.sqrt(C)),
    }


def features(D: np.ndarray, g: np.ndarray):
    """x [B][Mf*Mf][12] and the norms |D_b| (inputs scaled by 1/|D|)."""
    B = D.shape[0]
    nrm = np.sqrt(np.sum(np.abs(D.reshape(B, -1)) ** 2, axis=1))
    scale = np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1.0), 0.0)
    parts = []
    for arr in (D, g):
        a = arr * scale[:, None, None, None]
        for c in range(3):
            parts.append(a[:, c].real.reshape(B, -1))
            parts.append(a[:, c].imag.reshape(B, -1))
    return np.stack(parts, axis=-1), nrm


def shift_rows(h: np.ndarray, Mf: int, dky: int, dkx: int) -> np.ndarray:
    """out[m] = h[m + s] with zero outside the box; h: [B][Mf*Mf][C]."""
    B, _, C = h.shape
    g = h.reshape(B, Mf, Mf, C)
    out = np.zeros_like(g)
    ys = slice(max(0, -dky), Mf - max(0, dky))
    xs = slice(max(0, -dkx), Mf - max(0, dkx))
    ysrc = slice(max(0, dky), Mf - max(0, -dky))
    xsrc = slice(max(0, dkx), Mf - max(0, -dkx))
    out[:, ys, xs] = g[:, ysrc, xsrc]
    return out.reshape(B, Mf * Mf, C)


def layer_weights(V_l: np.ndarray, t: np.ndarray) -> np.ndarray:
    """W_{l,s}(t) for every sample: [B][5][C][C]."""
    phi = np.stack([np.ones_like(t), np.cos(t), np.sin(t)], axis=1)   # [B][3]
    return np.einsum("bj,jsio->bsio", phi, V_l)


def bf16(a: np.ndarray) -> np.ndarray:
    """The value the matrix-core kernels use for an FP32 operand in BF16
    mode: the number rounded to FP32, then to the nearest BF16 (8 significant
    bits, ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(a):
    return a


def forward(params: dict, x: np.ndarray, t: np.ndarray, Mf: int, rnd=None):
    """c [B][Mf*Mf][6] and the cache for backward.  rnd (default: none) is
    applied to both operands of every channel-mixing product, to evaluate the
    network with the operands the BF16 kernels use (``bf16``)."""
    q = rnd if rnd is not None else _ident
    h = x @ params["W_in"]
    cache = {"x": x, "t": t, "hs": [h], "ys": []}
    L = params["V"].shape[0]
    for l in range(L):
        W = q(layer_weights(params["V"][l], t))
        y = np.zeros_like(h)
        for s, (dy, dx) in enumerate(SHIFTS):
            y += np.einsum("bmi,bio->bmo", q(shift_rows(h, Mf, dy, dx)), W[:, s])
        cache["ys"].append(y)
        h = h + params["gamma"][l][None] * y
        cache["hs"].append(h)
    return h @ params["W_out"], cache


def loss_and_grad(params: dict, x, t, r, Mf: int, w=None, rnd=None):
    """Loss sum w_m |c - r|^2 / sum w_m |r|^2 (per-mode weights w, [Q]; None:
    all 1) and its gradients with respect to every parameter (manual
    backward).  rnd as in ``forward``, applied also to the operands of the
    backward channel-mixing products."""
    q = rnd if rnd is not None else _ident
    c, cache = forward(params, x, t, Mf, rnd)
    wm = np.ones(c.shape[1]) if w is None else np.asarray(w, dtype=np.float64)
    diff = c - r
    den = float(np.sum(wm[None, :, None] * r * r))
    loss = float(np.sum(wm[None, :, None] * diff * diff)) / den
    dc = 2.0 * wm[None, :, None] * diff / den
    L = params["V"].shape[0]
    grads = {}
    hL = cache["hs"][-1]
    grads["W_out"] = np.einsum("bmi,bmo->io", hL, dc)
    dh = dc @ params["W_out"].T
    grads["V"] = np.zeros_like(params["V"])
    grads["gamma"] = np.zeros_like(params["gamma"])
    phi = np.stack([np.ones_like(t), np.cos(t), np.sin(t)], axis=1)
    for l in reversed(range(L)):
        h, y = cache["hs"][l], cache["ys"][l]
        grads["gamma"][l] = np.sum(dh * y, axis=0)
        dy = dh * params["gamma"][l][None]
        W = q(layer_weights(params["V"][l], t))
        dh_prev = dh.copy()
        for s, (sy, sx) in enumerate(SHIFTS):
            hs = q(shift_rows(h, Mf, sy, sx))
            dWs = np.einsum("bmi,bmo->bio", hs, q(dy))              # per sample
            grads["V"][l, :, s] = np.einsum("bj,bio->jio", phi, dWs)
            # adjoint of the shift: contribution to h at m + s from y at m
            dh_prev += shift_rows(np.einsum("bmo,bio->bmi", q(dy), W[:, s]), Mf, -sy, -sx)
        dh = dh_prev
    grads["W_in"] = np.einsum("bmi,bmo->io", cache["x"], dh)
    return loss, grads


def apply(params: dict, D: np.ndarray, g: np.ndarray, t: np.ndarray) -> np.ndarray:
    """G_learned(D) = g + |D| c on the fine box, [B][3][Mf][Mf] complex."""
    B, _, Mf, _ = D.shape
    x, nrm = features(D, g)
    c, _ = forward(params, x, t, Mf)
    c = c.reshape(B, Mf, Mf, 6)
    corr = np.stack([c[..., 2 * k] + 1j * c[..., 2 * k + 1] for k in range(3)], axis=1)
    return g + nrm[:, None, None, None] * corr
