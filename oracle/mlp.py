"""FP64 reference of the learned residual-kernel network -- TEST INFRASTRUCTURE ONLY.

Not part of the paper.  A multilayer perceptron predicts the residual-w Fourier kernel
c_hat of Sect. 3.1 (w-projection, Fig. 1) from per-row inputs, so that the build of G
can skip the exact kernel construction for rows where the network is accurate; the
exact construction stays the fallback and the judge.

Definitions mirrored here (the GPU path implements them on its own):
  * inputs (5 per row): x0 = w_proj (o L)^2 / 4, x1 = L / L_ref with L_ref = 4 degrees
    in radians (the field side of the widest training field), x2 = u-offset and x3 = v-offset of the
    row from its nearest grid cell (in cells, [-1/2, 1/2)), x4 = n_k / 15 with n_k the
    uncapped kernel side of the bandwidth rule.  L = nx cell is the field side (square
    fields only).  n_k is a function of (w_proj, L); it is given to the network so that
    it can follow the kernel's jumps where the sampled side changes.
  * outputs (451): the thresholded kernel centred in a 15 x 15 window, row-major over
    (s_v, s_u), each tap as (re, im); then one error output predicting log10 of the
    relative L2 error of the 450 kernel outputs.
  * network: 5 -> 256 -> 256 -> 256 -> 256 -> 451, exact GELU g(z) = z Phi(z) (Phi the
    standard normal CDF, via erf) after every hidden layer, linear output.  Flat
    parameter vector: for each layer, W [in x out] row-major, then b [out].
  * loss over a batch of B rows: L = (1/B) sum_b [ sum_{j<450} (p_bj - t_bj)^2
    + (e_b - log10(max(r_b, 1e-8)))^2 ], with r_b = ||p_b - t_b|| / max(||t_b||, 1e-30)
    held constant; the error output's gradient reaches its own weights only (the
    hidden layers learn from the kernel outputs alone).
  * Adam (Kingma & Ba 2015): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
    p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from .wkernel import nk_rule, threshold_shrink, wkernel_exact

NIN, HID, NLAYERS, SIDE = 5, 256, 4, 15
NOUT = 2 * SIDE * SIDE + 1
SIZES = [NIN] + [HID] * NLAYERS + [NOUT]
L_REF = math.radians(4.0)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def n_params(sizes=SIZES) -> int:
    return sum(a * b + b for a, b in zip(sizes[:-1], sizes[1:]))


def unpack(theta, sizes=SIZES):
    """Flat vector -> [(W, b)] views."""
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = theta[o:o + a * b].reshape(a, b)
        o += a * b
        bb = theta[o:o + b]
        o += b
        out.append((W, bb))
    return out


def init(seed: int, sizes=SIZES):
    """Uniform(-1/sqrt(in), 1/sqrt(in)) weights, zero biases (oracle's own draw)."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = 1.0 / math.sqrt(a)
        parts.append(rng.uniform(-lim, lim, a * b))
        parts.append(np.zeros(b))
    return np.concatenate(parts)


def forward(theta, X, sizes=SIZES):
    """Returns (outputs [B, nout], cache of pre-activations and activations)."""
    layers = unpack(np.asarray(theta, dtype=np.float64), sizes)
    H = np.asarray(X, dtype=np.float64)
    Hs, Zs = [H], []
    for i, (W, b) in enumerate(layers):
        Z = H @ W + b
        Zs.append(Z)
        H = gelu(Z) if i + 1 < len(layers) else Z
        Hs.append(H)
    return H, (Hs, Zs)


def error_target(P, T):
    """log10 of the relative L2 error of the kernel outputs (held constant)."""
    nk = P.shape[1] - 1
    num = np.sqrt(np.sum((P[:, :nk] - T) ** 2, axis=1))
    den = np.maximum(np.sqrt(np.sum(T ** 2, axis=1)), 1e-30)
    return np.log10(np.maximum(num / den, 1e-8))


def loss(theta, X, T, sizes=SIZES, etgt=None):
    """(kernel loss, error-head loss); etgt: fixed error targets (None: from theta)."""
    P, _ = forward(theta, X, sizes)
    nk = P.shape[1] - 1
    B = X.shape[0]
    if etgt is None:
        etgt = error_target(P, T)
    lk = float(np.sum((P[:, :nk] - T) ** 2) / B)
    le = float(np.sum((P[:, nk] - etgt) ** 2) / B)
    return lk, le


def loss_grad(theta, X, T, sizes=SIZES):
    """Loss terms and the flat gradient of their sum (error target held constant)."""
    P, (Hs, Zs) = forward(theta, X, sizes)
    layers = unpack(np.asarray(theta, dtype=np.float64), sizes)
    nk = P.shape[1] - 1
    B = X.shape[0]
    et = error_target(P, T)
    dP = np.zeros_like(P)
    dP[:, :nk] = 2.0 * (P[:, :nk] - T) / B
    dP[:, nk] = 2.0 * (P[:, nk] - et) / B
    lk = float(np.sum((P[:, :nk] - T) ** 2) / B)
    le = float(np.sum((P[:, nk] - et) ** 2) / B)
    grads = [None] * len(layers)
    dZ = dP
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        gW = Hs[i].T @ dZ
        gb = dZ.sum(axis=0)
        grads[i] = (gW, gb)
        if i == 0:
            break
        if i == len(layers) - 1:
            dH = dZ[:, :nk] @ W[:, :nk].T      # no gradient from the error output below
        else:
            dH = dZ @ W.T
        dZ = dH * gelu_grad(Zs[i - 1])
    flat = np.concatenate([np.concatenate([g.ravel(), bb]) for g, bb in grads])
    return lk, le, flat


def adam(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def features(wproj, L, fu, fv, o: int = 2, alpha: float = 2.0):
    """Network inputs [n, 5] and the uncapped kernel sides n_k (square field of side L)."""
    wproj = np.asarray(wproj, dtype=np.float64)
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), wproj.shape)
    nk = np.array([int(nk_rule(np.array([w]), l, l, o, alpha, None)[0])
                   for w, l in zip(wproj.ravel(), L.ravel())], dtype=np.int64)
    x = np.stack([wproj * (o * L) ** 2 / 4.0, L / L_REF, np.asarray(fu, dtype=np.float64),
                  np.asarray(fv, dtype=np.float64), nk / 15.0], axis=1)
    return x, nk


def kernel_target(wproj: float, L: float, o: int = 2, alpha: float = 2.0,
                  eps: float = 1e-6):
    """Thresholded exact kernel centred in the 15 x 15 window as 450 reals (re, im
    interleaved, row-major over (s_v, s_u)), or None when its side exceeds 15."""
    nk = int(nk_rule(np.array([wproj]), L, L, o, alpha, None)[0])
    if nk > SIDE:
        return None
    c = wkernel_exact(np.array([wproj]), nk, L, L, o)[0]
    k2, _ = threshold_shrink(c, eps)
    n2 = k2.shape[0]
    win = np.zeros((SIDE, SIDE), dtype=np.complex128)
    a = (SIDE - n2) // 2
    win[a:a + n2, a:a + n2] = k2
    out = np.empty(2 * SIDE * SIDE)
    out[0::2] = win.real.ravel()
    out[1::2] = win.imag.ravel()
    return out
