"""Residual-w Fourier kernels (w-projection part), FP64 (oracle; test infrastructure only).

Sect. 3.1 (w-projection) and Fig. 1: the residual modulation C(.; w_proj) is sampled
at an adaptive resolution set by its spatial Fourier bandwidth, over o = 2 times the
field, with a Hamming taper outside the field of interest; a small FFT gives the
Fourier kernel, which is then compressed by an l2-energy hard threshold.
Readings (the paper's bandwidth formula is dimensionally incomplete and the taper,
sampling and threshold constants are unstated):
  * the kernel carries only the phase exp(-2i pi w (n-1)); the 1/n of eq. 2 is applied
    once, in the w-layer of Z_p;
  * bandwidth: the chirp's largest local frequency over the padded field is
    f = |w| l_p / n(l_p, m_p) with l_p = o Lx / 2, m_p = o Ly / 2 (Lx = nx cell); in
    grid cells its two-sided band is B = max(2 f_x o Lx, 2 f_y o Ly); the kernel side
    is n_k = 2 ceil(alpha B / 2) + 1 with alpha = 2, n_k = 1 iff w = 0, capped at S_max;
  * samples at l'_a = a o Lx / n_k, m'_b = b o Ly / n_k, a, b = -h..h (h = (n_k-1)/2);
  * taper T(l') = 1 for |l'| <= L/2, 0.54 + 0.46 cos(pi (|l'| - L/2) / (L/2)) beyond,
    applied to the chirp's phase: c = exp(-2i pi w (n-1) T(l') T(m')).  Inside the field
    this is the exact residual w-term; outside it the phase relaxes smoothly, so the
    periodic extension over the padded field has no kink and, as w -> 0, the kernel
    tends to a unit delta (G tends to the plain interpolation matrix, Sect. 3.4);
  * c_hat[s_v, s_u] = n_k^-2 sum_{b,a} c[b,a] exp(-2i pi (s_u a + s_v b) / n_k), so that
    c(l', m') ~ sum_s c_hat[s] exp(+2i pi (s_u l'/(o Lx) + s_v m'/(o Ly))) and w = 0 gives
    a unit delta;
  * threshold: drop the largest set of smallest-energy entries whose energy sum is at
    most eps * total (eps = 1e-6), i.e. keep the shortest descending-energy prefix
    holding at least (1 - eps) of the energy; entries within a relative 1e-9 of the
    smallest kept energy are kept too, so that mirror-symmetric entries (equal energy
    in exact arithmetic) are kept or dropped together; no renormalisation;
  * compression: the kernel is cut to the smallest centred odd square holding every
    kept entry.
"""
from __future__ import annotations

import math

import numpy as np

TIE_REL = 1e-9


def nk_rule(wproj, Lx: float, Ly: float, o: int = 2, alpha: float = 2.0,
            smax: int | None = 15):
    """Kernel side n_k for residual offsets wproj (array).  smax=None: uncapped."""
    wproj = np.asarray(wproj, dtype=np.float64)
    lp = (o * Lx) / 2.0
    mp = (o * Ly) / 2.0
    nn = math.sqrt(1.0 - lp * lp - mp * mp)
    aw = np.abs(wproj)
    bx = 2.0 * ((aw * lp) / nn) * (o * Lx)
    by = 2.0 * ((aw * mp) / nn) * (o * Ly)
    B = np.maximum(bx, by)
    nk = 2 * np.ceil((alpha * B) / 2.0).astype(np.int64) + 1
    nk = np.where(wproj == 0.0, 1, nk)
    if smax is not None:
        nk = np.minimum(nk, smax)
    return nk


def taper(lp, L: float):
    """Half-Hamming taper: 1 inside the field (|l| <= L/2), Hamming roll-off to |l| = L."""
    a = np.abs(lp)
    half = L / 2.0
    return np.where(a <= half, 1.0, 0.54 + 0.46 * np.cos(math.pi * (a - half) / half))


def wkernel_exact(wproj, nk: int, Lx: float, Ly: float, o: int = 2):
    """Untruncated kernels c_hat for a batch of offsets sharing one side nk.
    Returns [B, nk, nk] complex128 indexed [s_v + h, s_u + h]."""
    wproj = np.atleast_1d(np.asarray(wproj, dtype=np.float64))
    if nk == 1:
        return np.ones((wproj.size, 1, 1), dtype=np.complex128)
    h = (nk - 1) // 2
    a = np.arange(-h, h + 1, dtype=np.float64)
    lpa = (a * (o * Lx)) / nk
    mpb = (a * (o * Ly)) / nk
    L2 = lpa[None, :] ** 2 + mpb[:, None] ** 2
    nn = np.sqrt(1.0 - L2)
    d = -L2 / (1.0 + nn)                                   # n - 1, [b, a]
    tap = taper(mpb, Ly)[:, None] * taper(lpa, Lx)[None, :]
    c = np.exp(-2j * np.pi * wproj[:, None, None] * (d * tap)[None])
    s = np.arange(-h, h + 1, dtype=np.float64)
    D = np.exp(-2j * np.pi * np.outer(s, a) / nk)          # [s, a]
    # c_hat[s_v, s_u] = sum_{b,a} D[s_v,b] c[b,a] D[s_u,a] / nk^2
    return np.einsum("vb,kba,ua->kvu", D, c, D) / (nk * nk)


def threshold_shrink(chat, eps: float = 1e-6):
    """Hard threshold on l2 energy and compression to the smallest centred square.
    chat: [nk, nk].  Returns (kernel [n', n'], dropped_energy_fraction)."""
    nk = chat.shape[0]
    if nk == 1:
        return chat.copy(), 0.0
    E = (chat.real ** 2 + chat.imag ** 2).ravel()
    tot = E.sum()
    if tot == 0.0:
        return np.zeros((1, 1), dtype=chat.dtype), 0.0
    Es = np.sort(E)
    A = np.cumsum(Es)
    jdrop = int(np.searchsorted(A, eps * tot, side="right"))
    tau = Es[jdrop]
    keep = (E >= tau * (1.0 - TIE_REL)).reshape(nk, nk)
    h = (nk - 1) // 2
    sv, su = np.nonzero(keep)
    hp = int(max(np.abs(sv - h).max(), np.abs(su - h).max()))
    k2 = np.where(keep, chat, 0.0)[h - hp:h + hp + 1, h - hp:h + hp + 1]
    dropped = float(E[~keep.ravel()].sum() / tot)
    return k2, dropped
