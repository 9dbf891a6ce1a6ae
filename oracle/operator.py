"""Phi, Phi^dag, Phi^dag Phi and H_p in FP64, matrix-free (oracle; test infrastructure only).

Sect. 3.2, eq. 6: Phi = [Phi_1 .. Phi_P]^T with Phi_p = G_p F Z_p.
  * Z_p  = diag(s (x) C(.; w_p)): grid correction times the w-layer (eq. 2 with its 1/n);
  * F    = unnormalised forward 2-D DFT of the image zero-padded to (o ny) x (o nx),
           pixel (i, j) placed at ((i - nx/2) mod Kx, (j - ny/2) mod Ky);
  * G_p  = rows g_k[q] = sum_s c_hat_k[s] phi(u_k - s_u - q_u) phi(v_k - s_v - q_v): the
           Kaiser-Bessel taps at the row's fractional grid position convolved with its
           residual-w kernel (Sect. 3.1-3.2); a dense T x T patch, T = n' + J - 1, with
           grid indices taken modulo K (periodic grid).
Sect. 3.3, eq. 7-8: Phi^dag Phi = sum_p Z_p^dag F^dag G_p^dag G_p F Z_p, F^dag being the
unnormalised inverse DFT followed by the crop back to the image positions;
H_p = G_p^dag G_p.
Sect. 2, eq. 3: (u, v, w) are baseline components in wavelengths, u = u_m f / c.
Sect. 2 (data weighting, flags): a per-measurement weight omega_k scales row k of the
operator, Phi_W = diag(omega) Phi, so Phi_W^dag Phi_W = Phi^dag diag(omega^2) Phi; a
flagged measurement is discarded before anything else (planning included) and its
forward value is zero.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import os

import numpy as np
import scipy.fft
import scipy.sparse as sp

from . import wbins
from .kernels import pixel_lm, nm1, grid_correction, kb_taps
from .wkernel import nk_rule, wkernel_exact, TIE_REL

C_LIGHT = 299_792_458.0


@dataclass
class OperatorParams:
    nx: int
    ny: int
    cell: float
    J: int = 7
    beta: float = 2.34 * 7
    o: int = 2
    alpha: float = 2.0
    smax: int = 31
    eps: float = 1e-6


def threshold_shrink_batch(chat, eps):
    """Vectorised form of wkernel.threshold_shrink over a batch [B, nk, nk].
    Returns (list of (rows, kernels [b, n', n'])) grouped by n', and dropped energy."""
    B, nk, _ = chat.shape
    if nk == 1:
        return [(np.arange(B), chat.copy())], np.zeros(B)
    E = (chat.real ** 2 + chat.imag ** 2).reshape(B, -1)
    tot = E.sum(1)
    Es = np.sort(E, axis=1)
    A = np.cumsum(Es, axis=1)
    jdrop = (A <= (eps * tot)[:, None]).sum(1)
    jdrop = np.minimum(jdrop, nk * nk - 1)
    tau = Es[np.arange(B), jdrop]
    keep = E >= (tau * (1.0 - TIE_REL))[:, None]
    h = (nk - 1) // 2
    ii = np.arange(nk * nk)
    rad = np.maximum(np.abs(ii // nk - h), np.abs(ii % nk - h))
    hp = np.where(keep, rad[None, :], 0).max(1)
    dropped = np.where(keep, 0.0, E).sum(1) / np.where(tot > 0, tot, 1.0)
    kept = np.where(keep.reshape(B, nk, nk), chat, 0.0)
    groups = []
    for v in np.unique(hp):
        sel = np.nonzero(hp == v)[0]
        groups.append((sel, kept[sel, h - v:h + v + 1, h - v:h + v + 1]))
    return groups, dropped


class OracleOperator:
    """FP64 widefield operator for one channel.

    uvw_m: [M, 3] metres; freq_hz: scalar.  Bins: either `centroids` (ascending) or
    `nbins` (k-means on the planning subset drawn with `seed`, `plan_fraction`).
    weights: [M] real or None (all ones), scaling the rows of G; flags: [M] bool or None,
    True = discarded.  forward() returns all M values (zero where flagged) and adjoint()
    takes all M (flagged entries ignored); internally only the kept rows exist."""

    def __init__(self, uvw_m, freq_hz, prm: OperatorParams, nbins=None, centroids=None,
                 seed=0, plan_fraction=0.01, chunk=16384, cache_bytes=2 << 30,
                 weights=None, flags=None):
        self.prm = prm
        uvw_m = np.asarray(uvw_m, dtype=np.float64)
        self.M_all = uvw_m.shape[0]
        self.keep = (np.arange(self.M_all) if flags is None
                     else np.nonzero(~np.asarray(flags, dtype=bool))[0])
        uvw_m = uvw_m[self.keep]
        self.omega = (None if weights is None
                      else np.asarray(weights, dtype=np.float64)[self.keep])
        scale = freq_hz / C_LIGHT
        self.u = uvw_m[:, 0] * scale
        self.v = uvw_m[:, 1] * scale
        self.w = uvw_m[:, 2] * scale
        self.M = uvw_m.shape[0]
        if centroids is None:
            mask = wbins.plan_subset_mask(self.M, plan_fraction, seed)
            centroids = wbins.kmeans_1d(self.w[mask], int(nbins))
        self.centroids = np.asarray(centroids, dtype=np.float64)
        self.P = self.centroids.size
        self.bins = wbins.assign_bins(self.w, self.centroids)
        self.wproj = self.w - self.centroids[self.bins]
        nx, ny, cell, o = prm.nx, prm.ny, prm.cell, prm.o
        self.Kx, self.Ky = o * nx, o * ny
        self.Lx, self.Ly = nx * cell, ny * cell
        self.ubar = self.u * (self.Kx * cell)
        self.vbar = self.v * (self.Ky * cell)
        self.sx = grid_correction(nx, self.Kx, prm.J, prm.beta)
        self.sy = grid_correction(ny, self.Ky, prm.J, prm.beta)
        l, m = pixel_lm(nx, ny, cell)
        self.d, self.n = nm1(l[None, :], m[:, None])      # [ny, nx]
        self.rows_j = (np.arange(ny) - ny // 2) % self.Ky
        self.cols_i = (np.arange(nx) - nx // 2) % self.Kx
        self.chunk = chunk
        self.cache_bytes = cache_bytes
        self._cache = {}
        self._cache_used = 0
        self.bin_rows = [np.nonzero(self.bins == p)[0] for p in range(self.P)]

    # ------------------------------------------------------------------ pieces
    def zp(self, p):
        """Diagonal of Z_p: grid correction times the w-layer C(.; w_p) (eq. 2, eq. 6)."""
        s = self.sy[:, None] * self.sx[None, :]
        return s * np.exp(-2j * np.pi * self.centroids[p] * self.d) / self.n

    def fwd_fft(self, img):
        """F: unnormalised 2-D DFT of the zero-padded image (library FFT, all host cores)."""
        g = np.zeros((self.Ky, self.Kx), dtype=np.complex128)
        g[np.ix_(self.rows_j, self.cols_i)] = img
        return scipy.fft.fft2(g, workers=os.cpu_count())

    def inv_fft_crop(self, grid):
        """F^dag: unnormalised inverse 2-D DFT, then the crop back to the image."""
        full = scipy.fft.ifft2(grid, norm="forward", workers=os.cpu_count())
        return full[np.ix_(self.rows_j, self.cols_i)]

    def nk(self, idx):
        p = self.prm
        return nk_rule(self.wproj[idx], self.Lx, self.Ly, p.o, p.alpha, p.smax)

    def patches(self, idx):
        """Rows idx -> list of (rows, qv0, qu0, g [b, T, T]) grouped by patch side T."""
        key = (int(idx[0]), int(idx[-1]), idx.size) if idx.size else None
        if key in self._cache:
            return self._cache[key]
        p = self.prm
        half = (p.J - 1) // 2
        nks = self.nk(idx)
        ru, tu = kb_taps(self.ubar[idx], p.J, p.beta)
        rv, tv = kb_taps(self.vbar[idx], p.J, p.beta)
        out = []
        for nk in np.unique(nks):
            sel = np.nonzero(nks == nk)[0]
            chat = wkernel_exact(self.wproj[idx[sel]], int(nk), self.Lx, self.Ly, p.o)
            groups, _ = threshold_shrink_batch(chat, p.eps)
            for gsel, ker in groups:
                rows = sel[gsel]
                npr = ker.shape[1]
                hp = (npr - 1) // 2
                T = npr + p.J - 1
                a = np.arange(T)[:, None] - np.arange(npr)[None, :]     # [T, n']
                valid = (a >= 0) & (a < p.J)
                ac = np.clip(a, 0, p.J - 1)
                Ku = np.where(valid[None], tu[rows][:, ac], 0.0)       # [b, T, n']
                Kv = np.where(valid[None], tv[rows][:, ac], 0.0)
                g = Kv @ ker @ np.swapaxes(Ku, 1, 2)                    # [b, T, T]
                if self.omega is not None:
                    g = g * self.omega[idx[rows]][:, None, None]
                out.append((idx[rows], rv[rows] - half - hp, ru[rows] - half - hp, g))
        nbytes = sum(o[3].nbytes for o in out)
        if self._cache_used + nbytes <= self.cache_bytes:
            self._cache[key] = out
            self._cache_used += nbytes
        return out

    def flat_index(self, qv0, qu0, T):
        av = np.arange(T)
        rows = (qv0[:, None] + av[None, :]) % self.Ky                   # [b, T]
        cols = (qu0[:, None] + av[None, :]) % self.Kx
        return rows[:, :, None] * self.Kx + cols[:, None, :]             # [b, T, T]

    def _chunks(self, rows):
        for s in range(0, rows.size, self.chunk):
            yield rows[s:s + self.chunk]

    # ------------------------------------------------------------------ G_p products
    def degrid(self, p, X):
        """y_k = sum_q g_k[q] X[q] for the rows of bin p; returns (rows, y)."""
        Xf = X.ravel()
        rs, ys = [], []
        for ch in self._chunks(self.bin_rows[p]):
            for rows, qv0, qu0, g in self.patches(ch):
                idx = self.flat_index(qv0, qu0, g.shape[1])
                rs.append(rows)
                ys.append((g * Xf[idx]).sum((1, 2)))
        if not rs:
            return np.zeros(0, np.int64), np.zeros(0, np.complex128)
        return np.concatenate(rs), np.concatenate(ys)

    def grid(self, p, rows_y):
        """Y[q] = sum_k conj(g_k[q]) y_k over the rows of bin p (rows_y: full y vector)."""
        N = self.Kx * self.Ky
        Yr = np.zeros(N)
        Yi = np.zeros(N)
        for ch in self._chunks(self.bin_rows[p]):
            for rows, qv0, qu0, g in self.patches(ch):
                idx = self.flat_index(qv0, qu0, g.shape[1]).ravel()
                c = (np.conj(g) * rows_y[rows][:, None, None]).ravel()
                Yr += np.bincount(idx, weights=c.real, minlength=N)
                Yi += np.bincount(idx, weights=c.imag, minlength=N)
        return (Yr + 1j * Yi).reshape(self.Ky, self.Kx)

    def gtg(self, p, X):
        """G_p^dag G_p X (eq. 8)."""
        rows, y = self.degrid(p, X)
        full = np.zeros(self.M, dtype=np.complex128)
        full[rows] = y
        return self.grid(p, full)

    # ------------------------------------------------------------------ operators
    def forward(self, x):
        """Phi x (eq. 3, eq. 6); x: [ny, nx] real or complex -> y [M_all] complex."""
        y = np.zeros(self.M, dtype=np.complex128)
        for p in range(self.P):
            if self.bin_rows[p].size == 0:
                continue
            X = self.fwd_fft(self.zp(p) * x)
            rows, yp = self.degrid(p, X)
            y[rows] = yp
        full = np.zeros(self.M_all, dtype=np.complex128)
        full[self.keep] = y
        return full

    def adjoint(self, y):
        """Phi^dag y (y: [M_all]); returns [ny, nx] complex."""
        y = np.asarray(y)[self.keep]
        out = np.zeros((self.prm.ny, self.prm.nx), dtype=np.complex128)
        for p in range(self.P):
            if self.bin_rows[p].size == 0:
                continue
            Y = self.grid(p, y)
            out += np.conj(self.zp(p)) * self.inv_fft_crop(Y)
        return out

    def psf_layer(self, p, x):
        """Phi_p^dag Phi_p x (eq. 8)."""
        z = self.zp(p)
        X = self.fwd_fft(z * x)
        return np.conj(z) * self.inv_fft_crop(self.gtg(p, X))

    def psf(self, x):
        """Phi^dag Phi x = sum_p Phi_p^dag Phi_p x (eq. 7); complex [ny, nx]."""
        out = np.zeros((self.prm.ny, self.prm.nx), dtype=np.complex128)
        for p in range(self.P):
            if self.bin_rows[p].size:
                out += self.psf_layer(p, x)
        return out

    # ------------------------------------------------------------------ explicit matrices
    def G_matrix(self, p):
        """Explicit sparse G_p (rows in bin order) -- small problems only."""
        N = self.Kx * self.Ky
        data, ri, ci, order = [], [], [], []
        base = 0
        for ch in self._chunks(self.bin_rows[p]):
            for rows, qv0, qu0, g in self.patches(ch):
                T = g.shape[1]
                idx = self.flat_index(qv0, qu0, T)
                b = rows.size
                r = np.repeat(np.arange(base, base + b), T * T)
                ri.append(r)
                ci.append(idx.ravel())
                data.append(g.ravel())
                order.append(rows)
                base += b
        G = sp.csr_matrix((np.concatenate(data), (np.concatenate(ri), np.concatenate(ci))),
                          shape=(base, N))
        return G, np.concatenate(order)

    def H_matrix(self, p):
        """Holographic matrix H_p = G_p^dag G_p (Sect. 3.3), full Hermitian CSR."""
        G, _ = self.G_matrix(p)
        return (G.conj().T @ G).tocsr()

    def psf_via_H(self, x):
        out = np.zeros((self.prm.ny, self.prm.nx), dtype=np.complex128)
        for p in range(self.P):
            if self.bin_rows[p].size == 0:
                continue
            z = self.zp(p)
            H = self.H_matrix(p)
            X = self.fwd_fft(z * x).ravel()
            out += np.conj(z) * self.inv_fft_crop((H @ X).reshape(self.Ky, self.Kx))
        return out

    def taps_total(self):
        """K = number of stored values of G (sum of T_k^2)."""
        tot = 0
        for p in range(self.P):
            for ch in self._chunks(self.bin_rows[p]):
                for rows, _, _, g in self.patches(ch):
                    tot += rows.size * g.shape[1] * g.shape[2]
        return tot
