"""Briggs robust data weighting in FP64 -- TEST INFRASTRUCTURE ONLY.

Sect. 2 names a density-aware weighting of the data (Briggs weighting) as an optional
factor of the measurement operator.  The paper gives no formula; this follows the
published definition of robust weighting (D. S. Briggs, PhD thesis, New Mexico Tech,
1995):

* natural weights w_k (ones by default);
* gridded weight density W_c = sum of w_k over the samples whose (u, v) falls in uv
  cell c, the cells being the Fourier cells of the image (du = 1 / (nx cell),
  dv = 1 / (ny cell), index round(u / du) modulo nx, likewise for v).  The image is
  real, so every sample also samples (-u, -v): each sample is counted in both cells;
* f^2 = (5 10^-R)^2 / (sum_k w_k W_{c(k)} / sum_k w_k) for the robustness R;
* imaging weight  w'_k = w_k / (1 + W_{c(k)} f^2).

R -> +inf gives natural weighting (w'_k -> w_k), R -> -inf uniform weighting (w'_k
proportional to w_k / W_{c(k)}).  The imaging weight multiplies each sample once in the
gridded sum Phi^dag diag(w') y, so the operator weight is omega_k = sqrt(w'_k)
(Phi_W = diag(omega) Phi).  Flagged samples are left out of the density and get zero.
"""
from __future__ import annotations

import numpy as np


def uv_cells(u_lambda, v_lambda, nx: int, ny: int, cell: float):
    """Flat index iv * nx + iu of each (u, v) on the image's Fourier grid."""
    du = 1.0 / (nx * cell)
    dv = 1.0 / (ny * cell)
    iu = np.mod(np.floor(np.asarray(u_lambda, dtype=np.float64) / du + 0.5), nx).astype(np.int64)
    iv = np.mod(np.floor(np.asarray(v_lambda, dtype=np.float64) / dv + 0.5), ny).astype(np.int64)
    return iv * nx + iu


def density(u_lambda, v_lambda, nx: int, ny: int, cell: float, natural):
    """Gridded weight density W over nx * ny cells, each sample counted at (u, v) and at
    (-u, -v)."""
    w = np.asarray(natural, dtype=np.float64)
    c = uv_cells(u_lambda, v_lambda, nx, ny, cell)
    cc = uv_cells(-np.asarray(u_lambda), -np.asarray(v_lambda), nx, ny, cell)
    W = np.zeros(nx * ny)
    np.add.at(W, c, w)
    np.add.at(W, cc, w)
    return W


def briggs(u_lambda, v_lambda, nx: int, ny: int, cell: float, robust: float,
           natural=None, flags=None):
    """Imaging weights w'_k (zero where flagged)."""
    M = np.asarray(u_lambda).size
    w = np.ones(M) if natural is None else np.asarray(natural, dtype=np.float64).copy()
    if flags is not None:
        w[np.asarray(flags, dtype=bool)] = 0.0
    W = density(u_lambda, v_lambda, nx, ny, cell, w)
    Wk = W[uv_cells(u_lambda, v_lambda, nx, ny, cell)]
    S = float(np.sum(w * Wk))
    T = float(np.sum(w))
    if not (S > 0.0 and T > 0.0):
        return np.zeros(M)
    f2 = (5.0 * 10.0 ** (-robust)) ** 2 * T / S
    return w / (1.0 + Wk * f2)


def operator_weights(u_lambda, v_lambda, nx: int, ny: int, cell: float, robust: float,
                     natural=None, flags=None):
    """omega_k = sqrt(w'_k), the factor of row k of Phi_W."""
    return np.sqrt(briggs(u_lambda, v_lambda, nx, ny, cell, robust, natural, flags))
