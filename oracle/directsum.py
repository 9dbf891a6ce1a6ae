"""Brute-force widefield measurement equation (oracle; test infrastructure only).

y_k = sum_{j,i} x[j][i] * C(l_i, m_j; w_k) * exp(-2i pi (u_k l_i + v_k m_j))
with C the w-term of eq. 2: this is the discrete form of eq. 1 that eq. 3's Phi
models.  The adjoint is the exact conjugate transpose.  O(M N); chunked over rows.
"""
from __future__ import annotations

import numpy as np

from .kernels import pixel_lm, nm1


def _rows_matrix(u, v, w, nx, ny, cell):
    l, m = pixel_lm(nx, ny, cell)
    L = np.broadcast_to(l[None, :], (ny, nx)).ravel()
    Mm = np.broadcast_to(m[:, None], (ny, nx)).ravel()
    d, n = nm1(L, Mm)
    ph = (w[:, None] * d[None, :]) + (u[:, None] * L[None, :]) + (v[:, None] * Mm[None, :])
    return np.exp(-2j * np.pi * ph) / n[None, :]


def direct_matrix(uvw_lambda, nx, ny, cell):
    """Dense Phi (M x N) for tiny problems."""
    u, v, w = uvw_lambda[:, 0], uvw_lambda[:, 1], uvw_lambda[:, 2]
    return _rows_matrix(u, v, w, nx, ny, cell)


def direct_forward(x, uvw_lambda, cell, chunk=512):
    """Phi x by direct summation; x is [ny, nx] (real or complex)."""
    ny, nx = x.shape
    xf = x.ravel().astype(np.complex128)
    M = uvw_lambda.shape[0]
    y = np.empty(M, dtype=np.complex128)
    for s in range(0, M, chunk):
        e = min(M, s + chunk)
        A = _rows_matrix(uvw_lambda[s:e, 0], uvw_lambda[s:e, 1], uvw_lambda[s:e, 2],
                         nx, ny, cell)
        y[s:e] = A @ xf
    return y


def direct_adjoint(y, uvw_lambda, nx, ny, cell, chunk=512):
    """Phi^dag y by direct summation; returns [ny, nx] complex."""
    M = uvw_lambda.shape[0]
    out = np.zeros(nx * ny, dtype=np.complex128)
    for s in range(0, M, chunk):
        e = min(M, s + chunk)
        A = _rows_matrix(uvw_lambda[s:e, 0], uvw_lambda[s:e, 1], uvw_lambda[s:e, 2],
                         nx, ny, cell)
        out += A.conj().T @ y[s:e]
    return out.reshape(ny, nx)
