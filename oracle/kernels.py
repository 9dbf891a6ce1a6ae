"""Scalar building blocks of the operator, FP64 (oracle; test infrastructure only).

Conventions (the paper fixes none of them; readings listed in the design notes):
  * pixel (i, j) of an nx x ny image sits at direction cosines
    l_i = (i - nx/2) * cell, m_j = (j - ny/2) * cell; the image array is x[j][i].
  * the oversampled grid has Kx = o*nx, Ky = o*ny cells (o = 2, Sect. 3.2).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special


def pixel_lm(nx: int, ny: int, cell: float):
    """Direction cosines of the pixel centres (l along columns i, m along rows j)."""
    l = (np.arange(nx, dtype=np.float64) - nx // 2) * cell
    m = (np.arange(ny, dtype=np.float64) - ny // 2) * cell
    return l, m


def nm1(l, m):
    """n - 1 = sqrt(1 - l^2 - m^2) - 1, written as -(l^2+m^2)/(1+n) so that no
    cancellation occurs near the phase centre (same value, eq. 2)."""
    r2 = l * l + m * m
    n = np.sqrt(1.0 - r2)
    return -r2 / (1.0 + n), n


def chirp(l, m, w):
    """w-term C(l, m; w) = exp(-2i pi w (n - 1)) / n  (Sect. 2, eq. 2)."""
    d, n = nm1(l, m)
    return np.exp(-2j * np.pi * w * d) / n


def i0_series(x):
    """Modified Bessel function I0 from its power series sum_k ((x/2)^k / k!)^2.
    Used only to cross-check the library routine in the tests."""
    x = np.asarray(x, dtype=np.float64)
    term = np.ones_like(x)
    s = np.ones_like(x)
    q = (x / 2.0) ** 2
    for k in range(1, 200):
        term = term * q / (k * k)
        s = s + term
    return s


def kb_phi(t, J: int, beta: float):
    """Kaiser-Bessel interpolation kernel of support J (the NUFFT interpolation kernel
    of G_p, Sect. 3.2): phi(t) = I0(beta sqrt(1-(2t/J)^2)) / I0(beta) for |t| <= J/2."""
    t = np.asarray(t, dtype=np.float64)
    z = 1.0 - (2.0 * t / J) ** 2
    out = np.where(z >= 0.0, scipy.special.i0(beta * np.sqrt(np.maximum(z, 0.0))), 0.0)
    return out / scipy.special.i0(beta)


def kb_phihat(nu, J: int, beta: float):
    """Continuous Fourier transform of kb_phi, int phi(t) e^{2i pi nu t} dt
    = (J / I0(beta)) sinh(z)/z with z = sqrt(beta^2 - (pi J nu)^2)  (closed form of
    the Kaiser-Bessel window transform; real and even).  Valid for pi J |nu| < beta,
    which holds on the image (|nu| <= 1/(2o))."""
    nu = np.asarray(nu, dtype=np.float64)
    z = np.sqrt(beta * beta - (math.pi * J * nu) ** 2)
    return (J / scipy.special.i0(beta)) * np.sinh(z) / z


def grid_correction(n: int, K: int, J: int, beta: float):
    """Grid-correction factors s_i = 1 / phihat((i - n/2)/K), the part of Z_p that
    undoes the interpolation kernel's apodisation (Sect. 3.2, eq. 6)."""
    iota = np.arange(n, dtype=np.float64) - n // 2
    return 1.0 / kb_phihat(iota / K, J, beta)


def kb_taps(coord, J: int, beta: float):
    """Interpolation taps for grid coordinates coord (in cells).  The nearest cell is
    r = floor(coord + 1/2); the J taps sit at cells r + d, d = -(J-1)/2..(J-1)/2, with
    weights phi(coord - r - d).  Returns (r int64, taps [len, J])."""
    coord = np.asarray(coord, dtype=np.float64)
    r = np.floor(coord + 0.5)
    f = coord - r
    half = (J - 1) // 2
    d = np.arange(-half, half + 1, dtype=np.float64)
    taps = kb_phi(f[:, None] - d[None, :], J, beta)
    return r.astype(np.int64), taps
