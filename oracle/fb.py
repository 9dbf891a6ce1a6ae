"""FP64 forward-backward iteration on the oracle operator -- TEST INFRASTRUCTURE ONLY.

Sect. 2, eq. 4: x <- D(x + gamma (x_dirty - Re{Phi^dag Phi x})), x_dirty = Re{Phi^dag y},
the gradient step of f(x) = 1/2 ||Phi x - y||^2 followed by a denoiser D.  The
denoiser here is the proximal operator of lam ||x||_1 plus the positivity constraint,
with step gamma: D(z) = max(z - gamma lam, 0) elementwise (a non-learned prox; the
paper's SARA and learned denoisers are out of scope).  The step must satisfy
gamma < 2 / L with L the largest eigenvalue of Re{Phi^dag Phi}, estimated by power
iteration from the all-ones image.
"""
from __future__ import annotations

import numpy as np


def prox_pos_l1(z, t):
    """argmin_u 1/2 (u - z)^2 + t |u| subject to u >= 0, elementwise."""
    return np.maximum(np.asarray(z, dtype=np.float64) - t, 0.0)


def dirty(orc, y):
    """x_dirty = Re{Phi^dag y}."""
    return orc.adjoint(np.asarray(y, dtype=np.complex128)).real


def op_norm(orc, iters: int):
    """Power iteration on x -> Re{Phi^dag Phi x} from the normalised all-ones image;
    returns the Rayleigh quotient of the last iterate."""
    x = np.ones((orc.prm.ny, orc.prm.nx))
    x /= np.linalg.norm(x)
    L = 0.0
    for _ in range(iters):
        z = orc.psf(x).real
        L = float(np.vdot(x, z).real)
        x = z / np.linalg.norm(z)
    return L


def fb(orc, x_dirty, x0, gamma: float, lam: float, iters: int):
    """iters iterations of eq. 4 with D = prox_pos_l1(., gamma lam)."""
    x = np.asarray(x0, dtype=np.float64).copy()
    for _ in range(iters):
        x = prox_pos_l1(x + gamma * (x_dirty - orc.psf(x).real), gamma * lam)
    return x


def objective(orc, x, y, lam: float):
    """1/2 ||Phi x - y||^2 + lam ||x||_1 (x >= 0)."""
    r = orc.forward(x) - y
    return 0.5 * float(np.vdot(r, r).real) + lam * float(np.abs(x).sum())
