"""Pins of the FP64 forward-backward reference (oracle/fb.py): the prox against brute
force, the power-iteration norm against the largest eigenvalue of the dense
Re{Phi^dag Phi}, and the monotone decrease of the FB objective for gamma = 1/L (a
property of proximal gradient steps no larger than 1/L)."""
import numpy as np

import wfsynth as ws
from oracle import OracleOperator, OperatorParams
from oracle import fb


def _tiny():
    obs = ws.tiny(n=16, nant=8, nsteps=30, fov_deg=2.0, sky=False)
    orc = OracleOperator(obs.uvw_m, obs.freqs_hz[0], OperatorParams(16, 16, obs.cell_rad),
                         nbins=2)
    return obs, orc


def test_prox_matches_brute_force():
    u = np.linspace(0.0, 4.0, 400001)
    for z in (-1.3, -0.1, 0.0, 0.05, 0.3, 1.7, 3.2):
        for t in (0.0, 0.1, 0.7):
            f = 0.5 * (u - z) ** 2 + t * u
            assert abs(fb.prox_pos_l1(z, t) - u[np.argmin(f)]) <= 1e-5


def test_power_iteration_matches_dense_eigenvalue():
    _, orc = _tiny()
    n = 16 * 16
    A = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = orc.psf(e.reshape(16, 16)).real.ravel()
    assert np.allclose(A, A.T, atol=1e-10 * np.abs(A).max())
    lmax = np.linalg.eigvalsh(0.5 * (A + A.T))[-1]
    # the Rayleigh quotient approaches the largest eigenvalue from below, monotonically
    L1, L2 = fb.op_norm(orc, 30), fb.op_norm(orc, 300)
    assert L1 <= L2 <= lmax * (1 + 1e-12)
    assert L2 >= 0.995 * lmax


def test_fb_objective_decreases():
    obs, orc = _tiny()
    rng = np.random.default_rng(0)
    x_true = np.zeros((16, 16))
    x_true[rng.integers(0, 16, 6), rng.integers(0, 16, 6)] = rng.uniform(0.5, 2.0, 6)
    y = orc.forward(x_true)
    y = y + 0.01 * np.abs(y).mean() * (rng.standard_normal(y.size) + 1j * rng.standard_normal(y.size))
    L = fb.op_norm(orc, 100)
    xd = fb.dirty(orc, y)
    lam = 0.01 * np.abs(xd).max()
    x = np.zeros((16, 16))
    prev = fb.objective(orc, x, y, lam)
    for _ in range(15):
        x = fb.fb(orc, xd, x, 1.0 / L, lam, 1)
        cur = fb.objective(orc, x, y, lam)
        assert cur <= prev * (1 + 1e-12)
        prev = cur
    assert np.all(x >= 0)
