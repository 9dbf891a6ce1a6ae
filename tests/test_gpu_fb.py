"""Forward-backward driver (Sect. 2, eq. 4) through the C ABI against the FP64 reference
(oracle/fb.py): dirty image, power-iteration norm and ten FB iterations with the
positivity + l1 prox, all within 1e-4 relative L2 (FP32 operator, errors of 1e-6
amplified at most by the iteration's contraction)."""
import sys

import numpy as np
import pytest

import wfsynth as ws
from gpu_common import TOL, rel, oracle_for, gpu_operator, to_dev
from oracle import fb as ofb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_forward_backward_matches_oracle():
    obs = ws.widefield(n=64, nvis=20_000, fov_deg=3.0, npoints=20, nblobs=2,
                       blob_sigma=(1.0, 2.0))
    op = gpu_operator(obs, 2)
    orc = oracle_for(obs, 2)
    x_true = np.clip(obs.sky, 0, None).astype(np.float32)
    y = op.forward(to_dev(x_true[None]))
    yh = y.cpu().numpy().astype(np.complex128)
    xd = op.dirty_image(y)
    xd_ref = ofb.dirty(orc, yh)
    e = rel(xd.cpu().numpy()[0], xd_ref)
    say(f"[gpu] dirty image rel {e:.2e}")
    assert e <= TOL["f32"]
    L = op.op_norm(30)
    L_ref = ofb.op_norm(orc, 30)
    say(f"[gpu] norm {L:.6e} vs {L_ref:.6e}")
    assert abs(L - L_ref) <= 1e-4 * L_ref
    gamma = 1.0 / L_ref
    lam = 1e-3 * float(np.abs(xd_ref).max())
    x = torch.zeros((1, 64, 64), dtype=torch.float32, device="cuda:0")
    op.fb_iterate(xd, x, 10, gamma, lam)
    x_ref = ofb.fb(orc, xd_ref, np.zeros((64, 64)), gamma, lam, 10)
    e = rel(x.cpu().numpy()[0], x_ref)
    say(f"[gpu] 10 FB iterations rel {e:.2e}")
    assert e <= 1e-4
    assert float(x.min()) >= 0.0
