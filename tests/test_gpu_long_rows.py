"""Parity of the HIP operator with the FP64 oracle at the long row lengths (grid sides
2048 and 4096), where the row passes of F and F^dag run as three register-resident
radix-16/32 passes: element-wise F Z_p x per layer, Phi x, Phi^dag y and Phi^dag Phi x
on a seeded widefield subset (eq. 6-8)."""
import sys

import numpy as np
import pytest

import wfsynth as ws
from gpu_common import TOL, rel, oracle_for, gpu_operator, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("n,fov", [(1024, 2.0), (2048, 3.0)])
def test_long_rows_element_wise(n, fov):
    obs = ws.widefield(n=n, nvis=20_000, fov_deg=fov, npoints=60, nblobs=4)
    say(f"[gpu] long rows: {n}^2 over {fov} deg, 20k rows, P=3")
    op = gpu_operator(obs, 3)
    orc = oracle_for(obs, 3)
    assert np.allclose(op.centroids(), orc.centroids, rtol=1e-12, atol=1e-9)
    x = obs.sky.astype(np.float32)
    xd = to_dev(x[None])
    for p in range(orc.P):
        g = op.layer_grid(0, p, xd).cpu().numpy()
        e = rel(g, orc.fwd_fft(orc.zp(p) * x.astype(np.float64)))
        say(f"[gpu]   layer {p}: F Z_p x rel {e:.2e}")
        assert e <= 2e-6
    for probe in ("sky", "noise"):
        xi = (obs.sky if probe == "sky" else ws.gauss_image(n, 4)).astype(np.float32)
        out = op.psf_apply(to_dev(xi[None])).cpu().numpy()[0]
        e = rel(out, orc.psf(xi.astype(np.float64)))
        say(f"[gpu]   psf {probe} rel {e:.2e}")
        assert e <= TOL["f32"]
    y = op.forward(xd).cpu().numpy()
    assert rel(y, orc.forward(x.astype(np.float64))) <= TOL["f32"]
    r = np.random.default_rng(3)
    v = (r.standard_normal(orc.M) + 1j * r.standard_normal(orc.M)).astype(np.complex64)
    a = op.adjoint(to_dev(v)).cpu().numpy()[0]
    e = rel(a, orc.adjoint(v.astype(np.complex128)))
    say(f"[gpu]   adjoint rel {e:.2e}")
    assert e <= TOL["f32"]
    op.close()


def test_layer_transform_8192_unmasked():
    """F Z_p x of a 4096^2 image (8192-point passes, lines exchanged as floats) without a
    pruning mask, element-wise against the FP64 oracle (eq. 6): every output row of the
    column passes is written when no tile is masked out."""
    obs = ws.widefield(n=4096, nvis=20_000, fov_deg=3.0, npoints=60, nblobs=4)
    say("[gpu] layer transform: 4096^2 over 3 deg, 20k rows, P=3, no mask")
    op = gpu_operator(obs, 3)
    orc = oracle_for(obs, 3)
    assert np.allclose(op.centroids(), orc.centroids, rtol=1e-12, atol=1e-9)
    x = obs.sky.astype(np.float32)
    xd = to_dev(x[None])
    for p in (0, orc.P - 1):
        g = op.layer_grid(0, p, xd).cpu().numpy()
        e = rel(g, orc.fwd_fft(orc.zp(p) * x.astype(np.float64)))
        say(f"[gpu]   layer {p}: F Z_p x rel {e:.2e}")
        assert e <= 2e-6
    op.close()
