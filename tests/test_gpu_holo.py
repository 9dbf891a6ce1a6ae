"""Holographic strategy (Sect. 3.3, Fig. 2 branch (b)) through the C ABI: Phi^dag Phi
with H_p = G_p^dag G_p against the fused G^dag G operator (same arithmetic up to the
order of FP32 additions: 2e-6) and the FP64 oracle (1e-5 FP32, 1e-3 FP16 storage),
Hermitian symmetry of the applied operator, and the decision tree choosing H when G does
not fit the budget but H does."""
import sys

import numpy as np
import pytest

import wfsynth as ws
from gpu_common import TOL, rel, oracle_for, gpu_operator, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def obs():
    # 64^2 over 3 degrees, 20k rows; kernel sides capped at 15 keep the stencils small
    return ws.widefield(n=64, nvis=20_000, fov_deg=3.0, npoints=20, nblobs=2,
                        blob_sigma=(1.0, 2.0))


@pytest.fixture(scope="module")
def ops(obs):
    say("[gpu] build 64^2 / 20k rows / P=3, G and H")
    g = gpu_operator(obs, 3, smax=15)
    h = gpu_operator(obs, 3, smax=15, strategy="H")
    return g, h


def test_holographic_matches_fused_and_oracle(obs, ops):
    from paper_2605_26347_amd._lib import WfError
    g, h = ops
    ph = h.plan()
    assert ph["strategy"] == 2 and ph["mem_h_bytes"] > 0
    say(f"[gpu] H bytes {ph['mem_h_bytes'] / 1e6:.1f} MB vs G {g.plan()['mem_g_bytes'] / 1e6:.1f} MB")
    orc = oracle_for(obs, 3, smax=15)
    for x in (obs.sky, ws.gauss_image(64, 5)):
        x = x.astype(np.float32)
        xd = to_dev(x[None])
        yh = h.psf_apply(xd).cpu().numpy()[0]
        yg = g.psf_apply(xd).cpu().numpy()[0]
        ref = orc.psf(x.astype(np.float64))
        say(f"[gpu] H vs fused {rel(yh, yg):.2e}, H vs oracle {rel(yh, ref):.2e}")
        assert rel(yh, yg) <= 2e-6
        assert rel(yh, ref) <= TOL["f32"]
        assert rel(h.psf_apply_re(xd).cpu().numpy()[0], ref.real) <= TOL["f32"]
    with pytest.raises(WfError):
        h.forward(to_dev(obs.sky.astype(np.float32)[None]))


def test_holographic_is_hermitian(ops):
    _, h = ops
    x = ws.gauss_image(64, 8).astype(np.float32)
    y = ws.gauss_image(64, 9).astype(np.float32)
    hx = h.psf_apply(to_dev(x[None])).cpu().numpy()[0].astype(np.complex128)
    hy = h.psf_apply(to_dev(y[None])).cpu().numpy()[0].astype(np.complex128)
    a = np.vdot(y, hx)
    b = np.conj(np.vdot(x, hy))
    assert abs(a - b) <= 1e-5 * abs(a)
    assert abs(np.vdot(x, hx).imag) <= 1e-5 * abs(np.vdot(x, hx))


def test_holographic_fp16(obs):
    h = gpu_operator(obs, 3, smax=15, strategy="H", store="f16")
    orc = oracle_for(obs, 3, smax=15)
    x = obs.sky.astype(np.float32)
    e = rel(h.psf_apply(to_dev(x[None])).cpu().numpy()[0], orc.psf(x.astype(np.float64)))
    say(f"[gpu] H fp16 vs oracle {e:.2e}")
    assert e <= TOL["f16"]


def test_decision_tree_chooses_holographic():
    """Many visibilities per grid cell: G cannot fit the budget at any P (m_G stays
    above its asymptote) while H, whose size does not grow with M, does."""
    obs = ws.widefield(n=32, nvis=200_000, fov_deg=0.2, npoints=10, nblobs=1,
                       blob_sigma=(1.0, 2.0))
    big = gpu_operator(obs, 0)
    pg = big.plan()
    m_inf = 8 * obs.uvw_m.shape[0] * 49 + 12 * obs.uvw_m.shape[0]
    budget = 0.9 * m_inf / 0.65
    say(f"[gpu] G plan P={pg['nbins']} G {pg['mem_g_bytes'] / 1e6:.1f} MB; budget "
        f"{budget / 1e6:.1f} MB")
    h = gpu_operator(obs, 0, memory_budget=budget)
    ph = h.plan()
    say(f"[gpu] chosen strategy {ph['strategy']} P={ph['nbins']} H {ph['mem_h_bytes'] / 1e6:.1f} MB")
    assert ph["strategy"] == 2
    orc = oracle_for(obs, ph["nbins"])
    x = obs.sky.astype(np.float32)
    assert rel(h.psf_apply(to_dev(x[None])).cpu().numpy()[0],
               orc.psf(x.astype(np.float64))) <= TOL["f32"]
