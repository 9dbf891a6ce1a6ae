"""Parity of the HIP operator (through the C ABI) with the FP64 oracle.

Element-wise comparisons on the same seeded inputs: the 2-D layer transform F Z_p x,
stored rows of G, Phi x, Phi^dag y, Phi^dag Phi x and its real part, for FP32 / FP16 /
BF16 storage, several channels, empty bins and split work items.  Tolerances are the
relative-L2 bounds of the operator's precision forms (FP32 1e-5, FP16 1e-3, BF16 5e-3).
"""
import math
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
def wide():
    # 128^2 over 4 degrees, 64-antenna array thinned to 24k rows: grid 256^2 = 4 x 4
    # tiles, heavy wrapping of long baselines, many rows at the kernel-side cap.
    return ws.widefield(n=128, nvis=24_000, fov_deg=4.0, npoints=40, nblobs=3,
                        blob_sigma=(1.0, 3.0))


@pytest.fixture(scope="module")
def wide_pair(wide):
    say("[gpu] build widefield 128^2 / 24k rows / P=4")
    op = gpu_operator(wide, 4, max_rows_per_item=97)
    orc = oracle_for(wide, 4)
    return op, orc


def test_centroids_and_bins_match(wide_pair):
    op, orc = wide_pair
    c = op.centroids()
    assert np.allclose(c, orc.centroids, rtol=1e-12, atol=1e-9)
    assert np.array_equal(op.bin_rows(), np.bincount(orc.bins, minlength=orc.P))


def test_layer_transform(wide, wide_pair):
    op, orc = wide_pair
    x = wide.sky.astype(np.float32)
    xd = to_dev(x[None])
    for p in range(orc.P):
        g = op.layer_grid(0, p, xd).cpu().numpy()
        ref = orc.fwd_fft(orc.zp(p) * x.astype(np.float64))
        say(f"[gpu] layer {p} rel {rel(g, ref):.2e}")
        assert rel(g, ref) <= 2e-6


def test_stored_rows(wide_pair):
    op, orc = wide_pair
    rng = np.random.default_rng(0)
    rows = rng.choice(orc.M, 150, replace=False)
    nk_ok = 0
    for r in rows:
        T, qu0, qv0, b, vals = op.get_row(int(r))
        (rr, qv, qu, g), = orc.patches(np.array([r]))
        assert b == orc.bins[r]
        assert T == g.shape[1]
        assert qu0 == qu[0] % orc.Kx and qv0 == qv[0] % orc.Ky
        err = np.abs(vals - g[0]).max()
        assert err <= 1e-6 * np.abs(g[0]).max(), (r, err)
        nk_ok += 1
    assert nk_ok == len(rows)


@pytest.mark.parametrize("probe", ["sky", "noise"])
def test_psf_fp32(wide, wide_pair, probe):
    op, orc = wide_pair
    x = wide.sky if probe == "sky" else ws.gauss_image(128, 4)
    x = x.astype(np.float32)
    out = op.psf_apply(to_dev(x[None])).cpu().numpy()[0]
    ref = orc.psf(x.astype(np.float64))
    e = rel(out, ref)
    say(f"[gpu] psf fp32 {probe} rel {e:.2e}")
    assert e <= TOL["f32"]
    re = op.psf_apply_re(to_dev(x[None])).cpu().numpy()[0]
    assert rel(re, ref.real) <= TOL["f32"]


def test_forward_adjoint_fp32(wide, wide_pair):
    op, orc = wide_pair
    x = wide.sky.astype(np.float32)
    y = op.forward(to_dev(x[None])).cpu().numpy()
    yr = orc.forward(x.astype(np.float64))
    say(f"[gpu] forward rel {rel(y, yr):.2e}")
    assert rel(y, yr) <= TOL["f32"]
    r = np.random.default_rng(3)
    v = (r.standard_normal(orc.M) + 1j * r.standard_normal(orc.M)).astype(np.complex64)
    a = op.adjoint(to_dev(v)).cpu().numpy()[0]
    ar = orc.adjoint(v.astype(np.complex128))
    say(f"[gpu] adjoint rel {rel(a, ar):.2e}")
    assert rel(a, ar) <= TOL["f32"]


@pytest.mark.parametrize("store", ["f16", "bf16"])
def test_psf_low_precision_storage(wide, wide_pair, store):
    _, orc = wide_pair
    op = gpu_operator(wide, 4, store=store)
    for x in (wide.sky, ws.gauss_image(128, 4)):
        x = x.astype(np.float32)
        out = op.psf_apply(to_dev(x[None])).cpu().numpy()[0]
        e = rel(out, orc.psf(x.astype(np.float64)))
        say(f"[gpu] psf {store} rel {e:.2e}")
        assert e <= TOL[store]


def test_tiny_configuration_full():
    """64^2, 19,200 rows, one w-bin without residual kernel (FP32)."""
    obs = ws.tiny()
    op = gpu_operator(obs, 1, smax=1)
    orc = oracle_for(obs, 1, smax=1)
    x = obs.sky.astype(np.float32)
    out = op.psf_apply(to_dev(x[None])).cpu().numpy()[0]
    assert rel(out, orc.psf(x.astype(np.float64))) <= TOL["f32"]
    y = op.forward(to_dev(x[None])).cpu().numpy()
    assert rel(y, orc.forward(x.astype(np.float64))) <= TOL["f32"]


def test_two_channels_uneven_rows():
    base = ws.widefield(n=64, nvis=30_000, fov_deg=3.0, sky=False)
    counts = np.array([11_000, 19_000])
    obs = ws.Observation("two", base.uvw_m, np.array([1.0e9, 1.4e9]), 64, 64,
                         base.cell_rad, None, chan_rows=counts)
    op = gpu_operator(obs, 3)
    x = np.stack([ws.gauss_image(64, 1), ws.gauss_image(64, 2)]).astype(np.float32)
    out = op.psf_apply(to_dev(x)).cpu().numpy()
    y = op.forward(to_dev(x)).cpu().numpy()
    off = 0
    for c in range(2):
        orc = oracle_for(obs, 3, chan=c, uvw=base.uvw_m[off:off + counts[c]])
        assert rel(out[c], orc.psf(x[c].astype(np.float64))) <= TOL["f32"]
        assert rel(y[off:off + counts[c]], orc.forward(x[c].astype(np.float64))) <= TOL["f32"]
        off += counts[c]


def test_empty_bins_and_single_rows():
    """w quantised to two values but four bins: two bins receive no rows."""
    obs = ws.tiny(n=32, nant=8, nsteps=20, fov_deg=3.0, sky=False)
    uvw = obs.uvw_m.copy()
    uvw[:, 2] = np.where(uvw[:, 2] > 0, 50.0, -50.0)
    o2 = ws.Observation("q", uvw, obs.freqs_hz, 32, 32, obs.cell_rad)
    op = gpu_operator(o2, 4)
    orc = oracle_for(o2, 4)
    assert (op.bin_rows() == 0).sum() >= 1
    x = ws.gauss_image(32, 7).astype(np.float32)
    assert rel(op.psf_apply(to_dev(x[None])).cpu().numpy()[0],
               orc.psf(x.astype(np.float64))) <= TOL["f32"]
    # one row only
    o1 = ws.Observation("one", obs.uvw_m[:1], obs.freqs_hz, 32, 32, obs.cell_rad)
    op1 = gpu_operator(o1, 1)
    orc1 = oracle_for(o1, 1)
    assert rel(op1.psf_apply(to_dev(x[None])).cpu().numpy()[0],
               orc1.psf(x.astype(np.float64))) <= TOL["f32"]
