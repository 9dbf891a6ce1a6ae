"""Parity at the benchmark's full size (4096^2 over 3 degrees, 50M visibilities, planner
P, FP16-stored G -- the configuration bench.py times) on outputs the FP64 oracle can
compute one by one, plus identities that hold at any size:
  * stored rows of G at sampled visibilities, element by element;
  * Phi applied to a point source off the phase centre at sampled rows: the oracle's
    row of G times the point source's layer transform, y_k = sum_q g_k[q] X_p[q] with
    X_p[q] = Z_p(pixel) exp(-2 pi i q . pixel / K);
  * adjointness <Phi x, y> = <x, Phi^dag y> and Hermitian symmetry of Phi^dag Phi.
The oracle is built on the sampled rows only, with the GPU plan's centroids imported
(data, not code), so that both sides bin the rows alike."""
import math
import sys

import numpy as np
import pytest

import wfsynth as ws
from gpu_common import TOL, rel, to_dev
from oracle import OracleOperator, OperatorParams

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def full():
    from paper_2605_26347_amd import Operator
    say("[gpu] full size: inputs 4096^2 / 50M")
    obs = ws.precision_form(sky=False)
    op = Operator(obs.uvw_m, obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad, store="f16")
    say(f"[gpu] full size: built P={op.plan()['nbins']}")
    return obs, op


def _oracle(obs, op, rows):
    prm = OperatorParams(obs.nx, obs.ny, obs.cell_rad)
    return OracleOperator(obs.uvw_m[rows], obs.freqs_hz[0], prm, centroids=op.centroids())


def test_stored_rows_full_size(full):
    obs, op = full
    rows = np.sort(np.random.default_rng(21).choice(obs.uvw_m.shape[0], 60, replace=False))
    orc = _oracle(obs, op, rows)
    for i, r in enumerate(rows):
        T, qu0, qv0, b, vals = op.get_row(int(r))
        (_, qv, qu, g), = orc.patches(np.array([i]))
        assert b == orc.bins[i] and T == g.shape[1]
        assert qu0 == qu[0] % orc.Kx and qv0 == qv[0] % orc.Ky
        # FP16 storage: half an ulp of 2^-10 relative, against the row's largest value
        assert np.abs(vals - g[0]).max() <= 1e-3 * np.abs(g[0]).max(), r


def test_point_source_forward_full_size(full):
    obs, op = full
    nx, ny = obs.nx, obs.ny
    i0, j0 = nx // 2 + 1234, ny // 2 - 987
    img = np.zeros((ny, nx), dtype=np.float32)
    img[j0, i0] = 1.0
    y = op.forward(to_dev(img[None])).cpu().numpy()
    rows = np.sort(np.random.default_rng(22).choice(obs.uvw_m.shape[0], 2000, replace=False))
    orc = _oracle(obs, op, rows)
    ref = np.zeros(rows.size, dtype=np.complex128)
    ci, rj = (i0 - nx // 2) % orc.Kx, (j0 - ny // 2) % orc.Ky
    for p in range(orc.P):
        z = orc.sy[j0] * orc.sx[i0] * np.exp(-2j * np.pi * orc.centroids[p] * orc.d[j0, i0]) \
            / orc.n[j0, i0]
        sel = np.nonzero(orc.bins == p)[0]
        if sel.size == 0:
            continue
        for rr, qv0, qu0, g in orc.patches(sel):
            T = g.shape[1]
            a = np.arange(T)
            qv = (qv0[:, None] + a[None, :]) % orc.Ky
            qu = (qu0[:, None] + a[None, :]) % orc.Kx
            ph = np.exp(-2j * np.pi * (qv[:, :, None] * rj / orc.Ky + qu[:, None, :] * ci / orc.Kx))
            ref[rr] = z * np.sum(g * ph, axis=(1, 2))
    e = rel(y[rows], ref)
    say(f"[gpu] point-source forward at 2000 sampled rows: rel {e:.2e}")
    assert e <= TOL["f16"]


def test_adjoint_and_hermitian_full_size(full):
    obs, op = full
    r = np.random.default_rng(23)
    x = r.standard_normal((obs.ny, obs.nx)).astype(np.float32)
    M = obs.uvw_m.shape[0]
    yv = (r.standard_normal(M) + 1j * r.standard_normal(M)).astype(np.complex64)
    xd, yd = to_dev(x[None]), to_dev(yv)
    phix = op.forward(xd).to(torch.complex128)
    phity = op.adjoint(yd)[0].to(torch.complex128)
    a = torch.vdot(phix, yd.to(torch.complex128)).item()
    b = torch.vdot(xd[0].to(torch.complex128).flatten(), phity.flatten()).item()
    say(f"[gpu] adjointness: {abs(a - b) / abs(a):.2e}")
    assert abs(a - b) <= 1e-5 * abs(a)
    x2 = r.standard_normal((obs.ny, obs.nx)).astype(np.float32)
    x2d = to_dev(x2[None])
    h1 = op.psf_apply(xd)[0].to(torch.complex128)
    h2 = op.psf_apply(x2d)[0].to(torch.complex128)
    s1 = torch.vdot(x2d[0].to(torch.complex128).flatten(), h1.flatten()).item()
    s2 = torch.vdot(xd[0].to(torch.complex128).flatten(), h2.flatten()).item()
    say(f"[gpu] Hermitian: {abs(s1 - np.conj(s2)) / abs(s1):.2e}")
    assert abs(s1 - np.conj(s2)) <= 1e-5 * abs(s1)
