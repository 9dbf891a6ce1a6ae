"""Data weights and flags in G (Sect. 2 data weighting; the flag vector of Sect. 3.5's
inputs) and the Briggs robust weights, through the C ABI against the FP64 oracle.

Weighted + flagged Phi, Phi^dag, Phi^dag Phi and its real part at the precision forms'
tolerances (FP32 1e-5, FP16 1e-3); stored rows looked up by caller row; flagged rows
read as zero and ignored; flagging equal to building on the kept rows (bit for bit for
Phi, up to the order of FP32 atomic additions for Phi^dag Phi);
the holographic strategy with weights; FP16 overflow rejected; Briggs weights equal to
the oracle's element by element (FP32 output, 1e-6)."""
import sys

import numpy as np
import pytest

import wfsynth as ws
from gpu_common import TOL, rel, oracle_for, gpu_operator, to_dev
from oracle import weighting as owt
from oracle.operator import C_LIGHT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def obs():
    return ws.widefield(n=128, nvis=24_000, fov_deg=4.0, npoints=40, nblobs=3,
                        blob_sigma=(1.0, 3.0))


@pytest.fixture(scope="module")
def data(obs):
    M = obs.uvw_m.shape[0]
    sigma = ws.noise_sigma(M)
    flags = ws.flag_runs(M, 0.1)
    uvw = obs.uvw_m * (obs.freqs_hz[0] / C_LIGHT)
    omega = owt.operator_weights(uvw[:, 0], uvw[:, 1], obs.nx, obs.ny, obs.cell_rad, 0.5,
                                 natural=1.0 / sigma.astype(np.float64) ** 2, flags=flags)
    omega = (omega / omega.max()).astype(np.float32)
    return omega, flags


@pytest.fixture(scope="module")
def pair(obs, data):
    omega, flags = data
    say(f"[gpu] build weighted 128^2 / 24k rows / P=4, {flags.mean():.3f} flagged")
    op = gpu_operator(obs, 4, max_rows_per_item=97, weights=omega, flags=flags)
    orc = oracle_for(obs, 4, weights=omega.astype(np.float64), flags=flags)
    return op, orc


def test_weighted_flagged_operator_matches_oracle(obs, data, pair):
    omega, flags = data
    op, orc = pair
    pl = op.plan()
    assert pl["nflagged"] == int(flags.sum()) and pl["nrows"] == int((~flags).sum())
    assert np.allclose(op.centroids(), orc.centroids, rtol=1e-12, atol=1e-9)
    x = obs.sky.astype(np.float32)
    xd = to_dev(x[None])
    out = torch.full((flags.size,), float("nan"), dtype=torch.complex64, device="cuda:0")
    y = op.forward(xd, out=out).cpu().numpy()
    yr = orc.forward(x.astype(np.float64))
    say(f"[gpu] weighted forward rel {rel(y, yr):.2e}")
    assert np.all(y[flags] == 0)
    assert rel(y, yr) <= TOL["f32"]
    r = np.random.default_rng(61)
    yv = (r.standard_normal(flags.size) + 1j * r.standard_normal(flags.size))
    yv[flags] = 1e6      # flagged data must not reach the image
    a = op.adjoint(to_dev(yv.astype(np.complex64))).cpu().numpy()[0]
    ar = orc.adjoint(yv)
    say(f"[gpu] weighted adjoint rel {rel(a, ar):.2e}")
    assert rel(a, ar) <= TOL["f32"]
    p = op.psf_apply(xd).cpu().numpy()[0]
    pr = orc.psf(x.astype(np.float64))
    say(f"[gpu] weighted psf rel {rel(p, pr):.2e}")
    assert rel(p, pr) <= TOL["f32"]
    assert rel(op.psf_apply_re(xd).cpu().numpy()[0], pr.real) <= TOL["f32"]


def test_stored_rows_by_caller_row(data, pair):
    from paper_2605_26347_amd._lib import WfError
    omega, flags = data
    op, orc = pair
    kept = np.nonzero(~flags)[0]
    r = np.random.default_rng(62)
    for i in r.choice(kept.size, 40, replace=False):
        T, qu0, qv0, b, vals = op.get_row(int(kept[i]))
        (_, qv, qu, g), = orc.patches(np.array([i]))
        assert T == g.shape[1] and b == orc.bins[i]
        assert np.abs(vals - g[0]).max() <= 1e-6 * np.abs(g[0]).max()
    with pytest.raises(WfError):
        op.get_row(int(np.nonzero(flags)[0][0]))


def test_flags_equal_building_on_kept_rows(obs, data, pair):
    omega, flags = data
    op, _ = pair
    keep = ~flags
    from paper_2605_26347_amd import Operator
    sub = Operator(obs.uvw_m[keep], obs.freqs_hz, obs.nx, obs.ny, obs.cell_rad, nbins=4,
                   max_rows_per_item=97, weights=omega[keep])
    for x in (obs.sky, ws.gauss_image(128, 63)):
        xd = to_dev(x.astype(np.float32)[None])
        # the gather of Phi is deterministic: equal bit for bit; Phi^dag Phi sums with
        # FP32 atomics, whose order may differ between two applies
        assert np.array_equal(op.forward(xd).cpu().numpy()[keep], sub.forward(xd).cpu().numpy())
        assert rel(op.psf_apply(xd).cpu().numpy(), sub.psf_apply(xd).cpu().numpy()) <= 1e-6


def test_weighted_fp16_and_holographic(obs, data):
    omega, flags = data
    x = obs.sky.astype(np.float32)
    xd = to_dev(x[None])
    orc = oracle_for(obs, 4, weights=omega.astype(np.float64), flags=flags)
    ref = orc.psf(x.astype(np.float64))
    f16 = gpu_operator(obs, 4, store="f16", weights=omega, flags=flags)
    e16 = rel(f16.psf_apply(xd).cpu().numpy()[0], ref)
    orc15 = oracle_for(obs, 3, smax=15, weights=omega.astype(np.float64), flags=flags)
    ref15 = orc15.psf(x.astype(np.float64))
    h = gpu_operator(obs, 3, smax=15, strategy="H", weights=omega, flags=flags)
    eh = rel(h.psf_apply(xd).cpu().numpy()[0], ref15)
    say(f"[gpu] weighted psf rel: FP16 G {e16:.2e}, FP32 H {eh:.2e}")
    assert e16 <= TOL["f16"]
    assert eh <= TOL["f32"]


def test_fp16_overflow_is_rejected(obs):
    from paper_2605_26347_amd._lib import WfError
    w = np.full(obs.uvw_m.shape[0], 1e6, dtype=np.float32)
    with pytest.raises(WfError, match="FP16"):
        gpu_operator(obs, 2, store="f16", weights=w)


def test_briggs_weights_match_oracle(obs):
    from paper_2605_26347_amd import briggs_weights
    M = obs.uvw_m.shape[0]
    sigma = ws.noise_sigma(2 * M)
    flags = ws.flag_runs(2 * M, 0.05)
    nat = (1.0 / sigma.astype(np.float64) ** 2).astype(np.float32)
    freqs = np.array([1.0e9, 1.4e9])
    for R in (-1.0, 0.0, 2.0):
        got = briggs_weights(obs.uvw_m, freqs, obs.nx, obs.ny, obs.cell_rad, R,
                             natural=nat, flags=flags)
        worst = 0.0
        for c in range(2):
            sl = slice(c * M, (c + 1) * M)
            uvw = obs.uvw_m * (freqs[c] / C_LIGHT)
            ref = owt.operator_weights(uvw[:, 0], uvw[:, 1], obs.nx, obs.ny, obs.cell_rad,
                                       R, natural=nat[sl].astype(np.float64), flags=flags[sl])
            assert np.all(got[sl][flags[sl]] == 0)
            worst = max(worst, float(np.max(np.abs(got[sl] - ref) / ref.max())))
        say(f"[gpu] Briggs R={R}: max error {worst:.2e} of the largest weight")
        assert worst <= 1e-6
    # per-channel row blocks (chan_rows) and unit natural weights
    cr = np.array([M // 3, M - M // 3])
    got = briggs_weights(obs.uvw_m, freqs, obs.nx, obs.ny, obs.cell_rad, 0.0, chan_rows=cr)
    for c, sl in enumerate((slice(0, cr[0]), slice(cr[0], M))):
        uvw = obs.uvw_m[sl] * (freqs[c] / C_LIGHT)
        ref = owt.operator_weights(uvw[:, 0], uvw[:, 1], obs.nx, obs.ny, obs.cell_rad, 0.0)
        assert np.max(np.abs(got[sl] - ref)) <= 1e-6 * ref.max()


@pytest.mark.parametrize("strategy,form", [("G", "auto"), ("otf", "factorised"),
                                           ("otf", "rebuilt")])
def test_fully_flagged_channel(strategy, form):
    """Channel 0 has every row flagged (no row is built: zero visibilities, zero image);
    channel 1 is weighted and partly flagged and matches the oracle on its own rows."""
    base = ws.widefield(n=64, nvis=30_000, fov_deg=3.0, sky=False)
    counts = np.array([11_000, 19_000])
    obs = ws.Observation("two", base.uvw_m, np.array([1.0e9, 1.4e9]), 64, 64,
                         base.cell_rad, None, chan_rows=counts)
    flags = np.concatenate([np.ones(counts[0], bool), ws.flag_runs(counts[1], 0.2)])
    w = (1.0 / ws.noise_sigma(int(counts.sum()))).astype(np.float32)
    op = gpu_operator(obs, 3, weights=w, flags=flags, strategy=strategy, otf_form=form,
                      memory_budget=400e6 if strategy == "otf" else 288e9)
    assert op.plan(0)["nrows"] == 0 and op.plan(0)["nflagged"] == counts[0]
    x = np.stack([ws.gauss_image(64, 1), ws.gauss_image(64, 2)]).astype(np.float32)
    out = op.psf_apply(to_dev(x)).cpu().numpy()
    vis = torch.full((int(counts.sum()),), float("nan"), dtype=torch.complex64, device="cuda:0")
    y = op.forward(to_dev(x), out=vis).cpu().numpy()
    assert np.all(out[0] == 0) and np.all(y[:counts[0]] == 0)
    sl = slice(counts[0], None)
    orc = oracle_for(obs, 3, chan=1, uvw=base.uvw_m[sl], weights=w[sl].astype(np.float64),
                     flags=flags[sl])
    assert rel(out[1], orc.psf(x[1].astype(np.float64))) <= TOL["f32"]
    assert rel(y[sl], orc.forward(x[1].astype(np.float64))) <= TOL["f32"]
    assert np.all(y[sl][flags[sl]] == 0)


def test_holographic_with_network_is_refused(obs):
    """Branch (b) accumulates H from exact kernels only; a network is refused there
    (branch (c) takes it: tests/test_gpu_mlp.py)."""
    from paper_2605_26347_amd import Network
    from paper_2605_26347_amd._lib import WfError
    net = Network(5)
    with pytest.raises(WfError, match="exact kernels only"):
        gpu_operator(obs, 4, strategy="H", surrogate=net)
