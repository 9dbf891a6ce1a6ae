"""Strategy (c) of Sect. 3.4 / Fig. 2, G computed on the fly, through the C ABI.

The on-the-fly operator rebuilds G chunk by chunk at every apply with the same FP64
value pass as the build of a stored G, so its forward apply must equal the stored-G
operator's bit for bit and its other applies up to the order of FP32 atomic additions
(relative L2 <= 2e-6); against the FP64 oracle the precision forms' tolerances hold
(FP32 1e-5, FP16 1e-3), also with weights and flags.  The decision tree must reach (c)
when neither G nor H fits the budget; several chunks per bin, concurrent branches,
graph replays and the work-item autotuner are exercised."""
import sys

import numpy as np
import pytest

import wfsynth as ws
from gpu_common import TOL, rel, oracle_for, gpu_operator, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SAME = 2e-6
OTF = 3


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def obs():
    return ws.widefield(n=128, nvis=24_000, fov_deg=4.0, npoints=40, nblobs=3,
                        blob_sigma=(1.0, 3.0))


@pytest.fixture(scope="module")
def ops(obs):
    # a 50 MB budget cuts every bin into several chunks of ~100k values
    say("[gpu] build 128^2 / 24k rows / P=4: stored G and on the fly")
    g = gpu_operator(obs, 4, max_rows_per_item=97)
    f = gpu_operator(obs, 4, max_rows_per_item=97, strategy="otf", memory_budget=50e6)
    return g, f


def test_onthefly_equals_stored_and_oracle(obs, ops):
    g, f = ops
    pf = f.plan()
    say(f"[gpu] on the fly: row data {pf['mem_g_bytes'] / 1e6:.2f} MB, transient "
        f"{pf['mem_transient_bytes'] / 1e6:.2f} MB vs stored G {g.plan()['mem_g_bytes'] / 1e6:.1f} MB")
    assert pf["strategy"] == OTF
    assert pf["mem_transient_bytes"] < 0.3 * 8 * pf["ntaps"]   # several chunks
    assert pf["ntaps"] == g.plan()["ntaps"]
    orc = oracle_for(obs, 4)
    x = obs.sky.astype(np.float32)
    xd = to_dev(x[None])
    yf = f.forward(xd).cpu().numpy()
    assert np.array_equal(yf, g.forward(xd).cpu().numpy())
    assert rel(yf, orc.forward(x.astype(np.float64))) <= TOL["f32"]
    r = np.random.default_rng(71)
    v = (r.standard_normal(orc.M) + 1j * r.standard_normal(orc.M)).astype(np.complex64)
    af = f.adjoint(to_dev(v)).cpu().numpy()[0]
    assert rel(af, g.adjoint(to_dev(v)).cpu().numpy()[0]) <= SAME
    assert rel(af, orc.adjoint(v.astype(np.complex128))) <= TOL["f32"]
    for probe in (x, ws.gauss_image(128, 72).astype(np.float32)):
        pd = to_dev(probe[None])
        pf_ = f.psf_apply(pd).cpu().numpy()[0]
        ref = orc.psf(probe.astype(np.float64))
        e = rel(pf_, ref)
        say(f"[gpu] on-the-fly psf rel {e:.2e}")
        assert rel(pf_, g.psf_apply(pd).cpu().numpy()[0]) <= SAME
        assert e <= TOL["f32"]
        assert rel(f.psf_apply_re(pd).cpu().numpy()[0], ref.real) <= TOL["f32"]
    from paper_2605_26347_amd._lib import WfError
    with pytest.raises(WfError):
        f.get_row(0)


def test_onthefly_fp16_weights_flags(obs):
    M = obs.uvw_m.shape[0]
    omega = (1.0 / ws.noise_sigma(M)).astype(np.float32)
    flags = ws.flag_runs(M, 0.1)
    f = gpu_operator(obs, 4, strategy="otf", store="f16", weights=omega, flags=flags,
                     memory_budget=50e6)
    orc = oracle_for(obs, 4, weights=omega.astype(np.float64), flags=flags)
    x = obs.sky.astype(np.float32)
    xd = to_dev(x[None])
    y = f.forward(xd).cpu().numpy()
    assert np.all(y[flags] == 0)
    ey = rel(y, orc.forward(x.astype(np.float64)))
    ep = rel(f.psf_apply(xd).cpu().numpy()[0], orc.psf(x.astype(np.float64)))
    say(f"[gpu] on-the-fly FP16 weighted+flagged: forward {ey:.2e}, psf {ep:.2e}")
    assert ey <= TOL["f16"] and ep <= TOL["f16"]


def test_decision_tree_chooses_onthefly(obs):
    """Budget below the stored G's asymptote (every row at least J x J values, so no P
    fits) and below the holographic stencils of a sparse 256^2 grid: the tree must fall
    through to (c) (Fig. 2)."""
    big = gpu_operator(obs, 0)
    pg = big.plan()
    M = obs.uvw_m.shape[0]
    budget = 0.9 * (8 * M * 49 + 12 * M) / 0.65
    f = gpu_operator(obs, 0, memory_budget=budget)
    pf = f.plan()
    say(f"[gpu] G {pg['mem_g_bytes'] / 1e6:.1f} MB at P={pg['nbins']}; budget "
        f"{budget / 1e6:.1f} MB -> strategy {pf['strategy']} at P={pf['nbins']}")
    assert pf["strategy"] == OTF
    orc = oracle_for(obs, pf["nbins"])
    x = obs.sky.astype(np.float32)
    assert rel(f.psf_apply(to_dev(x[None])).cpu().numpy()[0],
               orc.psf(x.astype(np.float64))) <= TOL["f32"]


def test_onthefly_branches_graphs_autotune(obs):
    """Two channels on two branches (one transient buffer each), graph replays against
    the eager apply, and the autotuner's re-split of the work items."""
    M = obs.uvw_m.shape[0]
    cr = np.array([M // 2, M - M // 2])
    kw = dict(chan_rows=cr, strategy="otf", memory_budget=50e6, max_rows_per_item=128)
    from paper_2605_26347_amd import Operator
    one = Operator(obs.uvw_m, [1.2e9, 1.5e9], 128, 128, obs.cell_rad, nbins=3, branches=1, **kw)
    two = Operator(obs.uvw_m, [1.2e9, 1.5e9], 128, 128, obs.cell_rad, nbins=3, branches=2, **kw)
    x = to_dev(np.stack([obs.sky, ws.gauss_image(128, 73)]).astype(np.float32))
    ref = one.psf_apply_re(x).cpu().numpy()
    assert rel(two.psf_apply_re(x).cpu().numpy(), ref) <= SAME
    s = torch.cuda.Stream()
    out = torch.empty_like(x)
    g = two.capture("psf_re", x, out, s)
    for rep in range(3):
        with torch.cuda.stream(s):
            out.fill_(float("nan"))
        g.launch(s)
        s.synchronize()
        assert rel(out.cpu().numpy(), ref) <= SAME, rep
        two.psf_apply(x)          # eager work on the same grids between replays
        torch.cuda.synchronize()
    g.close()
    y0 = one.forward(x).cpu().numpy()
    info = one.autotune(x, torch.empty_like(x), reps=1)
    say(f"[gpu] on-the-fly autotune {info}")
    assert one.plan(0)["max_rows_per_item"] in (256, 512, 1024)
    assert np.array_equal(one.forward(x).cpu().numpy(), y0)
    assert rel(one.psf_apply_re(x).cpu().numpy(), ref) <= SAME
