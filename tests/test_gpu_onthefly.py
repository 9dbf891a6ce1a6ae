"""Strategy (c) of Sect. 3.4 / Fig. 2, G computed on the fly, through the C ABI.

Rebuilt form: G is rebuilt chunk by chunk at every apply with the same FP64 value pass
as the build of a stored G, so its forward apply must equal the stored-G operator's bit
for bit and its other applies up to the order of FP32 atomic additions (relative L2
<= 2e-6).  Factorised form: the build stores each row's thresholded residual kernel and
an apply convolves it with the Kaiser-Bessel taps in FP32, so it matches the stored G
to FP32 rounding (relative L2 <= 5e-6).  Against the FP64 oracle both meet the precision
forms' tolerances (FP32 1e-5, FP16 1e-3, BF16 5e-3), also with weights and flags.  The
decision tree must reach (c) when neither G nor H fits the budget and pick the
factorised form only when its kernels fit; several chunks per bin, concurrent
branches, graph replays and the work-item autotuner are exercised."""
import sys

import numpy as np
import pytest

import wfsynth as ws
from gpu_common import TOL, rel, oracle_for, gpu_operator, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SAME = 2e-6
FACT = 5e-6
OTF = 3
REBUILT, FACTORISED = 1, 2


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
    f = gpu_operator(obs, 4, max_rows_per_item=97, strategy="otf", memory_budget=50e6,
                     otf_form="rebuilt")
    return g, f


def test_onthefly_equals_stored_and_oracle(obs, ops):
    g, f = ops
    pf = f.plan()
    say(f"[gpu] on the fly: row data {pf['mem_g_bytes'] / 1e6:.2f} MB, transient "
        f"{pf['mem_transient_bytes'] / 1e6:.2f} MB vs stored G {g.plan()['mem_g_bytes'] / 1e6:.1f} MB")
    assert pf["strategy"] == OTF and pf["otf_form"] == REBUILT and pf["mem_khat_bytes"] == 0
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
                     memory_budget=50e6, otf_form="rebuilt")
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


def test_factorised_equals_stored_and_oracle(obs, ops):
    g, _ = ops
    # the kernels of this 4 degree field (n' ~ 17) need ~56 MB: a 400 MB budget holds them
    # and still cuts every bin into several chunks
    f = gpu_operator(obs, 4, max_rows_per_item=97, strategy="otf", memory_budget=400e6)
    pf, pg = f.plan(), g.plan()
    say(f"[gpu] factorised: kernels {pf['mem_khat_bytes'] / 1e6:.2f} MB, row data "
        f"{pf['mem_g_bytes'] / 1e6:.2f} MB vs stored G {pg['mem_g_bytes'] / 1e6:.1f} MB")
    assert pf["strategy"] == OTF and pf["otf_form"] == FACTORISED   # auto: the kernels fit
    assert pf["ntaps"] == pg["ntaps"]
    assert pf["mem_transient_bytes"] < 0.3 * 8 * pf["ntaps"]   # several chunks
    # kernel values: n'^2 per row against G's T^2, T = n' + J - 1
    assert 4 * pf["nrows"] < pf["mem_khat_bytes"] < 0.7 * 8 * pf["ntaps"]
    orc = oracle_for(obs, 4)
    x = obs.sky.astype(np.float32)
    xd = to_dev(x[None])
    yf = f.forward(xd).cpu().numpy()
    assert rel(yf, g.forward(xd).cpu().numpy()) <= FACT
    assert rel(yf, orc.forward(x.astype(np.float64))) <= TOL["f32"]
    assert np.array_equal(f.forward(xd).cpu().numpy(), yf)      # deterministic expansion
    r = np.random.default_rng(74)
    v = (r.standard_normal(orc.M) + 1j * r.standard_normal(orc.M)).astype(np.complex64)
    af = f.adjoint(to_dev(v)).cpu().numpy()[0]
    assert rel(af, g.adjoint(to_dev(v)).cpu().numpy()[0]) <= FACT
    assert rel(af, orc.adjoint(v.astype(np.complex128))) <= TOL["f32"]
    for probe in (x, ws.gauss_image(128, 75).astype(np.float32)):
        pd = to_dev(probe[None])
        p = f.psf_apply(pd).cpu().numpy()[0]
        ref = orc.psf(probe.astype(np.float64))
        e = rel(p, ref)
        say(f"[gpu] factorised psf rel {e:.2e}")
        assert rel(p, g.psf_apply(pd).cpu().numpy()[0]) <= FACT
        assert e <= TOL["f32"]
        assert rel(f.psf_apply_re(pd).cpu().numpy()[0], ref.real) <= TOL["f32"]


@pytest.mark.parametrize("store", ["f16", "bf16"])
def test_factorised_precision_forms_weights_flags(obs, store):
    M = obs.uvw_m.shape[0]
    omega = (1.0 / ws.noise_sigma(M)).astype(np.float32)
    flags = ws.flag_runs(M, 0.1)
    f = gpu_operator(obs, 4, strategy="otf", store=store, weights=omega, flags=flags,
                     memory_budget=400e6, otf_form="factorised")
    assert f.plan()["otf_form"] == FACTORISED
    orc = oracle_for(obs, 4, weights=omega.astype(np.float64), flags=flags)
    x = obs.sky.astype(np.float32)
    xd = to_dev(x[None])
    y = f.forward(xd).cpu().numpy()
    assert np.all(y[flags] == 0)
    ey = rel(y, orc.forward(x.astype(np.float64)))
    ep = rel(f.psf_apply(xd).cpu().numpy()[0], orc.psf(x.astype(np.float64)))
    say(f"[gpu] factorised {store} weighted+flagged: forward {ey:.2e}, psf {ep:.2e}")
    assert ey <= TOL[store] and ep <= TOL[store]


def test_factorised_only_when_its_kernels_fit(obs):
    """Budget share below the factorised form's kernels but above the rebuilt form's row
    data: auto takes the rebuilt form, and forcing the factorised one is refused."""
    from paper_2605_26347_amd._lib import WfError
    M = obs.uvw_m.shape[0]
    small = gpu_operator(obs, 4, strategy="otf", memory_budget=50e6, otf_form="rebuilt")
    fact = gpu_operator(obs, 4, strategy="otf", memory_budget=400e6, otf_form="factorised")
    tr = small.plan()["mem_transient_bytes"]
    kb = fact.plan()["mem_khat_bytes"]
    share = 44 * M + 4 * tr + 0.5 * kb       # row data + four branch buffers + half the kernels
    auto = gpu_operator(obs, 4, strategy="otf", memory_budget=share / 0.65)
    pa = auto.plan()
    say(f"[gpu] share {share / 1e6:.1f} MB: kernels {kb / 1e6:.1f} MB, transient "
        f"{pa['mem_transient_bytes'] / 1e6:.2f} MB -> form {pa['otf_form']}")
    assert pa["otf_form"] == REBUILT
    assert 44 * M + kb + 4 * pa["mem_transient_bytes"] > share   # the kernels do not fit
    with pytest.raises(WfError, match="factorised"):
        gpu_operator(obs, 4, strategy="otf", memory_budget=share / 0.65, otf_form="factorised")
    x = to_dev(obs.sky.astype(np.float32)[None])
    assert rel(auto.psf_apply(x).cpu().numpy(), fact.psf_apply(x).cpu().numpy()) <= FACT


def test_factorised_branches_and_graph(obs):
    """Two channels on two branches (a transient buffer each), graph replays against the
    eager apply, and the autotuner's re-split of the work items, in the factorised form."""
    M = obs.uvw_m.shape[0]
    cr = np.array([M // 2, M - M // 2])
    from paper_2605_26347_amd import Operator
    kw = dict(chan_rows=cr, strategy="otf", memory_budget=400e6, max_rows_per_item=128,
              otf_form="factorised")
    one = Operator(obs.uvw_m, [1.2e9, 1.5e9], 128, 128, obs.cell_rad, nbins=3, branches=1, **kw)
    two = Operator(obs.uvw_m, [1.2e9, 1.5e9], 128, 128, obs.cell_rad, nbins=3, branches=2, **kw)
    x = to_dev(np.stack([obs.sky, ws.gauss_image(128, 76)]).astype(np.float32))
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
        two.forward(x)            # eager work on the same transient buffers between replays
        torch.cuda.synchronize()
    g.close()
    y0 = one.forward(x).cpu().numpy()
    info = one.autotune(x, torch.empty_like(x), reps=1)
    say(f"[gpu] factorised autotune {info}")
    assert one.plan(0)["max_rows_per_item"] in (256, 512, 1024)
    assert np.array_equal(one.forward(x).cpu().numpy(), y0)
    assert rel(one.psf_apply_re(x).cpu().numpy(), ref) <= SAME


def test_factorised_large_launches():
    """200k rows on few chunks: the expansion launches hold tens of thousands of rows of
    one class, so that a workgroup expands many slot steps (the lanes that evaluate the
    rows' taps are then not the lanes that expand them).  Against the stored G, whose FP64
    value pass the oracle tests pin."""
    big = ws.widefield(n=256, nvis=200_000, fov_deg=3.0, sky=False)
    g = gpu_operator(big, 4)
    f = gpu_operator(big, 4, strategy="otf", otf_form="factorised", memory_budget=8e9)
    assert f.plan()["otf_form"] == FACTORISED
    x = to_dev(ws.gauss_image(256, 77).astype(np.float32)[None])
    ef = rel(f.forward(x).cpu().numpy(), g.forward(x).cpu().numpy())
    ep = rel(f.psf_apply(x).cpu().numpy(), g.psf_apply(x).cpu().numpy())
    say(f"[gpu] factorised 256^2 / 200k rows vs stored G: forward {ef:.2e}, psf {ep:.2e}")
    assert ef <= FACT and ep <= FACT


@pytest.mark.parametrize("J", [5, 9])
def test_other_kaiser_bessel_supports(obs, J):
    """Kaiser-Bessel supports other than 7 (J odd in [3, 15], beta = 2.34 J): the stored
    G and the factorised form, whose expansion carries 7 taps for J <= 7 (the taps past J
    zero) and 15 above, against the FP64 oracle."""
    kw = dict(J=J, beta=2.34 * J, smax=21)
    orc = oracle_for(obs, 3, **kw)
    x = obs.sky.astype(np.float32)
    ref = orc.psf(x.astype(np.float64))
    xd = to_dev(x[None])
    g = gpu_operator(obs, 3, **kw)
    f = gpu_operator(obs, 3, strategy="otf", otf_form="factorised", memory_budget=400e6, **kw)
    assert f.plan()["otf_form"] == FACTORISED
    eg = rel(g.psf_apply(xd).cpu().numpy()[0], ref)
    ef = rel(f.psf_apply(xd).cpu().numpy()[0], ref)
    y = f.forward(xd).cpu().numpy()
    ey = rel(y, orc.forward(x.astype(np.float64)))
    say(f"[gpu] J={J}: psf rel stored G {eg:.2e}, factorised {ef:.2e}; forward {ey:.2e}")
    assert max(eg, ef, ey) <= TOL["f32"]
