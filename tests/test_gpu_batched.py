"""Batched form of the operator through the C ABI: channels (or one channel's w-bins) on
concurrent branches, applies captured into HIP graphs, per-channel completion stamps
and the work-item autotuner.

Each result is compared with the one-branch eager apply of the same operator (only the
order of FP32 additions may differ: relative L2 <= 2e-6; the forward apply, which has
no cross-branch sum, must be bit-identical) and with the FP64 oracle per channel
(FP32 storage: 1e-5).
"""
import sys
import time

import numpy as np
import pytest

import wfsynth as ws
from gpu_common import TOL, rel, oracle_for, gpu_operator, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SAME = 2e-6


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def wb():
    # five channels over 0.9-1.67 GHz on one 64^2 / 3 degree image, uneven row counts
    # and one channel without rows
    base = ws.widefield(n=64, nvis=40_000, fov_deg=3.0, sky=False)
    counts = np.array([9_000, 0, 14_000, 3_000, 14_000])
    uvw = np.ascontiguousarray(base.uvw_m[:counts.sum()])
    return ws.Observation("wideband", uvw, np.linspace(0.9e9, 1.67e9, 5), 64, 64,
                          base.cell_rad, None, chan_rows=counts)


@pytest.fixture(scope="module")
def wb_images(wb):
    return np.stack([ws.gauss_image(64, 10 + c) for c in range(5)]).astype(np.float32)


@pytest.fixture(scope="module")
def wb_ops(wb):
    say("[gpu] build wideband 5 x 64^2, branches 1 and 3")
    return gpu_operator(wb, 3, branches=1), gpu_operator(wb, 3, branches=3)


def _vis(m, seed=3):
    r = np.random.default_rng(seed)
    return (r.standard_normal(m) + 1j * r.standard_normal(m)).astype(np.complex64)


def _nan_like(shape, dtype):
    return torch.full(shape, float("nan"), dtype=dtype, device="cuda:0")


def test_branches_match_one_branch(wb, wb_images, wb_ops):
    op1, op3 = wb_ops
    assert [op3.plan(c)["branch"] for c in (0, 2, 3, 4)] != [0, 0, 0, 0]
    x = to_dev(wb_images)
    shp = (5, 64, 64)
    for name in ("psf_apply", "psf_apply_re"):
        dt = torch.float32 if name.endswith("re") else torch.complex64
        a = getattr(op1, name)(x, out=_nan_like(shp, dt)).cpu().numpy()
        b = getattr(op3, name)(x, out=_nan_like(shp, dt)).cpu().numpy()
        assert np.all(b[1] == 0), "channel without rows must be zero-filled"
        e = rel(b, a)
        say(f"[gpu] {name} 3 branches vs 1: {e:.2e}")
        assert e <= SAME
    y1 = op1.forward(x).cpu().numpy()
    y3 = op3.forward(x).cpu().numpy()
    assert np.array_equal(y1, y3)
    v = to_dev(_vis(int(wb.chan_rows.sum())))
    a1 = op1.adjoint(v).cpu().numpy()
    a3 = op3.adjoint(v, out=_nan_like(shp, torch.complex64)).cpu().numpy()
    assert np.all(a3[1] == 0)
    assert rel(a3, a1) <= SAME


def test_branches_match_oracle(wb, wb_images, wb_ops):
    _, op3 = wb_ops
    x = to_dev(wb_images)
    out = op3.psf_apply(x).cpu().numpy()
    y = op3.forward(x).cpu().numpy()
    off = 0
    for c, m in enumerate(wb.chan_rows):
        if m == 0:
            continue
        orc = oracle_for(wb, 3, chan=c, uvw=wb.uvw_m[off:off + m])
        e = rel(out[c], orc.psf(wb_images[c].astype(np.float64)))
        ef = rel(y[off:off + m], orc.forward(wb_images[c].astype(np.float64)))
        say(f"[gpu] chan {c} psf rel {e:.2e} forward rel {ef:.2e}")
        assert e <= TOL["f32"] and ef <= TOL["f32"]
        off += m


def test_single_channel_bin_split():
    """One channel whose w-bins run on three branches with partial-sum accumulators."""
    obs = ws.widefield(n=128, nvis=24_000, fov_deg=4.0, npoints=40, nblobs=3,
                       blob_sigma=(1.0, 3.0))
    op = gpu_operator(obs, 5)
    x = to_dev(obs.sky.astype(np.float32)[None])
    v = to_dev(_vis(obs.uvw_m.shape[0]))
    ref = [op.psf_apply(x).cpu().numpy(), op.psf_apply_re(x).cpu().numpy(),
           op.forward(x).cpu().numpy(), op.adjoint(v).cpu().numpy()]
    op.set_branches(3)
    got = [op.psf_apply(x).cpu().numpy(), op.psf_apply_re(x).cpu().numpy(),
           op.forward(x).cpu().numpy(), op.adjoint(v).cpu().numpy()]
    for k in (0, 1, 3):
        say(f"[gpu] split bins, result {k}: {rel(got[k], ref[k]):.2e}")
        assert rel(got[k], ref[k]) <= SAME
    assert np.array_equal(got[2], ref[2])
    orc = oracle_for(obs, 5)
    assert rel(got[0][0], orc.psf(obs.sky.astype(np.float64))) <= TOL["f32"]
    op.set_branches(1)
    assert rel(op.psf_apply(x).cpu().numpy(), ref[0]) <= SAME


@pytest.mark.parametrize("branches", [1, 3])
def test_graph_replays_match_eager(wb, wb_images, branches):
    op = gpu_operator(wb, 3, branches=branches)
    x = to_dev(wb_images)
    v = to_dev(_vis(int(wb.chan_rows.sum()), 5))
    shp = (5, 64, 64)
    eager = {"psf_re": op.psf_apply_re(x).cpu().numpy(),
             "adjoint": op.adjoint(v).cpu().numpy(),
             "forward": op.forward(x).cpu().numpy()}
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    outs = {"psf_re": torch.empty(shp, dtype=torch.float32, device="cuda:0"),
            "adjoint": torch.empty(shp, dtype=torch.complex64, device="cuda:0"),
            "forward": torch.empty(int(wb.chan_rows.sum()), dtype=torch.complex64,
                                   device="cuda:0")}
    ins = {"psf_re": x, "adjoint": v, "forward": x}
    graphs = {k: op.capture(k, ins[k], outs[k], s) for k in outs}
    other = torch.empty(shp, dtype=torch.complex64, device="cuda:0")
    for rep in range(3):
        for k, g in graphs.items():
            with torch.cuda.stream(s):
                outs[k].fill_(float("nan"))
            g.launch(s)
            s.synchronize()
            got = outs[k].cpu().numpy()
            if k == "forward":
                assert np.array_equal(got, eager[k]), (rep, k)
            else:
                e = rel(got, eager[k])
                say(f"[gpu] graph {k} replay {rep} (branches {branches}): {e:.2e}")
                assert e <= SAME, (rep, k)
            # the program's own eager work between replays, on the same grids
            op.psf_apply(x, out=other)
            other.mul_(0.5)
            torch.cuda.synchronize()
    for g in graphs.values():
        g.close()


def test_graph_needs_created_stream(wb, wb_images, wb_ops):
    from paper_2605_26347_amd._lib import WfError
    _, op3 = wb_ops
    x = to_dev(wb_images)
    out = torch.empty_like(x)

    class Null:
        cuda_stream = 0
    with pytest.raises(WfError):
        op3.capture("psf_re", x, out, Null())


def test_latency_stamps(wb, wb_images):
    op = gpu_operator(wb, 3, branches=2)
    x = to_dev(wb_images)
    out = torch.empty_like(x)
    op.latency_enable(True)
    op.psf_apply_re(x, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op.psf_apply_re(x, out=out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    lat = op.read_latency()
    say(f"[gpu] latency ms {np.round(lat, 3)} wall {wall:.2f}")
    assert np.all(np.isfinite(lat)) and np.all(lat >= 0)
    assert lat.max() <= wall + 0.5
    s = torch.cuda.Stream()
    g = op.capture("psf_re", x, out, s)
    g.launch(s)
    s.synchronize()
    lat2 = op.read_latency()
    assert np.all(lat2 >= 0) and lat2.max() > 0
    g.close()


def test_autotune_keeps_results(wb, wb_images):
    from paper_2605_26347_amd._lib import WfError
    op = gpu_operator(wb, 3, max_rows_per_item=64, branches=1)
    x = to_dev(wb_images)
    ref = op.psf_apply(x).cpu().numpy()
    yref = op.forward(x).cpu().numpy()
    nwork0 = [op.plan(c)["nwork"] for c in range(5)]
    s = torch.cuda.Stream()
    out = torch.empty_like(x)
    g = op.capture("psf_re", x, out, s)
    info = op.autotune(x, out, reps=1)
    say(f"[gpu] autotune {info}")
    assert info["branches"] in (1, 2, 4)
    assert info["retuned_chans"] == 4
    for c in (0, 2, 3, 4):
        p = op.plan(c)
        assert p["max_rows_per_item"] in (256, 512, 1024)
        assert p["nwork"] <= nwork0[c]
    with pytest.raises(WfError):
        g.launch(s)
    g.close()
    assert rel(op.psf_apply(x).cpu().numpy(), ref) <= SAME
    assert np.array_equal(op.forward(x).cpu().numpy(), yref)
