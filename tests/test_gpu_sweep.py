"""Layer-batched sweep (wf_set_sweep): every stage of an apply as one launch over all
(channel, bin) layers -- the row kernels as one persistent launch per patch class
draining the items of every layer, the inverse row pass summing each channel's layers
in registers.  Compared with the branch apply of the same operator (only the order of
FP32 additions differs: relative L2 <= 2e-6; the forward apply is bit-identical), with
the FP64 oracle per channel (FP32 storage, 1e-5), under graph capture and replay, and
for its per-channel completion stamps."""
import sys

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
def wide3():
    # three channels of a 1024^2 / 2 degree image (grid 2048^2), uneven rows, one empty
    base = ws.widefield(n=1024, nvis=40_000, fov_deg=2.0, sky=False)
    counts = np.array([14_000, 0, 22_000])
    uvw = np.ascontiguousarray(base.uvw_m[:counts.sum()])
    return ws.Observation("sweep3", uvw, np.array([0.95e9, 1.2e9, 1.45e9]), 1024, 1024,
                          base.cell_rad, None, chan_rows=counts)


@pytest.fixture(scope="module")
def imgs(wide3):
    return np.stack([ws.gauss_image(1024, 20 + c) for c in range(3)]).astype(np.float32)


def _vis(m, seed=4):
    r = np.random.default_rng(seed)
    return (r.standard_normal(m) + 1j * r.standard_normal(m)).astype(np.complex64)


def test_sweep_matches_branches_and_oracle(wide3, imgs):
    say("[gpu] sweep: 3 channels x 1024^2, P=3")
    op = gpu_operator(wide3, 3, branches=2)
    x = to_dev(imgs)
    M = int(wide3.chan_rows.sum())
    v = to_dev(_vis(M))
    ref = {"psf": op.psf_apply(x).cpu().numpy(), "psf_re": op.psf_apply_re(x).cpu().numpy(),
           "fwd": op.forward(x).cpu().numpy(), "adj": op.adjoint(v).cpu().numpy()}
    op.set_sweep(True)
    got = {"psf": op.psf_apply(x).cpu().numpy(), "psf_re": op.psf_apply_re(x).cpu().numpy(),
           "fwd": op.forward(x).cpu().numpy(), "adj": op.adjoint(v).cpu().numpy()}
    for k in ("psf", "psf_re", "adj"):
        e = rel(got[k], ref[k])
        say(f"[gpu]   sweep {k} vs branches {e:.2e}")
        assert e <= SAME, k
    assert np.array_equal(got["fwd"], ref["fwd"])
    assert np.all(got["psf"][1] == 0) and np.all(got["adj"][1] == 0)   # channel without rows
    off = 0
    for c in (0, 2):
        if c == 2:
            off = int(wide3.chan_rows[0])
        orc = oracle_for(wide3, 3, chan=c,
                         uvw=wide3.uvw_m[off:off + int(wide3.chan_rows[c])])
        e = rel(got["psf"][c], orc.psf(imgs[c].astype(np.float64)))
        say(f"[gpu]   sweep channel {c} psf vs oracle {e:.2e}")
        assert e <= TOL["f32"]
    op.set_sweep(False)
    assert rel(op.psf_apply(x).cpu().numpy(), ref["psf"]) <= SAME
    op.close()


def test_sweep_graph_replays_and_stamps(wide3, imgs):
    op = gpu_operator(wide3, 3, store="f16")
    x = to_dev(imgs)
    op.set_sweep(True)
    eager = op.psf_apply_re(x).cpu().numpy()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    out = torch.empty_like(x)
    g = op.capture("psf_re", x, out, s)
    other = torch.empty((3, 1024, 1024), dtype=torch.complex64, device="cuda:0")
    for rep in range(3):
        with torch.cuda.stream(s):
            out.fill_(float("nan"))
        g.launch(s)
        s.synchronize()
        e = rel(out.cpu().numpy(), eager)
        say(f"[gpu]   sweep graph replay {rep}: {e:.2e}")
        assert e <= SAME
        op.psf_apply(x, out=other)        # eager work on the same grids between replays
        torch.cuda.synchronize()
    g.close()
    op.latency_enable(True)
    op.psf_apply_re(x, out=out)
    torch.cuda.synchronize()
    lat = op.read_latency()
    say(f"[gpu]   sweep completion (ms): {lat}")
    assert np.all(np.isfinite(lat)) and np.all(lat > 0)
    op.close()


@pytest.mark.parametrize("lanes", [2, 3])
def test_sweep_lanes(wide3, imgs, lanes):
    """The sweep on several lanes (channel ranges on streams of their own, each lane
    starting once the previous one has issued its forward passes): same results as the
    branch apply, eager and as a replayed graph, with per-channel stamps."""
    say(f"[gpu] sweep on {lanes} lanes: 3 channels x 1024^2, P=3")
    op = gpu_operator(wide3, 3, store="f16")
    x = to_dev(imgs)
    M = int(wide3.chan_rows.sum())
    v = to_dev(_vis(M))
    ref = {"psf_re": op.psf_apply_re(x).cpu().numpy(), "fwd": op.forward(x).cpu().numpy(),
           "adj": op.adjoint(v).cpu().numpy()}
    op.set_sweep(True, lanes=lanes)
    got = {"psf_re": op.psf_apply_re(x).cpu().numpy(), "fwd": op.forward(x).cpu().numpy(),
           "adj": op.adjoint(v).cpu().numpy()}
    for k in ("psf_re", "adj"):
        e = rel(got[k], ref[k])
        say(f"[gpu]   {lanes} lanes {k} vs branches {e:.2e}")
        assert e <= SAME, k
    assert np.array_equal(got["fwd"], ref["fwd"])
    s = torch.cuda.Stream()
    out = torch.empty_like(x)
    op.latency_enable(True)
    g = op.capture("psf_re", x, out, s)
    k, n = g.nodes()
    say(f"[gpu]   {lanes} lanes: graph of {k} kernel nodes ({n} nodes)")
    for rep in range(2):
        with torch.cuda.stream(s):
            out.fill_(float("nan"))
        g.launch(s)
        s.synchronize()
        assert rel(out.cpu().numpy(), ref["psf_re"]) <= SAME
        op.forward(x)                     # eager work between replays
        torch.cuda.synchronize()
    lat = op.read_latency()
    assert np.all(np.isfinite(lat)) and np.all(lat > 0)
    g.close()
    op.close()


def test_sweep_needs_long_grids():
    from paper_2605_26347_amd._lib import WfError
    obs = ws.tiny(n=64, nant=8, nsteps=20, fov_deg=2.0, sky=False)
    op = gpu_operator(obs, 2)
    with pytest.raises(WfError, match="sweep"):
        op.set_sweep(True)
    op.close()
