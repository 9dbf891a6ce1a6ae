"""Work-item tile side per bin (wf_set_bin_tiles / wf_get_bin_tiles, and the autotuner's
choice): items over 2 x 2 base tiles re-split the stored rows and rewrite their patch
words, never their values.  Phi is then bit-identical (each row gathers the same grid
cells in the same order), Phi^dag and Phi^dag Phi differ only in the order of FP32
additions (relative L2 <= 2e-6), in the branch apply and in the layer-batched sweep, and
Phi^dag Phi stays within the FP32 tolerance of the FP64 oracle (eq. 7-8)."""
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
def wide():
    # one channel of a 1024^2 / 2 degree image (grid 2048^2), 3 bins, every patch class
    return ws.widefield(n=1024, nvis=40_000, fov_deg=2.0, sky=False)


def _vis(m, seed=6):
    r = np.random.default_rng(seed)
    return (r.standard_normal(m) + 1j * r.standard_normal(m)).astype(np.complex64)


def _applies(op, x, v):
    return {"psf": op.psf_apply(x).cpu().numpy(), "fwd": op.forward(x).cpu().numpy(),
            "adj": op.adjoint(v).cpu().numpy()}


def _same(got, ref, label):
    for k in ("psf", "adj"):
        e = rel(got[k], ref[k])
        say(f"[gpu]   {label} {k} vs base tiles {e:.2e}")
        assert e <= SAME, (label, k)
    assert np.array_equal(got["fwd"], ref["fwd"]), label


@pytest.mark.parametrize("store", ["f32", "f16"])
def test_wide_items_match_base_tiles_and_oracle(wide, store):
    say(f"[gpu] bin tiles: 1024^2, 40000 rows, P=3, {store}")
    op = gpu_operator(wide, 3, store=store)
    assert list(op.bin_tiles()) == [32, 32, 32]
    x = to_dev(ws.gauss_image(1024, 8).astype(np.float32)[None])
    v = to_dev(_vis(wide.uvw_m.shape[0]))
    ref = _applies(op, x, v)
    op.set_bin_tiles([64, 32, 64])
    assert list(op.bin_tiles()) == [64, 32, 64]
    _same(_applies(op, x, v), ref, "tiles 64/32/64")
    op.set_bin_tiles([64, 64, 64])
    wide_all = _applies(op, x, v)
    _same(wide_all, ref, "tiles 64")
    if store == "f32":
        orc = oracle_for(wide, 3)
        e = rel(wide_all["psf"][0], orc.psf(ws.gauss_image(1024, 8)))
        say(f"[gpu]   tiles 64 psf vs oracle {e:.2e}")
        assert e <= TOL["f32"]
    # the sweep's item lists follow the tiles
    op.set_sweep(True)
    _same(_applies(op, x, v), ref, "sweep, tiles 64")
    op.set_bin_tiles([32, 64, 32])
    _same(_applies(op, x, v), ref, "sweep, tiles 32/64/32")
    op.set_sweep(False)
    op.set_bin_tiles([32, 32, 32])
    _same(_applies(op, x, v), ref, "back to base tiles")
    op.close()


def test_autotuner_picks_tiles(wide):
    op = gpu_operator(wide, 3, store="f16")
    x = to_dev(ws.gauss_image(1024, 8).astype(np.float32)[None])
    out = torch.empty_like(x)
    ref = op.psf_apply_re(x).cpu().numpy()
    tune = op.autotune(x, out, reps=2)
    tiles = op.bin_tiles()
    say(f"[gpu] autotune {tune}, tiles {list(tiles)}")
    assert set(tiles.tolist()) <= {32, 64}
    assert tune["wide_tile_bins"] == int((tiles == 64).sum())
    assert rel(op.psf_apply_re(x).cpu().numpy(), ref) <= SAME
    op.close()


def test_bin_tile_arguments(wide):
    from paper_2605_26347_amd import _lib
    op = gpu_operator(wide, 3)
    with pytest.raises(_lib.WfError, match="tile"):
        op.set_bin_tiles([48, 32, 32])
    with pytest.raises(_lib.WfError, match="one entry per bin"):
        op.set_bin_tiles([32, 32])
    with pytest.raises(_lib.WfError, match="bad channel"):
        op.set_bin_tiles([32, 32, 32], chan=3)
    assert list(op.bin_tiles()) == [32, 32, 32]
    op.close()
