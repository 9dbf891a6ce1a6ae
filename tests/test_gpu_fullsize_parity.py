"""Element-wise parity of the HIP operator with the FP64 oracle at the benchmark's
size (eq. 6-8): P = 22 w-bins as the benchmark's plan, FP32 / FP16 / BF16 storage.

  sub4096 -- the 4096^2 / 3 degree image with a seeded 300k-row subset of the 50M rows:
             the 8192-point row and column passes (two-column groups) run in full;
  crop512 -- all 50M rows on the central 512^2 crop (same cell), the protocol the
             precision configuration states for its oracle.

The oracle's values at seeded samples of 32768 pixels (Phi^dag Phi x, Phi^dag y) and
20000 rows (Phi x) were written by tests/golden/make_fullsize_parity.py (oracle only);
this test rebuilds the same seeded inputs, checks that the library clusters the w-bins
exactly as the oracle did, and compares the samples within the precision forms'
relative-L2 bounds."""
import os
import sys

import numpy as np
import pytest

import wfsynth as ws
from gpu_common import TOL, rel, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("case", ["sub4096", "crop512"])
def test_fullsize_element_wise(case):
    from paper_2605_26347_amd import Operator
    fx = np.load(os.path.join(GOLDEN, f"fullsize_{case}.npz"))
    uvw, f, n, cell = ws.fullsize_case(case)
    M = uvw.shape[0]
    pix, rows = ws.fullsize_samples(n, M)
    assert np.array_equal(pix, fx["pix"]) and np.array_equal(rows, fx["rows"])
    x = to_dev(ws.gauss_image(n, 4).astype(np.float32)[None])
    y = to_dev(ws.complex_probe(M, 5).astype(np.complex64))
    pixd = torch.from_numpy(pix).to("cuda:0")
    rowd = torch.from_numpy(rows).to("cuda:0")
    for store in ("f32", "f16", "bf16"):
        say(f"[gpu] fullsize {case}: {M} rows, {n}^2, P={ws.FULLSIZE_P}, {store}")
        op = Operator(uvw, [f], n, n, cell, nbins=ws.FULLSIZE_P, store=store)
        assert np.allclose(op.centroids(), fx["centroids"], rtol=1e-12, atol=1e-9)
        assert np.array_equal(op.bin_rows(), fx["bin_rows"])
        psf = op.psf_apply(x)[0].flatten()[pixd].cpu().numpy()
        adj = op.adjoint(y)[0].flatten()[pixd].cpu().numpy()
        fwd = op.forward(x)[rowd].cpu().numpy()
        e = (rel(psf, fx["psf"]), rel(adj, fx["adj"]), rel(fwd, fx["fwd"]))
        say(f"[gpu]   rel L2: Phi^dag Phi {e[0]:.2e}, Phi^dag {e[1]:.2e}, Phi {e[2]:.2e}")
        assert max(e) <= TOL[store], e
        op.close()
        del op
        torch.cuda.empty_cache()
