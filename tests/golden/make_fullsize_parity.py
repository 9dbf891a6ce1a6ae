"""Write the oracle fixtures of the full-size parity tests (tests/test_gpu_fullsize_parity.py).

Two cases of the benchmark's setup (64-antenna array over 16 h at 1.28 GHz, a 3 degree
field at 4096^2, i.e. a cell of 3 deg / 4096), both with P = 22 w-bins forced (the
planner's choice for the benchmark) and the oracle's own k-means centroids:
  crop512  -- all 50M rows on the central 512^2 crop of the image (same cell, 0.375
              degree field), the protocol the precision configuration states for its
              oracle;
  sub4096  -- the full 4096^2 image (grid 8192^2) with a seeded 300k-row subset of the
              50M rows, so that the 8192-point transforms run in full.
For each case, with the probe x = N(0,1) image (seed 4) and y = complex N(0,1) data
(seed 5), the FP64 oracle's Phi^dag Phi x and Phi^dag y at a seeded sample of pixels
and Phi x at a seeded sample of rows are stored as complex64 (rounding below 1e-7 of
each value) with the sample indices, the centroids and the row counts per bin.
Calls only oracle/ and the seeded input generators; run from the repository root:
    python tests/golden/make_fullsize_parity.py [crop512|sub4096]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import wfsynth as ws  # noqa: E402
from oracle import OracleOperator, OperatorParams  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def run(name):
    t0 = time.time()
    uvw, f, n, cell = ws.fullsize_case(name)
    M = uvw.shape[0]
    op = OracleOperator(uvw, f, OperatorParams(n, n, cell), nbins=ws.FULLSIZE_P)
    pix, rows = ws.fullsize_samples(n, M)
    x = ws.gauss_image(n, 4)
    y = ws.complex_probe(M, 5)
    print(f"{name}: {M} rows, {n}^2, inputs {time.time() - t0:.0f} s", flush=True)
    psf = op.psf(x).ravel()[pix]
    print(f"{name}: psf {time.time() - t0:.0f} s", flush=True)
    adj = op.adjoint(y).ravel()[pix]
    print(f"{name}: adjoint {time.time() - t0:.0f} s", flush=True)
    fwd = op.forward(x)[rows]
    print(f"{name}: forward {time.time() - t0:.0f} s", flush=True)
    np.savez(os.path.join(HERE, f"fullsize_{name}.npz"), pix=pix, rows=rows,
             psf=psf.astype(np.complex64), adj=adj.astype(np.complex64),
             fwd=fwd.astype(np.complex64), centroids=op.centroids,
             bin_rows=np.array([r.size for r in op.bin_rows], dtype=np.int64))


if __name__ == "__main__":
    for nm in (sys.argv[1:] or ["sub4096", "crop512"]):
        run(nm)
