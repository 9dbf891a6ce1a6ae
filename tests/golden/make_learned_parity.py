"""Write the oracle fixture of the learned configuration's parity checks
(tests/test_gpu_mlp.py and bench.py's learned line).

The learned configuration (a seeded 20M-row subset of the benchmark's tracks, 64-antenna
array over 16 h at 1.28 GHz, on a 4096^2 image over 3 degrees with 16 w-bins), reduced
to a seeded 2M-row subset of its rows so that the oracle finishes in minutes (its wide
residual kernels cost ~0.3 ms per row): P = 16 w-bins forced with the oracle's own
k-means centroids.  With the probe x = N(0,1) image (seed 4), the
FP64 oracle's Phi^dag Phi x (exact residual kernels) at the seeded sample of pixels of
the full-size fixtures is stored as complex64 with the sample indices, the centroids and
the row counts per bin.  Calls only oracle/ and the seeded input generators; run from
the repository root:
    python tests/golden/make_learned_parity.py
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
NBINS = 16
NROWS = 2_000_000


def run():
    t0 = time.time()
    obs = ws.learned_form(sky=False)
    uvw = np.ascontiguousarray(obs.uvw_m[ws.seeded_subset(obs.uvw_m.shape[0], NROWS, 3)])
    M = uvw.shape[0]
    # G's patches of a bin are needed twice (de-gridding, then gridding): a cache large
    # enough for one bin, emptied between bins, computes them once
    op = OracleOperator(uvw, obs.freqs_hz[0], OperatorParams(obs.nx, obs.ny, obs.cell_rad),
                        nbins=NBINS, cache_bytes=12 << 30)
    pix, _ = ws.fullsize_samples(obs.nx, M)
    x = ws.gauss_image(obs.nx, 4)
    print(f"learned: {M} rows, {obs.nx}^2, inputs {time.time() - t0:.0f} s", flush=True)
    acc = np.zeros((obs.ny, obs.nx), dtype=np.complex128)
    for p in range(op.P):            # eq. 7: the sum of the layers' Phi_p^dag Phi_p x
        if op.bin_rows[p].size:
            acc += op.psf_layer(p, x)
        op._cache.clear()         # the next bin's rows are other rows
        op._cache_used = 0
        print(f"learned: layer {p} {time.time() - t0:.0f} s", flush=True)
    psf = acc.ravel()[pix]
    print(f"learned: psf {time.time() - t0:.0f} s", flush=True)
    np.savez(os.path.join(HERE, "learned_4096sq_2M.npz"), pix=pix,
             psf=psf.astype(np.complex64), centroids=op.centroids,
             bin_rows=np.array([r.size for r in op.bin_rows], dtype=np.int64))


if __name__ == "__main__":
    run()
