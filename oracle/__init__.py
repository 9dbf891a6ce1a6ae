"""FP64 CPU oracle of the widefield measurement operator -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from this package.  The product path (the HIP
library and its Python binding) never calls into it, and the oracle shares no code,
table or constant generator with that path; the two meet only in the seeded input
generators of ``wfsynth``.

What it computes (Dabbech & Wiaux, "A distributed resource-adaptive implementation
of the widefield radio-interferometric measurement model"):

* ``directsum``  -- the discrete widefield measurement equation (Sect. 2, eq. 1-3)
                    evaluated by brute force, and its exact conjugate transpose.
* ``kernels``    -- Kaiser-Bessel interpolation taps and their closed-form Fourier
                    transform (grid correction, Sect. 3.2 / eq. 6 Z_p), w-term chirp
                    (eq. 2).
* ``wbins``      -- k-means w-binning on a seeded subset (Sect. 3.1, w-stacking).
* ``wkernel``    -- residual w-kernels: chirp sampled over twice the field, Hamming
                    taper outside it, small DFT, l2-energy hard threshold (Sect. 3.1,
                    w-projection; Fig. 1).
* ``operator``   -- Phi = [G_p F Z_p]_p (eq. 6), its adjoint, Phi^dag Phi (eq. 7-8)
                    and the holographic matrix H_p = G_p^dag G_p (Sect. 3.3), all in
                    FP64, matrix-free over row chunks.
* ``weighting``  -- Briggs robust data weights (published definition; the paper names
                    the scheme in Sect. 2 without a formula); the operator itself takes
                    per-row weights and flags (``OracleOperator(weights=, flags=)``).
* ``planner``    -- WSClean bin bound (eq. 5), memory model (eq. 9, GPU byte form),
                    cost model (eq. 10) and the decision tree (Sect. 3.4, Fig. 2).
* ``fb``         -- forward-backward iteration (Sect. 2, eq. 4) with the positivity +
                    l1 prox as denoiser, and the power iteration for its step bound.
* ``mlp``        -- (not in the paper) FP64 forward, backward and Adam step of the
                    network that predicts residual-w kernels, its input definition and
                    its training targets (thresholded exact kernels).

Pins (tests/test_oracle_*.py): brute-force direct sum, adjointness to 1e-12,
Hermitian positive semi-definiteness, w-stacking exactness on quantised w,
residual-kernel convergence towards the true-w direct sum, closed forms (delta
images, w = 0 PSF convolution), k-means against an exact dynamic programme, and
hand-computed planner values; weighted rows against the weighted direct sum, flags
against building on the kept rows, Briggs weights against a hand-computed example and
their natural / uniform limits; the forward-backward iteration against a brute-force
prox, a dense eigenvalue bound and its monotone objective.
"""
from .kernels import (kb_phi, kb_phihat, grid_correction, chirp, nm1, i0_series)  # noqa: F401
from .directsum import direct_forward, direct_adjoint, direct_matrix  # noqa: F401
from .wbins import splitmix64, plan_subset_mask, kmeans_1d, assign_bins  # noqa: F401
from .wkernel import nk_rule, wkernel_exact, threshold_shrink  # noqa: F401
from .operator import OracleOperator, OperatorParams  # noqa: F401
from .planner import p_wsclean, plan  # noqa: F401
