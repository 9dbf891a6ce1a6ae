"""Compute-resource planning (oracle; test infrastructure only).

Sect. 3.1 eq. 5: WSClean's uniform-bin rule P >= 2 pi (w_max - w_min) max_Omega(1 - n),
used as the upper end of the search over P.
Sect. 3.4 eq. 9: memory of G; the MATLAB constants (24 B per non-zero, 4 N') are
re-derived for the GPU formats: b_v bytes per stored value (8 complex FP32, 4 complex
FP16/BF16), 12 B per row (packed patch origin, value offset, caller-order index) and
the per-bin work grids 8 (2 N' + ny Kx + nx ny).
Sect. 3.4 eq. 10: c(P) ~= 2 (10 N' log2 sqrt(N') P + 6 K(P)).
Sect. 3.4 and Fig. 2: (a) precompute G at the minimiser P* of c, or at the feasible P
closest to it; (b) otherwise precompute H at the P where m_G stabilises (within 5% of
its large-P asymptote b_v M J^2 + ...) if m_H fits; (c) otherwise compute G on the fly.
m* = budget_fraction * memory budget (65%, Sect. 5.2).  K(P) is estimated from the
planning subset (1% of the rows, Sect. 5.2) with the kernel-side rule uncapped; a P is
feasible only if m_G fits and at least 99% of the subset rows need n_k <= S_max (the
kernel-side cap is an implementation limit; the paper has none).
"""
from __future__ import annotations

import math

import numpy as np

from . import wbins
from .wkernel import nk_rule

STORE_BYTES = {"f32": 8, "f16": 4, "bf16": 4}
ROW_BYTES = 12
OK_FRACTION = 0.99
STABLE_FACTOR = 1.05


def p_wsclean(wmin: float, wmax: float, nx: int, ny: int, cell: float) -> float:
    """Right-hand side of eq. 5 over the image's field (largest |l|, |m| at pixel 0)."""
    lmax = (nx // 2) * cell
    mmax = (ny // 2) * cell
    return 2.0 * math.pi * (wmax - wmin) * (1.0 - math.sqrt(1.0 - lmax * lmax - mmax * mmax))


def grid_bytes(nx, ny, o=2):
    Kx, Ky = o * nx, o * ny
    return 8 * (2 * Kx * Ky + ny * Kx + nx * ny)


def mem_G(K: float, M: int, nx: int, ny: int, store: str = "f32", o: int = 2) -> float:
    """GPU form of eq. 9."""
    return STORE_BYTES[store] * K + ROW_BYTES * M + grid_bytes(nx, ny, o)


def cost(P: int, K: float, nx: int, ny: int, o: int = 2) -> float:
    """eq. 10."""
    Np = (o * nx) * (o * ny)
    return 2.0 * (10.0 * Np * math.log2(math.sqrt(Np)) * P + 6.0 * K)


def k_of_p(wsub, M: int, P: int, nx, ny, cell, J=7, o=2, alpha=2.0, smax=31):
    """(K(P) estimate scaled to M rows, fraction of subset rows with n_k <= smax, centroids)."""
    c = wbins.kmeans_1d(wsub, P)
    b = wbins.assign_bins(wsub, c)
    wproj = wsub - c[b]
    nk = nk_rule(wproj, nx * cell, ny * cell, o, alpha, None)
    T = nk + J - 1
    K = float(np.sum(T.astype(np.float64) ** 2)) * (M / wsub.size)
    ok = float(np.mean(nk <= smax))
    return K, ok, c


def plan(w_lambda, nx, ny, cell, memory_budget, store="f32", J=7, o=2, alpha=2.0, smax=31,
         plan_fraction=0.01, budget_fraction=0.65, seed=0, m_H=None, p_max=None):
    """Decision tree of Sect. 3.4.  w_lambda: all rows' w in wavelengths.
    m_H: optional callable P -> bytes of the holographic matrix.  Returns a dict."""
    M = w_lambda.size
    mask = wbins.plan_subset_mask(M, plan_fraction, seed)
    wsub = w_lambda[mask]
    pw = p_wsclean(float(w_lambda.min()), float(w_lambda.max()), nx, ny, cell)
    Pmax = max(1, int(math.ceil(pw))) if p_max is None else p_max
    table = []
    for P in range(1, Pmax + 1):
        K, ok, _ = k_of_p(wsub, M, P, nx, ny, cell, J, o, alpha, smax)
        table.append((P, K, ok, mem_G(K, M, nx, ny, store, o), cost(P, K, nx, ny, o)))
    mstar = budget_fraction * memory_budget
    Pstar = min(table, key=lambda r: (r[4], r[0]))[0]
    feas = [r for r in table if r[3] <= mstar and r[2] >= OK_FRACTION]
    out = {"P_wsclean": pw, "P_max": Pmax, "P_star": Pstar, "table": table, "m_star": mstar}
    if feas:
        best = min(feas, key=lambda r: (abs(r[0] - Pstar), r[4]))
        out.update(strategy="G", P=best[0])
        return out
    m_inf = STORE_BYTES[store] * M * J * J + ROW_BYTES * M + grid_bytes(nx, ny, o)
    stab = [r for r in table if r[3] <= STABLE_FACTOR * m_inf]
    Pbar = stab[0][0] if stab else Pmax
    mh = m_H(Pbar) if m_H is not None else float("inf")
    out.update(P=Pbar, m_H=mh, strategy="H" if mh <= mstar else "otf")
    return out
