"""w-binning by 1-D k-means on a seeded data subset (oracle; test infrastructure only).

Sect. 3.1 (w-stacking): the w-bin values are the centroids of a k-means clustering
of the w components, run on a random subset; Sect. 5.2 plans on 1% of the data.
Readings (the paper leaves them open):
  * subset: row k is drawn iff SplitMix64(seed)[k] < f * 2^64 with
    f = min(1, max(fraction, 20000/M)) -- a counter-based generator (Steele, Lea &
    Flood 2014) so that any implementation draws the same rows;
  * initial centroids at the sorted subset's quantiles floor((p + 1/2) n / P);
  * Lloyd iterations until no assignment changes, at most 100; an empty cluster
    keeps its centroid; centroids are returned in ascending order;
  * assignment: bin p collects the w with mid_{p-1} < w <= mid_p, where
    mid_p = (c_p + c_{p+1}) / 2 -- the nearest centroid, ties to the lower bin.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MIN_PLAN_ROWS = 20000


def splitmix64(seed: int, idx: np.ndarray) -> np.ndarray:
    """k-th output (k = idx, 0-based) of SplitMix64 started from state `seed`:
    z = seed + (k+1)*gamma; z ^= z>>30; z *= m1; z ^= z>>27; z *= m2; z ^= z>>31."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (idx.astype(np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def plan_fraction(M: int, fraction: float) -> float:
    return min(1.0, max(fraction, MIN_PLAN_ROWS / float(M))) if M > 0 else 1.0


def plan_subset_mask(M: int, fraction: float, seed: int) -> np.ndarray:
    """Boolean mask of the rows in the planning / clustering subset."""
    f = plan_fraction(M, fraction)
    if f >= 1.0:
        return np.ones(M, dtype=bool)
    thr = np.uint64(int(f * 18446744073709551616.0))
    return splitmix64(seed, np.arange(M, dtype=np.uint64)) < thr


def assign_bins(w, centroids):
    """Bin index of every w: nearest centroid, ties to the lower bin (midpoint rule)."""
    c = np.asarray(centroids, dtype=np.float64)
    mid = 0.5 * (c[:-1] + c[1:])
    return np.searchsorted(mid, w, side="left").astype(np.int64)


def kmeans_1d(wsub, P: int, max_iter: int = 100):
    """Lloyd's algorithm in 1-D (Sect. 3.1).  Returns ascending centroids (length P)."""
    ws = np.sort(np.asarray(wsub, dtype=np.float64))
    n = ws.size
    if n == 0:
        return np.zeros(P)
    idx = np.floor(((np.arange(P, dtype=np.float64) + 0.5) * n) / P).astype(np.int64)
    c = ws[np.minimum(idx, n - 1)].copy()
    prev = None
    for _ in range(max_iter):
        a = assign_bins(ws, c)
        if prev is not None and np.array_equal(a, prev):
            break
        prev = a
        for p in range(P):
            sel = ws[a == p]
            if sel.size:
                c[p] = sel.mean()
        c = np.sort(c)
    return np.sort(c)


def kmeans_1d_optimal(w, P: int):
    """Globally optimal 1-D k-means by dynamic programming over the sorted data
    (O(P n^2)); used only to bound Lloyd's gap on small inputs.
    Returns (centroids, sse)."""
    ws = np.sort(np.asarray(w, dtype=np.float64))
    n = ws.size
    s1 = np.concatenate([[0.0], np.cumsum(ws)])
    s2 = np.concatenate([[0.0], np.cumsum(ws * ws)])

    def cost(a, b):  # sse of ws[a:b]
        cnt = b - a
        s = s1[b] - s1[a]
        return (s2[b] - s2[a]) - s * s / cnt

    INF = float("inf")
    D = np.full((P + 1, n + 1), INF)
    arg = np.zeros((P + 1, n + 1), dtype=np.int64)
    D[0, 0] = 0.0
    for k in range(1, P + 1):
        for b in range(1, n + 1):
            best, ba = INF, 0
            for a in range(k - 1, b):
                if D[k - 1, a] == INF:
                    continue
                v = D[k - 1, a] + cost(a, b)
                if v < best:
                    best, ba = v, a
            D[k, b], arg[k, b] = best, ba
    cents = []
    b = n
    for k in range(P, 0, -1):
        a = arg[k, b]
        cents.append(ws[a:b].mean())
        b = a
    return np.sort(np.array(cents)), D[P, n]
