"""Seeded synthetic inputs for the widefield measurement operator.

This module only *generates inputs*: antenna layouts, baseline (u,v,w) tracks in
metres, channel frequencies, sky images and probe vectors.  It holds none of the
operator's arithmetic (no gridding kernel, no w-term, no FFT) and is shared by the
FP64 oracle, the tests and the benchmark so that both sides of every parity check
see bit-identical inputs.

Geometry follows the standard interferometer conventions (Thompson, Moran &
Swenson, ch. 4): planar antennas in local East/North/Up, rotated to equatorial
baseline coordinates and projected onto (u,v,w) for an hour angle H and a
declination delta.  The paper's own workload (simulated MeerKAT L-band, Sect. 5.1)
is not available; these arrays stand in for it.

Seeds: array 1, sampling 2, sky 3, probe 4, MLP 5, data weights and flags 6.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 299_792_458.0  # m/s
LAT_DEG = -30.7
DEC_DEG = -30.0

SEED_ARRAY, SEED_SAMPLING, SEED_SKY, SEED_PROBE, SEED_MLP = 1, 2, 3, 4, 5
SEED_DATA = 6


# --------------------------------------------------------------------------- array

def disc_positions(n: int, r_min: float, r_max: float, rng: np.random.Generator) -> np.ndarray:
    """n antennas uniform in area in the annulus r_min <= r <= r_max (metres), ENU with U=0."""
    u = rng.random(n)
    r = np.sqrt(r_min * r_min + u * (r_max * r_max - r_min * r_min))
    th = rng.random(n) * 2.0 * math.pi
    return np.stack([r * np.cos(th), r * np.sin(th), np.zeros(n)], axis=1)


def array_16() -> np.ndarray:
    """16 antennas uniform in a 1 km-radius disc (the tiny configuration)."""
    rng = np.random.default_rng(SEED_ARRAY)
    return disc_positions(16, 0.0, 1000.0, rng)


def array_64() -> np.ndarray:
    """64 antennas: 45 uniform in a 1 km core, 19 uniform in the 1-4 km annulus (70% core)."""
    rng = np.random.default_rng(SEED_ARRAY)
    core = disc_positions(45, 0.0, 1000.0, rng)
    outer = disc_positions(19, 1000.0, 4000.0, rng)
    return np.concatenate([core, outer], axis=0)


def enu_to_xyz(enu: np.ndarray, lat_deg: float = LAT_DEG) -> np.ndarray:
    """Local East/North/Up to equatorial (X towards H=0, Y towards H=-6h, Z to the pole)."""
    lat = math.radians(lat_deg)
    e, n, up = enu[:, 0], enu[:, 1], enu[:, 2]
    x = -math.sin(lat) * n + math.cos(lat) * up
    y = e
    z = math.cos(lat) * n + math.sin(lat) * up
    return np.stack([x, y, z], axis=1)


def baseline_vectors(xyz: np.ndarray) -> np.ndarray:
    """All antenna pairs a<b, in row-major pair order: xyz[b]-xyz[a]."""
    na = xyz.shape[0]
    a, b = np.triu_indices(na, k=1)
    return xyz[b] - xyz[a]


def uvw_tracks(bl_xyz: np.ndarray, hour_angles_rad: np.ndarray,
               dec_deg: float = DEC_DEG) -> np.ndarray:
    """(u,v,w) in metres for every (hour angle, baseline), row index = t*nbl + b."""
    dec = math.radians(dec_deg)
    sd, cd = math.sin(dec), math.cos(dec)
    sh = np.sin(hour_angles_rad)[:, None]
    ch = np.cos(hour_angles_rad)[:, None]
    lx, ly, lz = bl_xyz[None, :, 0], bl_xyz[None, :, 1], bl_xyz[None, :, 2]
    u = sh * lx + ch * ly
    v = -sd * ch * lx + sd * sh * ly + cd * lz
    w = cd * ch * lx - cd * sh * ly + sd * lz
    out = np.stack([u, v, w], axis=-1)
    return out.reshape(-1, 3)


def hour_angles(h_start: float, h_stop: float, nsteps: int) -> np.ndarray:
    """nsteps hour angles (radians) evenly spanning [h_start, h_stop] hours."""
    return np.linspace(h_start, h_stop, nsteps) * (math.pi / 12.0)


def seeded_subset(nrows: int, nkeep: int, seed: int) -> np.ndarray:
    """Sorted indices of a seeded random subset of size nkeep (without replacement)."""
    if nkeep >= nrows:
        return np.arange(nrows, dtype=np.int64)
    rng = np.random.default_rng(seed)
    idx = rng.choice(nrows, size=nkeep, replace=False)
    idx.sort()
    return idx.astype(np.int64)


# --------------------------------------------------------------------------- data weights, flags

def noise_sigma(nrows: int, seed: int = SEED_DATA) -> np.ndarray:
    """Per-visibility noise standard deviations: log-normal around 1 (spread of
    antenna system temperatures), float32."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.normal(0.0, 0.35, nrows)).astype(np.float32)


def flag_runs(nrows: int, fraction: float, seed: int = SEED_DATA + 100,
              mean_run: int = 40) -> np.ndarray:
    """Boolean flag mask with about `fraction` of the rows set, in contiguous runs of
    geometric length (mean mean_run rows), as time ranges or baselines are flagged."""
    rng = np.random.default_rng(seed)
    target = int(round(fraction * nrows))
    cover = np.zeros(nrows + 1, dtype=np.int64)   # run starts +1, run ends -1
    m = np.zeros(nrows, dtype=bool)
    count = 0
    while count < target:
        # a batch of runs sized to the remaining deficit; overlaps leave some behind
        k = max(1, (target - count) // mean_run)
        a = rng.integers(0, nrows, k)
        e = np.minimum(a + rng.geometric(1.0 / mean_run, k), nrows)
        np.add.at(cover, a, 1)
        np.add.at(cover, e, -1)
        m = np.cumsum(cover[:nrows]) > 0
        count = int(m.sum())
    return m


# --------------------------------------------------------------------------- images

def point_blob_sky(n: int, npoints: int, nblobs: int, flux_lo: float, flux_hi: float,
                   sigma_lo: float, sigma_hi: float, blob_lo: float, blob_hi: float,
                   seed: int = SEED_SKY) -> np.ndarray:
    """n x n float64 sky: npoints log-uniform point sources at uniform pixels plus
    nblobs circular Gaussians (sigma uniform in px, peak log-uniform)."""
    rng = np.random.default_rng(seed)
    x = np.zeros((n, n), dtype=np.float64)
    pj = rng.integers(0, n, npoints)
    pi = rng.integers(0, n, npoints)
    fl = np.exp(rng.uniform(math.log(flux_lo), math.log(flux_hi), npoints))
    np.add.at(x, (pj, pi), fl)
    yy, xx = np.mgrid[0:n, 0:n]
    for _ in range(nblobs):
        cj, ci = rng.uniform(0, n, 2)
        s = rng.uniform(sigma_lo, sigma_hi)
        a = math.exp(rng.uniform(math.log(blob_lo), math.log(blob_hi)))
        x += a * np.exp(-((yy - cj) ** 2 + (xx - ci) ** 2) / (2 * s * s))
    return x


def gauss_image(n: int, seed: int = SEED_PROBE) -> np.ndarray:
    """i.i.d. N(0,1) image, the dense worst-case probe."""
    return np.random.default_rng(seed).standard_normal((n, n))


def complex_probe(shape, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# --------------------------------------------------------------------------- configs

@dataclass
class Observation:
    """One synthetic observation: uvw in metres, channel frequencies, image geometry."""
    name: str
    uvw_m: np.ndarray            # [nrows, 3] float64 metres
    freqs_hz: np.ndarray         # [nchan] float64
    nx: int
    ny: int
    cell_rad: float              # direction-cosine step
    sky: np.ndarray | None = None
    chan_rows: np.ndarray | None = None   # per-channel row counts (concatenated uvw) or None
    extra: dict = field(default_factory=dict)


def tiny(n: int = 64, nant: int = 16, nsteps: int = 160, fov_deg: float = 0.5,
         freq_hz: float = 1.28e9, sky: bool = True) -> Observation:
    """The tiny configuration: 16 antennas in a 1 km disc, dec -30, one channel at
    1.28 GHz, HA -2h..+2h in 160 steps (120 baselines x 160 = 19,200 rows), a 64^2
    sky of 10 point sources (log-uniform 1e-3..1) and 2 Gaussian blobs (sigma 2-4 px)
    over a 0.5 degree field.  Smaller variants keep the recipe and shrink n/nant/nsteps."""
    rng = np.random.default_rng(SEED_ARRAY)
    enu = disc_positions(nant, 0.0, 1000.0, rng)
    bl = baseline_vectors(enu_to_xyz(enu))
    uvw = uvw_tracks(bl, hour_angles(-2.0, 2.0, nsteps))
    cell = math.radians(fov_deg) / n
    s = point_blob_sky(n, 10, 2, 1e-3, 1.0, 2.0, 4.0, 1e-2, 1e-1) if sky else None
    return Observation("tiny", uvw, np.array([freq_hz]), n, n, cell, s)


def widefield(n: int = 1024, nvis: int = 2_000_000, fov_deg: float = 2.0,
              hours: float = 8.0, dt_s: float = 8.0, freq_hz: float = 1.28e9,
              npoints: int = 300, nblobs: int = 10, blob_sigma=(2.0, 8.0),
              sky: bool = True) -> Observation:
    """64-antenna array (70% in a 1 km core, the rest to 4 km), HA -hours/2..+hours/2 in
    dt_s steps, thinned to a seeded subset of nvis rows at one channel."""
    bl = baseline_vectors(enu_to_xyz(array_64()))
    nsteps = int(round(hours * 3600.0 / dt_s))
    uvw = uvw_tracks(bl, hour_angles(-hours / 2, hours / 2, nsteps))
    if nvis < uvw.shape[0]:
        uvw = uvw[seeded_subset(uvw.shape[0], nvis, SEED_SAMPLING)]
    cell = math.radians(fov_deg) / n
    s = None
    if sky:
        s = point_blob_sky(n, npoints, nblobs, 1e-4, 1.0, blob_sigma[0], blob_sigma[1],
                           1e-3, 1e-1)
    return Observation("widefield", np.ascontiguousarray(uvw), np.array([freq_hz]),
                       n, n, cell, s)


def precision_form(n: int = 4096, nvis: int = 50_000_000, fov_deg: float = 3.0,
                   sky: bool = True) -> Observation:
    """4096^2 over 3 degrees, 50M rows: the 64-antenna array over 16 h (HA -8..+8 h) in
    24,802 steps (2016 x 24,802 = 50,000,832 rows), 832 seeded rows dropped."""
    bl = baseline_vectors(enu_to_xyz(array_64()))
    nsteps = 24_802
    uvw = uvw_tracks(bl, hour_angles(-8.0, 8.0, nsteps))
    if nvis < uvw.shape[0]:
        uvw = uvw[seeded_subset(uvw.shape[0], nvis, SEED_SAMPLING)]
    cell = math.radians(fov_deg) / n
    s = None
    if sky:
        s = point_blob_sky(n, 2000, 50, 1e-4, 1.0, 2.0, 16.0, 1e-3, 1e-1)
    return Observation("precision", np.ascontiguousarray(uvw), np.array([1.28e9]),
                       n, n, cell, s)


FULLSIZE_P = 22            # w-bins of the benchmark's plan, forced in the parity cases
FULLSIZE_NPIX = 32768      # sampled output pixels of the full-size parity cases
FULLSIZE_NROWS = 20000     # sampled visibilities of the full-size parity cases


def fullsize_case(name: str):
    """Inputs of the full-size parity cases of the precision form, (uvw_m, freq_hz, n,
    cell_rad): 'crop512' = all 50M rows on the central 512^2 of the 4096^2 / 3 degree image
    (same cell); 'sub4096' = the full 4096^2 image with a seeded 300k-row subset."""
    obs = precision_form(sky=False)
    if name == "crop512":
        return obs.uvw_m, float(obs.freqs_hz[0]), 512, obs.cell_rad
    if name != "sub4096":
        raise ValueError(name)
    rows = seeded_subset(obs.uvw_m.shape[0], 300_000, 7)
    return np.ascontiguousarray(obs.uvw_m[rows]), float(obs.freqs_hz[0]), 4096, obs.cell_rad


def fullsize_samples(n: int, nrows: int):
    """Seeded sorted samples of output pixels (flat [ny*nx] indices) and of rows."""
    rng = np.random.default_rng(11)
    pix = np.sort(rng.choice(n * n, FULLSIZE_NPIX, replace=False))
    rows = np.sort(rng.choice(nrows, FULLSIZE_NROWS, replace=False))
    return pix, rows


def learned_form(n: int = 4096, nvis: int = 20_000_000, fov_deg: float = 3.0,
                 sky: bool = True) -> Observation:
    """4096^2 over 3 degrees, 20M rows: a seeded subset of the 16 h sample set of the
    64-antenna array (the precision form's tracks)."""
    o = precision_form(n, 50_000_000, fov_deg, sky)
    uvw = o.uvw_m[seeded_subset(o.uvw_m.shape[0], nvis, SEED_SAMPLING + 7)]
    return Observation("learned", np.ascontiguousarray(uvw), o.freqs_hz, n, n, o.cell_rad,
                       o.sky)


def kernel_examples(wproj_pool: np.ndarray, n: int, seed: int = SEED_MLP,
                    fovs_deg=(1.0, 2.0, 3.0, 4.0)):
    """Training examples of the residual-kernel network: residual w drawn (seeded, with
    replacement) from a pool, field side uniform over fovs_deg (as nx cell, radians),
    cell offsets uniform in [-1/2, 1/2).  Returns (w, L, fu, fv) float64 arrays."""
    rng = np.random.default_rng(seed)
    w = np.asarray(wproj_pool, dtype=np.float64)[rng.integers(0, len(wproj_pool), n)]
    L = np.radians(rng.choice(np.asarray(fovs_deg, dtype=np.float64), n))
    return w, L, rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n)


def batched_counts(nchan: int = 16, total: int = 48_000_000, lo: float = 0.5e6,
                   hi: float = 6e6, seed: int = SEED_SAMPLING) -> np.ndarray:
    """Seeded log-uniform per-channel counts in [lo, hi], rescaled (clamped,
    integer-fixed) to sum exactly to total."""
    rng = np.random.default_rng(seed + 100)
    c = np.exp(rng.uniform(math.log(lo), math.log(hi), nchan))
    c = c * (total / c.sum())
    c = np.clip(c, lo, hi)
    c = np.floor(c).astype(np.int64)
    i = 0
    while c.sum() != total:
        d = total - int(c.sum())
        step = 1 if d > 0 else -1
        j = i % nchan
        if lo <= c[j] + step <= hi:
            c[j] += step
        i += 1
    return c


def batched(n: int = 2048, nchan: int = 16, total: int = 48_000_000,
            f_lo: float = 0.9e9, f_hi: float = 1.67e9, fov_deg: float = 3.0,
            hours: float = 16.0, dt_s: float = 8.0, lo: float = 0.5e6,
            hi: float = 6e6) -> Observation:
    """16 channels over 0.9-1.67 GHz with uneven row counts (log-uniform, summing to
    48M); each channel is a seeded subset of the 16 h / 8 s sample set."""
    bl = baseline_vectors(enu_to_xyz(array_64()))
    nsteps = int(round(hours * 3600.0 / dt_s))
    full = uvw_tracks(bl, hour_angles(-hours / 2, hours / 2, nsteps))
    counts = batched_counts(nchan, total, lo, hi)
    blocks = [full[seeded_subset(full.shape[0], int(m), SEED_SAMPLING + 1000 + c)]
              for c, m in enumerate(counts)]
    uvw = np.ascontiguousarray(np.concatenate(blocks, axis=0))
    freqs = np.linspace(f_lo, f_hi, nchan)
    cell = math.radians(fov_deg) / n
    return Observation("batched", uvw, freqs, n, n, cell, None, chan_rows=counts)
