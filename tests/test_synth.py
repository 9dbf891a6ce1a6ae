"""The seeded input generators shared by the oracle, the tests and the benchmark.

They hold none of the operator's arithmetic; these checks pin them to the textbook
interferometer geometry (Thompson, Moran & Swenson, ch. 4) and to the recipes the
workloads are stated with: sizes, seeded determinism, distributions of the noise levels,
flag runs and per-channel row counts."""
import math

import numpy as np
import pytest

import wfsynth as ws


def test_enu_and_uvw_are_rotations():
    rng = np.random.default_rng(11)
    enu = rng.normal(0, 1000, (50, 3))
    xyz = ws.enu_to_xyz(enu)
    assert np.allclose(np.linalg.norm(xyz, axis=1), np.linalg.norm(enu, axis=1), rtol=1e-13)
    H = ws.hour_angles(-6, 6, 7)
    uvw = ws.uvw_tracks(xyz, H).reshape(7, 50, 3)
    assert np.allclose(np.linalg.norm(uvw, axis=2), np.linalg.norm(xyz, axis=1)[None],
                       rtol=1e-13)


def test_uvw_special_cases():
    L = 1234.5
    H = np.linspace(-math.pi, math.pi, 25)
    # pole: w is the polar component at every hour angle
    b = np.array([[300.0, -200.0, 700.0]])
    assert np.allclose(ws.uvw_tracks(b, H, dec_deg=90.0)[:, 2], 700.0, rtol=1e-13)
    # east-west baseline: the (u, v) track is the ellipse u^2 + (v / sin dec)^2 = L^2
    # and w = -L cos(dec) sin(H)
    dec = -30.0
    t = ws.uvw_tracks(np.array([[0.0, L, 0.0]]), H, dec_deg=dec)
    sd, cd = math.sin(math.radians(dec)), math.cos(math.radians(dec))
    assert np.allclose(t[:, 0] ** 2 + (t[:, 1] / sd) ** 2, L * L, rtol=1e-12)
    assert np.allclose(t[:, 2], -L * cd * np.sin(H), atol=1e-9)
    # hour angle 0: u is the east-west component
    b = np.array([[10.0, 20.0, 30.0]])
    assert math.isclose(ws.uvw_tracks(b, np.array([0.0]))[0, 0], 20.0, rel_tol=1e-15)


def test_arrays_and_discs():
    a = ws.array_64()
    assert a.shape == (64, 3) and np.all(a[:, 2] == 0)
    r = np.hypot(a[:, 0], a[:, 1])
    assert np.all(r[:45] <= 1000.0) and np.all((r[45:] >= 1000.0) & (r[45:] <= 4000.0))
    assert ws.baseline_vectors(ws.enu_to_xyz(a)).shape == (64 * 63 // 2, 3)
    # uniform in area: a quarter of a disc's points lie inside half its radius
    p = ws.disc_positions(200_000, 0.0, 1.0, np.random.default_rng(3))
    assert abs(np.mean(np.hypot(p[:, 0], p[:, 1]) < 0.5) - 0.25) < 0.005


def test_tiny_and_widefield_recipes():
    t = ws.tiny()
    assert t.uvw_m.shape == (120 * 160, 3) and t.freqs_hz.tolist() == [1.28e9]
    assert (t.nx, t.ny) == (64, 64) and math.isclose(t.cell_rad * 64, math.radians(0.5))
    assert t.sky.shape == (64, 64) and t.sky.min() >= 0
    assert np.array_equal(t.uvw_m, ws.tiny().uvw_m) and np.array_equal(t.sky, ws.tiny().sky)
    w = ws.widefield(n=128, nvis=24_000, fov_deg=4.0, npoints=40, nblobs=3,
                     blob_sigma=(1.0, 3.0))
    assert w.uvw_m.shape == (24_000, 3) and w.uvw_m.flags["C_CONTIGUOUS"]
    assert np.unique(w.uvw_m, axis=0).shape[0] == 24_000


def test_seeded_subset():
    s = ws.seeded_subset(1000, 300, 5)
    assert s.size == 300 and np.all(np.diff(s) > 0) and s[0] >= 0 and s[-1] < 1000
    assert np.array_equal(s, ws.seeded_subset(1000, 300, 5))
    assert not np.array_equal(s, ws.seeded_subset(1000, 300, 6))
    assert np.array_equal(ws.seeded_subset(10, 20, 5), np.arange(10))


def test_noise_levels_lognormal():
    s = ws.noise_sigma(400_000)
    assert s.dtype == np.float32 and np.all(s > 0)
    ls = np.log(s.astype(np.float64))
    assert abs(ls.mean()) < 0.003 and abs(ls.std() - 0.35) < 0.003
    assert np.array_equal(s[:1000], ws.noise_sigma(1000))


@pytest.mark.parametrize("frac,mean_run", [(0.1, 40), (0.05, 10), (0.3, 40)])
def test_flag_runs(frac, mean_run):
    n = 500_000
    m = ws.flag_runs(n, frac, mean_run=mean_run)
    assert m.dtype == bool and m.size == n
    assert np.array_equal(m, ws.flag_runs(n, frac, mean_run=mean_run))
    f = m.mean()
    # at least the target; the last batch of runs overshoots by at most a few runs
    assert frac <= f <= frac + 2e-3
    edges = np.diff(np.concatenate([[0], m.astype(np.int8), [0]]))
    starts, ends = np.nonzero(edges == 1)[0], np.nonzero(edges == -1)[0]
    runs = ends - starts
    # geometric lengths of mean mean_run; overlapping runs merge into longer ones
    assert mean_run * 0.9 <= runs.mean() <= mean_run * (1.0 + 2.5 * frac)


def test_batched_counts_and_small_batched():
    c = ws.batched_counts()
    assert c.size == 16 and c.sum() == 48_000_000
    assert c.min() >= 0.5e6 and c.max() <= 6e6
    assert np.array_equal(c, ws.batched_counts())
    assert c.max() / c.min() > 4   # uneven per-channel counts
    o = ws.batched(n=64, nchan=4, total=40_000, hours=2.0, lo=5_000, hi=15_000)
    assert o.chan_rows.sum() == 40_000 and o.uvw_m.shape == (40_000, 3)
    assert np.allclose(o.freqs_hz, np.linspace(0.9e9, 1.67e9, 4))
    assert np.all((o.chan_rows >= 5_000) & (o.chan_rows <= 15_000))


def test_probes():
    g = ws.gauss_image(256, 9)
    assert g.shape == (256, 256) and abs(g.mean()) < 0.02 and abs(g.std() - 1) < 0.02
    assert np.array_equal(g, ws.gauss_image(256, 9))
    p = ws.complex_probe((1000,), 4)
    assert np.iscomplexobj(p) and np.array_equal(p, ws.complex_probe((1000,), 4))
